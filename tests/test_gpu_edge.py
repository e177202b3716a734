"""Edge cases of the plain and batched paths against the FP64 oracle: a single
partition and a single feature block, partitions with fewer rows than a tile,
one feature, kappa = n (the l0 constraint inactive), all-zero data (every |z|
tied: the support is the kappa lowest indices), and the largest block width of
the batched form."""
import numpy as np
import pytest

import datagen
import oracle
from datagen import Workload
from parity import assert_coef_close, rel

pytestmark = pytest.mark.gpu

LOSS_NAME = {0: "squared", 1: "logistic", 2: "softmax"}


def _bca():
    import paper_2405_16267_amd as bca
    return bca


def run_gpu(w, iters):
    bca = _bca()
    P = bca.Problem(LOSS_NAME[w.loss], w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma,
                    rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=max(iters, 1), dtype=w.dtype, n_classes=w.n_classes)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    P.step(iters)
    out = dict(support=P.support(), coef=P.coef(), z=P.get_vector(bca.VEC_Z),
               hist=P.history(), objective=P.objective())
    P.close()
    return out


def run_oracle(w, iters):
    o = oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                       w.gamma, w.rho_c, w.rho_b, w.rho_l)
    o.iterate(iters, w.inner_iters)
    return o


def check(w, iters, tol):
    g = run_gpu(w, iters)
    o = run_oracle(w, iters)
    if o.topk_margin() > 1e-6:
        assert np.array_equal(g["support"], o.support())
    assert rel(g["z"], o.state.z) < tol
    assert_coef_close(g["coef"], o.coef(), tol)
    ho = np.array(o.state.history)
    assert np.max(np.abs(g["hist"] - ho) / np.maximum(np.abs(ho), 1e-3)) < 1e3 * tol
    return g, o


def test_single_partition_single_block_f64():
    w = datagen.linear_workload(61, N=1, m_per=[333], n=45, kappa=5, k_true=5, noise=0.01,
                                n_blocks=1, dtype="f64", max_iters=30)
    check(w, 30, 1e-12)


def test_partitions_smaller_than_a_tile_f64():
    # 1, 2 and 5 rows per partition; 7 features in blocks of 3, 2, 2
    w = datagen.linear_workload(62, N=3, m_per=[1, 2, 5], n=7, kappa=2, k_true=2, noise=0.01,
                                n_blocks=3, dtype="f64", max_iters=25)
    check(w, 25, 1e-12)


def test_single_feature_logistic_f64():
    w = datagen.logistic_workload(63, N=2, m_per=[50, 41], n=1, kappa=1, k_true=1, n_blocks=1,
                                  dtype="f64", max_iters=20)
    check(w, 20, 1e-12)


def test_kappa_equals_n_f32():
    w = datagen.linear_workload(64, N=2, m_per=[300, 280], n=40, kappa=40, k_true=8, noise=0.05,
                                n_blocks=2, dtype="f32", max_iters=30)
    g, o = check(w, 30, 1e-5)
    assert len(g["support"]) == 40


def test_all_zero_data_ties_to_lowest_indices():
    n, kappa = 33, 4
    A = [np.zeros((40, n)), np.zeros((37, n))]
    b = [np.zeros(40), np.zeros(37)]
    w = Workload(name="zeros", loss=0, A=A, b=b, n=n, kappa=kappa, n_blocks=3, dtype="f64",
                 max_iters=5)
    g = run_gpu(w, 5)
    o = run_oracle(w, 5)
    assert np.array_equal(g["support"], np.arange(kappa))
    assert np.array_equal(o.support(), np.arange(kappa))
    assert np.all(g["z"] == 0.0) and np.all(g["coef"] == 0.0)
    assert g["objective"] == 0.0


def test_batched_widest_block_matches_solo_f32():
    bca = _bca()
    # n = 2048 FP32: 512 16-byte chunks per row (the widest batched row) and
    # feature blocks of 1024 columns (the widest batched block)
    w = datagen.batched_instance(11, 700, 2048, dtype="f32", max_iters=6)
    w.n_blocks = 2

    def make():
        P = bca.Problem(LOSS_NAME[w.loss], w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma,
                        rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                        max_iters=w.max_iters, dtype=w.dtype)
        for i in range(w.N):
            P.set_data(i, w.A[i], w.b[i])
        P.finalize()
        return P

    B, S = make(), make()
    bca.batch_step([B], 6)
    S.step(6)
    assert rel(B.get_vector(bca.VEC_Z), S.get_vector(bca.VEC_Z)) < 1e-5
    assert np.array_equal(B.support(), S.support())
    B.close()
    S.close()
