"""Sparse SVM (hinge loss) on the GPU against the FP64 oracle.

The hinge loss changes only the per-sample omega-bar prox (a closed form) and
the objective; everything else is the path the other losses take.  Checks: the
state after each of the first outer iterations (FP64, 1e-12), a full FP32 run
(support exact, coefficients and objective 1e-5), label validation, and the
batched form (a hinge problem inside a mix equals its solo run and the oracle).
"""
import numpy as np
import pytest

import datagen
import oracle
from parity import assert_coef_close, rel

pytestmark = pytest.mark.gpu


def _bca():
    import paper_2405_16267_amd as bca
    return bca


def make(w):
    bca = _bca()
    P = bca.Problem("hinge", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=w.dtype)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def make_oracle(w):
    return oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                          w.gamma, w.rho_c, w.rho_b, w.rho_l)


def test_svm_f64_state_matches_each_outer_iteration():
    """Uneven partitions (401, 377, 350 rows) and blocks (75, 75 of n = 150)."""
    bca = _bca()
    w = datagen.svm_workload(61, N=3, m_per=[401, 377, 350], n=150, kappa=8, k_true=8,
                             n_blocks=2, dtype="f64", max_iters=60)
    P = make(w)
    o = make_oracle(w)
    for _ in range(3):
        P.step(1)
        o.iterate(1, w.inner_iters)
        st = o.state
        for i in range(w.N):
            assert rel(P.get_vector(bca.VEC_X, i), st.x[i]) < 1e-12
            assert rel(P.get_vector(bca.VEC_OMEGA, i), st.omega[i]) < 1e-12
            assert rel(P.get_vector(bca.VEC_NU, i), st.nu[i]) < 1e-12
        assert rel(P.get_vector(bca.VEC_Z), st.z) < 1e-12
    P.step(w.max_iters - 3)
    o.iterate(w.max_iters - 3, w.inner_iters)
    assert o.topk_margin() > 1e-6
    assert np.array_equal(P.support(), o.support())
    assert np.array_equal(P.support(), np.nonzero(w.x_true)[0])
    assert_coef_close(P.coef(), o.coef(), 1e-11)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= 1e-11 * abs(fo)
    P.close()


def test_svm_f32_parity():
    """FP32 storage; 4 blocks of n = 531 (133, 133, 133, 132 columns: ragged tiles)."""
    w = datagen.svm_workload(62, N=3, m_per=[701, 650, 613], n=531, kappa=12, k_true=12,
                             n_blocks=4, dtype="f32", max_iters=30)
    P = make(w)
    P.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    assert o.topk_margin() > 1e-4
    assert np.array_equal(P.support(), o.support())
    assert_coef_close(P.coef(), o.coef(), 1e-5)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= 1e-5 * abs(fo)
    P.close()


def test_svm_rejects_labels_other_than_plus_minus_one():
    bca = _bca()
    w = datagen.svm_workload(63, N=1, m_per=[100], n=20, kappa=3, k_true=3, n_blocks=1,
                             dtype="f64", max_iters=5)
    P = bca.Problem("hinge", w.n, w.rows, 1, w.kappa, dtype="f64")
    b = w.b[0].copy()
    b[7] = 0.5
    with pytest.raises(bca.BcaError):
        P.set_data(0, w.A[0], b)
    P.close()


def test_svm_in_batched_mix_matches_solo_and_oracle():
    """A hinge problem batched with a squared and a logistic problem (FP64)."""
    bca = _bca()
    ws = [datagen.svm_workload(64, N=4, m_per=[300, 280, 260, 240], n=90, kappa=6, k_true=6,
                               n_blocks=2, dtype="f64", max_iters=12),
          datagen.batched_instance(0, 700, 53, dtype="f64", max_iters=12),
          datagen.batched_instance(1, 1300, 130, dtype="f64", max_iters=12)]
    names = {0: "squared", 1: "logistic", 3: "hinge"}
    probs = []
    for w in ws:
        P = bca.Problem(names[w.loss], w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma,
                        rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                        max_iters=w.max_iters, dtype=w.dtype)
        for i in range(w.N):
            P.set_data(i, w.A[i], w.b[i])
        P.finalize()
        probs.append(P)
    bca.batch_solve(probs)
    solo = make(ws[0])
    solo.step(ws[0].max_iters)
    o = make_oracle(ws[0])
    o.iterate(ws[0].max_iters, ws[0].inner_iters)
    z = probs[0].get_vector(bca.VEC_Z)
    assert rel(z, solo.get_vector(bca.VEC_Z)) < 1e-12
    assert rel(z, o.state.z) < 1e-12
    assert np.array_equal(probs[0].support(), o.support())
    for P in probs + [solo]:
        P.close()
