"""Sample-space (Woodbury) x_ij-step (BCA_FLAG_WOODBURY) against the FP64 oracle's
Algorithm 2 as written: the form computes the same iterates through
S_ij = rho_l A_ij A_ij^T + shift I (m_i x m_i) instead of K_ij (n_j x n_j), so
the oracle needs no mode of its own.  Every sample-space sum is carried in FP64
from the exactly widened stored values, so FP32 and BF16 storage are compared
with FP64 tolerances on the widened data; the cases have m_i < n_j, partitions
of uneven height (rows padded to the tallest in the sample-space layout) that
span several 64-row tiles with a ragged tail, and more than one feature block.
"""
import numpy as np
import pytest

import datagen
import oracle
from parity import assert_coef_close, rel

pytestmark = pytest.mark.gpu

LOSS_NAME = {0: "squared", 1: "logistic", 3: "hinge"}


def _bca():
    import paper_2405_16267_amd as bca
    return bca


def make(w, woodbury=True, dtype=None):
    bca = _bca()
    P = bca.Problem(LOSS_NAME[w.loss], w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma,
                    rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=dtype or w.dtype, woodbury=woodbury)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def make_oracle(w):
    return oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                          w.gamma, w.rho_c, w.rho_b, w.rho_l)


def _final_matches(P, o, tol, dtype):
    """z to tol; support and x_hat whenever the oracle's top-kappa margin is
    wider than the FP64-level error (else the selection is a tie).  The objective
    pass forms A x_hat with products in the storage's arithmetic type (FP32 for
    FP32 and BF16 storage), so f(x_hat) is held to the FP32 bar, 1e-5, there."""
    bca = _bca()
    assert rel(P.get_vector(bca.VEC_Z), o.state.z) < tol
    if o.topk_margin() > 1e-8:
        assert np.array_equal(P.support(), o.support())
        assert_coef_close(P.coef(), o.coef(), tol)
        f, fo = P.objective(), o.objective(o.coef())
        assert abs(f - fo) <= (tol if dtype == "f64" else 1e-5) * abs(fo)


def _state_matches(P, o, w, tol):
    bca = _bca()
    for i in range(w.N):
        assert rel(P.get_vector(bca.VEC_X, i), o.state.x[i]) < tol
        assert rel(P.get_vector(bca.VEC_U, i), o.state.u[i]) < tol
        assert rel(P.get_vector(bca.VEC_OMEGA, i), o.state.omega[i]) < tol
        assert rel(P.get_vector(bca.VEC_NU, i), o.state.nu[i]) < tol
    assert rel(P.get_vector(bca.VEC_Z), o.state.z) < tol


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_woodbury_squared_state_matches_each_outer_iteration(dtype):
    """m_i = 130, 101, 77 (three, two and two 64-row tiles, all ragged) under
    n_j = 150, 150 of n = 300."""
    w = datagen.linear_workload(81, N=3, m_per=[130, 101, 77], n=300, kappa=8, k_true=8,
                                noise=0.05, n_blocks=2, dtype=dtype, max_iters=40)
    P = make(w)
    o = make_oracle(w)
    for _ in range(3):
        P.step(1)
        o.iterate(1, w.inner_iters)
        _state_matches(P, o, w, 1e-10)
        pr, dr, br, it = P.residuals()
        opr, odr, obr = o.state.history[-1]
        assert abs(pr - opr) <= 1e-9 * max(1, opr) and abs(dr - odr) <= 1e-9 * max(1, odr)
    P.step(w.max_iters - 3)
    o.iterate(w.max_iters - 3, w.inner_iters)
    assert o.topk_margin() > 1e-8
    _final_matches(P, o, 1e-9, dtype)
    P.close()


def test_woodbury_logistic_f32_parity():
    w = datagen.logistic_workload(82, N=4, m_per=[210, 190, 171, 150], n=900, kappa=12,
                                  k_true=12, n_blocks=3, dtype="f32", max_iters=30)
    P = make(w)
    P.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    _final_matches(P, o, 1e-9, w.dtype)
    P.close()


def test_woodbury_hinge_bf16_parity():
    """BF16 storage: the oracle runs on the stored BF16 values widened to FP64."""
    w = datagen.svm_workload(83, N=2, m_per=[140, 129], n=400, kappa=10, k_true=10, n_blocks=2,
                             dtype="bf16", max_iters=25)
    P = make(w)
    P.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    _final_matches(P, o, 1e-9, w.dtype)
    P.close()


def test_woodbury_matches_default_form_at_feature_scaling_shape():
    """The paper's feature-scaling shape (partitions of 800 rows, one block of
    n = 4,000 columns, kappa = 0.2 n), FP32: the sample-space form against the
    oracle and against the default form (n_j x n_j inverse, FP32 products)."""
    w = datagen.linear_workload(84, N=4, m_per=[800, 800, 800, 800], n=4000, kappa=800,
                                k_true=800, noise=0.05, n_blocks=1, dtype="f32", normalize=True,
                                max_iters=15)
    P = make(w)
    Q = make(w, woodbury=False)
    P.step(w.max_iters)
    Q.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    bca = _bca()
    _final_matches(P, o, 1e-9, w.dtype)
    assert rel(Q.get_vector(bca.VEC_Z), o.state.z) < 1e-5
    P.close()
    Q.close()


def test_woodbury_checkpoint_resume_is_bitwise():
    """Every outer iteration re-derives d = A_ij x_ij + e from the state a
    checkpoint holds, so runs resumed from one equal the uninterrupted run bit
    for bit."""
    bca = _bca()
    w = datagen.logistic_workload(85, N=2, m_per=[120, 99], n=260, kappa=6, k_true=6,
                                  n_blocks=2, dtype="f32", max_iters=20)
    A = make(w)
    A.step(10)
    blob = A.get_state()
    A.step(10)
    B = make(w)
    B.step(20)
    assert np.array_equal(A.history(), B.history())
    assert np.array_equal(A.get_vector(bca.VEC_Z), B.get_vector(bca.VEC_Z))
    C = make(w)
    C.set_state(blob)
    C.step(10)
    assert np.array_equal(C.get_vector(bca.VEC_Z), A.get_vector(bca.VEC_Z))
    for i in range(w.N):
        assert np.array_equal(C.get_vector(bca.VEC_X, i), A.get_vector(bca.VEC_X, i))
        assert np.array_equal(C.get_vector(bca.VEC_NU, i), A.get_vector(bca.VEC_NU, i))
    for P in (A, B, C):
        P.close()


def test_woodbury_parameter_checks():
    bca = _bca()
    with pytest.raises(bca.BcaError):
        bca.Problem("softmax", 20, [50], 1, 3, dtype="f64", n_classes=3, woodbury=True)
    with pytest.raises(bca.BcaError):
        bca.Problem("squared", 20, [50], 1, 3, dtype="f64", exact_x=True, woodbury=True)
    w = datagen.linear_workload(86, N=2, m_per=[30, 25], n=80, kappa=3, k_true=3, noise=0.05,
                                n_blocks=2, dtype="f64", max_iters=5)
    P = make(w)
    with pytest.raises(bca.BcaError):
        P.inverse(0, 0)
    with pytest.raises(bca.BcaError):
        bca.batch_solve([P])
    P.close()


def test_woodbury_edge_shapes_f64():
    """A one-row partition beside one of exactly one 64-row tile (mw = 64), and
    three ragged feature blocks (44, 43, 43 of n = 130): state after each outer
    iteration against the oracle."""
    w = datagen.linear_workload(87, N=2, m_per=[1, 64], n=130, kappa=4, k_true=4, noise=0.05,
                                n_blocks=3, dtype="f64", max_iters=6)
    P = make(w)
    o = make_oracle(w)
    for _ in range(w.max_iters):
        P.step(1)
        o.iterate(1, w.inner_iters)
        _state_matches(P, o, w, 1e-10)
    P.close()


def test_woodbury_all_zero_data_stays_at_zero():
    """A = 0 and b = 0: S_ij = shift I, and every iterate stays exactly zero."""
    bca = _bca()
    rows = [70, 33]
    P = bca.Problem("squared", 90, rows, 2, 5, dtype="f32", max_iters=5, woodbury=True)
    for i, m in enumerate(rows):
        P.set_data(i, np.zeros((m, 90), dtype=np.float32), np.zeros(m))
    P.finalize()
    P.step(5)
    assert not np.any(P.get_vector(bca.VEC_Z))
    for i in range(len(rows)):
        assert not np.any(P.get_vector(bca.VEC_X, i))
        assert not np.any(P.get_vector(bca.VEC_NU, i))
    pr, dr, br, it = P.residuals()
    assert (pr, dr, br, it) == (0.0, 0.0, 0.0, 5)
    assert np.array_equal(P.support(), np.arange(5))   # ties go to the lowest indices
    P.close()


def test_woodbury_full_size_matches_default_form():
    """The benchmark shape of the sample-space form (8 partitions of 800 x 10,000
    FP32, one block, kappa = 2,000), where the oracle's 10,000 x 10,000 factors are
    too slow for a test: against the default form on the GPU, a property that
    holds at any size (the two forms compute the same iterates up to rounding)."""
    bca = _bca()
    N, m, n, kappa = 8, 800, 10000, 2000
    supp, val = datagen.linear_model(31, n, kappa)
    probs = []
    for wb in (True, False):
        P = bca.Problem("squared", n, [m] * N, 1, kappa, dtype="f32", max_iters=10, woodbury=wb)
        for i in range(N):
            A, b = datagen.linear_partition(31, i, m, n, supp, val, 0.05, "f32", True)
            P.set_data(i, A, b)
        P.finalize()
        P.step(10)
        probs.append(P)
    W, D = probs
    assert rel(D.get_vector(bca.VEC_Z), W.get_vector(bca.VEC_Z)) < 1e-5
    for i in (0, N - 1):
        assert rel(D.get_vector(bca.VEC_X, i), W.get_vector(bca.VEC_X, i)) < 1e-5
    hw, hd = W.history(), D.history()
    assert np.allclose(hw, hd, rtol=1e-3, atol=1e-6)
    for P in probs:
        P.close()


@pytest.mark.parametrize("woodbury", [False, True])
def test_rho_b_study_regime_f64(woodbury):
    """The recipe of the paper's rho_b study (unit-norm columns, kappa = 0.2 n planted
    nonzeros) at its largest penalties, rho_b = 16 and rho_c = rho_l = 32, on a size
    the oracle finishes in seconds (4 partitions of 90 rows, n = 200, one block, so
    m_i < n_j): the default and the sample-space x-step against the oracle after
    every outer iteration."""
    w = datagen.linear_workload(21, N=4, m_per=[90, 90, 90, 90], n=200, kappa=40, k_true=40,
                                noise=0.05, n_blocks=1, dtype="f64", normalize=True, max_iters=8,
                                rho=32.0)
    w.rho_b = 16.0
    P = make(w, woodbury=woodbury)
    o = make_oracle(w)
    for _ in range(w.max_iters):
        P.step(1)
        o.iterate(1, w.inner_iters)
        _state_matches(P, o, w, 1e-10)
    P.close()
