"""Exact x-update (BCA_FLAG_EXACT_X) against the FP64 oracle's exact mode (itself
pinned to Algorithm 2's inner-loop limit, the global ridge solution and, for the
logistic loss, SciPy's trust-region Newton minimiser and the regularised MLE).
Squared loss: the cached H_i^-1, the state after each outer iteration (FP64,
1e-12), a full FP32 run (support exact, coefficients and objective 1e-5), the
nontemporal tile path.  Logistic loss (Newton-CG): the state per outer iteration
and a full run in FP64 (1e-10) and FP32 (1e-5).  Parameter checks.
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
    P = bca.Problem("squared", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=w.dtype, exact_x=True)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def make_oracle(w):
    return oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                          w.gamma, w.rho_c, w.rho_b, w.rho_l, exact_x=True)


def test_exact_inverse_and_state_match_oracle_f64():
    """n = 300 (five 64-wide tiles, the last ragged) over uneven partitions; the
    n_blocks = 3 given is ignored by the exact x-update."""
    bca = _bca()
    w = datagen.linear_workload(71, N=3, m_per=[420, 390, 351], n=300, kappa=9, k_true=9, noise=0.05,
                                n_blocks=3, dtype="f64", max_iters=40)
    P = make(w)
    shift = 1.0 / (w.N * w.gamma) + w.rho_c
    for i in range(w.N):
        A = w.A[i]
        H = 2.0 * A.T @ A + shift * np.eye(w.n)
        Kinv = P.inverse(i, 0)
        assert np.max(np.abs(Kinv @ H - np.eye(w.n))) < 1e-12
    o = make_oracle(w)
    for _ in range(3):
        P.step(1)
        o.iterate(1, w.inner_iters)
        for i in range(w.N):
            assert rel(P.get_vector(bca.VEC_X, i), o.state.x[i]) < 1e-12
            assert rel(P.get_vector(bca.VEC_U, i), o.state.u[i]) < 1e-12
        assert rel(P.get_vector(bca.VEC_Z), o.state.z) < 1e-12
        pr, dr, br, it = P.residuals()
        opr, odr, obr = o.state.history[-1]
        assert abs(pr - opr) <= 1e-11 * max(1, opr) and abs(dr - odr) <= 1e-11 * max(1, odr)
    P.step(w.max_iters - 3)
    o.iterate(w.max_iters - 3, w.inner_iters)
    assert o.topk_margin() > 1e-6
    assert np.array_equal(P.support(), o.support())
    assert_coef_close(P.coef(), o.coef(), 1e-11)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= 1e-11 * abs(fo)
    P.close()


def test_exact_f32_parity():
    w = datagen.linear_workload(72, N=4, m_per=[800, 760, 700, 650], n=530, kappa=10, k_true=10,
                                noise=0.1, n_blocks=1, dtype="f32", normalize=True, max_iters=30)
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


def test_exact_x_parameter_checks():
    bca = _bca()
    with pytest.raises(bca.BcaError):
        bca.Problem("hinge", 20, [50], 1, 3, dtype="f64", exact_x=True)
    w = datagen.linear_workload(73, N=2, m_per=[60, 55], n=20, kappa=3, k_true=3, noise=0.05,
                                n_blocks=1, dtype="f64", max_iters=5)
    P = make(w)
    with pytest.raises(bca.BcaError):
        bca.batch_solve([P])
    P.close()


def test_exact_nontemporal_tile_path_matches_oracle():
    """With more than 1 GB of H_i^-1 tiles the symmetric product reads them with
    nontemporal loads (the path the precision-sized exact runs take): 2 partitions of
    n = 11,600 (182 tiles per side, 2 x 16,653 stored 64 x 64 FP64 tiles = 1.09 GB),
    FP64 data with unit-norm columns (cond(H_i) about 100, so the explicitly inverted
    H_i^-1 is accurate to FP64 level), state against the oracle's exact mode at 1e-11
    over three outer iterations."""
    bca = _bca()
    w = datagen.linear_workload(74, N=2, m_per=[300, 277], n=11600, kappa=40, k_true=40,
                                noise=0.05, n_blocks=1, dtype="f64", normalize=True, max_iters=3)
    tiles = 2 * (182 * 183 // 2) * 64 * 64 * 8
    assert tiles > (1 << 30)
    P = make(w)
    o = make_oracle(w)
    for _ in range(3):
        P.step(1)
        o.iterate(1, w.inner_iters)
        for i in range(w.N):
            assert rel(P.get_vector(bca.VEC_X, i), o.state.x[i]) < 1e-11
        assert rel(P.get_vector(bca.VEC_Z), o.state.z) < 1e-11
        pr, dr, br, it = P.residuals()
        opr, odr, obr = o.state.history[-1]
        assert abs(pr - opr) <= 1e-10 * max(1, opr) and abs(dr - odr) <= 1e-10 * max(1, odr)
    P.close()


# ------------------------------------------------------------------ logistic: Newton-CG
def make_logistic(w):
    bca = _bca()
    P = bca.Problem("logistic", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=w.dtype, exact_x=True)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def test_exact_logistic_state_matches_oracle_f64():
    """Logistic exact x-update (Newton's method on each partition's whole x-subproblem,
    conjugate gradients preconditioned with (A_i^T A_i / 4 + s I)^-1 on the GPU, exact
    Hessian solves in the oracle) on uneven partitions, one of them with fewer rows than
    features: x, u, z after each of the first outer iterations and the final support,
    coefficients and objective against the oracle's exact mode, FP64 at 1e-10."""
    bca = _bca()
    w = datagen.logistic_workload(75, N=3, m_per=[420, 390, 150], n=230, kappa=9, k_true=9,
                                  n_blocks=1, dtype="f64", max_iters=25)
    P = make_logistic(w)
    o = make_oracle(w)
    for _ in range(3):
        P.step(1)
        o.iterate(1, w.inner_iters)
        for i in range(w.N):
            assert rel(P.get_vector(bca.VEC_X, i), o.state.x[i]) < 1e-10
            assert rel(P.get_vector(bca.VEC_U, i), o.state.u[i]) < 1e-10
        assert rel(P.get_vector(bca.VEC_Z), o.state.z) < 1e-10
    P.step(w.max_iters - 3)
    o.iterate(w.max_iters - 3, w.inner_iters)
    assert o.topk_margin() > 1e-6
    assert np.array_equal(P.support(), o.support())
    assert_coef_close(P.coef(), o.coef(), 1e-10)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= 1e-10 * abs(fo)
    P.close()


def test_exact_logistic_f32_parity():
    """The same in FP32 storage on the sparse logistic recipe (AR(1) rows): support
    exact, coefficients and objective within 1e-5 of the FP64 oracle."""
    w = datagen.logistic_workload(76, N=4, m_per=[900, 820, 760, 700], n=300, kappa=12, k_true=12,
                                  n_blocks=1, dtype="f32", max_iters=20)
    P = make_logistic(w)
    P.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    assert o.topk_margin() > 1e-4
    assert np.array_equal(P.support(), o.support())
    assert_coef_close(P.coef(), o.coef(), 1e-5)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= 1e-5 * abs(fo)
    P.close()
