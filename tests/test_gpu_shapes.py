"""Oracle parity at the launch shapes the streaming pass takes for wide rows.

The fused streaming pass (block matvecs, sample-space average, prox, nu update,
A_i^T e; Sec. 3.1, Algorithm 2) picks its workgroup shape from the row length:
threads per workgroup x 16-byte chunks per thread.  Full-size workloads run
shapes that small parity cases never reach, so each case below takes few rows
(so the FP64 oracle finishes in seconds) and a row length that selects one of
those shapes:

  BF16 (8 columns per chunk):  n = 10,000 -> 448 x 3 (the precision workload's
    shape), 11,000 -> 512 x 3, 14,000 -> 512 x 4, 20,000 -> 1,024 x 3;
  FP32 (4 columns per chunk):  n = 10,000 -> 512 x 5 (the FP32 side of the
    precision workload), 14,000 -> 1,024 x 4;
  FP64 (2 columns per chunk):  n = 3,500 -> 512 x 4, 7,000 -> 1,024 x 4.

Squared-loss cases take 203 and 170 rows (4-row tiles with a ragged tail).
Each case runs three outer iterations of Algorithm 1 and compares the whole state
with the oracle (BF16 data widened exactly to FP64, reading R21 (i)): z, every
x_i, omega and nu element-wise, the residuals, and the support where the
oracle's top-kappa margin is clear of the tolerance.  Tolerances: FP64 1e-11,
FP32 and BF16 1e-5 (reading R20).

The sampled full-size case runs the precision workload's launch configuration
itself (16 partitions of 100,000 x 10,000, BF16 beside FP32) and recomputes one
partition's x-update and the global step with the oracle from the GPU's state.
"""
import numpy as np
import pytest

import datagen
import oracle
from oracle.bicadmm import LOSS_SQUARED
from parity import assert_coef_close, rel

pytestmark = pytest.mark.gpu

LOSS_NAME = {0: "squared", 1: "logistic"}


def _bca():
    import paper_2405_16267_amd as bca
    return bca


def make_gpu(w):
    bca = _bca()
    P = bca.Problem(LOSS_NAME[w.loss], w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma,
                    rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=w.dtype)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def close_vec(got, ref, tol, what):
    """Norm-wise and element-wise (every entry within tol * ||ref||_inf)."""
    got = np.asarray(got, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    inf = max(float(np.max(np.abs(ref))), 1e-300)
    assert rel(got, ref) <= tol, (what, rel(got, ref))
    assert float(np.max(np.abs(got - ref))) <= tol * inf, (what, float(np.max(np.abs(got - ref))) / inf)


SHAPES = [
    # dtype, n, feature blocks, loss, seed
    ("bf16", 10000, 4, "squared", 81),
    ("bf16", 11000, 4, "squared", 82),
    ("bf16", 14000, 6, "squared", 83),
    ("bf16", 20000, 8, "squared", 84),
    ("f32", 10000, 4, "squared", 85),
    ("f32", 10000, 8, "logistic", 86),
    ("f32", 14000, 6, "squared", 87),
    ("f64", 3500, 2, "squared", 88),
    ("f64", 7000, 3, "squared", 89),
]


@pytest.mark.parametrize("dtype,n,M,loss,seed", SHAPES,
                         ids=["%s-n%d-%s" % (s[0], s[1], s[3]) for s in SHAPES])
def test_wide_row_launch_shapes_match_oracle(dtype, n, M, loss, seed):
    bca = _bca()
    K = 3
    if loss == "squared":
        kappa = 40
        w = datagen.linear_workload(seed, N=2, m_per=[203, 170], n=n, kappa=kappa, k_true=kappa,
                                    noise=0.05, n_blocks=M, dtype=dtype, normalize=True, max_iters=K)
    else:
        # The logistic recipe has no column normalisation: with fewer rows than block
        # columns the row-space eigenvalues of A_ij^T A_ij (about 4,000 at 200 rows)
        # against the shift (1.05) leave K_ij so ill-conditioned that FP32 rounding of the
        # row dots alone moves x by more than 1e-5.  More rows than block columns keep
        # K_ij well conditioned, as in the full-size logistic workload.
        kappa = 30
        w = datagen.logistic_workload(seed, N=2, m_per=[6007, 5990], n=n, kappa=kappa, k_true=kappa,
                                      n_blocks=M, dtype=dtype, max_iters=K)
    tol = 1e-11 if dtype == "f64" else 1e-5
    P = make_gpu(w)
    o = oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                       w.gamma, w.rho_c, w.rho_b, w.rho_l)
    for k in range(K):
        P.step(1)
        o.iterate(1, w.inner_iters)
        st = o.state
        close_vec(P.get_vector(bca.VEC_Z), st.z, tol, "z, iteration %d" % (k + 1))
        for i in range(w.N):
            close_vec(P.get_vector(bca.VEC_X, i), st.x[i], tol, "x_%d, iteration %d" % (i, k + 1))
            close_vec(P.get_vector(bca.VEC_OMEGA, i), st.omega[i], tol, "omega_%d" % i)
            close_vec(P.get_vector(bca.VEC_NU, i), st.nu[i], tol, "nu_%d" % i)
        pr, dr, br, it = P.residuals()
        opr, odr, obr = st.history[-1]
        assert it == k + 1
        assert abs(pr - opr) <= tol * max(1.0, opr) and abs(dr - odr) <= tol * max(1.0, odr)
        assert abs(br - obr) <= tol * max(1.0, abs(obr))
    if o.topk_margin() > 100 * tol * float(np.max(np.abs(o.state.z))):
        assert np.array_equal(P.support(), o.support())
        assert_coef_close(P.coef(), o.coef(), tol)
        f, fo = P.objective(), o.objective(o.coef())
        assert abs(f - fo) <= tol * abs(fo)
    P.close()


# ------------------------------------------------------------------ softmax, MFMA streaming pass
# FP32 and BF16 storage run the multi-class pass on MFMA: the sample-space average
# kernel picks (wavefronts x steps of 32 features) from n -- n = 100 -> 4 x 1,
# 250 -> 4 x 2, 500 -> 4 x 4, 1,000 -> 4 x 8, 2,000 -> 8 x 8 -- and the A^T E
# kernel covers strips of 128 features (a ragged last strip unless 128 divides n)
# and row ranges of at least 256 samples (several per partition here).  Rows are
# at least twice the block width, so that K_ij stays well conditioned.
MC_SHAPES = [
    # dtype, n, C, feature blocks, rows, seed
    ("f32", 100, 3, 2, [700, 531], 91),
    ("f32", 250, 16, 2, [1100, 1037], 92),
    ("f32", 500, 10, 2, [1100, 613], 93),
    ("f32", 1000, 10, 2, [1100, 1037], 94),
    ("f32", 2000, 5, 4, [1100, 1037], 95),
    ("bf16", 1000, 10, 2, [1100, 1037], 96),
    ("bf16", 1930, 7, 4, [1100, 1037], 97),
]


@pytest.mark.parametrize("dtype,n,C,M,rows,seed", MC_SHAPES,
                         ids=["%s-n%d-C%d" % (s[0], s[1], s[2]) for s in MC_SHAPES])
def test_softmax_mfma_launch_shapes_match_oracle(dtype, n, C, M, rows, seed):
    bca = _bca()
    K = 3
    w = datagen.softmax_workload(seed, N=2, m_per=rows, n=n, C=C, kappa=6, k_true=6, n_blocks=M,
                                 dtype=dtype, max_iters=K)
    tol = 1e-5
    P = bca.Problem("softmax", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters, max_iters=w.max_iters,
                    dtype=dtype, n_classes=C)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    o = oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                       w.gamma, w.rho_c, w.rho_b, w.rho_l, n_classes=C)
    for k in range(K):
        P.step(1)
        o.iterate(1, w.inner_iters)
        st = o.state
        close_vec(P.get_vector(bca.VEC_Z), st.z, tol, "z, iteration %d" % (k + 1))
        for i in range(w.N):
            close_vec(P.get_vector(bca.VEC_X, i), st.x[i], tol, "x_%d, iteration %d" % (i, k + 1))
            close_vec(P.get_vector(bca.VEC_OMEGA, i), st.omega[i], tol, "omega_%d" % i)
            close_vec(P.get_vector(bca.VEC_NU, i), st.nu[i], tol, "nu_%d" % i)
    if o.topk_margin() > 100 * tol * float(np.max(np.abs(o.state.z))):
        assert np.array_equal(P.support(), o.support())
        assert_coef_close(P.coef(), o.coef(), tol)
        f, fo = P.objective(), o.objective(o.coef())
        assert abs(f - fo) <= tol * abs(fo)
    P.close()


# ------------------------------------------------------------------ precision workload, sampled
@pytest.fixture(scope="module")
def precision_data():
    """Two partitions of the precision workload's recipe (100,000 x 10,000, unit-norm
    columns, planted 100-sparse model), each drawn once as canonical FP32 and its BF16
    rounding; the 16 partitions of the launch alternate between the two."""
    n, m, kappa = 10000, 100000, 100
    supp, val = datagen.linear_model(2, n, kappa)
    parts = []
    for i in range(2):
        (A32, Abf), b = datagen.linear_partition(2, i, m, n, supp, val, 0.05, "f32+bf16", True)
        parts.append((A32, Abf, b))
    return dict(n=n, m=m, kappa=kappa, parts=parts)


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_precision_workload_full_size_sampled_parity(precision_data, dtype):
    """16 partitions of 100,000 x 10,000 (the precision workload's launch: BF16 rows
    on the 448 x 3 shape, FP32 rows on 512 x 5, 4 feature blocks of 2,500), three
    outer iterations, then a fourth whose partition-0 x-update (Algorithm 2, five
    inner iterations over the full partition) and global step the oracle recomputes
    from the GPU's state before it.  BF16 is compared with the oracle on the BF16
    data widened to FP64 (arithmetic error only) at 1e-5, like FP32."""
    bca = _bca()
    d = precision_data
    n, m, kappa, N, M = d["n"], d["m"], d["kappa"], 16, 4
    P = bca.Problem("squared", n, [m] * N, M, kappa, gamma=10.0, rho_c=1.0, rho_b=0.5, rho_l=1.0,
                    inner_iters=5, max_iters=10, dtype=dtype)
    for i in range(N):
        A32, Abf, b = d["parts"][i % 2]
        P.set_data(i, Abf if dtype == "bf16" else A32, b)
    P.finalize()
    P.step(3)
    before = dict(x=[P.get_vector(bca.VEC_X, i) for i in range(N)],
                  u=[P.get_vector(bca.VEC_U, i) for i in range(N)],
                  z=P.get_vector(bca.VEC_Z), s=P.get_vector(bca.VEC_S), tv=P.get_vector(bca.VEC_TV),
                  om0=P.get_vector(bca.VEC_OMEGA, 0), nu0=P.get_vector(bca.VEC_NU, 0))
    P.step(1)
    after = dict(x=[P.get_vector(bca.VEC_X, i) for i in range(N)],
                 u=[P.get_vector(bca.VEC_U, i) for i in range(N)],
                 z=P.get_vector(bca.VEC_Z), s=P.get_vector(bca.VEC_S), tv=P.get_vector(bca.VEC_TV),
                 om0=P.get_vector(bca.VEC_OMEGA, 0), nu0=P.get_vector(bca.VEC_NU, 0),
                 res=P.residuals())
    P.close()

    A32, Abf, b = d["parts"][0]
    A0 = datagen.widen(Abf if dtype == "bf16" else A32)
    o = oracle.BiCADMM([A0], [b], LOSS_SQUARED, M, kappa, 10.0, 1.0, 0.5, 1.0,
                       n_partitions=N)
    del A0
    st = o.zero_state()
    st.x[0] = before["x"][0]
    st.u = np.array(before["u"])
    st.z = before["z"]
    st.omega[0] = before["om0"]
    st.nu[0] = before["nu0"]
    o.x_update(0, 5, st)
    close_vec(after["x"][0], st.x[0], 1e-5, "x_0")
    close_vec(after["om0"], st.omega[0], 1e-5, "omega_0")
    close_vec(after["nu0"], st.nu[0], 1e-5, "nu_0")

    # the global step at full size from the GPU's x_i of this iteration
    st.x = np.array(after["x"])
    st.u = np.array(before["u"])
    st.z = before["z"]
    st.s = before["s"]
    st.t, st.v = before["tv"]
    pr, dr, br = o.global_update(st)
    close_vec(after["z"], st.z, 1e-9, "z")
    close_vec(np.array(after["u"]), st.u, 1e-9, "u")
    r = np.sort(np.abs(st.z))[::-1]
    if r[kappa - 1] - r[kappa] > 1e-9 * r[0]:
        assert np.array_equal(np.nonzero(after["s"])[0], np.nonzero(st.s)[0])
    close_vec(after["s"], st.s, 1e-9, "s")
    gpr, gdr, gbr, _ = after["res"]
    assert abs(gpr - pr) <= 1e-9 * max(1.0, pr) and abs(gdr - dr) <= 1e-9 * max(1.0, dr)
    assert abs(gbr - br) <= 1e-9 * max(1.0, abs(br))
