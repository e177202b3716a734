"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances: FP64 storage 1e-12 relative on
coefficients and objective; FP32 storage 1e-5 relative (norm-wise) on
coefficients and objective; supports and top-kappa selections bit-exact whenever
the oracle's top-kappa margin is wider than the precision's error bound.
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


LOSS_NAME = {0: "squared", 1: "logistic", 2: "softmax"}


def make_gpu(w, dtype=None, device_data=False):
    bca = _bca()
    dtype = dtype or w.dtype
    P = bca.Problem(LOSS_NAME[w.loss], w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma,
                    rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=dtype)
    for i in range(w.N):
        if device_data:
            import torch
            A = torch.from_numpy(np.ascontiguousarray(w.A[i])).cuda()
            if dtype == "bf16":
                A = A.view(torch.int16)
            b = torch.from_numpy(np.ascontiguousarray(w.b[i], dtype=np.float64)).cuda()
            P.set_data(i, A, b)
        else:
            P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def make_oracle(w):
    return oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                          w.gamma, w.rho_c, w.rho_b, w.rho_l)


# ------------------------------------------------------------------ setup: Gram, Cholesky, inverse
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_cached_inverse_matches_ridge_matrix(dtype):
    """P_ij K_ij = I, with K_ij = rho_l A_ij^T A_ij + (1/(N gamma) + rho_c) I
    formed on the host from the stored data: pins the MFMA Gram, the Cholesky
    factor, the triangular inverse, P = W^T W and its tiled storage together.
    n_j = 150 and 149 span three 64-wide tiles with a ragged tail."""
    w = datagen.linear_workload(21, N=2, m_per=[333, 290], n=299, kappa=5, k_true=5, noise=0.1,
                                n_blocks=2, dtype=dtype, max_iters=3, rho=1.3)
    P = make_gpu(w)
    bounds = oracle.split_columns(w.n, w.n_blocks)
    tol = {"f64": 1e-12, "f32": 1e-5, "bf16": 1e-5}[dtype]
    for i in range(w.N):
        A = datagen.widen(w.A[i])
        for j, (c0, c1) in enumerate(bounds):
            Aj = A[:, c0:c1]
            K = w.rho_l * Aj.T @ Aj + (1.0 / (w.N * w.gamma) + w.rho_c) * np.eye(c1 - c0)
            Kinv = P.inverse(i, j)
            assert np.max(np.abs(Kinv - Kinv.T)) < 1e-14 * np.max(np.abs(Kinv))
            E = Kinv @ K - np.eye(c1 - c0)
            assert np.max(np.abs(E)) < tol, (i, j, np.max(np.abs(E)))
    P.close()


@pytest.mark.parametrize("n,M,rows", [(1201, 2, [1000, 777]), (1300, 2, [1000, 777]),
                                      (1536, 2, [1000, 777]), (700, 1, [1000, 777]),
                                      (1203, 3, [40, 5])],
                         ids=["odd-block-start", "4-byte-block-start", "16-byte-block-start", "one-block",
                              "fewer-rows-than-the-pipeline"])
def test_bf16_gram_tiles_match_ridge_matrix(n, M, rows):
    """The BF16 Gram's 256 x 256 tiles (several tile rows and columns, ragged last
    tiles, block starts at odd, 4-byte and 16-byte aligned columns, row counts not a
    multiple of the 32-row stage, and partitions of fewer rows than the stages in
    flight), through P_ij K_ij = I with K_ij formed on the host from the BF16 data
    widened to FP64 (unit-norm columns, so FP32 accumulation keeps the products
    within 1e-5)."""
    w = datagen.linear_workload(22, N=2, m_per=rows, n=n, kappa=5, k_true=5, noise=0.1,
                                n_blocks=M, dtype="bf16", normalize=True, max_iters=3)
    P = make_gpu(w)
    bounds = oracle.split_columns(w.n, w.n_blocks)
    for i in range(w.N):
        A = datagen.widen(w.A[i])
        for j, (c0, c1) in enumerate(bounds):
            Aj = A[:, c0:c1]
            K = w.rho_l * Aj.T @ Aj + (1.0 / (w.N * w.gamma) + w.rho_c) * np.eye(c1 - c0)
            E = P.inverse(i, j) @ K - np.eye(c1 - c0)
            assert np.max(np.abs(E)) < 1e-5, (i, j, np.max(np.abs(E)))
    P.close()


# ------------------------------------------------------------------ top-kappa
def test_topk_bit_exact_on_ties():
    import torch
    bca = _bca()
    r = np.random.default_rng(5)
    cases = []
    z = np.array([0.0, -0.0, 3.0, -3.0, 3.0, 1e-310, -1e-310, 2.0, 5e-324, -2.0])
    cases += [(z, k) for k in range(1, len(z) + 1)]
    cases.append((np.full(3001, -1.5), 7))
    v = np.round(r.standard_normal(5000), 1)          # many exact ties
    cases += [(v, 1), (v, 50), (v, 2500), (v, 4999), (v, 5000)]
    v2 = r.standard_normal(70000)
    cases += [(v2, 1000)]
    # mostly zeros: fewer nonzero entries than kappa (threshold 0, lowest-index zeros
    # kept), exactly kappa nonzero entries, and one fewer
    v3 = np.zeros(60000)
    v3[r.choice(60000, 1000, replace=False)] = r.standard_normal(1000)
    cases += [(v3, 3000), (v3, 1000), (v3, 999), (v3, 1001)]
    for z, k in cases:
        ref = oracle.topk_support(z, k)
        for dt in (torch.float64, torch.float32):
            zz = z.astype(np.float32) if dt == torch.float32 else z
            if dt == torch.float32:
                ref = oracle.topk_support(zz.astype(np.float64), k)
            got = bca.topk(torch.from_numpy(np.ascontiguousarray(zz)).cuda(), k).cpu().numpy()
            assert np.array_equal(got, ref), (len(z), k, dt)


# ------------------------------------------------------------------ config 0 (FP64)
def test_config0_one_outer_iteration_state_matches():
    bca = _bca()
    w = datagen.config0()
    P = make_gpu(w)
    o = make_oracle(w)
    for k in range(3):
        P.step(1)
        o.iterate(1, w.inner_iters)
        st = o.state
        for i in range(w.N):
            assert rel(P.get_vector(bca.VEC_X, i), st.x[i]) < 1e-12
            assert rel(P.get_vector(bca.VEC_U, i), st.u[i]) < 1e-12
            assert rel(P.get_vector(bca.VEC_OMEGA, i), st.omega[i]) < 1e-12
            assert rel(P.get_vector(bca.VEC_NU, i), st.nu[i]) < 1e-12
        assert rel(P.get_vector(bca.VEC_Z), st.z) < 1e-12
        assert rel(P.get_vector(bca.VEC_S), st.s) < 1e-12
        t, v = P.get_vector(bca.VEC_TV)
        assert abs(t - st.t) <= 1e-12 * max(1, abs(st.t)) and abs(v - st.v) <= 1e-12 * max(1, abs(st.v))
        pr, dr, br, it = P.residuals()
        assert it == k + 1
        opr, odr, obr = st.history[-1]
        assert abs(pr - opr) <= 1e-11 * max(1, opr) and abs(dr - odr) <= 1e-11 * max(1, odr)
        assert abs(br - obr) <= 1e-11 * max(1, abs(obr))
    P.close()


def test_config0_full_run_parity():
    w = datagen.config0()
    P = make_gpu(w)
    P.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    assert o.topk_margin() > 1e-6
    assert np.array_equal(P.support(), o.support())
    assert_coef_close(P.coef(), o.coef(), 1e-12)
    f = P.objective()
    fo = o.objective(o.coef())
    assert abs(f - fo) <= 1e-12 * abs(fo)
    h, ho = P.history(), np.array(o.state.history)
    assert h.shape == ho.shape
    assert np.max(np.abs(h - ho) / np.maximum(np.abs(ho), 1e-3)) < 1e-9
    P.close()


def test_config0_solve_stops_on_tolerance():
    bca = _bca()
    w = datagen.config0()
    P = bca.Problem("squared", w.n, w.rows, w.n_blocks, w.kappa, max_iters=200, dtype="f64",
                    tol=(0.05, 1e-3, 0.01), check_every=5)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    k, conv = P.solve()
    assert conv and k % 5 == 0 and k < 200
    pr, dr, br, it = P.residuals()
    assert it == k and pr <= 0.05 and dr <= 1e-3 and br <= 0.01
    P.close()


# ------------------------------------------------------------------ FP32 logistic (config-1 recipe, small)
def test_logistic_f32_parity_small():
    w = datagen.logistic_workload(31, N=3, m_per=[701, 650, 613], n=531, kappa=12, k_true=12,
                                  n_blocks=4, dtype="f32", max_iters=30)
    P = make_gpu(w)
    P.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    margin = o.topk_margin()
    assert margin > 1e-4, margin
    assert np.array_equal(P.support(), o.support())
    assert_coef_close(P.coef(), o.coef(), 1e-5)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= 1e-5 * abs(fo)
    P.close()


def test_table1_recipe_dense_support_parity():
    """The recipe of the paper's Table 1 shapes (unit-norm columns per partition,
    kappa = 0.4 n with a planted model of that many nonzeros) at a size the oracle
    finishes in seconds: FP32, one feature block (n_j = 200: four 64-wide tiles of the
    cached inverse, the last one ragged), a top-kappa that keeps 40 % of the entries."""
    w = datagen.linear_workload(5, N=4, m_per=[500, 500, 500, 500], n=200, kappa=80, k_true=80,
                                noise=0.05, n_blocks=1, dtype="f32", normalize=True, max_iters=30)
    P = make_gpu(w)
    P.step(w.max_iters)
    o = make_oracle(w)
    o.iterate(w.max_iters, w.inner_iters)
    assert o.topk_margin() > 1e-4
    assert np.array_equal(P.support(), o.support())
    assert np.array_equal(P.support(), np.nonzero(w.x_true)[0])
    assert_coef_close(P.coef(), o.coef(), 1e-5)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= 1e-5 * abs(fo)
    P.close()


def test_squared_f32_device_input_matches_host_input():
    w = datagen.linear_workload(41, N=2, m_per=[400, 377], n=130, kappa=6, k_true=6, noise=0.05,
                                n_blocks=3, dtype="f32", max_iters=20)
    P1 = make_gpu(w)
    P2 = make_gpu(w, device_data=True)
    P1.step(20)
    P2.step(20)
    assert np.array_equal(P1.coef(), P2.coef())
    assert np.array_equal(P1.history(), P2.history())
    P1.close()
    P2.close()


def test_bitwise_determinism_and_checkpoint_resume():
    bca = _bca()
    w = datagen.logistic_workload(51, N=2, m_per=[300, 280], n=97, kappa=5, k_true=5,
                                  n_blocks=2, dtype="f32", max_iters=20)
    A = make_gpu(w)
    A.step(10)
    blob = A.get_state()
    A.step(10)
    B = make_gpu(w)
    B.step(20)
    assert np.array_equal(A.get_vector(bca.VEC_Z), B.get_vector(bca.VEC_Z))
    assert np.array_equal(A.history(), B.history())
    C = make_gpu(w)
    C.set_state(blob)
    C.step(10)
    assert np.array_equal(C.get_vector(bca.VEC_Z), A.get_vector(bca.VEC_Z))
    for i in range(w.N):
        assert np.array_equal(C.get_vector(bca.VEC_X, i), A.get_vector(bca.VEC_X, i))
        assert np.array_equal(C.get_vector(bca.VEC_NU, i), A.get_vector(bca.VEC_NU, i))
    assert np.array_equal(C.history(), A.history())
    for P in (A, B, C):
        P.close()


def test_set_state_rejects_inconsistent_blobs():
    """The state blob's iteration count indexes the residual history on the device:
    a negative count, a count that disagrees with the stored scalar copy, and
    non-finite scalars are refused (BCA_E_INVALID) before anything is uploaded."""
    import struct
    bca = _bca()
    w = datagen.linear_workload(52, N=2, m_per=[120, 100], n=40, kappa=4, k_true=4, noise=0.05,
                                n_blocks=2, dtype="f64", max_iters=6)
    P = make_gpu(w)
    P.step(2)
    blob = bytearray(P.get_state())
    # header: magic u64, n C N kappa i32, m_total i64, iter hist_cap i32, scal[8] f64
    assert struct.unpack_from("<i", blob, 32)[0] == 2 and struct.unpack_from("<d", blob, 80)[0] == 2.0
    bad = []
    b1 = bytearray(blob); struct.pack_into("<i", b1, 32, -1); struct.pack_into("<d", b1, 80, -1.0)
    b2 = bytearray(blob); struct.pack_into("<d", b2, 80, 5.0)
    b3 = bytearray(blob); struct.pack_into("<d", b3, 40, float("nan"))
    for b in (b1, b2, b3):
        with pytest.raises(bca.BcaError) as e:
            P.set_state(bytes(b))
        assert e.value.code == -1
    P.set_state(bytes(blob))              # the untouched blob is still accepted
    assert P.residuals()[3] == 2
    P.close()


def test_error_paths():
    bca = _bca()
    w = datagen.linear_workload(61, N=2, m_per=50, n=20, kappa=3, k_true=3, noise=0.1,
                                n_blocks=2, dtype="f64", max_iters=5)
    P = bca.Problem("squared", w.n, w.rows, 2, 3, dtype="f64", max_iters=5)
    with pytest.raises(bca.BcaError) as e:
        P.step(1)
    assert e.value.code == -3
    with pytest.raises(bca.BcaError) as e:
        P.finalize()
    assert e.value.code == -3
    A = w.A[0].copy()
    A[3, 4] = np.nan
    with pytest.raises(bca.BcaError) as e:
        P.set_data(0, A, w.b[0])
    assert e.value.code == -4
    with pytest.raises(bca.BcaError) as e:
        bca.Problem("squared", 20, [50, 50], 2, 0, dtype="f64")
    assert e.value.code == -1
    Q = bca.Problem("logistic", w.n, w.rows, 2, 3, dtype="f64", max_iters=5)
    with pytest.raises(bca.BcaError) as e:
        Q.set_data(0, w.A[0], w.b[0])          # real-valued targets are not labels
    assert e.value.code == -1
    P.close()
    Q.close()


# ------------------------------------------------------------------ softmax (C classes, row sparsity)
def _softmax_gpu(w, dtype):
    bca = _bca()
    P = bca.Problem("softmax", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=dtype, n_classes=w.n_classes)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def _softmax_oracle(w):
    return oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                          w.gamma, w.rho_c, w.rho_b, w.rho_l, n_classes=w.n_classes)


@pytest.mark.parametrize("dtype,C,tol", [("f64", 3, 1e-10), ("f32", 10, 1e-5)])
def test_softmax_parity(dtype, C, tol):
    bca = _bca()
    w = datagen.softmax_workload(71, N=2, m_per=[300, 257], n=150, C=C, kappa=4, k_true=4,
                                 n_blocks=2, dtype=dtype, max_iters=15)
    P = _softmax_gpu(w, dtype)
    o = _softmax_oracle(w)
    P.step(1)
    o.iterate(1, w.inner_iters)
    for i in range(w.N):
        assert rel(P.get_vector(bca.VEC_X, i).reshape(w.n, C), o.state.x[i]) < tol
        assert rel(P.get_vector(bca.VEC_OMEGA, i).reshape(-1, C), o.state.omega[i]) < tol
    assert rel(P.get_vector(bca.VEC_Z).reshape(w.n, C), o.state.z) < tol
    P.step(w.max_iters - 1)
    o.iterate(w.max_iters - 1, w.inner_iters)
    assert o.topk_margin() > 10 * tol
    assert np.array_equal(P.support(), o.support())
    assert_coef_close(P.coef(), o.coef(), tol)
    f, fo = P.objective(), o.objective(o.coef())
    assert abs(f - fo) <= tol * abs(fo)
    h, ho = P.history(), np.array(o.state.history)
    assert np.max(np.abs(h - ho) / np.maximum(np.abs(ho), 1e-2)) < 100 * tol
    P.close()


def test_softmax_rejects_bad_labels_and_shapes():
    bca = _bca()
    with pytest.raises(bca.BcaError) as e:
        bca.Problem("softmax", 3000, [10], 1, 2, dtype="f32", n_classes=4)
    assert e.value.code == -1
    P = bca.Problem("softmax", 20, [30], 2, 2, dtype="f32", n_classes=4)
    y = np.zeros(30, dtype=np.int32)
    y[5] = 4
    with pytest.raises(bca.BcaError) as e:
        P.set_data(0, np.ones((30, 20), dtype=np.float32), y)
    assert e.value.code == -1
    P.close()
