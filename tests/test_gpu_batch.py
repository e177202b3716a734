"""Batched form: many uneven problems in one persistent launch.

Checks: each problem of a batch matches its solo run of the one-problem path
(FP64 1e-12, FP32 1e-5) and the FP64 oracle; a problem gives the same bits alone
and inside a mix; the tile-shape autotuner leaves the ADMM state untouched.
"""
import numpy as np
import pytest

import datagen
import oracle
from parity import assert_coef_close, rel

pytestmark = pytest.mark.gpu

LOSS_NAME = {0: "squared", 1: "logistic"}


def _bca():
    import paper_2405_16267_amd as bca
    return bca


def make(w):
    bca = _bca()
    P = bca.Problem(LOSS_NAME[w.loss], w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma,
                    rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=w.dtype)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def mix(dtype="f32", K=12):
    specs = [(0, 700, 53), (1, 1300, 130), (2, 4100, 517), (3, 950, 1100), (4, 2600, 260),
             (5, 520, 77)]
    out = []
    for r, m, n in specs:
        w = datagen.batched_instance(r, m, n, dtype=dtype, max_iters=K)
        out.append(w)
    return out


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
def test_batch_matches_solo_runs(dtype, tol):
    bca = _bca()
    ws = mix(dtype)
    if dtype == "f64":
        ws = [w for w in ws if w.n <= 1024]
    batch = [make(w) for w in ws]
    solo = [make(w) for w in ws]
    bca.batch_step(batch, 12)
    for w, B, S in zip(ws, batch, solo):
        S.step(12)
        assert B.residuals()[3] == 12
        hb, hs = B.history(), S.history()
        assert hb.shape == hs.shape == (12, 3)
        assert np.max(np.abs(hb - hs) / np.maximum(np.abs(hs), 1e-2)) < 100 * tol, w.name
        assert rel(B.get_vector(bca.VEC_Z), S.get_vector(bca.VEC_Z)) < tol, w.name
        assert np.array_equal(B.support(), S.support()), w.name
    for P in batch + solo:
        P.close()


def test_batch_problem_alone_equals_in_mix():
    bca = _bca()
    ws = mix("f32", K=8)
    alone = make(ws[2])
    together = [make(w) for w in ws]
    bca.batch_step([alone], 8)
    bca.batch_step(together, 8)
    assert np.array_equal(alone.get_vector(bca.VEC_Z), together[2].get_vector(bca.VEC_Z))
    assert np.array_equal(alone.history(), together[2].history())
    for i in range(ws[2].N):
        assert np.array_equal(alone.get_vector(bca.VEC_NU, i), together[2].get_vector(bca.VEC_NU, i))
    for P in [alone] + together:
        P.close()


def test_batch_against_oracle_f64():
    bca = _bca()
    w = datagen.batched_instance(6, 1200, 90, dtype="f64", max_iters=20)
    P = make(w)
    bca.batch_step([P], 7)
    bca.batch_step([P], 13)          # two launches: the state carries over
    o = oracle.BiCADMM(w.A, w.b, w.loss, w.n_blocks, w.kappa, w.gamma, w.rho_c, w.rho_b, w.rho_l)
    o.iterate(20, w.inner_iters)
    assert rel(P.get_vector(bca.VEC_Z), o.state.z) < 1e-12
    assert np.array_equal(P.support(), o.support())
    h, ho = P.history(), np.array(o.state.history)
    assert np.max(np.abs(h - ho) / np.maximum(np.abs(ho), 1e-3)) < 1e-9
    P.close()


# Every batched tile shape (chunks per lane NC, rows per tile R, segments per
# wavefront S) forced on an FP32 instance whose row length selects it: S = 4 for
# n <= 64, S = 2 for n <= 128, NC = 1, 2, 4, 8 up to n = 256, 512, 1024, 2048.
SHAPE_CASES = [(60, R) for R in (1, 2, 4, 8)] + [(120, R) for R in (1, 2, 4, 8)] + \
              [(250, R) for R in (1, 2, 4, 8)] + [(500, R) for R in (1, 2, 4)] + \
              [(1000, R) for R in (1, 2)] + [(2000, 1)]


def test_batch_every_tile_shape_against_oracle_f32():
    """One persistent launch over 18 FP32 instances (squared and logistic), each
    forced onto its own tile shape and rows per item (16, 32, 64, 256, 1024 in turn), against
    the FP64 oracle: z element-wise at 1e-5, the support where the oracle's top-kappa
    margin is clear of that, coefficients and objective at 1e-5 (reading R20)."""
    bca = _bca()
    K = 10
    ws, P = [], []
    for q, (n, R) in enumerate(SHAPE_CASES):
        m = 2400 + 131 * q
        w = datagen.batched_instance(40 + q, m, n, dtype="f32", max_iters=K)
        p = make(w)
        p.set_batch_shape(R, (16, 32, 64, 256, 1024)[q % 5])
        assert p.batch_shape() == (R, (16, 32, 64, 256, 1024)[q % 5])
        ws.append(w)
        P.append(p)
    bca.batch_step(P, K)
    for w, p in zip(ws, P):
        o = oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                           w.gamma, w.rho_c, w.rho_b, w.rho_l)
        o.iterate(K, w.inner_iters)
        z, oz = p.get_vector(bca.VEC_Z), o.state.z
        inf = float(np.max(np.abs(oz)))
        assert rel(z, oz) < 1e-5 and float(np.max(np.abs(z - oz))) <= 1e-5 * inf, (w.name, p.batch_shape())
        if o.topk_margin() > 1e-3 * inf:
            assert np.array_equal(p.support(), o.support()), w.name
            assert_coef_close(p.coef(), o.coef(), 1e-5, w.name)
            f, fo = p.objective(), o.objective(o.coef())
            assert abs(f - fo) <= 1e-5 * abs(fo), w.name
        h, ho = p.history(), np.array(o.state.history)
        assert np.max(np.abs(h - ho) / np.maximum(np.abs(ho), 1e-2)) < 1e-3, w.name
    for p in P:
        p.close()


def test_batch_respects_each_max_iters_and_mixes_with_plain_steps():
    bca = _bca()
    a = datagen.batched_instance(8, 800, 64, dtype="f64", max_iters=5)
    b = datagen.batched_instance(9, 900, 70, dtype="f64", max_iters=9)
    A, B = make(a), make(b)
    bca.batch_solve([A, B])
    assert A.residuals()[3] == 5 and B.residuals()[3] == 9
    # plain and batched steps interleave on one problem
    C = make(b)
    C.step(4)
    bca.batch_step([C], 3)
    C.step(2)
    assert C.residuals()[3] == 9
    assert rel(C.get_vector(bca.VEC_Z), B.get_vector(bca.VEC_Z)) < 1e-12
    for P in (A, B, C):
        P.close()


def test_batch_autotune_keeps_state_and_results():
    bca = _bca()
    ws = mix("f32", K=6)
    P = [make(w) for w in ws]
    Q = [make(w) for w in ws]
    bca.batch_step(P, 3)
    bca.batch_step(Q, 3)
    z_before = [p.get_vector(bca.VEC_Z) for p in P]
    bca.batch_autotune(P)
    for p, zb in zip(P, z_before):
        assert np.array_equal(p.get_vector(bca.VEC_Z), zb)
        t, i = p.batch_shape()
        assert t in (1, 2, 4, 8) and i in (16, 32, 64, 256, 1024)
    bca.batch_step(P, 3)
    bca.batch_step(Q, 3)
    for w, p, q in zip(ws, P, Q):
        assert rel(p.get_vector(bca.VEC_Z), q.get_vector(bca.VEC_Z)) < 1e-5
        # the autotuned shapes against the oracle
        o = oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                           w.gamma, w.rho_c, w.rho_b, w.rho_l)
        o.iterate(6, w.inner_iters)
        z, oz = p.get_vector(bca.VEC_Z), o.state.z
        assert rel(z, oz) < 1e-5 and float(np.max(np.abs(z - oz))) <= 1e-5 * float(np.max(np.abs(oz))), w.name
    for x in P + Q:
        x.close()


def test_batch_rejects_out_of_scope_problems():
    bca = _bca()
    w = datagen.softmax_workload(3, N=2, m_per=40, n=20, C=3, kappa=2, k_true=2, n_blocks=2)
    S = bca.Problem("softmax", w.n, w.rows, 2, 2, dtype="f32", n_classes=3)
    for i in range(2):
        S.set_data(i, w.A[i], w.b[i])
    S.finalize()
    with pytest.raises(bca.BcaError) as e:
        bca.batch_step([S], 1)
    assert e.value.code == -1
    S.close()


def test_batch_phase_tracing_accounts_for_the_launch():
    """Phase tracing (bca_batch_set_tracing): every phase kind of the launches made
    while it is on is summed, the sums cover the launches' duration (one timestamp
    per grid barrier; the host side of a launch is outside them), results are the
    same bits as untraced launches, and turning tracing on again clears the sums."""
    import time
    bca = _bca()
    ws = mix("f32", K=8)
    P = [make(w) for w in ws]
    Q = [make(w) for w in ws]
    bca.batch_step(P, 1)
    bca.batch_step(Q, 1)
    bca.batch_set_tracing(True)
    t = time.perf_counter()
    bca.batch_step(P, 4)
    wall_us = (time.perf_counter() - t) * 1e6
    us, n = bca.batch_get_tracing()
    bca.batch_set_tracing(False)
    bca.batch_step(Q, 4)
    assert n == 1
    assert set(us) == set(bca.BATCH_PHASES)
    for k in ("rhs", "symv", "xupd", "stream", "global"):
        assert us[k] > 0.0, k
    total = sum(us.values())
    assert 0.2 * wall_us < total <= wall_us, (total, wall_us)
    for p, q in zip(P, Q):
        assert np.array_equal(p.get_vector(bca.VEC_Z), q.get_vector(bca.VEC_Z))
    bca.batch_step(P, 1)             # untraced: the sums stay
    assert bca.batch_get_tracing()[1] == 1
    bca.batch_set_tracing(True)
    assert bca.batch_get_tracing() == ({k: 0.0 for k in bca.BATCH_PHASES}, 0)
    bca.batch_set_tracing(False)
    for p in P + Q:
        p.close()


def test_batch_reports_a_problem_whose_iterates_overflow():
    """A problem whose iterates overflow (labels of 1e308: the squared-loss prox's 2 b
    exceeds the FP64 range) makes the batched launch fail with BCA_E_NONFINITE -- the per-problem
    flags are gathered and read back once per launch -- while the same launch's other
    problems keep their results (they match their solo runs)."""
    bca = _bca()
    good = datagen.batched_instance(11, 600, 40, dtype="f64", max_iters=4)
    bad = datagen.batched_instance(12, 600, 40, dtype="f64", max_iters=4)
    G, S = make(good), make(good)
    B = bca.Problem("squared", bad.n, bad.rows, bad.n_blocks, bad.kappa, gamma=bad.gamma,
                    rho_c=bad.rho_c, rho_b=bad.rho_b, rho_l=bad.rho_l,
                    inner_iters=bad.inner_iters, max_iters=bad.max_iters, dtype="f64")
    for i in range(bad.N):
        B.set_data(i, bad.A[i], np.full_like(bad.b[i], 1e308))
    B.finalize()
    with pytest.raises(bca.BcaError) as e:
        bca.batch_step([G, B], 2)
    assert e.value.code == -4
    S.step(2)
    assert rel(G.get_vector(bca.VEC_Z), S.get_vector(bca.VEC_Z)) < 1e-12
    for P in (G, S, B):
        P.close()
