"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test checks the oracle against something other than itself: a closed form,
a generic optimiser or root finder from SciPy, brute force on tiny inputs, a
textbook special case, or a hand-worked example.  A plausible slip in the
oracle (a dropped term, a wrong sign or index, a transposed operand) fails at
least one of them.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest
from scipy.optimize import brentq, linprog, minimize

import datagen
import oracle
from oracle.bicadmm import LOSS_HINGE, LOSS_LOGISTIC, LOSS_SOFTMAX, LOSS_SQUARED

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rng(seed):
    return np.random.default_rng(seed)


def _problem(seed, N, m, n, loss=LOSS_SQUARED, C=1):
    r = _rng(seed)
    A = [r.standard_normal((m, n)) for _ in range(N)]
    if loss == LOSS_SQUARED:
        b = [r.standard_normal(m) for _ in range(N)]
    elif loss == LOSS_LOGISTIC:
        b = [np.where(r.random(m) < 0.5, -1.0, 1.0) for _ in range(N)]
    else:
        b = [r.integers(0, C, m).astype(np.int32) for _ in range(N)]
    return A, b


# ------------------------------------------------------------------ P1
@pytest.mark.parametrize("M", [1, 2, 4])
def test_split_x_update_reaches_closed_form_prox_squared(M):
    """Squared loss: Algorithm 2 run to convergence equals the closed-form local
    prox (2 A^T A + (1/(N gamma) + rho_c) I)^-1 (2 A^T b + rho_c (z - u))."""
    N, m, n = 3, 60, 11
    A, b = _problem(1, N, m, n)
    gam, rc, rl = 10.0, 1.3, 0.8
    o = oracle.BiCADMM(A, b, LOSS_SQUARED, M, 3, gam, rc, 0.5 * rc, rl)
    r = _rng(2)
    o.state.z = r.standard_normal(n)
    o.state.u = r.standard_normal((N, n))
    o.x_update(1, 4000)
    A1 = A[1]
    K = 2 * A1.T @ A1 + (1 / (N * gam) + rc) * np.eye(n)
    x = np.linalg.solve(K, 2 * A1.T @ b[1] + rc * (o.state.z - o.state.u[1]))
    assert np.linalg.norm(o.state.x[1] - x) / np.linalg.norm(x) < 1e-12


# ------------------------------------------------------------------ P2
def _logistic_prox_unsplit(A, b, v, N, gam, rc):
    def f(x):
        q = A @ x
        return np.sum(np.logaddexp(0, -b * q)) + x @ x / (2 * N * gam) + 0.5 * rc * np.sum((x - v) ** 2)

    def g(x):
        q = A @ x
        sg = 1 / (1 + np.exp(b * q))
        return A.T @ (-b * sg) + x / (N * gam) + rc * (x - v)

    def h(x):
        q = A @ x
        sg = 1 / (1 + np.exp(b * q))
        w = sg * (1 - sg)
        return A.T @ (w[:, None] * A) + (1 / (N * gam) + rc) * np.eye(len(x))

    res = minimize(f, np.zeros(A.shape[1]), jac=g, hess=h, method="trust-exact",
                   options=dict(gtol=1e-13, maxiter=500))
    x = res.x
    for _ in range(4):          # polish: plain Newton steps on the same gradient/Hessian
        x = x - np.linalg.solve(h(x), g(x))
    return x


@pytest.mark.parametrize("M", [1, 2, 4])
def test_split_x_update_equals_unsplit_prox_logistic(M):
    """Sharing ADMM over feature blocks reaches the same x_i as the unsplit
    proximal problem of the local loss (solved here by SciPy's trust-region Newton)."""
    N, m, n = 2, 80, 9
    A, b = _problem(3, N, m, n, LOSS_LOGISTIC)
    gam, rc, rl = 10.0, 1.0, 1.0
    o = oracle.BiCADMM(A, b, LOSS_LOGISTIC, M, 3, gam, rc, 0.5, rl)
    r = _rng(4)
    o.state.z = r.standard_normal(n)
    o.state.u = 0.3 * r.standard_normal((N, n))
    o.x_update(0, 1500)
    x = _logistic_prox_unsplit(A[0], b[0], o.state.z - o.state.u[0], N, gam, rc)
    assert np.linalg.norm(o.state.x[0] - x) / np.linalg.norm(x) < 1e-12


# ------------------------------------------------------------------ P3
def test_prox_squared_is_the_minimiser():
    r = _rng(5)
    c, b = r.standard_normal(50), r.standard_normal(50)
    for M, rl in [(1, 1.0), (4, 0.7)]:
        w = oracle.prox_squared(c, b, M, rl)
        # derivative of (M w - b)^2 + (M rl / 2)(w - c)^2 vanishes
        d = 2 * M * (M * w - b) + M * rl * (w - c)
        assert np.max(np.abs(d)) < 1e-12


def test_prox_logistic_matches_brent_root():
    r = _rng(6)
    M, rl = 4, 1.0
    c = 3.0 * r.standard_normal(40)
    c[:3] = [40.0, -40.0, 0.0]
    b = np.where(r.random(40) < 0.5, -1.0, 1.0)
    w = oracle.prox_logistic(c, b, M, rl)
    beta = rl / M
    for k in range(40):
        f = lambda q: -b[k] / (1 + math.exp(b[k] * q)) + beta * (q - M * c[k])
        q = brentq(f, M * c[k] - 1 / beta - 1, M * c[k] + 1 / beta + 1, xtol=1e-15, rtol=1e-15)
        assert abs(w[k] * M - q) <= 1e-12 * max(1.0, abs(q))


def test_prox_hinge_is_the_minimiser():
    """The closed-form hinge prox against a bounded scalar minimiser and a dense
    grid of the per-sample objective max(0, 1 - b q) + (beta/2)(q - Mc)^2, over
    inputs that reach all three branches (loss inactive, linear piece, kink)."""
    from scipy.optimize import minimize_scalar
    r = _rng(23)
    seen = set()
    for M in (1, 2, 4):
        for rho in (0.3, 1.0, 5.0):
            beta = rho / M
            c = r.uniform(-3.0, 3.0, 40) / M
            b = np.where(r.random(40) < 0.5, -1.0, 1.0)
            w = oracle.prox_hinge(c, b, M, rho)
            for k in range(40):
                f = lambda q: max(0.0, 1.0 - b[k] * q) + 0.5 * beta * (q - M * c[k]) ** 2
                lo, hi = M * c[k] - 2.0 / beta - 2.0, M * c[k] + 2.0 / beta + 2.0
                ref = minimize_scalar(f, bounds=(lo, hi), method="bounded",
                                      options=dict(xatol=1e-12)).x
                grid = np.linspace(lo, hi, 20001)
                fq = f(M * w[k])
                assert fq <= min(f(q) for q in grid) + 1e-12
                assert abs(M * w[k] - ref) < 1e-6
                d = b[k] * M * c[k]
                seen.add(0 if d >= 1 else (1 if d + 1 / beta <= 1 else 2))
    assert seen == {0, 1, 2}


def test_prox_softmax_matches_generic_minimiser():
    r = _rng(7)
    M, rl, C = 2, 1.0, 5
    c = 2.0 * r.standard_normal((6, C))
    y = r.integers(0, C, 6)
    w = oracle.prox_softmax(c, y, M, rl)
    beta = rl / M
    for k in range(6):
        def F(q):
            return np.log(np.sum(np.exp(q - q.max()))) + q.max() - q[y[k]] + 0.5 * beta * np.sum((q - M * c[k]) ** 2)

        def G(q):
            p = np.exp(q - q.max()); p /= p.sum()
            e = np.zeros(C); e[y[k]] = 1
            return p - e + beta * (q - M * c[k])

        res = minimize(F, M * c[k], jac=G, method="BFGS", options=dict(gtol=1e-12))
        assert np.max(np.abs(w[k] * M - res.x)) < 1e-7
        assert np.linalg.norm(G(w[k] * M)) < 1e-12


# ------------------------------------------------------------------ P4
def _zt_generic(wbar, s, v, a, rb):
    """Generic solver: variables (z, t); ||z||_1 <= t written as the 2^n linear
    constraints sigma^T z <= t."""
    n = len(wbar)

    def f(y):
        z, t = y[:n], y[n]
        return 0.5 * a * np.sum((z - wbar) ** 2) + 0.5 * rb * (s @ z - t + v) ** 2

    def g(y):
        z, t = y[:n], y[n]
        r = s @ z - t + v
        return np.concatenate([a * (z - wbar) + rb * r * s, [-rb * r]])

    cons = []
    for sig in itertools.product([-1.0, 1.0], repeat=n):
        sg = np.array(sig)
        cons.append(dict(type="ineq", fun=lambda y, sg=sg: y[n] - sg @ y[:n],
                         jac=lambda y, sg=sg: np.concatenate([-sg, [1.0]])))
    y0 = np.concatenate([wbar, [np.sum(np.abs(wbar)) + 1.0]])
    res = minimize(f, y0, jac=g, constraints=cons, method="SLSQP",
                   options=dict(ftol=1e-15, maxiter=1000))
    return res.x[:n], res.x[n], f(res.x)


@pytest.mark.parametrize("seed", range(12))
def test_zt_step_is_the_qp_minimiser(seed):
    r = _rng(100 + seed)
    n = int(r.integers(2, 7))
    wbar = r.standard_normal(n)
    if seed % 4 == 0:
        wbar[0] = 0.0
    s = np.clip(r.standard_normal(n), -1, 1)
    if seed % 3 == 0:
        s[:] = 0.0
    v = float(r.standard_normal()) * (3.0 if seed % 5 == 0 else 0.5)
    a, rb = float(r.uniform(0.5, 5)), float(r.uniform(0.2, 3))
    z, t, theta = oracle.zt_step(wbar, s, v, a, rb)
    assert np.sum(np.abs(z)) <= t + 1e-12
    fo = 0.5 * a * np.sum((z - wbar) ** 2) + 0.5 * rb * (s @ z - t + v) ** 2
    zg, tg, fg = _zt_generic(wbar, s, v, a, rb)
    assert fo <= fg + 1e-9
    assert np.max(np.abs(z - zg)) < 2e-5 and abs(t - tg) < 2e-5


def test_zt_step_branches():
    # theta = 0: s^T wbar + v >= ||wbar||_1
    w = np.array([1.0, -2.0, 0.5])
    z, t, th = oracle.zt_step(w, np.zeros(3), 10.0, 2.0, 1.0)
    assert th == 0.0 and np.array_equal(z, w) and t == 10.0
    # root beyond every breakpoint: all z_k with d_k > 0 vanish, theta = -v rho_b
    z, t, th = oracle.zt_step(w, np.zeros(3), -1e3, 1.0, 0.5)
    assert np.all(z == 0) and t == 0.0 and abs(th - 500.0) < 1e-9
    # s = sign(wbar) keeps those coordinates (d_k = 0): z = wbar there
    s = np.array([1.0, -1.0, 0.0])
    z, t, th = oracle.zt_step(w, s, -100.0, 1.0, 1.0)
    assert z[0] == 1.0 and z[1] == -2.0 and z[2] == 0.0


# ------------------------------------------------------------------ P5
@pytest.mark.parametrize("seed", range(20))
def test_s_step_attains_the_lp_range_optimum(seed):
    r = _rng(200 + seed)
    n = int(r.integers(3, 12))
    kappa = int(r.integers(1, n + 1))
    z = r.standard_normal(n)
    tau = float(r.standard_normal() * r.choice([0.1, 1.0, 10.0]))
    s, T = oracle.s_step(z, tau, kappa)
    # feasibility in S^kappa
    assert np.max(np.abs(s)) <= 1 + 1e-15 and np.sum(np.abs(s)) <= kappa + 1e-12
    # LP: max z^T s over S^kappa (variables s, w with |s| <= w <= 1, sum w <= kappa)
    c = np.concatenate([-z, np.zeros(n)])
    Aub = np.block([[np.eye(n), -np.eye(n)], [-np.eye(n), -np.eye(n)],
                    [np.zeros((1, n)), np.ones((1, n))]])
    bub = np.concatenate([np.zeros(2 * n), [kappa]])
    lp = linprog(c, A_ub=Aub, b_ub=bub, bounds=[(None, None)] * n + [(0, 1)] * n, method="highs")
    Mk = -lp.fun
    assert abs((z @ s - tau) ** 2 - max(abs(tau) - Mk, 0.0) ** 2) < 1e-9 * max(1, tau * tau)


def test_topk_ties_break_toward_lower_index():
    z = np.array([0.0, -0.0, 3.0, -3.0, 3.0, 1e-310, -1e-310, 2.0, 5e-324, -2.0])
    for kappa in range(1, len(z) + 1):
        ref = sorted(range(len(z)), key=lambda k: (-abs(z[k]), k))[:kappa]
        assert list(oracle.topk_support(z, kappa)) == sorted(ref)
    allsame = np.full(17, -1.5)
    assert list(oracle.topk_support(allsame, 5)) == [0, 1, 2, 3, 4]


# ------------------------------------------------------------------ residuals, worked example
@pytest.mark.parametrize("which", [0, 1])
def test_global_update_worked_example(which):
    """Hand-worked global step (Sec. 3: the (z,t), s, v, u updates and the
    Termination residuals); the values are in tests/golden."""
    ex = json.load(open(os.path.join(GOLDEN, "global_step_worked_example.json")))["examples"][which]
    inp, out = ex["input"], ex["expected"]
    N = inp["N"]
    A = [np.zeros((1, 2)) for _ in range(N)]
    o = oracle.BiCADMM(A, [np.zeros(1)] * N, LOSS_SQUARED, 1, inp["kappa"], 10.0,
                       inp["rho_c"], inp["rho_b"], 1.0)
    st = o.state
    st.x = np.array(inp["x"], dtype=float)
    st.u = np.array(inp["u"], dtype=float)
    st.s = np.array(inp["s"], dtype=float)
    st.v = inp["v"]
    pr, dr, br = o.global_update()
    np.testing.assert_allclose(st.z, out["z"], rtol=0, atol=1e-15)
    assert st.t == pytest.approx(out["t"], abs=1e-15)
    np.testing.assert_allclose(st.s, out["s"], atol=1e-15)
    assert st.v == pytest.approx(out["v"], abs=1e-15)
    np.testing.assert_allclose(st.u, out["u"], atol=1e-15)
    assert pr == pytest.approx(out["p_r"], rel=1e-15)
    assert dr == pytest.approx(out["d_r"], rel=1e-15)
    assert br == pytest.approx(out["b_r"], abs=1e-15)


# ------------------------------------------------------------------ P6, P10
def test_config0_support_and_residual_decay():
    w = datagen.config0()
    o = oracle.BiCADMM(w.A, w.b, w.loss, w.n_blocks, w.kappa, w.gamma, w.rho_c, w.rho_b, w.rho_l)
    o.iterate(200, 5)
    x = o.coef()
    assert np.count_nonzero(x) <= w.kappa
    h = np.array(o.state.history)
    assert h[-1, 0] < h[0, 0] / 100 and h[-1, 1] < h[0, 1] / 1000 and h[-1, 2] < 0.01
    # Hempel: at the end z^T s is close to t >= ||z||_1 on the kappa-support
    assert list(o.support()) == list(np.nonzero(w.x_true)[0])


# ------------------------------------------------------------------ P7
@pytest.mark.parametrize("M", [1, 2])
def test_kappa_equal_n_gives_global_ridge(M):
    """With kappa = n the l0 constraint is void and Bi-cADMM converges to the
    global ridge solution (2 sum A_i^T A_i + I/gamma)^-1 2 sum A_i^T b_i for any
    number of partitions and blocks."""
    N, m, n = 3, 30, 8
    A, b = _problem(8, N, m, n)
    gam = 10.0
    o = oracle.BiCADMM(A, b, LOSS_SQUARED, M, n, gam, 5.0, 2.5, 5.0)
    o.iterate(1500, 5)
    S = sum(Ai.T @ Ai for Ai in A)
    x = np.linalg.solve(2 * S + np.eye(n) / gam, 2 * sum(Ai.T @ bi for Ai, bi in zip(A, b)))
    assert np.linalg.norm(o.state.z - x) / np.linalg.norm(x) < 1e-10


def test_kappa_equal_n_logistic_gives_regularised_mle():
    N, m, n = 2, 50, 5
    A, b = _problem(9, N, m, n, LOSS_LOGISTIC)
    gam = 2.0
    o = oracle.BiCADMM(A, b, LOSS_LOGISTIC, 2, n, gam, 2.0, 1.0, 2.0)
    o.iterate(1200, 5)
    Aall, ball = np.vstack(A), np.concatenate(b)
    f = lambda x: np.sum(np.logaddexp(0, -ball * (Aall @ x))) + x @ x / (2 * gam)
    gr = lambda x: Aall.T @ (-ball / (1 + np.exp(ball * (Aall @ x)))) + x / gam
    res = minimize(f, np.zeros(n), jac=gr, method="BFGS", options=dict(gtol=1e-12))
    assert np.linalg.norm(o.state.z - res.x) / np.linalg.norm(res.x) < 1e-7


def test_kappa_equal_n_softmax_gives_regularised_mle():
    N, m, n, C = 2, 40, 4, 3
    A, b = _problem(10, N, m, n, LOSS_SOFTMAX, C)
    gam = 2.0
    o = oracle.BiCADMM(A, b, LOSS_SOFTMAX, 2, n, gam, 2.0, 1.0, 2.0, n_classes=C)
    o.iterate(800, 5)
    Aall, yall = np.vstack(A), np.concatenate(b)
    Y = np.zeros((len(yall), C)); Y[np.arange(len(yall)), yall] = 1

    def f(w):
        Q = Aall @ w.reshape(n, C)
        mx = Q.max(axis=1, keepdims=True)
        return np.sum(np.log(np.exp(Q - mx).sum(axis=1)) + mx[:, 0] - np.sum(Q * Y, axis=1)) + w @ w / (2 * gam)

    def g(w):
        W = w.reshape(n, C)
        Q = Aall @ W
        P = np.exp(Q - Q.max(axis=1, keepdims=True)); P /= P.sum(axis=1, keepdims=True)
        return (Aall.T @ (P - Y) + W / gam).ravel()

    res = minimize(f, np.zeros(n * C), jac=g, method="BFGS", options=dict(gtol=1e-12))
    Z = o.state.z
    assert np.linalg.norm(Z.ravel() - res.x) / np.linalg.norm(res.x) < 1e-6


def test_kappa_equal_n_hinge_gives_regularised_svm():
    """Hinge loss (the sparse SVM) with kappa = n: Bi-cADMM converges to the
    L2-regularised SVM, min sum max(0, 1 - b a^T x) + ||x||^2 / (2 gamma), here
    the QP in (x, xi) solved by SLSQP; and its KKT conditions hold: x / gamma =
    sum_k alpha_k b_k a_k with alpha_k = 1 inside the margin, 0 outside it, and
    alpha_k in [0, 1] on it."""
    N, m, n, gam = 2, 30, 5, 2.0
    r = _rng(12)
    A = [r.standard_normal((m, n)) for _ in range(N)]
    xt = r.standard_normal(n)
    b = [np.where(Ai @ xt + 0.5 * r.standard_normal(m) >= 0, 1.0, -1.0) for Ai in A]
    o = oracle.BiCADMM(A, b, LOSS_HINGE, 2, n, gam, 2.0, 1.0, 2.0)
    o.iterate(1200, 5)
    z = o.state.z
    Aall, ball = np.vstack(A), np.concatenate(b)
    K = len(ball)
    f = lambda v: np.sum(v[n:]) + v[:n] @ v[:n] / (2 * gam)
    g = lambda v: np.concatenate([v[:n] / gam, np.ones(K)])
    cons = [{"type": "ineq", "fun": lambda v: v[n:],
             "jac": lambda v: np.hstack([np.zeros((K, n)), np.eye(K)])},
            {"type": "ineq", "fun": lambda v: v[n:] - (1 - ball * (Aall @ v[:n])),
             "jac": lambda v: np.hstack([ball[:, None] * Aall, np.eye(K)])}]
    v0 = np.concatenate([np.zeros(n), np.ones(K)])
    res = minimize(f, v0, jac=g, constraints=cons, method="SLSQP", options=dict(ftol=1e-15, maxiter=1000))
    assert np.linalg.norm(z - res.x[:n]) / np.linalg.norm(res.x[:n]) < 1e-7
    fz = np.sum(np.maximum(0.0, 1.0 - ball * (Aall @ z))) + z @ z / (2 * gam)
    assert abs(fz - f(res.x)) <= 1e-9 * fz
    # KKT
    mar = ball * (Aall @ z)
    inside, onm = mar < 1 - 1e-8, np.abs(mar - 1) <= 1e-8
    rest = z / gam - (ball[inside, None] * Aall[inside]).sum(axis=0)
    B = (ball[onm, None] * Aall[onm]).T
    alpha = np.linalg.lstsq(B, rest, rcond=None)[0]
    assert np.linalg.norm(B @ alpha - rest) <= 1e-7 * max(1.0, np.linalg.norm(z / gam))
    assert np.all(alpha >= -1e-7) and np.all(alpha <= 1 + 1e-7)


def test_exact_x_update_is_the_limit_of_algorithm_2():
    """The exact x-update (squared loss) is what Algorithm 2's inner loop converges
    to: with 200 warm-started inner iterations per outer iteration the two runs
    agree to rounding over several outer iterations, with 50 they do not yet."""
    N, m, n = 3, 40, 12
    A, b = _problem(3, N, m, n)
    args = (A, b, LOSS_SQUARED, 2, 4, 10.0, 1.0, 0.5, 1.0)
    oe = oracle.BiCADMM(*args, exact_x=True)
    oa = oracle.BiCADMM(*args)
    oa50 = oracle.BiCADMM(*args)
    for _ in range(3):
        oe.iterate(1, 5)
        oa.iterate(1, 200)
        oa50.iterate(1, 50)
        for i in range(N):
            assert np.linalg.norm(oa.state.x[i] - oe.state.x[i]) <= 1e-13 * np.linalg.norm(oe.state.x[i])
        assert np.linalg.norm(oa.state.z - oe.state.z) <= 1e-13 * np.linalg.norm(oe.state.z)
    assert np.linalg.norm(oa50.state.z - oe.state.z) > 1e-10 * np.linalg.norm(oe.state.z)
    # kappa = n: the exact variant reaches the global ridge solution as well
    o = oracle.BiCADMM(A, b, LOSS_SQUARED, 1, n, 10.0, 5.0, 2.5, 5.0, exact_x=True)
    o.iterate(1500, 5)
    S = sum(Ai.T @ Ai for Ai in A)
    x = np.linalg.solve(2 * S + np.eye(n) / 10.0, 2 * sum(Ai.T @ bi for Ai, bi in zip(A, b)))
    assert np.linalg.norm(o.state.z - x) / np.linalg.norm(x) < 1e-10
    with pytest.raises(ValueError):
        oracle.BiCADMM(A, [np.sign(bi) for bi in b], LOSS_HINGE, 1, 4, 10.0, 1.0, 0.5, 1.0, exact_x=True)


def test_exact_logistic_x_update_is_the_unsplit_prox():
    """Logistic exact x-update (Newton's method on the unsplit x-subproblem of Sec. 3)
    against SciPy's trust-region Newton minimiser of the same function, from a cold
    and a warm start, on a random consensus state."""
    N, m, n = 3, 70, 11
    A, b = _problem(21, N, m, n, LOSS_LOGISTIC)
    gam, rc = 10.0, 1.3
    o = oracle.BiCADMM(A, b, LOSS_LOGISTIC, 2, 3, gam, rc, 0.5 * rc, 1.0, exact_x=True)
    r = _rng(22)
    o.state.z = r.standard_normal(n)
    o.state.u = 0.3 * r.standard_normal((N, n))
    for i in range(N):
        ref = _logistic_prox_unsplit(A[i], b[i], o.state.z - o.state.u[i], N, gam, rc)
        o.state.x[i] = 0.0
        o.x_update_exact(i)
        assert np.linalg.norm(o.state.x[i] - ref) <= 1e-11 * np.linalg.norm(ref)
        o.state.x[i] = ref + 0.1 * r.standard_normal(n)        # warm start off the minimiser
        o.x_update_exact(i)
        assert np.linalg.norm(o.state.x[i] - ref) <= 1e-11 * np.linalg.norm(ref)


def test_exact_logistic_x_update_is_the_limit_of_algorithm_2():
    """Algorithm 2's inner loop (logistic loss, M = 2 feature blocks) run long enough
    per outer iteration approaches the exact x-update (linearly: 300 inner iterations
    are much further off than 3000); and with kappa = n the exact variant converges
    to the L2-regularised logistic MLE, like Algorithm 2."""
    N, m, n = 3, 50, 10
    A, b = _problem(23, N, m, n, LOSS_LOGISTIC)
    args = (A, b, LOSS_LOGISTIC, 2, 4, 10.0, 1.0, 0.5, 1.0)
    oe = oracle.BiCADMM(*args, exact_x=True)
    oa = oracle.BiCADMM(*args)
    oa3 = oracle.BiCADMM(*args)
    for _ in range(2):
        oe.iterate(1, 5)
        oa.iterate(1, 3000)
        oa3.iterate(1, 300)
        ne = np.linalg.norm(oe.state.x)
        d3000 = np.linalg.norm(oa.state.x - oe.state.x)
        assert d3000 <= 5e-9 * ne
        assert np.linalg.norm(oa3.state.x - oe.state.x) >= 10 * d3000
    o = oracle.BiCADMM(A, b, LOSS_LOGISTIC, 1, n, 2.0, 2.0, 1.0, 2.0, exact_x=True)
    o.iterate(400, 5)
    Aall, ball = np.vstack(A), np.concatenate(b)
    f = lambda x: np.sum(np.logaddexp(0, -ball * (Aall @ x))) + x @ x / 4.0
    gf = lambda x: Aall.T @ (-ball / (1 + np.exp(ball * (Aall @ x)))) + x / 2.0
    res = minimize(f, np.zeros(n), jac=gf, method="BFGS", options=dict(gtol=1e-12))
    assert np.linalg.norm(o.state.z - res.x) / np.linalg.norm(res.x) < 1e-7


# ------------------------------------------------------------------ P8
def test_orthogonal_design_closed_form():
    """sum A_i^T A_i = I and squared loss: the l0-constrained optimum is hard
    thresholding H_kappa(A^T b / (1 + 1/(2 gamma)))."""
    N, m, n, kappa, gam = 4, 25, 12, 3, 10.0
    r = _rng(11)
    Q, _ = np.linalg.qr(r.standard_normal((N * m, n)))
    A = [Q[i * m:(i + 1) * m] for i in range(N)]
    xt = np.zeros(n); xt[[2, 5, 9]] = [3.0, -2.5, 2.0]
    bb = Q @ xt + 0.05 * r.standard_normal(N * m)
    b = [bb[i * m:(i + 1) * m] for i in range(N)]
    o = oracle.BiCADMM(A, b, LOSS_SQUARED, 2, kappa, gam, 1.0, 0.5, 1.0)
    o.iterate(600, 5)
    c = (Q.T @ bb) / (1 + 1 / (2 * gam))
    T = np.sort(np.argsort(-np.abs(c))[:kappa])
    xh = np.zeros(n); xh[T] = c[T]
    assert list(o.support()) == list(T)
    assert np.linalg.norm(o.coef() - xh) / np.linalg.norm(xh) < 1e-8


# ------------------------------------------------------------------ P9
def test_tiny_planted_support_matches_brute_force():
    N, m, n, kappa, gam = 2, 30, 10, 2, 10.0
    r = _rng(12)
    A = [r.standard_normal((m, n)) for _ in range(N)]
    xt = np.zeros(n); xt[[3, 7]] = [1.5, -1.2]
    b = [Ai @ xt + 0.05 * r.standard_normal(m) for Ai in A]
    o = oracle.BiCADMM(A, b, LOSS_SQUARED, 2, kappa, gam, 1.0, 0.5, 1.0)
    o.iterate(300, 5)
    Aall, ball = np.vstack(A), np.concatenate(b)
    best, bestT = np.inf, None
    for T in itertools.combinations(range(n), kappa):
        AT = Aall[:, T]
        xT = np.linalg.solve(2 * AT.T @ AT + np.eye(kappa) / gam, 2 * AT.T @ ball)
        f = np.sum((AT @ xT - ball) ** 2) + xT @ xT / (2 * gam)
        if f < best:
            best, bestT = f, T
    assert tuple(o.support()) == bestT


def test_objective_definition():
    A = [np.array([[1.0, 2.0]]), np.array([[0.0, -1.0]])]
    b = [np.array([1.0]), np.array([-1.0])]
    x = np.array([1.0, 1.0])
    # (3 - 1)^2 + (-1 + 1)^2 + ||x||^2 / (2*2) = 4 + 0 + 0.5
    assert oracle.objective(LOSS_SQUARED, A, b, x, 2.0) == 4.5
    bl = [np.array([1.0]), np.array([-1.0])]
    expect = math.log1p(math.exp(-3.0)) + math.log1p(math.exp(-1.0)) + 0.5
    assert abs(oracle.objective(LOSS_LOGISTIC, A, bl, x, 2.0) - expect) < 1e-15


def test_objective_worked_examples_softmax_and_hinge():
    """Objective of Sec. 2 for the softmax loss (row sparsity, classes from 0) and the
    hinge loss of the sparse SVM, against hand-worked values in tests/golden: a wrong
    class index, LSE replaced by the max, a dropped max(0, .) or a flipped label sign
    each changes the value."""
    ex = json.load(open(os.path.join(GOLDEN, "loss_worked_examples.json")))["examples"]
    for e in ex:
        A = [np.array(a, dtype=float) for a in e["A"]]
        if e["loss"] == "softmax":
            loss = LOSS_SOFTMAX
            b = [np.array(y, dtype=np.int32) for y in e["b"]]
        else:
            loss = LOSS_HINGE
            b = [np.array(y, dtype=float) for y in e["b"]]
        x = np.array(e["x"], dtype=float)
        ls = sum(oracle.loss_value(loss, Ai @ x, bi) for Ai, bi in zip(A, b))
        assert abs(ls - e["loss_sum"]) <= 4e-16 * abs(e["loss_sum"]), (e["loss"], ls)
        f = oracle.objective(loss, A, b, x, e["gamma"])
        assert abs(f - e["objective"]) <= 4e-16 * abs(e["objective"]), (e["loss"], f)


def _zt_matrix_generic(W, s, v, a, rb, rng, starts=6):
    """Generic solver of the row-sparse (z, t) problem of the softmax model:
        min_{Z, t}  (a/2)||Z - W||_F^2 + (rb/2)(sum_r s_r ||Z_r|| - t + v)^2
        s.t.        sum_r ||Z_r|| <= t,
    written without the reduction to row norms.  The row norms are not smooth at
    Z_r = 0, so every subset P of rows is tried as the set of nonzero rows (the
    others fixed at 0), each smooth problem by SLSQP from several starts; the best
    feasible point over all subsets is returned."""
    n, C = W.shape
    best = (np.inf, None, None)
    for mask in itertools.product([False, True], repeat=n):
        P = [r for r in range(n) if mask[r]]
        k = len(P)
        Wz = float(np.sum(W[[r for r in range(n) if not mask[r]]] ** 2))

        def unpack(y):
            return y[:k * C].reshape(k, C), y[k * C]

        def f(y):
            Z, t = unpack(y)
            nr = np.sqrt(np.sum(Z * Z, axis=1))
            res = float(s[P] @ nr) - t + v
            return 0.5 * a * (np.sum((Z - W[P]) ** 2) + Wz) + 0.5 * rb * res * res

        def g(y):
            Z, t = unpack(y)
            nr = np.maximum(np.sqrt(np.sum(Z * Z, axis=1)), 1e-300)
            res = float(s[P] @ nr) - t + v
            gz = a * (Z - W[P]) + rb * res * (s[P] / nr)[:, None] * Z
            return np.concatenate([gz.ravel(), [-rb * res]])

        def cf(y):
            Z, t = unpack(y)
            return t - np.sum(np.sqrt(np.sum(Z * Z, axis=1)))

        def cj(y):
            Z, t = unpack(y)
            nr = np.maximum(np.sqrt(np.sum(Z * Z, axis=1)), 1e-300)
            return np.concatenate([(-Z / nr[:, None]).ravel(), [1.0]])

        for st in range(starts if k else 1):
            if st == 0:
                Z0 = W[P] + (np.abs(W[P]) < 1e-12) * 1e-3
            else:
                Z0 = rng.standard_normal((k, C)) * (1.0 + np.abs(W[P]))
            y0 = np.concatenate([Z0.ravel(), [np.sum(np.sqrt(np.sum(Z0 * Z0, axis=1))) + 1.0]])
            res = minimize(f, y0, jac=g, constraints=[dict(type="ineq", fun=cf, jac=cj)],
                           method="SLSQP", options=dict(ftol=1e-16, maxiter=2000))
            y = res.x
            if cf(y) < -1e-10:
                continue
            fy = f(y)
            if fy < best[0]:
                Z = np.zeros((n, C))
                Z[P] = unpack(y)[0]
                best = (fy, Z, unpack(y)[1])
    return best


@pytest.mark.parametrize("seed", range(10))
def test_softmax_row_sparse_zt_step_is_the_matrix_minimiser(seed):
    """Row-sparse (z, t) step of the softmax model (reading: Hempel's theorem on the row
    norms of X, Sec. 2.1, with the (z, t) minimisation of the ADMM iterations, Sec. 3),
    run through the oracle's global step with kappa < n, against a generic solver of the
    matrix problem that does not use the reduction to row norms."""
    r = _rng(700 + seed)
    N, n, C = 2, int(r.integers(2, 5)), int(r.integers(2, 4))
    kappa = int(r.integers(1, n))
    rc, rb = float(r.uniform(0.5, 2.0)), float(r.uniform(0.3, 2.0))
    A = [np.zeros((1, n)) for _ in range(N)]
    b = [np.zeros(1, dtype=np.int32) for _ in range(N)]
    o = oracle.BiCADMM(A, b, LOSS_SOFTMAX, 1, kappa, 10.0, rc, rb, 1.0, n_classes=C)
    st = o.state
    st.x = r.standard_normal((N, n, C))
    st.u = 0.5 * r.standard_normal((N, n, C))
    if seed % 3 == 0:                      # a zero row of the consensus target
        st.x[:, 0, :] = 0.0
        st.u[:, 0, :] = 0.0
    s = r.uniform(-1.0, 1.0, n)
    if seed % 4 == 1:
        s = np.abs(s)                      # the s-step's own sign pattern on row norms
    if seed % 5 == 2:
        s[:] = 0.0
    st.s = s.copy()
    v = float(r.standard_normal()) * (3.0 if seed % 2 else 0.7)
    st.v = v
    W = np.mean(st.x + st.u, axis=0)
    a = N * rc
    o.global_update()
    Z, t = st.z, st.t
    nr = np.sqrt(np.sum(Z * Z, axis=1))
    assert np.sum(nr) <= t + 1e-12
    fo = 0.5 * a * np.sum((Z - W) ** 2) + 0.5 * rb * (s @ nr - t + v) ** 2
    fg, Zg, tg = _zt_matrix_generic(W, s, v, a, rb, _rng(900 + seed))
    assert fo <= fg + 1e-10 * max(1.0, abs(fg)), (fo, fg)
    assert np.max(np.abs(Z - Zg)) < 1e-4 and abs(t - tg) < 1e-4, (np.max(np.abs(Z - Zg)), t, tg)
