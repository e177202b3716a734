"""Plain FP64 CPU reference of Bi-cADMM (Olama et al., "A GPU-Accelerated
Bi-linear ADMM Algorithm for Distributed Sparse Machine Learning").

TEST INFRASTRUCTURE ONLY.  This module is the oracle against which the GPU
library is checked.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never calls it and the two
share no code.  Inputs reach both sides from the seeded generator in
``datagen``.

Everything is FP64.  The steps are taken in the paper's order and notation:

* problem: min sum_i l_i(A_i x; b_i) + 1/(2 gamma) ||x||^2  s.t. ||x||_0 <= kappa
  (Sec. 2, the SML problem);
* Hempel's theorem turns ||x||_0 <= kappa into x^T s = t, ||x||_1 <= t,
  s in S^kappa = {||s||_inf <= 1, ||s||_1 <= kappa} (Sec. 2.1);
* consensus copies x_i = z, scaled duals u_i and v = lambda / rho_b; one outer
  iteration is x -> (z, t) -> s -> v -> u (Sec. 3, the ADMM iterations, the
  u-update, the s- and v-updates);
* the x-step of every partition is the feature-split sharing ADMM of Sec. 3.1
  (Algorithm 2): per block j an x_ij ridge solve with a cached Cholesky factor,
  the block predictions A_ij x_ij averaged over the M blocks, the per-sample
  omega-bar prox and the nu dual update;
* termination residuals p_r, d_r, b_r (Sec. 3, Termination).

Readings where the paper is silent or inconsistent:
  - scaled consensus form as printed: x_i = prox(z - u_i), u_i += x_i - z, so the
    (z, t) target is w = mean_i (x_i + u_i);
  - the (z, t) step is solved exactly (unique minimiser of a strictly convex
    problem, found from its KKT conditions as a 1-D monotone root);
  - s-step: among the minimisers, s = clip(tau / M_kappa, -1, 1) sign(z) on the
    kappa largest |z| (ties to the lower index), 0 elsewhere, tau = t - v;
  - all state starts at zero; a fixed number K_in of warm-started inner
    iterations per outer iteration; rho_l as given by the caller;
  - losses: squared sum (q - b)^2 (no 1/2, as in the experimental SLS problem),
    logistic sum log(1 + exp(-b q)), softmax sum LSE(Q_k) - Q_{k, y_k}, and for
    the sparse SVM the paper names without a formulation the hinge loss
    sum max(0, 1 - b q), b in {-1, +1}, with the same ridge term;
  - softmax sparsity is row sparsity: Hempel applied to the row norms of X.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
from scipy.linalg import cho_factor, cho_solve, cholesky, solve_triangular
from scipy.special import expit, logsumexp, softmax as _softmax

LOSS_SQUARED, LOSS_LOGISTIC, LOSS_SOFTMAX, LOSS_HINGE = 0, 1, 2, 3


def split_columns(n: int, M: int):
    """Feature blocks x_i = [x_i1 .. x_iM] (Sec. 3.1): contiguous column ranges,
    the first n mod M blocks one column wider."""
    q, r = divmod(n, M)
    bounds, c = [], 0
    for j in range(M):
        w = q + (1 if j < r else 0)
        bounds.append((c, c + w))
        c += w
    return bounds


# ---------------------------------------------------------------- losses
def loss_value(loss: int, q: np.ndarray, b: np.ndarray) -> float:
    """l(q; b) summed over samples (q = A x, rows of Q for softmax)."""
    if loss == LOSS_SQUARED:
        return float(np.sum((q - b) ** 2))
    if loss == LOSS_LOGISTIC:
        return float(np.sum(np.logaddexp(0.0, -b * q)))
    if loss == LOSS_HINGE:
        return float(np.sum(np.maximum(0.0, 1.0 - b * q)))
    rows = np.arange(q.shape[0])
    return float(np.sum(logsumexp(q, axis=1) - q[rows, b.astype(np.int64)]))


def objective(loss: int, A_parts, b_parts, x: np.ndarray, gamma: float) -> float:
    """Objective of the SML problem (Sec. 2): sum_i l_i(A_i x; b_i) + ||x||^2 / (2 gamma)."""
    f = sum(loss_value(loss, A @ x, b) for A, b in zip(A_parts, b_parts))
    return f + float(np.sum(x * x)) / (2.0 * gamma)


# ---------------------------------------------------------------- omega-bar prox
# The omega-bar step of Sec. 3.1 minimises l(M w; b) + (M rho_l / 2)||w - c||^2
# with c = (average of A_ij x_ij) + nu.  With q = M w this is, per sample,
#   l(q; b) + (beta / 2)(q - M c)^2,  beta = rho_l / M.
def prox_squared(c: np.ndarray, b: np.ndarray, M: int, rho_l: float) -> np.ndarray:
    """Squared loss (q - b)^2: 2(q - b) + beta (q - Mc) = 0, so
    w = q / M = (2 b + rho_l c) / (2 M + rho_l)."""
    return (2.0 * b + rho_l * c) / (2.0 * M + rho_l)


def prox_logistic(c: np.ndarray, b: np.ndarray, M: int, rho_l: float,
                  max_iter: int = 200) -> np.ndarray:
    """Logistic loss log(1 + exp(-b q)), b in {-1, +1}.  The minimiser is the unique
    root of phi'(q) = -b sigmoid(-b q) + beta (q - Mc), which lies in
    [Mc - 1/beta, Mc + 1/beta] because |b sigmoid| <= 1.  Newton steps,
    safeguarded by bisection of that bracket, until the step is below a few ulp."""
    beta = rho_l / M
    q0 = M * np.asarray(c, dtype=np.float64)
    lo = q0 - 1.0 / beta
    hi = q0 + 1.0 / beta
    q = q0.copy()
    active = np.ones(q.shape, dtype=bool)
    for _ in range(max_iter):
        sg = expit(-b * q)
        g = -b * sg + beta * (q - q0)
        h = sg * (1.0 - sg) + beta
        lo = np.where(g < 0, q, lo)
        hi = np.where(g > 0, q, hi)
        qn = q - g / h
        outside = (qn <= lo) | (qn >= hi)
        qn = np.where(outside, 0.5 * (lo + hi), qn)
        step = np.abs(qn - q)
        done = (g == 0) | (step <= 4 * np.spacing(np.abs(q))) | (hi - lo <= 4 * np.spacing(np.abs(q)))
        q = np.where(active, qn, q)
        active &= ~done
        if not active.any():
            break
    return q / M


def prox_hinge(c: np.ndarray, b: np.ndarray, M: int, rho_l: float) -> np.ndarray:
    """Hinge loss max(0, 1 - b q), b in {-1, +1}.  With s = b q and d = b M c
    (b^2 = 1) the problem is max(0, 1 - s) + (beta/2)(s - d)^2, whose minimiser is
      s = d            if d >= 1           (loss inactive at the quadratic's minimum),
      s = d + 1/beta   if d + 1/beta <= 1  (on the linear piece: -1 + beta (s - d) = 0),
      s = 1            otherwise           (at the kink);
    q = b s and w = q / M."""
    beta = rho_l / M
    d = b * M * np.asarray(c, dtype=np.float64)
    s = np.where(d >= 1.0, d, np.where(d + 1.0 / beta <= 1.0, d + 1.0 / beta, 1.0))
    return b * s / M


def prox_softmax(c: np.ndarray, y: np.ndarray, M: int, rho_l: float,
                 max_iter: int = 100, tol: float = 1e-14) -> np.ndarray:
    """Softmax loss LSE(q) - q_y per sample (q in R^C).  Newton on
    F(q) = LSE(q) - q_y + (beta/2)||q - Mc||^2 with the Hessian diag(p) - p p^T
    + beta I inverted by Sherman-Morrison (D = diag(p + beta)):
      H^-1 g = D^-1 g + D^-1 p (p^T D^-1 g) / (1 - p^T D^-1 p),
    plus backtracking (Armijo on F, or a decrease of ||grad|| once F is flat to
    rounding), until ||grad|| <= tol."""
    beta = rho_l / M
    c = np.asarray(c, dtype=np.float64)
    m, C = c.shape
    onehot = np.zeros((m, C))
    onehot[np.arange(m), y.astype(np.int64)] = 1.0
    q0 = M * c
    q = q0.copy()

    def F(qq):
        return logsumexp(qq, axis=1) - np.sum(qq * onehot, axis=1) + 0.5 * beta * np.sum((qq - q0) ** 2, axis=1)

    def gnorm(qq):
        g = _softmax(qq, axis=1) - onehot + beta * (qq - q0)
        return np.sqrt(np.sum(g * g, axis=1))

    for _ in range(max_iter):
        p = _softmax(q, axis=1)
        g = p - onehot + beta * (q - q0)
        gn = np.sqrt(np.sum(g * g, axis=1))
        act = gn > tol
        if not act.any():
            break
        Dinv = 1.0 / (p + beta)
        Dg = Dinv * g
        Dp = Dinv * p
        denom = 1.0 - np.sum(p * Dp, axis=1)
        step = Dg + Dp * (np.sum(p * Dg, axis=1) / denom)[:, None]
        f0 = F(q)
        slope = np.sum(g * step, axis=1)
        tstep = np.ones(m)
        for _ls in range(60):
            qn = q - tstep[:, None] * step
            # Armijo decrease, or (once F is flat to rounding) a smaller gradient
            ok = (F(qn) <= f0 - 1e-4 * tstep * slope) | (gnorm(qn) < gn)
            ok |= ~act
            if ok.all():
                break
            tstep = np.where(ok, tstep, 0.5 * tstep)
        q = np.where(act[:, None], q - tstep[:, None] * step, q)
    return q / M


def omega_prox(loss: int, c, b, M, rho_l):
    if loss == LOSS_SQUARED:
        return prox_squared(c, b, M, rho_l)
    if loss == LOSS_LOGISTIC:
        return prox_logistic(c, b, M, rho_l)
    if loss == LOSS_HINGE:
        return prox_hinge(c, b, M, rho_l)
    return prox_softmax(c, b, M, rho_l)


# ---------------------------------------------------------------- global steps
def zt_step(wbar: np.ndarray, s: np.ndarray, v: float, a: float, rho_b: float):
    """(z, t) step of the ADMM iterations (Sec. 3):
        min_{||z||_1 <= t} (a/2)||z - wbar||^2 + (rho_b/2)(s^T z - t + v)^2,
    a = N rho_c, wbar = mean_i (x_i + u_i).  Strictly convex, so the minimiser is
    unique.  KKT with multiplier theta >= 0 of ||z||_1 <= t gives
        z(theta) = S_{theta/a}(wbar + theta s / a)   (soft threshold),
        rho_b (s^T z - t + v) = -theta,  theta (||z||_1 - t) = 0.
    theta = 0 holds when s^T wbar + v >= ||wbar||_1 (then z = wbar,
    t = s^T wbar + v).  Otherwise t = ||z(theta)||_1 and theta is the root of
        psi(theta) = s^T z(theta) - ||z(theta)||_1 + v + theta / rho_b,
    which is continuous, increasing and piecewise linear with a breakpoint
    theta_k = a |wbar_k| / d_k, d_k = 1 - sign(wbar_k) s_k, where z_k reaches 0.
    On a segment with active set S (theta_k > theta):
        psi = v - sum_S d_k |wbar_k| + theta (1/rho_b + sum_S d_k^2 / a).
    The breakpoints are sorted and the segment holding the root is found."""
    wbar = np.asarray(wbar, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    aw = np.abs(wbar)
    d = 1.0 - np.sign(wbar) * s
    psi0 = v - float(np.sum(d * aw))
    if psi0 >= 0.0:
        return wbar.copy(), float(s @ wbar + v), 0.0
    pos = d > 0
    th = np.full(wbar.shape, np.inf)
    th[pos] = a * aw[pos] / d[pos]
    order = np.argsort(th[pos], kind="stable")
    thk = th[pos][order]
    c1 = (d * aw)[pos][order]
    c2 = (d * d / a)[pos][order]
    # suffix sums: active set for theta in [thk[l-1], thk[l]) is order[l:]
    S1 = np.concatenate([np.cumsum(c1[::-1])[::-1], [0.0]])
    S2 = np.concatenate([np.cumsum(c2[::-1])[::-1], [0.0]])
    theta = None
    lo = 0.0
    for l in range(len(thk) + 1):
        hi = thk[l] if l < len(thk) else np.inf
        if hi <= lo and l < len(thk):
            continue
        root = (S1[l] - v) / (1.0 / rho_b + S2[l])
        if root <= hi:
            theta = max(root, lo)
            break
        lo = hi
    z = np.sign(wbar + theta * s / a) * np.maximum(np.abs(wbar + theta * s / a) - theta / a, 0.0)
    return z, float(np.sum(np.abs(z))), float(theta)


def topk_support(z: np.ndarray, kappa: int) -> np.ndarray:
    """T_kappa(z): indices of the kappa largest |z|, ties broken toward the lower
    index (-0 equals +0), returned in ascending index order."""
    n = z.shape[0]
    order = np.lexsort((np.arange(n), -np.abs(z)))
    return np.sort(order[:kappa])


def s_step(z: np.ndarray, tau: float, kappa: int):
    """s-step (Sec. 3, scaled bilinear term): min_{s in S^kappa} (z^T s - tau)^2,
    tau = t - v.  The attainable values of z^T s fill [-M_k, M_k], M_k = sum of
    the kappa largest |z|; the minimiser taken is
    s = clip(tau / M_k, -1, 1) sign(z) on T_kappa(z), 0 elsewhere (s = 0 if M_k = 0)."""
    T = topk_support(z, kappa)
    Mk = float(np.sum(np.abs(z[T])))
    s = np.zeros_like(z)
    if Mk > 0:
        s[T] = np.clip(tau / Mk, -1.0, 1.0) * np.sign(z[T])
    return s, T


# ---------------------------------------------------------------- the solver
@dataclass
class State:
    x: np.ndarray            # N x n (x C)   local estimates x_i
    u: np.ndarray            # N x n (x C)   scaled consensus duals u_i
    omega: List[np.ndarray]  # per partition, m_i (x C)   omega-bar
    nu: List[np.ndarray]     # per partition, m_i (x C)   nu
    z: np.ndarray
    s: np.ndarray
    t: float = 0.0
    v: float = 0.0
    k: int = 0
    history: list = field(default_factory=list)


class BiCADMM:
    """FP64 Bi-cADMM over N sample partitions with M feature blocks each.

    A_parts are FP64 arrays m_i x n; b_parts targets (squared), +-1 labels
    (logistic) or class ids (softmax).  For softmax the variables are n x C and
    the sparsity counts rows."""

    def __init__(self, A_parts, b_parts, loss: int, n_blocks: int, kappa: int, gamma: float,
                 rho_c: float, rho_b: float, rho_l: float, n_classes: int = 1,
                 n_partitions: Optional[int] = None, exact_x: bool = False):
        """n_partitions: the problem's N when only some partitions' data are given
        (x-updates are then run for those partitions only).  exact_x (squared and
        logistic loss): the x-update of every partition is its exact minimiser, the
        limit of Algorithm 2's inner loop, instead of K_in inner iterations (the
        closed form for the squared loss, Newton's method for the logistic loss)."""
        if exact_x and loss not in (LOSS_SQUARED, LOSS_LOGISTIC):
            raise ValueError("the exact x-update is built for the squared and logistic losses")
        self.A = [np.asarray(A, dtype=np.float64) for A in A_parts]
        self.b = [np.asarray(b) for b in b_parts]
        self.loss = loss
        self.N = len(self.A) if n_partitions is None else n_partitions
        self.n = self.A[0].shape[1]
        self.M = n_blocks
        self.kappa = kappa
        self.gamma, self.rho_c, self.rho_b, self.rho_l = gamma, rho_c, rho_b, rho_l
        self.C = n_classes if loss == LOSS_SOFTMAX else 1
        self.blocks = split_columns(self.n, self.M)
        # Cached factors of the x_ij ridge problems (Sec. 3.1, x_ij-step):
        # K_ij = rho_l A_ij^T A_ij + (1/(N gamma) + rho_c) I = L L^T.
        shift = 1.0 / (self.N * gamma) + rho_c
        self.L = []
        for A in self.A:
            Li = []
            for (c0, c1) in self.blocks:
                Aij = A[:, c0:c1]
                G = Aij.T @ Aij
                K = rho_l * G + shift * np.eye(c1 - c0)
                Li.append(cholesky(K, lower=True))
            self.L.append(Li)
        # Exact x-update of partition i (squared loss): the minimiser of
        # ||A_i x - b_i||^2 + ||x||^2 / (2 N gamma) + (rho_c/2)||x - z + u_i||^2 solves
        # H_i x = 2 A_i^T b_i + rho_c (z - u_i),  H_i = 2 A_i^T A_i + (1/(N gamma) + rho_c) I.
        self.exact_x = exact_x
        if exact_x and loss == LOSS_SQUARED:
            self.H = [cho_factor(2.0 * A.T @ A + shift * np.eye(self.n), lower=True) for A in self.A]
            self.c = [2.0 * A.T @ b for A, b in zip(self.A, self.b)]
        self.state = self.zero_state()

    # -- state
    def _shape(self):
        return (self.n,) if self.C == 1 else (self.n, self.C)

    def _mshape(self, m):
        return (m,) if self.C == 1 else (m, self.C)

    def zero_state(self) -> State:
        sh = self._shape()
        return State(x=np.zeros((self.N,) + sh), u=np.zeros((self.N,) + sh),
                     omega=[np.zeros(self._mshape(A.shape[0])) for A in self.A],
                     nu=[np.zeros(self._mshape(A.shape[0])) for A in self.A],
                     z=np.zeros(sh), s=np.zeros(self.n))

    def block_predictions(self, i: int, x_i: np.ndarray):
        """p_ij = A_ij x_ij for every block j."""
        return [self.A[i][:, c0:c1] @ x_i[c0:c1] for (c0, c1) in self.blocks]

    # -- Algorithm 2 (node level), one partition
    def x_update(self, i: int, inner_iters: int, st: Optional[State] = None):
        st = self.state if st is None else st
        A, b, M = self.A[i], self.b[i], self.M
        x_i = st.x[i]
        z, u_i = st.z, st.u[i]
        p = self.block_predictions(i, x_i)
        for _ in range(inner_iters):
            a = sum(p) / M
            e = st.omega[i] - a - st.nu[i]
            for j, (c0, c1) in enumerate(self.blocks):
                # x_ij-step: argmin r_j(x) + (rho_l/2)||A_ij x - p_ij - e||^2, i.e.
                # K_ij x = rho_l A_ij^T (p_ij + e) + rho_c (z_j - u_ij)
                rhs = self.rho_l * (A[:, c0:c1].T @ (p[j] + e)) + self.rho_c * (z[c0:c1] - u_i[c0:c1])
                y = solve_triangular(self.L[i][j], rhs, lower=True)
                x_i[c0:c1] = solve_triangular(self.L[i][j], y, lower=True, trans="T")
                p[j] = A[:, c0:c1] @ x_i[c0:c1]
            a = sum(p) / M                                   # sample-space average (AllReduce)
            st.omega[i] = omega_prox(self.loss, a + st.nu[i], b, M, self.rho_l)
            st.nu[i] = st.nu[i] + a - st.omega[i]            # nu-update
        st.x[i] = x_i

    def x_update_exact(self, i: int, st: Optional[State] = None):
        st = self.state if st is None else st
        if self.loss == LOSS_LOGISTIC:
            st.x[i] = self.x_update_newton(i, st)
            return
        st.x[i] = cho_solve(self.H[i], self.c[i] + self.rho_c * (st.z - st.u[i]))

    def x_update_newton(self, i: int, st: State, max_iter: int = 100) -> np.ndarray:
        """Exact x-update of partition i for the logistic loss: the unique minimiser of
            phi(x) = sum_k log(1 + exp(-b_k a_k^T x)) + ||x||^2 / (2 N gamma)
                     + (rho_c / 2) ||x - z + u_i||^2
        (the x-subproblem of the ADMM iterations, Sec. 3, without the feature split
        of Sec. 3.1).  Newton's method: gradient A^T(-b sigmoid(-b q)) + s x - rho_c v
        with q = A x, v = z - u_i, s = 1/(N gamma) + rho_c; Hessian
        A^T diag(sigmoid(q) sigmoid(-q)) A + s I, solved exactly; backtracking until
        phi decreases by the Armijo amount or, once phi is flat to rounding, the
        gradient norm decreases; warm-started at the current x_i; stopped once a
        full Newton step is at the rounding level of x."""
        A, b = self.A[i], self.b[i]
        s = 1.0 / (self.N * self.gamma) + self.rho_c
        v = st.z - st.u[i]
        x = st.x[i].copy()

        def phi(xx):
            q = A @ xx
            return (float(np.sum(np.logaddexp(0.0, -b * q))) + float(xx @ xx) / (2.0 * self.N * self.gamma)
                    + 0.5 * self.rho_c * float(np.sum((xx - v) ** 2)))

        def grad(xx):
            sg = expit(-b * (A @ xx))
            return A.T @ (-b * sg) + s * xx - self.rho_c * v, sg

        for _ in range(max_iter):
            g, sg = grad(x)
            D = sg * (1.0 - sg)
            H = A.T @ (D[:, None] * A) + s * np.eye(self.n)
            d = -cho_solve(cho_factor(H, lower=True), g)
            f0, slope, gn, t = phi(x), float(g @ d), float(np.linalg.norm(g)), 1.0
            while t > 1e-12:
                xt = x + t * d
                if phi(xt) <= f0 + 1e-4 * t * slope or np.linalg.norm(grad(xt)[0]) < gn:
                    break
                t *= 0.5
            x = x + t * d
            if t == 1.0 and np.max(np.abs(d)) <= 4 * np.finfo(float).eps * max(np.max(np.abs(x)), 1e-300):
                break
        return x

    def _row_norms(self, X):
        return X if self.C == 1 else np.sqrt(np.sum(X * X, axis=1))

    # -- global level (Algorithm 1) + u-update + residuals
    def global_update(self, st: Optional[State] = None):
        st = self.state if st is None else st
        N, a = self.N, self.N * self.rho_c
        z_old = st.z.copy()
        wbar = np.mean(st.x + st.u, axis=0)
        if self.C == 1:
            z, t, _ = zt_step(wbar, st.s, st.v, a, self.rho_b)
        else:
            # Row sparsity: the (z, t) problem in Z reduces to the vector problem on
            # the row norms omega_r = ||W_r|| (its solution rho >= 0), Z_r = rho_r W_r / omega_r.
            om = self._row_norms(wbar)
            rho, t, _ = zt_step(om, st.s, st.v, a, self.rho_b)
            scale = np.where(om > 0, rho / np.where(om > 0, om, 1.0), 0.0)
            z = wbar * scale[:, None]
        zr = self._row_norms(z)
        s, _ = s_step(zr, t - st.v, self.kappa)
        g = float(zr @ s - t)
        v = st.v + g                                               # v-update
        st.u = st.u + st.x - z[None]                               # u-update
        pr = float(sum(np.linalg.norm((st.x[i] - z).ravel()) for i in range(N)))
        dr = math.sqrt(N) * self.rho_c * float(np.linalg.norm((z - z_old).ravel()))
        br = abs(g)
        st.z, st.t, st.s, st.v = z, t, s, v
        st.k += 1
        st.history.append((pr, dr, br))
        return pr, dr, br

    def iterate(self, outer_iters: int, inner_iters: int, st: Optional[State] = None):
        st = self.state if st is None else st
        for _ in range(outer_iters):
            for i in range(self.N):
                if self.exact_x:
                    self.x_update_exact(i, st)
                else:
                    self.x_update(i, inner_iters, st)
            self.global_update(st)
        return st

    # -- outputs
    def support(self, st: Optional[State] = None) -> np.ndarray:
        st = self.state if st is None else st
        return topk_support(self._row_norms(st.z), self.kappa)

    def coef(self, st: Optional[State] = None) -> np.ndarray:
        """x_hat = z restricted to T_kappa(z) (rows for softmax), zero elsewhere."""
        st = self.state if st is None else st
        T = self.support(st)
        x = np.zeros_like(st.z)
        x[T] = st.z[T]
        return x

    def objective(self, x: np.ndarray) -> float:
        return objective(self.loss, self.A, self.b, x, self.gamma)

    def topk_margin(self, st: Optional[State] = None) -> float:
        """|z|_(kappa) - |z|_(kappa+1): distance of the support decision from a tie."""
        st = self.state if st is None else st
        r = np.sort(self._row_norms(np.abs(st.z)))[::-1]
        if self.kappa >= len(r):
            return float("inf")
        return float(r[self.kappa - 1] - r[self.kappa])
