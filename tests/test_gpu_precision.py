"""Precision form: A stored in BF16 (FP32 products, FP64 long sums, BF16 MFMA
Gram with FP32 accumulation, FP64 Cholesky / residuals), run beside the FP32
form on the same data.

Two references (the stated BF16 bound):
  (i)  the FP64 oracle on the BF16-rounded data widened exactly to FP64 -- this
       isolates the arithmetic of the path and must agree to 1e-5 like FP32;
  (ii) the FP64 oracle on the canonical FP32 data -- this adds the quantisation
       of A (unit roundoff u = 2^-8 per element); the measured coefficient error
       must stay within the first-order bound 4 cond(K) u, with cond(K) the
       largest condition number of the block ridge matrices K_ij.
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


def make(w, dtype):
    bca = _bca()
    P = bca.Problem("squared", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype=dtype)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def test_bf16_form_against_both_references():
    kw = dict(N=3, m_per=[800, 750, 777], n=602, kappa=12, k_true=12, noise=0.05, n_blocks=4,
              normalize=True, max_iters=25)
    wb = datagen.linear_workload(2, dtype="bf16", **kw)
    w32 = datagen.linear_workload(2, dtype="f32", **kw)
    Pb = make(wb, "bf16")
    P32 = make(w32, "f32")
    Pb.step(wb.max_iters)
    P32.step(w32.max_iters)
    # (i) oracle on the BF16-rounded data
    ob = oracle.BiCADMM([datagen.widen(a) for a in wb.A], wb.b, wb.loss, wb.n_blocks, wb.kappa,
                        wb.gamma, wb.rho_c, wb.rho_b, wb.rho_l)
    ob.iterate(wb.max_iters, wb.inner_iters)
    assert ob.topk_margin() > 1e-4
    assert np.array_equal(Pb.support(), ob.support())
    assert_coef_close(Pb.coef(), ob.coef(), 1e-5)
    assert abs(Pb.objective() - ob.objective(ob.coef())) <= 1e-5 * abs(ob.objective(ob.coef()))
    # (ii) oracle on the canonical FP32 data; FP32 form matches it to 1e-5
    o32 = oracle.BiCADMM([datagen.widen(a) for a in w32.A], w32.b, w32.loss, w32.n_blocks,
                         w32.kappa, w32.gamma, w32.rho_c, w32.rho_b, w32.rho_l)
    o32.iterate(w32.max_iters, w32.inner_iters)
    assert_coef_close(P32.coef(), o32.coef(), 1e-5)
    cond = 0.0
    shift = 1.0 / (w32.N * w32.gamma) + w32.rho_c
    for A in w32.A:
        A = datagen.widen(A)
        for c0, c1 in oracle.split_columns(w32.n, w32.n_blocks):
            ev = np.linalg.eigvalsh(w32.rho_l * A[:, c0:c1].T @ A[:, c0:c1] + shift * np.eye(c1 - c0))
            cond = max(cond, ev[-1] / ev[0])
    err = rel(Pb.coef(), o32.coef())
    bound = 4 * cond * 2.0 ** -8
    assert err <= bound, (err, bound)
    Pb.close()
    P32.close()
