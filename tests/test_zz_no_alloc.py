"""bca_batch_step_noalloc (the batched step without device allocation) against
bca_batch_step: two calls in a row on fresh problem sets, the second batch
smaller than the first, every result bitwise equal to the allocating entry
point's (same kernels) and within 1e-5 of the FP64 oracle (FP32 storage); a
batch beyond the fixed scratch is refused with BCA_E_INVALID."""
import ctypes

import numpy as np
import pytest

import datagen
import oracle
from parity import rel

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


def _same_state(bca, p, q, N):
    assert np.array_equal(p.get_vector(bca.VEC_Z), q.get_vector(bca.VEC_Z))
    assert np.array_equal(p.history(), q.history())
    for i in range(N):
        assert np.array_equal(p.get_vector(bca.VEC_X, i), q.get_vector(bca.VEC_X, i))
        assert np.array_equal(p.get_vector(bca.VEC_NU, i), q.get_vector(bca.VEC_NU, i))


def test_noalloc_batch_step_matches_allocating_entry_point():
    bca = _bca()
    big = [(0, 2300, 60), (1, 1900, 130), (2, 4100, 517), (3, 1500, 1100), (4, 2600, 260)]
    small = [(5, 700, 53), (6, 900, 90)]
    for k, specs in enumerate((big, small)):
        K = 8 - 2 * k
        ws = [datagen.batched_instance(r, m, n, dtype="f32", max_iters=K) for r, m, n in specs]
        A = [make(w) for w in ws]
        B = [make(w) for w in ws]
        bca.batch_step_noalloc(A, 3)
        bca.batch_step_noalloc(A, K - 3)
        bca.batch_step(B, 3)
        bca.batch_step(B, K - 3)
        for w, p, q in zip(ws, A, B):
            assert p.residuals()[3] == K
            _same_state(bca, p, q, w.N)
            o = oracle.BiCADMM([datagen.widen(a) for a in w.A], w.b, w.loss, w.n_blocks, w.kappa,
                               w.gamma, w.rho_c, w.rho_b, w.rho_l)
            o.iterate(K, w.inner_iters)
            z, oz = p.get_vector(bca.VEC_Z), o.state.z
            assert rel(z, oz) < 1e-5 and float(np.max(np.abs(z - oz))) <= 1e-5 * float(np.max(np.abs(oz)))
        for p in A + B:
            p.close()


def test_noalloc_batch_step_refuses_more_than_its_scratch():
    bca = _bca()
    # one phase counter per phase: 1 + outer x (4 K_in + 1) counters of 4 bytes
    # exceed 16 MiB for 300,000 outer iterations
    w = datagen.batched_instance(7, 600, 40, dtype="f32", max_iters=300000)
    P = make(w)
    with pytest.raises(bca.BcaError) as e:
        bca.batch_step_noalloc([P], 300000)
    assert e.value.code == -1 and "scratch" in str(e.value)
    assert P.residuals()[3] == 0
    P.close()
