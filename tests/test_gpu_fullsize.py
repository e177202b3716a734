"""Parity at the benchmark's full size and launch configuration: 8 partitions of
50,000 x 5,000 FP32 rows (sparse logistic regression, 4 feature blocks).

The oracle cannot rerun the whole solve at this size in seconds, so it
recomputes sampled outputs from the GPU's own state: the x-update (Algorithm 2,
K_in inner iterations) of partition 0 over its full 50,000 x 5,000 data, and the
full-size global step (consensus, (z,t), top-kappa s-step, v, u, residuals)
from the GPU's x_i of that iteration.
"""
import numpy as np
import pytest

import datagen
import oracle
from parity import rel

pytestmark = pytest.mark.gpu


def test_config1_full_size_sampled_parity():
    import paper_2405_16267_amd as bca
    w = datagen.config1()
    P = bca.Problem("logistic", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=w.max_iters, dtype="f32")
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    P.step(3)
    before = dict(x=[P.get_vector(bca.VEC_X, i) for i in range(w.N)],
                  u=[P.get_vector(bca.VEC_U, i) for i in range(w.N)],
                  z=P.get_vector(bca.VEC_Z), s=P.get_vector(bca.VEC_S),
                  tv=P.get_vector(bca.VEC_TV), om0=P.get_vector(bca.VEC_OMEGA, 0),
                  nu0=P.get_vector(bca.VEC_NU, 0))
    P.step(1)
    after = dict(x=[P.get_vector(bca.VEC_X, i) for i in range(w.N)],
                 u=[P.get_vector(bca.VEC_U, i) for i in range(w.N)],
                 z=P.get_vector(bca.VEC_Z), s=P.get_vector(bca.VEC_S),
                 tv=P.get_vector(bca.VEC_TV), om0=P.get_vector(bca.VEC_OMEGA, 0),
                 nu0=P.get_vector(bca.VEC_NU, 0), res=P.residuals())
    P.close()

    # x-update of partition 0 at full size
    o = oracle.BiCADMM([datagen.widen(w.A[0])], [w.b[0]], w.loss, w.n_blocks, w.kappa, w.gamma,
                       w.rho_c, w.rho_b, w.rho_l, n_partitions=w.N)
    st = o.zero_state()
    st.x[0] = before["x"][0]
    st.u = np.array(before["u"])
    st.z = before["z"]
    st.omega[0] = before["om0"]
    st.nu[0] = before["nu0"]
    o.x_update(0, w.inner_iters, st)
    assert rel(after["x"][0], st.x[0]) < 1e-5
    assert rel(after["om0"], st.omega[0]) < 1e-5
    assert rel(after["nu0"], st.nu[0]) < 1e-5

    # global step at full size from the GPU's x_i of this iteration
    st.x = np.array(after["x"])
    st.u = np.array(before["u"])
    st.z = before["z"]
    st.s = before["s"]
    st.t, st.v = before["tv"]
    pr, dr, br = o.global_update(st)
    assert rel(after["z"], st.z) < 1e-9
    assert rel(np.array(after["u"]), st.u) < 1e-9
    margin = np.sort(np.abs(st.z))[::-1]
    if margin[w.kappa - 1] - margin[w.kappa] > 1e-9 * margin[0]:
        assert np.array_equal(np.nonzero(after["s"])[0], np.nonzero(st.s)[0])
    assert rel(after["s"], st.s) < 1e-9
    assert abs(after["tv"][0] - st.t) <= 1e-9 * max(1.0, abs(st.t))
    gpr, gdr, gbr, _ = after["res"]
    assert abs(gpr - pr) <= 1e-9 * max(1.0, pr) and abs(gdr - dr) <= 1e-9 * max(1.0, dr)
    assert abs(gbr - br) <= 1e-9 * max(1.0, abs(br))


def test_config1_full_size_last_iteration_and_support():
    """The whole solve at full size (K = 100 outer iterations of the benchmark's
    launch), checked at its last iteration: the oracle recomputes the 100th outer
    iteration from the GPU's state after 99 -- the x-update of EVERY partition over
    its 50,000 x 5,000 data (Algorithm 2, K_in inner iterations), then the global
    step from those x_i -- and the GPU's x_i, z and support after 100 iterations are
    compared with it (support where the top-kappa margin is clear of the FP32 error)."""
    import paper_2405_16267_amd as bca
    w = datagen.config1()
    K = w.max_iters
    P = bca.Problem("logistic", w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=K, dtype="f32")
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    P.step(K - 1)
    before = dict(x=[P.get_vector(bca.VEC_X, i) for i in range(w.N)],
                  u=[P.get_vector(bca.VEC_U, i) for i in range(w.N)],
                  om=[P.get_vector(bca.VEC_OMEGA, i) for i in range(w.N)],
                  nu=[P.get_vector(bca.VEC_NU, i) for i in range(w.N)],
                  z=P.get_vector(bca.VEC_Z), s=P.get_vector(bca.VEC_S), tv=P.get_vector(bca.VEC_TV))
    P.step(1)
    assert P.residuals()[3] == K
    after = dict(x=[P.get_vector(bca.VEC_X, i) for i in range(w.N)], z=P.get_vector(bca.VEC_Z),
                 support=P.support())
    P.close()

    xs = []
    for i in range(w.N):
        o = oracle.BiCADMM([datagen.widen(w.A[i])], [w.b[i]], w.loss, w.n_blocks, w.kappa, w.gamma,
                           w.rho_c, w.rho_b, w.rho_l, n_partitions=w.N)
        st = o.zero_state()
        st.x[0] = before["x"][i]
        st.u = np.array(before["u"])
        st.u[0] = before["u"][i]     # this oracle holds partition i as its partition 0
        st.z = before["z"]
        st.omega[0] = before["om"][i]
        st.nu[0] = before["nu"][i]
        o.x_update(0, w.inner_iters, st)
        assert rel(after["x"][i], st.x[0]) < 1e-5, i
        xs.append(st.x[0].copy())
    st.x = np.array(xs)
    st.u = np.array(before["u"])
    st.z = before["z"]
    st.s = before["s"]
    st.t, st.v = before["tv"]
    o.global_update(st)
    assert rel(after["z"], st.z) < 1e-5
    assert o.topk_margin(st) > 1e-4 * float(np.max(np.abs(st.z)))
    assert np.array_equal(after["support"], o.support(st))
