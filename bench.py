"""Benchmark of the Bi-cADMM hot path on one MI355X.

Workload (default): sparse logistic regression, 8 sample partitions of
50,000 x 5,000 FP32 rows (AR(1) rows with Toeplitz covariance 0.3^|i-j|), planted
50-sparse model, kappa = 50, 4 feature blocks per partition, 5 inner iterations
per outer iteration.  One step = one outer Bi-cADMM iteration (5 passes of the
node-level loop over all partitions, then the global step).  Inputs are resident
in HBM before the timed region starts.

Prints one JSON line with the step rate, the roofline of the dominant kernel
(the fused A-streaming pass, timed with HIP events on the library's stream) and
the FP64 oracle timed on a bounded sample on the host cores.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP64_PEAK_TFLOPS = 78.6


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


# Sources that define the A-streaming kernel; counter-based traffic figures are
# only reported for the exact source they were taken on.
STREAM_SOURCES = ("paper_2405_16267_amd/csrc/stream.hip", "paper_2405_16267_amd/csrc/prox_impl.h",
                  "paper_2405_16267_amd/csrc/bca_internal.h")


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_traffic(kernel, workload_name, src_hash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summaries
    (FETCH_SIZE and WRITE_SIZE passes, each scaled by the plain-copy calibration),
    or None when no summary was taken on the current kernel source."""
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as fh:
            for line in fh:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
                if (kv.get("kernel") == kernel and kv.get("workload") == workload_name
                        and kv.get("source") == src_hash):
                    return float(kv["read_bytes"]) + float(kv["write_bytes"]), os.path.basename(path)
    return None, None


def workload(name):
    import datagen
    if name == "slogr_8x50000x5000_f32":
        return datagen.config1()
    if name == "slinr_4x500x200_f64":
        return datagen.config0()
    if name.startswith("slogr_small"):
        return datagen.config1(N=8, m_per=5000, n=1000, kappa=20)
    if name == "slinr_8x50000x5000_f32":
        # the same shape with the squared loss (closed-form prox)
        return datagen.linear_workload(1, N=8, m_per=50000, n=5000, kappa=50, k_true=50,
                                       noise=0.1, n_blocks=4, dtype="f32", max_iters=100,
                                       name=name)
    if name == "ssvm_8x50000x5000_f32":
        # the same shape, sparse SVM (hinge loss) on the sparse linear recipe's rows
        return datagen.svm_workload(1, N=8, m_per=50000, n=5000, kappa=50, k_true=50,
                                    n_blocks=4, dtype="f32", max_iters=100, name=name)
    if name == "ssr_4x5000x1000x10_f32":
        # the serving trace's softmax request: 4 partitions of 5,000 rows, n = 1,000,
        # C = 10 classes, 30 nonzero rows of W*
        w = datagen.softmax_request(4007, max_iters=100)
        w.name = name
        return w
    raise SystemExit("unknown workload " + name)


def host_info():
    """Logical CPUs, CPU model and socket count of the host that runs the oracle."""
    model, sockets = "unknown", set()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "sockets": max(len(sockets), 1)}


def oracle_baseline(w, min_seconds=10.0, max_outer=10):
    """The FP64 oracle, as it is, on the whole problem: full outer iterations (the
    x-update of every partition, K_in inner iterations each, then the global step)
    from the zero state, repeated until `min_seconds` of CPU work or `max_outer`
    iterations; its one-time factorisation is not timed."""
    import datagen
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    A = [datagen.widen(a) for a in w.A]
    t0 = time.perf_counter()
    o = oracle.BiCADMM(A, w.b, w.loss, w.n_blocks, w.kappa, w.gamma, w.rho_c, w.rho_b, w.rho_l,
                       n_classes=w.n_classes)
    setup_s = time.perf_counter() - t0
    k = 0
    t0 = time.perf_counter()
    while k < max_outer and (k == 0 or time.perf_counter() - t0 < min_seconds):
        o.iterate(1, w.inner_iters)
        k += 1
    el = time.perf_counter() - t0
    out = {"value": k / el, "unit": "iter/s", "cores": int(cores), "kind": "oracle",
           "sample": "%d full outer iterations (all %d partitions, %d inner iterations each, "
                     "then the global step) from the zero state: %.1f s of CPU work; the "
                     "oracle's factorisation (%.1f s) is not timed" % (k, w.N, w.inner_iters, el, setup_s)}
    out.update(host_info())
    return out


def make_problem(bca, w):
    P = bca.Problem({0: "squared", 1: "logistic", 2: "softmax"}[w.loss], w.n, w.rows, w.n_blocks,
                    w.kappa, gamma=w.gamma, rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l,
                    inner_iters=w.inner_iters, max_iters=w.max_iters, dtype=w.dtype,
                    n_classes=w.n_classes)
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    P.finalize()
    return P


def batched_bench(args):
    """Many uneven problems (sizes log-uniform in m in [500, 20000], n in [50, 2000];
    half squared, half logistic; FP32; 4 partitions x 2 blocks) solved for
    `iters` outer iterations each in one persistent launch, tile shapes from the
    autotuner."""
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    t = time.perf_counter()
    ms, ns = datagen.config3_sizes(3, args.instances)
    ws = [datagen.batched_instance(r, int(ms[r]), int(ns[r]), max_iters=args.iters)
          for r in range(args.instances)]
    log("generated %d instances in %.1f s" % (len(ws), time.perf_counter() - t))
    t = time.perf_counter()
    probs = [make_problem(bca, w) for w in ws]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    log("setup of %d problems %.1f s" % (len(ws), setup_s))
    t = time.perf_counter()
    bca.batch_autotune(probs)
    tune_s = time.perf_counter() - t
    shapes = {}
    for P in probs:
        shapes[str(P.batch_shape())] = shapes.get(str(P.batch_shape()), 0) + 1
    log("autotune %.1f s, shapes %s" % (tune_s, shapes))
    torch.cuda.synchronize()
    bca.batch_set_tracing(True)
    t0 = time.perf_counter()
    bca.batch_solve(probs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    phase_us, _ = bca.batch_get_tracing()
    bca.batch_set_tracing(False)
    a_bytes = sum(sum(w.rows) * w.n * 4 for w in ws)
    fac_bytes = 0
    for w in ws:
        for j in range(w.n_blocks):
            nj = w.n // w.n_blocks + (1 if j < w.n % w.n_blocks else 0)
            fac_bytes += w.N * nj * (nj + 1) // 2 * 8   # distinct entries of K_ij^-1
    inner = args.iters * ws[0].inner_iters
    gbps = (a_bytes + fac_bytes) * inner / el / 1e9
    its = [P.residuals()[3] for P in probs]
    for P in probs:
        P.close()
    out = {"metric": "batched solves/s + ADMM iter/s + HBM GB/s", "value": len(ws) / el,
           "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": el * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "batched_%d_instances" % len(ws), "iters": args.iters,
                      "inner_iters": ws[0].inner_iters, "N": 4, "M": 2,
                      "sum_A_GB": a_bytes / 1e9},
           "admm_iter_per_s": sum(its) / el,
           "hbm_gbps_algorithmic": gbps, "hbm_frac": gbps / HBM_PEAK_GBPS,
           "setup_s": setup_s, "autotune_s": tune_s, "shapes": shapes,
           # per inner iteration (global: per outer iteration), each with its grid barrier
           "phase_us": {k: round(v / (inner if k in ("rhs", "symv", "xupd", "stream") else
                                      (args.iters if k == "global" else 1)), 1)
                        for k, v in phase_us.items()}}
    print(json.dumps(out), flush=True)


def precision_bench(args):
    """Precision form: sparse linear regression on 16 partitions of 100,000 x 10,000
    (A iid N(0,1), unit-norm columns per partition, planted 100-sparse +-U(1,2)
    model, noise 0.05, kappa = 100, 4 feature blocks), stored as BF16 and, beside
    it on the same GPU, as the canonical FP32 matrix the BF16 values were rounded
    from.  Both forms run the same iterations; reported: iter/s and the streaming
    roofline of each, the Gram's MFMA utilisation for each dtype, and the BF16
    result's deviation from the FP32 result with the first-order BF16 bound
    4 cond(K) 2^-8 (cond of feature block 0 of partition 0, from its cached inverse)."""
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    N, m, n, kappa, Mb = 16, args.m_per or 100000, 10000 if not args.m_per else max(1000, args.m_per // 10), 100, 4
    supp, val = datagen.linear_model(2, n, kappa)
    rows = [m] * N
    kw = dict(gamma=10.0, rho_c=1.0, rho_b=0.5, rho_l=1.0, inner_iters=5,
              max_iters=args.warmup + args.steps)
    kw["max_iters"] += 1             # one more outer iteration, sampled by the oracle
    Pb = bca.Problem("squared", n, rows, Mb, kappa, dtype="bf16", **kw)
    P32 = bca.Problem("squared", n, rows, Mb, kappa, dtype="f32", **kw)
    t = time.perf_counter()
    for i in range(N):
        (A32, Abf), b = datagen.linear_partition(2, i, m, n, supp, val, 0.05, "f32+bf16", True)
        Pb.set_data(i, Abf, b)
        P32.set_data(i, A32, b)
        del A32, Abf, b
        log("partition %d of %d resident (%.1f s)" % (i + 1, N, time.perf_counter() - t))
    bounds = [(n // Mb + (1 if j < n % Mb else 0)) for j in range(Mb)]
    gram_flops = sum(m * nj * (nj + 1) for nj in bounds) * N
    res = {}
    for name, P, esize, peak in (("bf16", Pb, 2, BF16_MFMA_PEAK_TFLOPS),
                                 ("f32", P32, 4, FP32_MFMA_PEAK_TFLOPS)):
        P.set_timing(True)
        t = time.perf_counter()
        P.finalize()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        n_gram, gram_ms = P.timing(bca.KC_GRAM)
        n_fac, fac_ms = P.timing(bca.KC_FACTOR)
        P.set_timing(False)
        P.step(args.warmup)
        torch.cuda.synchronize()
        P.set_timing(True)
        t0 = time.perf_counter()
        P.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n_st, st_ms = P.timing(bca.KC_STREAM)
        n_so, so_ms = P.timing(bca.KC_SOLVE)
        n_gl, gl_ms = P.timing(bca.KC_GLOBAL)
        stream_bytes = N * m * n * esize + 32 * N * m
        avg_s = st_ms / max(n_st, 1) / 1e3
        ach = stream_bytes / avg_s / 1e9
        gtf = gram_flops / (gram_ms / 1e3) / 1e12 if gram_ms > 0 else None
        log("%s: %.2f iter/s, stream %.3f ms (%.0f GB/s), gram %.1f ms" % (name, args.steps / el, avg_s * 1e3, ach, gram_ms))
        res[name] = {"iter_per_s": args.steps / el, "ms_per_step": el / args.steps * 1e3,
                     "roofline": {"bound": "hbm", "kernel": "stream_kernel", "achieved": ach,
                                  "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS,
                                  "bytes_per_launch": stream_bytes, "avg_launch_ms": avg_s * 1e3,
                                  "launches": n_st},
                     "kernels_ms_per_step": {"stream": st_ms / args.steps, "solve": so_ms / args.steps,
                                             "global": gl_ms / args.steps},
                     "setup": {"seconds": setup_s, "gram_ms": gram_ms, "factor_ms": fac_ms,
                               "gram_tflops": gtf, "gram_mfma_peak_tflops": peak,
                               "gram_mfma_frac": gtf / peak if gtf else None}}
    xb, x32 = Pb.coef(), P32.coef()
    fb, f32 = Pb.objective(), P32.objective()
    same_support = bool(np.array_equal(Pb.support(), P32.support()))
    ev = np.linalg.eigvalsh(P32.inverse(0, 0))
    condK = float(ev[-1] / ev[0])
    # error against the FP64 oracle, sampled: one more outer iteration of each form, and
    # the oracle's x-update of partition 0 (five inner iterations over its full
    # 100,000 x 10,000 data) from the GPU's state before it
    snap = {}
    for name, P in (("bf16", Pb), ("f32", P32)):
        before = dict(x0=P.get_vector(bca.VEC_X, 0), u=np.array([P.get_vector(bca.VEC_U, i) for i in range(N)]),
                      z=P.get_vector(bca.VEC_Z), om0=P.get_vector(bca.VEC_OMEGA, 0), nu0=P.get_vector(bca.VEC_NU, 0))
        P.step(1)
        snap[name] = (before, P.get_vector(bca.VEC_X, 0))
    Pb.close()
    P32.close()
    oracle_err = precision_oracle_check(snap, N, m, n, Mb, kappa, supp, val)
    err = float(np.linalg.norm(xb - x32) / np.linalg.norm(x32))
    out = {"metric": "ADMM iter/s + HBM GB/s (precision form, BF16 beside FP32)",
           "value": res["bf16"]["iter_per_s"], "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["bf16"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic",
           "config": {"workload": "slinr_%dx%dx%d_bf16_beside_f32" % (N, m, n), "N": N,
                      "m_per_partition": m, "n": n, "M": Mb, "kappa": kappa, "inner_iters": 5},
           "bf16": res["bf16"], "f32": res["f32"],
           "bf16_vs_f32": {"coef_rel": err, "objective_rel": abs(fb - f32) / abs(f32),
                           "same_support": same_support, "cond_K_block0": condK,
                           "first_order_bound": 4 * condK * 2.0 ** -8},
           "vs_fp64_oracle": oracle_err}
    print(json.dumps(out), flush=True)


def precision_oracle_check(snap, N, m, n, M, kappa, supp, val):
    """Relative error of partition 0's x after one outer iteration, against the FP64
    oracle's x-update (Algorithm 2, five inner iterations) from the GPU's own state:
    BF16 against the oracle on the BF16 data widened to FP64 (arithmetic error) and on
    the canonical FP32 data (plus quantisation); FP32 against the canonical data."""
    import numpy as np
    import datagen
    import oracle
    from oracle.bicadmm import LOSS_SQUARED
    t = time.perf_counter()
    (A32, Abf), b = datagen.linear_partition(2, 0, m, n, supp, val, 0.05, "f32+bf16", True)
    out = {}
    for ref, A in (("bf16_data", Abf), ("canonical_f32_data", A32)):
        o = oracle.BiCADMM([datagen.widen(A)], [b], LOSS_SQUARED, M, kappa, 10.0, 1.0, 0.5, 1.0,
                           n_partitions=N)
        for name in ("bf16", "f32"):
            if ref == "bf16_data" and name == "f32":
                continue
            before, x_after = snap[name]
            st = o.zero_state()
            st.x[0] = before["x0"]
            st.u = before["u"]
            st.z = before["z"]
            st.omega[0] = before["om0"]
            st.nu[0] = before["nu0"]
            o.x_update(0, 5, st)
            d = x_after - st.x[0]
            out["%s_vs_oracle_on_%s" % (name, ref)] = {
                "x_rel": float(np.linalg.norm(d) / np.linalg.norm(st.x[0])),
                "x_max_abs_rel": float(np.max(np.abs(d)) / np.max(np.abs(st.x[0])))}
        del o
    out["sample"] = ("partition 0's x after the last outer iteration (Algorithm 2's five inner "
                     "iterations over its 100,000 x 10,000 data), from the GPU's state before it")
    log("oracle check of the precision form %.1f s" % (time.perf_counter() - t))
    return out


def setup_bench(args):
    """One-time setup at the precision workload's shape (16 partitions of 100,000 x
    10,000, 4 feature blocks of 2,500 columns): the Gram A_ij^T A_ij on MFMA and the
    FP64 factorisation (Cholesky, W = L^-1, K^-1 = W^T W), for BF16 and FP32 storage.
    A is drawn on the device with torch's seeded normal generator, N(0, 1/m) (the
    Gram's speed does not depend on the values)."""
    import math
    import torch
    import paper_2405_16267_amd as bca
    N, m, n, M = 16, args.m_per or 100000, 10000, 4
    bounds = [(n // M + (1 if j < n % M else 0)) for j in range(M)]
    flops = N * sum(m * nj * (nj + 1) for nj in bounds)
    res = {}
    for dtype, peak in (("bf16", BF16_MFMA_PEAK_TFLOPS), ("f32", FP32_MFMA_PEAK_TFLOPS)):
        P = bca.Problem("squared", n, [m] * N, M, 100, dtype=dtype, max_iters=1)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(5)
        b = torch.zeros(m, device="cuda", dtype=torch.float64)
        for i in range(N):
            X = torch.randn(m, n, device="cuda", generator=gen) / math.sqrt(m)
            if dtype == "bf16":
                X = X.to(torch.bfloat16).view(torch.int16)
            P.set_data(i, X, b)
            del X
        torch.cuda.synchronize()
        P.set_timing(True)
        t = time.perf_counter()
        P.finalize()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        _, gram_ms = P.timing(bca.KC_GRAM)
        _, fac_ms = P.timing(bca.KC_FACTOR)
        P.close()
        torch.cuda.empty_cache()
        tf = flops / (gram_ms / 1e3) / 1e12
        log("%s: Gram %.2f ms (%.1f TFLOP/s, %.3f of peak), factorisation %.2f ms" % (dtype, gram_ms, tf, tf / peak, fac_ms))
        res[dtype] = {"gram_ms": gram_ms, "gram_tflops": tf, "gram_peak_tflops": peak,
                      "gram_mfma_frac": tf / peak, "factor_ms": fac_ms, "setup_s": setup_s}
    out = {"metric": "Gram TFLOP/s (MFMA, once per problem) + factorisation ms",
           "value": res["bf16"]["gram_tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": res["bf16"]["gram_ms"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
           "config": {"workload": "gram_%dx%dx%d_M%d" % (N, m, n, M), "N": N, "m_per_partition": m,
                      "n": n, "M": M, "flops": flops},
           "roofline": {"bound": "mfma", "kernel": "gram_dma_bf16_kernel",
                        "achieved": res["bf16"]["gram_tflops"], "peak": BF16_MFMA_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": res["bf16"]["gram_mfma_frac"], "traffic": None},
           "bf16": res["bf16"], "f32": res["f32"]}
    print(json.dumps(out), flush=True)


# End-to-end solve times of Bi-cADMM in the paper's Table 1 (sparse least squares,
# 4 nodes sharing one RTX 4070 GPU with an i7-13700 host; PyTorch + mpi4py), in
# seconds, keyed by (s_l, total rows m, features n).  Context, not a target: other
# hardware, and the paper does not state its precision, parameters or stopping rule.
PAPER_TABLE1_S = {
    (0.6, 100000, 2000): 1.1, (0.6, 100000, 4000): 1.8,
    (0.6, 200000, 2000): 1.7, (0.6, 200000, 4000): 3.0,
    (0.6, 300000, 2000): 2.2, (0.6, 300000, 4000): 4.0,
    (0.9, 100000, 2000): 1.1, (0.9, 100000, 4000): 1.9,
    (0.9, 200000, 2000): 1.7, (0.9, 200000, 4000): 2.9,
    (0.9, 300000, 2000): 2.2, (0.9, 300000, 4000): 4.1,
}


def paper_shapes_bench(args):
    """The shapes of the paper's Table 1 solved end to end on one GPU: sparse least
    squares on N = 4 sample partitions of m/4 rows, m in {1e5, 2e5, 3e5}, n in
    {2,000, 4,000}, kappa = round(n (1 - s_l)) for sparsity levels s_l in {0.6, 0.9};
    A iid N(0,1) with unit-norm columns per partition (FP32), a planted model with
    kappa nonzeros of values +-U(1,2), noise 0.05.  One feature block per partition
    (the paper's nodes share one GPU), gamma = 10, rho_c = rho_l = 1, rho_b = 0.5,
    K_in = 5, stopping when p_r, d_r and b_r are all below 1e-4 (checked every 10
    outer iterations) or after 500.  Timed: Gram, factorisation and iterations with
    the data already in HBM ("solve"), and separately the host-to-device copy."""
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    N, seed, noise = 4, 5, 0.05
    rows_out = []
    total_solve = 0.0
    for n in (2000, 4000):
        for m in (100000, 200000, 300000):
            mp = m // N
            models = {}
            for sl in (0.6, 0.9):
                kappa = int(round(n * (1 - sl)))
                models[sl] = (kappa,) + datagen.linear_model(seed + int(10 * sl), n, kappa)
            probs = {}
            copy_s = {}
            for sl, (kappa, supp, val) in models.items():
                probs[sl] = bca.Problem("squared", n, [mp] * N, 1, kappa, gamma=10.0, rho_c=1.0,
                                        rho_b=0.5, rho_l=1.0, inner_iters=5, max_iters=500,
                                        dtype="f32", tol=(1e-4, 1e-4, 1e-4), check_every=10)
                copy_s[sl] = 0.0
            for i in range(N):
                k6, s6, v6 = models[0.6]
                A, b6 = datagen.linear_partition(seed, i, mp, n, s6, v6, noise, "f32", True)
                k9, s9, v9 = models[0.9]
                b9 = datagen.linear_targets(seed, i, A, s9, v9, noise)
                for sl, b in ((0.6, b6), (0.9, b9)):
                    torch.cuda.synchronize()
                    t = time.perf_counter()
                    probs[sl].set_data(i, A, b)
                    torch.cuda.synchronize()
                    copy_s[sl] += time.perf_counter() - t
                del A, b6, b9
            for sl, (kappa, supp, val) in models.items():
                P = probs[sl]
                torch.cuda.synchronize()
                t = time.perf_counter()
                P.finalize()
                k, conv = P.solve()
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                total_solve += el
                found = np.intersect1d(P.support(), supp).size
                paper = PAPER_TABLE1_S[(sl, m, n)]
                log("s_l %.1f m %d n %d kappa %d: %.3f s (%d iterations, converged %s), copy %.3f s, "
                    "planted support found %d/%d; paper %.1f s" % (sl, m, n, kappa, el, k, conv,
                                                                    copy_s[sl], found, kappa, paper))
                rows_out.append({"s_l": sl, "m": m, "n": n, "kappa": kappa, "solve_s": el,
                                 "iterations": k, "converged": conv, "copy_s": copy_s[sl],
                                 "planted_found": int(found), "paper_s": paper,
                                 "paper_over_ours": paper / el})
                P.close()
    ratios = [r["paper_over_ours"] for r in rows_out]
    out = {"metric": "end-to-end solve time at the paper's Table 1 shapes (context)",
           "value": total_solve, "unit": "s", "n_gpus": 1, "steps": len(rows_out), "warmup": 0,
           "ms_per_step": total_solve / len(rows_out) * 1e3, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "sls_table1_shapes_4_partitions", "N": N, "M": 1,
                      "m": [100000, 200000, 300000], "n": [2000, 4000], "s_l": [0.6, 0.9],
                      "tol": 1e-4, "max_iters": 500, "inner_iters": 5},
           "paper_hardware": "RTX 4070 (12 GB) + i7-13700; PyTorch 2.3 + mpi4py",
           "geomean_paper_over_ours": float(np.exp(np.mean(np.log(ratios)))),
           "cases": rows_out}
    print(json.dumps(out), flush=True)


def paper_sweeps_bench(args):
    """The remaining experiments of the paper's Sec. 4 run on one GPU (sparse least
    squares, A iid N(0,1) with unit-norm columns per partition, planted model of
    kappa = round(n (1 - s_l)) nonzeros of values +-U(1,2), noise 0.05, one feature
    block per partition, gamma = 10, K_in = 5):
      rho_b   the convergence study (Fig. 1): n = 4,000, m = 10,000 on N = 4
              partitions, s_l = 0.8, rho_b in {2, 4, 8, 16} with rho_c = rho_b / 0.5
              (alpha = 0.5), 200 outer iterations; reported: p_r, d_r, b_r along the run.
      features  feature scaling (Fig. 2): N in {2, 4, 8} partitions of 800 rows,
              n from 1,000 to 10,000, s_l = 0.8; each case solved with the default
              x-step and with the sample-space (Woodbury) x-step.
      samples   sample scaling (Fig. 3): N in {2, 4, 8}, n = 4,000, s_l = 0.8, rows
              per partition from 25,000 to 300,000.
    The scaling runs stop when p_r, d_r and b_r are all below 1e-4 (checked every
    10 outer iterations) or after 500, with rho_c = rho_l = 1, rho_b = 0.5, and time
    Gram, factorisation and iterations with the data in HBM.  For the sample
    scaling the 300,000-row matrices are drawn once per partition and each case
    takes their leading rows, re-normalised on the device."""
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    sweeps = ["rho_b", "features", "samples"] if args.sweep == "all" else [args.sweep]
    out = {"metric": "residual curves and end-to-end solve times of the paper's Sec. 4 "
                     "experiments (context)",
           "n_gpus": 1, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic", "unit": "s",
           "config": {"workload": "sls_sec4_sweeps", "sweeps": sweeps, "M": 1,
                      "inner_iters": 5, "gamma": 10.0, "noise": 0.05}}
    noise, total = 0.05, 0.0

    def solve_case(P, supp):
        torch.cuda.synchronize()
        t = time.perf_counter()
        P.finalize()
        k, conv = P.solve()
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        return el, k, conv, int(np.intersect1d(P.support(), supp).size)

    if "rho_b" in sweeps:
        n, m, N, sl = 4000, 10000, 4, 0.8
        kappa = int(round(n * (1 - sl)))
        supp, val = datagen.linear_model(21, n, kappa)
        parts = [datagen.linear_partition(21, i, m // N, n, supp, val, noise, "f32", True)
                 for i in range(N)]
        curves = []
        for rho_b in (2.0, 4.0, 8.0, 16.0):
            rho_c = rho_b / 0.5
            K = 200
            P = bca.Problem("squared", n, [m // N] * N, 1, kappa, gamma=10.0, rho_c=rho_c,
                            rho_b=rho_b, rho_l=rho_c, inner_iters=5, max_iters=K, dtype="f32")
            for i, (A, b) in enumerate(parts):
                P.set_data(i, A, b)
            torch.cuda.synchronize()
            t = time.perf_counter()
            P.finalize()
            P.step(K)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            total += el
            h = P.history()
            found = int(np.intersect1d(P.support(), supp).size)
            at = [1, 10, 25, 50, 100, 150, 200]
            pts = {str(k): [float(v) for v in h[k - 1]] for k in at if k <= len(h)}
            log("rho_b %4.1f rho_c %4.1f: %.3f s for %d iterations; (p_r, d_r, b_r) at 1: %s, "
                "200: %s; planted support %d/%d" % (rho_b, rho_c, el, len(h), pts.get("1"),
                                                     pts.get("200"), found, kappa))
            curves.append({"rho_b": rho_b, "rho_c": rho_c, "seconds": el, "iterations": len(h),
                           "residuals_p_d_b_at": pts, "planted_found": found, "kappa": kappa})
            P.close()
        del parts
        out["rho_b_sweep"] = {"n": n, "m": m, "N": N, "s_l": sl, "alpha": 0.5, "runs": curves}

    kw = dict(gamma=10.0, rho_c=1.0, rho_b=0.5, rho_l=1.0, inner_iters=5, max_iters=500,
              dtype="f32", tol=(1e-4, 1e-4, 1e-4), check_every=10)
    if "features" in sweeps:
        rows_out = []
        for N in (2, 4, 8):
            for n in (1000, 2500, 5000, 7500, 10000):
                kappa = int(round(n * 0.2))
                supp, val = datagen.linear_model(31, n, kappa)
                parts = [datagen.linear_partition(31, i, 800, n, supp, val, noise, "f32", True)
                         for i in range(N)]
                # the default x-step (n x n inverse per partition) and the sample-space
                # form (800 x 800 per partition), same iterates up to rounding
                rec = {"N": N, "m_per": 800, "n": n, "kappa": kappa}
                for form in ("default", "woodbury"):
                    P = bca.Problem("squared", n, [800] * N, 1, kappa, woodbury=form == "woodbury",
                                    **kw)
                    for i, (A, b) in enumerate(parts):
                        P.set_data(i, A, b)
                    el, k, conv, found = solve_case(P, supp)
                    if form == "default":
                        total += el
                    log("features (%s x-step): N %d n %5d kappa %4d: %.3f s (%d iterations, "
                        "converged %s), planted support %d/%d" % (form, N, n, kappa, el, k, conv,
                                                                  found, kappa))
                    rec.update({form + "_solve_s": el, form + "_iterations": k,
                                form + "_converged": conv, form + "_planted_found": found})
                    P.close()
                rec["woodbury_speedup"] = rec["default_solve_s"] / rec["woodbury_solve_s"]
                rows_out.append(rec)
                del parts
        out["feature_scaling"] = rows_out

    if "samples" in sweeps:
        n, kappa, m_max = 4000, 800, 300000
        supp, val = datagen.linear_model(41, n, kappa)
        x_true = torch.zeros(n, dtype=torch.float64, device="cuda")
        x_true[torch.as_tensor(supp, dtype=torch.long, device="cuda")] = torch.as_tensor(
            val, dtype=torch.float64, device="cuda")
        src = []
        t = time.perf_counter()
        for i in range(8):
            A32 = np.empty((m_max, n), dtype=np.float32)
            datagen.lib().bcd_gaussian_block(41, datagen.S_A + i, m_max, n, 0, 0, datagen._p(A32),
                                             None, n)
            src.append(torch.from_numpy(A32).cuda())
            del A32
        log("samples: 8 x %d x %d drawn and resident (%.1f s)" % (m_max, n, time.perf_counter() - t))
        rows_out = []
        for N in (2, 4, 8):
            for mp in (25000, 50000, 100000, 200000, 300000):
                P = bca.Problem("squared", n, [mp] * N, 1, kappa, **kw)
                for i in range(N):
                    A = src[i][:mp].double()
                    A /= A.norm(dim=0, keepdim=True)
                    gen = torch.Generator(device="cuda").manual_seed(41000 + 8 * mp + i)
                    b = A @ x_true + noise * torch.randn(mp, dtype=torch.float64, device="cuda",
                                                          generator=gen)
                    P.set_data(i, A.float(), b)
                    del A, b
                el, k, conv, found = solve_case(P, supp)
                total += el
                log("samples: N %d m_i %6d: %.3f s (%d iterations, converged %s), planted "
                    "support %d/%d" % (N, mp, el, k, conv, found, kappa))
                rows_out.append({"N": N, "m_per": mp, "n": n, "kappa": kappa, "solve_s": el,
                                 "iterations": k, "converged": conv, "planted_found": found})
                P.close()
        del src
        out["sample_scaling"] = rows_out
    out["value"] = total
    out["steps"] = 0
    out["warmup"] = 0
    out["ms_per_step"] = None
    print(json.dumps(out), flush=True)


def woodbury_bench(args):
    """Sample-space (Woodbury) x-step beside the default one on a wide problem:
    sparse linear regression on 8 partitions of 800 x 10,000 FP32 (the largest
    shape of the paper's feature-scaling runs: iid N(0,1), unit-norm columns per
    partition, planted model of kappa = 2,000 nonzeros of values +-U(1,2), noise
    0.05), one feature block, K_in = 5.  Timed over `steps` outer iterations with
    the kernel split; the sample-space symmetric products read the distinct
    entries of every S_ij^-1 (800 x 800) once per inner iteration, against the
    default form's A pass and 10,000 x 10,000 inverse per partition."""
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    N, m, n, kappa = 8, 800, 10000, 2000
    supp, val = datagen.linear_model(31, n, kappa)
    kw = dict(gamma=10.0, rho_c=1.0, rho_b=0.5, rho_l=1.0, inner_iters=5, dtype="f32",
              max_iters=args.warmup + args.steps)
    parts = [datagen.linear_partition(31, i, m, n, supp, val, 0.05, "f32", True) for i in range(N)]
    res, probs = {}, {}
    for name in ("default", "woodbury"):
        P = bca.Problem("squared", n, [m] * N, 1, kappa, woodbury=name == "woodbury", **kw)
        for i, (A, b) in enumerate(parts):
            P.set_data(i, A, b)
        P.set_timing(True)
        t = time.perf_counter()
        P.finalize()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        _, gram_ms = P.timing(bca.KC_GRAM)
        _, fac_ms = P.timing(bca.KC_FACTOR)
        P.set_timing(False)
        P.step(args.warmup)
        torch.cuda.synchronize()
        P.set_timing(True)
        t0 = time.perf_counter()
        P.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n_so, so_ms = P.timing(bca.KC_SOLVE)
        n_st, st_ms = P.timing(bca.KC_STREAM)
        n_gl, gl_ms = P.timing(bca.KC_GLOBAL)
        P.set_timing(False)
        r = {"iter_per_s": args.steps / el, "ms_per_step": el / args.steps * 1e3,
             "kernels_ms_per_step": {"stream": st_ms / args.steps, "solve": so_ms / args.steps,
                                     "global": gl_ms / args.steps},
             "setup": {"seconds": setup_s, "gram_ms": gram_ms, "factor_ms": fac_ms}}
        if name == "woodbury":
            # per inner iteration: the stored tiles of every S_ij^-1 (one block per partition)
            T = (m + 63) // 64
            sym_bytes = N * T * (T + 1) // 2 * 64 * 64 * 8
            inner_ms = (so_ms - 0.0) / max(n_so, 1)
            ach = sym_bytes / (inner_ms / 1e3) / 1e9
            # two passes over A per outer iteration (A w, then A^T r)
            a_bytes = N * m * n * 4
            pass_ms = st_ms / max(n_st, 1)
            r["sample_space_symv"] = {"bytes_per_launch": sym_bytes, "avg_launch_ms": inner_ms,
                                      "achieved_gbps": ach}
            r["a_pass"] = {"bytes_per_launch": a_bytes, "avg_launch_ms": pass_ms,
                           "achieved_gbps": a_bytes / (pass_ms / 1e3) / 1e9}
        log("%s: %.1f iter/s, setup %.3f s, kernels ms/iter %s" % (name, args.steps / el, setup_s,
                                                                 r["kernels_ms_per_step"]))
        res[name] = r
        probs[name] = P
    d, wb = probs["default"], probs["woodbury"]
    zd, zw = d.get_vector(bca.VEC_Z), wb.get_vector(bca.VEC_Z)
    agree = {"z_rel_diff": float(np.linalg.norm(zd - zw) / max(np.linalg.norm(zw), 1e-300)),
             "same_support": bool(np.array_equal(d.support(), wb.support()))}
    for P in probs.values():
        P.close()
    out = {"metric": "ADMM iter/s (sample-space x-step beside the default one)",
           "value": res["woodbury"]["iter_per_s"], "unit": "iter/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["woodbury"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "slinr_8x800x10000_f32_woodbury", "N": N, "m_per_partition": m,
                      "n": n, "M": 1, "kappa": kappa, "inner_iters": 5},
           "woodbury": res["woodbury"], "default": res["default"], "agreement": agree}
    print(json.dumps(out), flush=True)


def exact_bench(args):
    """Exact x-update (squared loss) beside Algorithm 2 on the same data: sparse
    linear regression, 16 partitions of 100,000 x 10,000 FP32 (the precision
    form's canonical matrix: iid N(0,1), unit-norm columns per partition, planted
    100-sparse model, noise 0.05), kappa = 100.  Each variant is set up, timed over
    `steps` outer iterations, then restarted and run to p_r, d_r, b_r <= 1e-3
    (checked every 10 iterations, at most 400): iterations, time to solution and
    the two results' agreement.  The exact variant's x-update reads the n x n
    inverse of every partition once per outer iteration and no A."""
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    N, m, n, kappa, Mb = 16, args.m_per or 100000, 10000 if not args.m_per else max(1000, args.m_per // 10), 100, 4
    supp, val = datagen.linear_model(2, n, kappa)
    kw = dict(gamma=10.0, rho_c=1.0, rho_b=0.5, rho_l=1.0, inner_iters=5, dtype="f32",
              max_iters=400, tol=(1e-3, 1e-3, 1e-3), check_every=10)
    variants = {"algorithm2": bca.Problem("squared", n, [m] * N, Mb, kappa, **kw),
                "exact": bca.Problem("squared", n, [m] * N, Mb, kappa, exact_x=True, **kw)}
    t = time.perf_counter()
    for i in range(N):
        A32, b = datagen.linear_partition(2, i, m, n, supp, val, 0.05, "f32", True)
        for P in variants.values():
            P.set_data(i, A32, b)
        del A32, b
    log("data resident (%.1f s)" % (time.perf_counter() - t))
    res = {}
    for name, P in variants.items():
        P.set_timing(True)
        t = time.perf_counter()
        P.finalize()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        _, gram_ms = P.timing(bca.KC_GRAM)
        _, fac_ms = P.timing(bca.KC_FACTOR)
        state0 = P.get_state()
        P.set_timing(False)
        P.step(args.warmup)
        torch.cuda.synchronize()
        P.set_timing(True)
        t0 = time.perf_counter()
        P.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n_so, so_ms = P.timing(bca.KC_SOLVE)
        n_st, st_ms = P.timing(bca.KC_STREAM)
        n_gl, gl_ms = P.timing(bca.KC_GLOBAL)
        P.set_timing(False)
        P.set_state(state0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k, conv = P.solve()
        torch.cuda.synchronize()
        sol_s = time.perf_counter() - t0
        r = {"iter_per_s": args.steps / el, "ms_per_step": el / args.steps * 1e3,
             "kernels_ms_per_step": {"stream": st_ms / args.steps, "solve": so_ms / args.steps,
                                     "global": gl_ms / args.steps},
             "setup": {"seconds": setup_s, "gram_ms": gram_ms, "factor_ms": fac_ms},
             "to_tolerance": {"iterations": k, "converged": conv, "seconds": sol_s}}
        if name == "exact":
            # the solve reads the distinct entries of every partition's H_i^-1 once
            sym_bytes = N * n * (n + 1) // 2 * 8
            ach = sym_bytes / (so_ms / max(n_so, 1) / 1e3) / 1e9
            r["roofline"] = {"bound": "hbm", "kernel": "symv_kernel (+ rhs, x update)",
                             "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                             "frac": ach / HBM_PEAK_GBPS, "bytes_per_launch": sym_bytes,
                             "avg_launch_ms": so_ms / max(n_so, 1)}
        log("%s: %.1f iter/s, setup %.2f s, %d iterations to 1e-3 (%s) in %.3f s"
            % (name, args.steps / el, setup_s, k, conv, sol_s))
        res[name] = r
    a2, ex = variants["algorithm2"], variants["exact"]
    same = bool(np.array_equal(a2.support(), ex.support()))
    diff = float(np.linalg.norm(a2.coef() - ex.coef()) / np.linalg.norm(ex.coef()))
    planted = int(np.intersect1d(ex.support(), supp).size)
    for P in variants.values():
        P.close()
    out = {"metric": "ADMM iter/s + time to tolerance (exact x-update beside Algorithm 2)",
           "value": res["exact"]["iter_per_s"], "unit": "iter/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res["exact"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "slinr_16x100000x10000_f32_exact_x", "N": N, "m_per_partition": m,
                      "n": n, "M": Mb, "kappa": kappa, "inner_iters": 5, "tol": 1e-3},
           "exact": res["exact"], "algorithm2": res["algorithm2"],
           "agreement": {"same_support": same, "coef_rel_diff": diff, "planted_found": planted}}
    print(json.dumps(out), flush=True)


def exact_logistic_bench(args):
    """Exact x-update of the logistic loss (Newton-CG) beside Algorithm 2 on the
    default workload's data (sparse logistic regression, 8 partitions of 50,000 x
    5,000 FP32, AR(1) rows): both run the same `steps` outer iterations from the
    zero state.  Reported: iter/s, passes over A per outer iteration (gradient and
    Hessian-vector passes against Algorithm 2's K_in fused passes), the residuals
    reached, and the two results' agreement."""
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    w = datagen.config1()
    res, probs = {}, {}
    for name, exact in (("algorithm2", False), ("exact_newton_cg", True)):
        P = bca.Problem("logistic", w.n, w.rows, 1 if exact else w.n_blocks, w.kappa, gamma=w.gamma,
                        rho_c=w.rho_c, rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                        max_iters=args.steps, dtype=w.dtype, exact_x=exact)
        for i in range(w.N):
            P.set_data(i, w.A[i], w.b[i])
        P.set_timing(True)
        t = time.perf_counter()
        P.finalize()
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t
        _, gram_ms = P.timing(bca.KC_GRAM)
        _, fac_ms = P.timing(bca.KC_FACTOR)
        t0 = time.perf_counter()
        P.step(args.steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        n_st, st_ms = P.timing(bca.KC_STREAM)
        n_so, so_ms = P.timing(bca.KC_SOLVE)
        n_gl, gl_ms = P.timing(bca.KC_GLOBAL)
        pr, dr, br, it = P.residuals()
        log("%s: %.2f iter/s, %.1f streaming launches per outer iteration, p_r %.3e d_r %.3e"
            % (name, args.steps / el, n_st / args.steps, pr, dr))
        res[name] = {"iter_per_s": args.steps / el, "ms_per_step": el / args.steps * 1e3,
                     "stream_launches_per_outer": n_st / args.steps,
                     "kernels_ms_per_step": {"stream": st_ms / args.steps, "solve": so_ms / args.steps,
                                             "global": gl_ms / args.steps},
                     "setup": {"seconds": setup_s, "gram_ms": gram_ms, "factor_ms": fac_ms},
                     "residuals": {"iter": it, "p_r": pr, "d_r": dr, "b_r": br}}
        probs[name] = P
    a2, ex = probs["algorithm2"], probs["exact_newton_cg"]
    same = bool(np.array_equal(a2.support(), ex.support()))
    diff = float(np.linalg.norm(a2.coef() - ex.coef()) / max(np.linalg.norm(ex.coef()), 1e-300))
    for P in probs.values():
        P.close()
    out = {"metric": "ADMM iter/s (logistic exact x-update by Newton-CG beside Algorithm 2)",
           "value": res["exact_newton_cg"]["iter_per_s"], "unit": "iter/s", "n_gpus": 1,
           "steps": args.steps, "warmup": 0, "ms_per_step": res["exact_newton_cg"]["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "slogr_8x50000x5000_f32_exact_x", "N": w.N, "m_per_partition": w.rows[0],
                      "n": w.n, "kappa": w.kappa, "inner_iters": w.inner_iters},
           "exact_newton_cg": res["exact_newton_cg"], "algorithm2": res["algorithm2"],
           "agreement_after_equal_iterations": {"same_support": same, "coef_rel_diff": diff}}
    print(json.dumps(out), flush=True)


# Offered rate of the serving trace, frozen: 1.5 x the plain method's rate on the
# trace's first 20 requests, measured on one MI355X (32.9-33.6 solves/s over four
# runs with the MFMA softmax kernels; `--rate 0` measures it again and uses that).
SERVE_PLAIN_RATE = 33.3
SERVE_RATE = 1.5 * SERVE_PLAIN_RATE


def serve_bench(args):
    """Continuous batching on a Poisson trace versus the plain one-at-a-time method
    on the same trace.  Requests: 80% sparse-fit problems of the batched size
    distribution (even: squared, odd: logistic), 20% softmax (C = 10, n = 1000,
    m = 20,000, 30 nonzero rows); each runs `iters` outer iterations.  Arrivals are
    Poisson at a frozen rate (1.5 x plain).  Reported for both methods: completions
    per second over the whole trace and over its steady window (the releases of
    requests R/10 .. 9R/10), latency percentiles after the first R/10 requests, and
    the backlog (submitted, not finished) sampled through the window: a stable
    queue keeps it flat, an overloaded one grows it."""
    import threading
    import numpy as np
    import torch
    import datagen
    import paper_2405_16267_amd as bca
    R = args.requests
    kind = datagen.uniform_vector(4, datagen.S_KIND, R) < 0.2
    ms, ns = datagen.instance_sizes(4, R)
    t = time.perf_counter()
    ws = []
    for r in range(R):
        if kind[r]:
            ws.append(datagen.softmax_request(4000 + r, max_iters=args.iters))
        else:
            ws.append(datagen.batched_instance(r, int(ms[r]), int(ns[r]), base_seed=4000,
                                               max_iters=args.iters))
        if (r + 1) % 250 == 0:
            log("generated %d of %d requests (%.0f s)" % (r + 1, R, time.perf_counter() - t))
    log("generated %d requests (%d softmax) in %.1f s" % (R, int(kind.sum()), time.perf_counter() - t))

    def plain_solve(w):
        P = make_problem(bca, w)
        P.step(w.max_iters)
        out = P.support(), P.coef(), P.objective()
        P.close()
        return out

    # calibration: plain one-at-a-time solves/s on the first requests, back to back
    ncal = min(20, R)
    plain_solve(ws[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for w in ws[:ncal]:
        plain_solve(w)
    plain_rate = ncal / (time.perf_counter() - t)
    lam = args.rate if args.rate > 0 else 1.5 * plain_rate
    gaps = -np.log(datagen.uniform_vector(4, datagen.S_ARRIVAL, R)) / lam
    release = np.cumsum(gaps)
    w0, w1 = R // 10, (9 * R) // 10
    log("plain calibration %.2f solves/s; offered rate %.2f req/s (%s)"
        % (plain_rate, lam, "frozen" if args.rate > 0 else "1.5 x this calibration"))

    def summarise(done_at, lat, backlog):
        """done_at: completion times from the trace start; backlog: (t, count) samples."""
        win = release[w1] - release[w0]
        in_win = np.sum((done_at >= release[w0]) & (done_at < release[w1]))
        b = np.array([c for (tt, c) in backlog if release[w0] <= tt < release[w1]] or [0])
        q = max(1, len(b) // 4)
        return {"solves_per_s": R / float(np.max(done_at)),
                "steady_solves_per_s": float(in_win / win),
                "p50_s": float(np.percentile(lat[w0:], 50)), "p99_s": float(np.percentile(lat[w0:], 99)),
                "backlog_mean": float(np.mean(b)), "backlog_max": int(np.max(b)),
                "backlog_first_quarter": float(np.mean(b[:q])), "backlog_last_quarter": float(np.mean(b[-q:]))}

    # plain method on the trace: one FIFO worker
    lat_plain = np.zeros(R)
    done_plain = np.zeros(R)
    backlog_plain = []
    t0 = time.perf_counter()
    for r, w in enumerate(ws):
        now = time.perf_counter() - t0
        if now < release[r]:
            time.sleep(release[r] - now)
        plain_solve(w)
        done_plain[r] = time.perf_counter() - t0
        lat_plain[r] = done_plain[r] - release[r]
        backlog_plain.append((done_plain[r], int(np.searchsorted(release, done_plain[r])) - (r + 1)))
        if (r + 1) % 200 == 0:
            log("plain: %d of %d done at %.1f s (latency %.2f s)" % (r + 1, R, done_plain[r], lat_plain[r]))
    log("plain trace done in %.1f s" % (time.perf_counter() - t0))

    # served on the same trace
    S = bca.Server(64 << 30, max_slots=256, round_iters=5)
    tickets = [None] * R
    t0 = time.perf_counter()

    def submitter():
        for r, w in enumerate(ws):
            now = time.perf_counter() - t0
            if now < release[r]:
                time.sleep(release[r] - now)
            tickets[r] = S.submit({0: "squared", 1: "logistic", 2: "softmax"}[w.loss], w.A, w.b,
                                  w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                                  rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                                  max_iters=w.max_iters, dtype=w.dtype, n_classes=w.n_classes)

    th = threading.Thread(target=submitter)
    th.start()
    lat_srv = np.zeros(R)
    done_srv = np.full(R, np.inf)
    done = np.zeros(R, dtype=bool)
    backlog_srv = []
    failed = 0
    next_log = 200
    while not done.all():
        now = time.perf_counter() - t0
        for r in range(R):
            if not done[r] and tickets[r] is not None:
                st = S.poll(tickets[r])
                if st in (bca.REQ_DONE, bca.REQ_FAILED, bca.REQ_CANCELLED):
                    done[r] = True
                    done_srv[r] = now
                    if st == bca.REQ_DONE:
                        lat_srv[r] = S.fetch(tickets[r])[3]
                    else:
                        failed += 1
        submitted = sum(1 for tk in tickets if tk is not None)
        backlog_srv.append((now, submitted - int(done.sum())))
        if done.sum() >= next_log:
            log("served: %d of %d done at %.1f s (backlog %d)" % (int(done.sum()), R, now, backlog_srv[-1][1]))
            next_log += 200
        time.sleep(0.005)
    th.join()
    span_srv = time.perf_counter() - t0
    stats = S.stats()
    srv_times = S.timing()
    S.close()
    log("server time split (s): " + ", ".join("%s %.2f" % kv for kv in srv_times.items()))
    srv = summarise(done_srv, lat_srv, backlog_srv)
    pln = summarise(done_plain, lat_plain, backlog_plain)
    log("served %.2f solves/s (steady %.2f), p50 %.3f s, p99 %.3f s; plain %.2f (steady %.2f), p50 %.3f s, "
        "p99 %.3f s" % (srv["solves_per_s"], srv["steady_solves_per_s"], srv["p50_s"], srv["p99_s"],
                        pln["solves_per_s"], pln["steady_solves_per_s"], pln["p50_s"], pln["p99_s"]))
    out = {"metric": "served solves/s + p99 latency vs plain", "value": srv["steady_solves_per_s"],
           "unit": "solves/s", "n_gpus": 1, "steps": R, "warmup": w0,
           "ms_per_step": span_srv / R * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "serve_%d_requests_poisson" % R, "offered_rate": lam,
                      "offered_rate_source": ("frozen: 1.5 x %.1f solves/s (plain, first 20 requests)"
                                              % (lam / 1.5)) if args.rate > 0 else
                      "1.5 x this run's plain calibration",
                      "softmax_fraction": float(kind.mean()), "iters": args.iters,
                      "hbm_budget_GiB": 64, "max_slots": 256, "round_iters": 5,
                      "steady_window_s": [float(release[w0]), float(release[w1])]},
           "served": srv, "plain": dict(pln, calibration_solves_per_s=plain_rate),
           "failed": failed, "server_rounds": stats["rounds"],
           "server_seconds": {k: round(v, 3) for k, v in srv_times.items()}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slogr_8x50000x5000_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    ap.add_argument("--mode", default="plain", choices=["plain", "batched", "serve", "precision",
                                                         "paper-shapes", "paper-sweeps", "exact", "woodbury",
                                                         "setup", "exact-logistic"],
                    help="plain: one problem (default); batched: many uneven problems in one "
                         "persistent launch; serve: continuous batching on a Poisson trace; precision: "
                         "BF16 beside FP32 at 16 x 100,000 x 10,000; paper-shapes: the sparse least-squares "
                         "shapes of the paper's Table 1, end to end; paper-sweeps: the paper's rho_b convergence study and its feature and sample scaling runs; exact: the exact squared-loss x-update beside "
                         "Algorithm 2 at 16 x 100,000 x 10,000 FP32; woodbury: the sample-space x-step beside the "
                         "default one at 8 x 800 x 10,000 FP32; setup: the Gram and factorisation at "
                         "the precision workload's shape, BF16 and FP32; exact-logistic: the logistic "
                         "exact x-update (Newton-CG) beside Algorithm 2 on the default workload")
    ap.add_argument("--instances", type=int, default=512, help="batched: number of problems")
    ap.add_argument("--requests", type=int, default=2000, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=SERVE_RATE,
                    help="serve: offered rate in requests/s (0: 1.5 x the plain rate measured first)")
    ap.add_argument("--iters", type=int, default=100, help="batched/serve: outer iterations per problem")
    ap.add_argument("--m-per", type=int, default=0,
                    help="precision: rows per partition (default 100,000; smaller values shrink n too)")
    ap.add_argument("--sweep", default="all", choices=["all", "rho_b", "features", "samples"],
                    help="paper-sweeps: which of the paper's Sec. 4 runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: all partitions live in one GPU's memory and "
              "there is no multi-GPU path (requested --gpus %d)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4}), flush=True)
        return
    import paper_2405_16267_amd as bca
    if args.mode == "batched":
        return batched_bench(args)
    if args.mode == "serve":
        return serve_bench(args)
    if args.mode == "precision":
        return precision_bench(args)
    if args.mode == "paper-shapes":
        return paper_shapes_bench(args)
    if args.mode == "exact":
        return exact_bench(args)
    if args.mode == "paper-sweeps":
        return paper_sweeps_bench(args)
    if args.mode == "woodbury":
        return woodbury_bench(args)
    if args.mode == "setup":
        return setup_bench(args)
    if args.mode == "exact-logistic":
        return exact_logistic_bench(args)

    t = time.perf_counter()
    w = workload(args.workload)
    log("generated %s in %.1f s" % (w.name, time.perf_counter() - t))
    loss = {0: "squared", 1: "logistic", 2: "softmax", 3: "hinge"}[w.loss]
    total_iters = args.warmup + args.steps
    P = bca.Problem(loss, w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=max(total_iters, 1), dtype=w.dtype, n_classes=w.n_classes)
    t = time.perf_counter()
    for i in range(w.N):
        P.set_data(i, w.A[i], w.b[i])
    torch.cuda.synchronize()
    log("data resident in HBM (%.1f s)" % (time.perf_counter() - t))
    P.set_timing(True)
    t = time.perf_counter()
    P.finalize()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    n_gram, gram_ms = P.timing(bca.KC_GRAM)
    n_fac, fac_ms = P.timing(bca.KC_FACTOR)
    log("setup (Gram + Cholesky + inverse factor) %.3f s" % setup_s)

    P.set_timing(False)
    P.step(args.warmup)
    torch.cuda.synchronize()
    P.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    n_st, st_ms = P.timing(bca.KC_STREAM)
    n_so, so_ms = P.timing(bca.KC_SOLVE)
    n_gl, gl_ms = P.timing(bca.KC_GLOBAL)
    pr, dr, br, it = P.residuals()
    log("residuals after %d iterations: p_r %.3e d_r %.3e b_r %.3e" % (it, pr, dr, br))
    zv = P.get_vector(bca.VEC_Z)
    if w.n_classes > 1:   # row sparsity: the support is the rows of largest norm
        zv = np.linalg.norm(zv.reshape(w.n, w.n_classes), axis=1)
    zr = np.sort(np.abs(zv))[::-1]
    margin = float(zr[w.kappa - 1] - zr[w.kappa]) if w.kappa < w.n else float("inf")

    m_total = sum(w.rows)
    esize = {"f64": 8, "f32": 4, "bf16": 2}[w.dtype]
    C = w.n_classes
    if C == 1:
        # algorithmic bytes of one A-streaming pass: A once, plus b (read), nu (read and
        # write) and omega-bar (write) per row
        stream_bytes = m_total * w.n * esize + 32 * m_total
        stream_kernel = "stream_kernel"
    else:
        # the multi-class pass's three kernels: A twice (sample-space averages, then
        # A^T E), the C-vector of averages written and read, omega-bar and nu read and
        # written, e written and read, the labels read
        stream_bytes = 2 * m_total * w.n * esize + 8 * 8 * C * m_total + 4 * m_total
        stream_kernel = "dot_mfma_kernel+prox_mc_kernel+acc_mfma_kernel"
    stream_avg_s = st_ms / max(n_st, 1) / 1e3
    achieved = stream_bytes / stream_avg_s / 1e9
    bounds = [(w.n // w.n_blocks + (1 if j < w.n % w.n_blocks else 0)) for j in range(w.n_blocks)]
    # bytes of one block solve: the distinct entries of the symmetric K_ij^-1 (FP64)
    factor_bytes = w.N * sum(nj * (nj + 1) // 2 * 8 for nj in bounds)
    inner_bytes = stream_bytes + factor_bytes
    ms_per_step = elapsed / args.steps * 1e3
    src_hash = source_hash(STREAM_SOURCES)
    traffic, traffic_file = counter_traffic(stream_kernel, w.name, src_hash)
    gram_flops = sum(m * nj * (nj + 1) for m in w.rows for nj in bounds)
    gram_peak = {"f64": FP64_PEAK_TFLOPS, "f32": FP32_MFMA_PEAK_TFLOPS, "bf16": BF16_MFMA_PEAK_TFLOPS}[w.dtype]
    gram_tflops = gram_flops / (gram_ms / 1e3) / 1e12 if gram_ms > 0 else None

    out = {
        "metric": "ADMM iter/s + HBM GB/s (plain)",
        "value": args.steps / elapsed,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "loss": loss, "N": w.N, "m_per_partition": w.rows[0],
                   "n": w.n, "M": w.n_blocks, "kappa": w.kappa, "inner_iters": w.inner_iters,
                   "rho_c": w.rho_c, "rho_b": w.rho_b, "rho_l": w.rho_l, "gamma": w.gamma},
        "inner_iters_per_s": args.steps * w.inner_iters / elapsed,
        "hbm_gbps_algorithmic": inner_bytes * w.inner_iters * args.steps / elapsed / 1e9,
        "roofline": {"bound": "hbm", "kernel": stream_kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic, "traffic_unit": "bytes per launch",
                     "traffic_source": traffic_file, "kernel_source": src_hash,
                     "bytes_per_launch": stream_bytes,
                     "avg_launch_ms": stream_avg_s * 1e3, "launches": n_st},
        "kernels_ms_per_step": {"stream": st_ms / args.steps, "solve": so_ms / args.steps,
                                "global": gl_ms / args.steps},
        "setup": {"seconds": setup_s, "gram_ms": gram_ms, "factor_ms": fac_ms,
                  "gram_tflops": gram_tflops,
                  "gram_mfma_frac": (gram_tflops / gram_peak) if gram_tflops else None},
        "residuals": {"iter": it, "p_r": pr, "d_r": dr, "b_r": br},
        # |z|_(kappa) - |z|_(kappa+1) of the last timed iteration: how far the support
        # decision is from a tie (a support comparison with the oracle is only
        # meaningful where this exceeds the FP32 error of z)
        "topk_margin": {"value": margin, "relative": margin / float(zr[0]) if zr[0] > 0 else None},
    }
    P.close()
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        out["cpu_baseline"] = oracle_baseline(w)
        log("cpu baseline %.1f s" % (time.perf_counter() - t))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
