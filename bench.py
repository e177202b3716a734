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


def workload(name):
    import datagen
    if name == "slogr_8x50000x5000_f32":
        return datagen.config1()
    if name == "slinr_4x500x200_f64":
        return datagen.config0()
    if name.startswith("slogr_small"):
        return datagen.config1(N=8, m_per=5000, n=1000, kappa=20)
    raise SystemExit("unknown workload " + name)


def oracle_baseline(w, max_parts=2):
    """The FP64 oracle, as it is, on a bounded sample: the x-update (K_in inner
    iterations of the node-level loop) of `max_parts` partitions and one global
    step on the full-size vectors; scaled to outer iterations per second of the
    whole problem."""
    import numpy as np
    import datagen
    import oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    parts = list(range(min(max_parts, w.N)))
    A = [datagen.widen(w.A[i]) for i in parts]
    b = [w.b[i] for i in parts]
    o = oracle.BiCADMM(A, b, w.loss, w.n_blocks, w.kappa, w.gamma, w.rho_c, w.rho_b, w.rho_l)
    t0 = time.perf_counter()
    for i in range(len(parts)):
        o.x_update(i, w.inner_iters)
    tx = time.perf_counter() - t0
    # global step at full size (N partitions of n-vectors)
    st = o.zero_state()
    st.x = np.random.default_rng(0).standard_normal((w.N, w.n))
    st.u = np.zeros((w.N, w.n))
    g = oracle.BiCADMM.__new__(oracle.BiCADMM)
    g.N, g.n, g.M, g.kappa, g.C = w.N, w.n, w.n_blocks, w.kappa, 1
    g.rho_c, g.rho_b = w.rho_c, w.rho_b
    t1 = time.perf_counter()
    g.global_update(st)
    tg = time.perf_counter() - t1
    per_outer = tx * (w.N / len(parts)) + tg
    return {"value": 1.0 / per_outer, "unit": "iter/s", "cores": int(cores), "kind": "oracle",
            "sample": "x-update (%d inner iterations) of %d of %d partitions plus one full-size "
                      "global step, scaled to all %d partitions; %.1f s of CPU work"
                      % (w.inner_iters, len(parts), w.N, w.N, tx + tg)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="slogr_8x50000x5000_f32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the partitions of this build live in one GPU's "
              "memory and no multi-GPU path exists (requested --gpus %d)" % args.gpus,
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

    t = time.perf_counter()
    w = workload(args.workload)
    log("generated %s in %.1f s" % (w.name, time.perf_counter() - t))
    loss = {0: "squared", 1: "logistic"}[w.loss]
    total_iters = args.warmup + args.steps
    P = bca.Problem(loss, w.n, w.rows, w.n_blocks, w.kappa, gamma=w.gamma, rho_c=w.rho_c,
                    rho_b=w.rho_b, rho_l=w.rho_l, inner_iters=w.inner_iters,
                    max_iters=max(total_iters, 1), dtype=w.dtype)
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

    m_total = sum(w.rows)
    esize = {"f64": 8, "f32": 4, "bf16": 2}[w.dtype]
    # algorithmic bytes of one A-streaming pass: A once, plus b (read), nu (read and
    # write) and omega-bar (write) per row
    stream_bytes = m_total * w.n * esize + 32 * m_total
    stream_avg_s = st_ms / max(n_st, 1) / 1e3
    achieved = stream_bytes / stream_avg_s / 1e9
    bounds = [(w.n // w.n_blocks + (1 if j < w.n % w.n_blocks else 0)) for j in range(w.n_blocks)]
    # factor bytes of one block solve: both packed triangles of W_ij = L_ij^-1 (FP64)
    factor_bytes = w.N * sum(nj * (nj + 1) * 8 for nj in bounds)
    inner_bytes = stream_bytes + factor_bytes
    ms_per_step = elapsed / args.steps * 1e3
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
        "roofline": {"bound": "hbm", "kernel": "stream_kernel", "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": None, "bytes_per_launch": stream_bytes,
                     "avg_launch_ms": stream_avg_s * 1e3, "launches": n_st},
        "kernels_ms_per_step": {"stream": st_ms / args.steps, "solve": so_ms / args.steps,
                                "global": gl_ms / args.steps},
        "setup": {"seconds": setup_s, "gram_ms": gram_ms, "factor_ms": fac_ms,
                  "gram_tflops": gram_tflops,
                  "gram_mfma_frac": (gram_tflops / gram_peak) if gram_tflops else None},
    }
    P.close()
    if not args.no_cpu_baseline:
        t = time.perf_counter()
        out["cpu_baseline"] = oracle_baseline(w)
        log("cpu baseline %.1f s" % (time.perf_counter() - t))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
