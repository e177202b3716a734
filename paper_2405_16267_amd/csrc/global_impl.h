// Device-side pieces of the global level of Algorithm 1 (see global.hip), templated
// on the workgroup size so that the one-problem kernel (1024 threads) and the
// batched persistent kernel (256 threads) run the same code.
#pragma once
#include "bca_internal.h"

namespace bca {

constexpr int PSECT = 15;  // interior points per multisection round

// Sum of one value per thread; every thread receives the same total (fixed order).
template <int BT>
__device__ double block_sum(double v, double* sh) {
  constexpr int GW = BT / 64;
  v = wave_sum_dpp(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < GW; ++w) t += sh[w];
  return t;
}

template <int BT, int K>
__device__ void block_sum_n(double (&v)[K], double* sh /* GW * K */) {
  constexpr int GW = BT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < K; ++q) v[q] = wave_sum_dpp(v[q]);
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < K; ++q) sh[q * GW + wv] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < K; ++q) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < GW; ++w) t += sh[q * GW + w];
    v[q] = t;
  }
}

template <int BT>
__device__ double block_max(double v, double* sh) {
  constexpr int GW = BT / 64;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wv] = v;
  __syncthreads();
  double t = sh[0];
  for (int w = 1; w < GW; ++w) t = fmax(t, sh[w]);
  return t;
}

// Exclusive prefix sum over threads (in thread order) of one int per thread.
template <int BT>
__device__ int block_exscan(int v, int* sh /* GW + 1 */, int* total) {
  constexpr int GW = BT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(inc, o, 64);
    if (lane >= o) inc += t;
  }
  __syncthreads();
  if (lane == 63) sh[wv] = inc;
  __syncthreads();
  int base = 0, tot = 0;
  for (int w = 0; w < GW; ++w) {
    if (w < wv) base += sh[w];
    tot += sh[w];
  }
  *total = tot;
  return base + inc - v;
}

__device__ __forceinline__ uint64_t abs_key(double x) {
  return (uint64_t)__double_as_longlong(x) & 0x7FFFFFFFFFFFFFFFull;
}
__device__ __forceinline__ uint64_t abs_key(float x) {
  return (uint64_t)(__float_as_uint(x) & 0x7FFFFFFFu);
}

template <int BT>
struct TopkShared {
  unsigned int hist[256];
  uint64_t prefix;
  int need;
  int done;
  int scan[BT / 64 + 1];
};

// Select T_kappa of |z| (z of type Z, n entries): returns the threshold key and,
// through *take_eq, how many entries equal to it are kept (lowest indices).
// Digit passes stop once the chosen bin holds exactly the entries still needed:
// the whole bin is then kept, with the threshold at the bin's lowest key pattern
// (the same set the remaining passes would select); with fewer than kappa
// nonzero entries the first pass ends the walk at threshold 0.
template <int BT, typename Z>
__device__ uint64_t topk_threshold(const Z* z, int64_t n, int kappa, TopkShared<BT>& sh, int* take_eq) {
  constexpr int GT = BT;
  constexpr int BITS = sizeof(Z) * 8;
  uint64_t prefix = 0, mask = 0;
  int need = kappa;
  if (threadIdx.x == 0) sh.done = 0;
  for (int d = BITS - 8; d >= 0; d -= 8) {
    for (int b = threadIdx.x; b < 256; b += GT) sh.hist[b] = 0;
    __syncthreads();
    int nzl = 0;
    for (int64_t k = threadIdx.x; k < n; k += GT) {
      const uint64_t key = abs_key(z[k]);
      nzl += key != 0;
      if ((key & mask) == prefix) atomicAdd(&sh.hist[(key >> d) & 255u], 1u);
    }
    if (d == BITS - 8) {
      // fewer than kappa nonzero entries: the threshold is 0 and the
      // lowest-index zeros fill T_kappa, which is where the digit walk would end
      int nz;
      (void)block_exscan<BT>(nzl, sh.scan, &nz);
      if (nz < kappa) {
        *take_eq = kappa - nz;
        return 0;
      }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // digit D: the highest bin where the count from the top reaches `need`.
      // Lane l sums bins 4l..4l+3; a suffix scan over lanes finds the lane
      // whose 4 bins hold D, and that lane walks them from the top.
      const int l = threadIdx.x;
      int loc = 0;
#pragma unroll
      for (int b = 0; b < 4; ++b) loc += (int)sh.hist[4 * l + b];
      int suf = loc;  // sum over lanes >= l
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_down(suf, o, 64);
        if (l + o < 64) suf += t;
      }
      const int above = suf - loc;  // sum over lanes > l
      if ((suf >= need && above < need) || (l == 0 && suf < need)) {
        int cum = above, D = 4 * l + 3;
        for (; D > 4 * l; --D) {
          if (cum + (int)sh.hist[D] >= need) break;
          cum += (int)sh.hist[D];
        }
        sh.prefix = prefix | ((uint64_t)D << d);
        sh.need = need - cum;
        sh.done = (need - cum) == (int)sh.hist[D];
      }
    }
    __syncthreads();
    prefix = sh.prefix;
    need = sh.need;
    mask |= (uint64_t)255 << d;
    const bool whole_bin = sh.done != 0;
    __syncthreads();
    if (whole_bin) break;
  }
  *take_eq = need;
  return prefix;
}

// Marks T_kappa: calls f(k, selected) for every k in ascending order within each
// thread's contiguous range; support positions are returned through pos().
template <int BT, typename Z, typename F>
__device__ void topk_apply(const Z* z, int64_t n, uint64_t thr, int take_eq, TopkShared<BT>& sh, F f) {
  constexpr int GT = BT;
  const int64_t chunk = (n + GT - 1) / GT;
  const int64_t lo = (int64_t)threadIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  int eq = 0;
  for (int64_t k = lo; k < hi; ++k) eq += (abs_key(z[k]) == thr);
  int tot;
  const int eq_base = block_exscan<BT>(eq, sh.scan, &tot);
  int sel = 0, r = eq_base;
  for (int64_t k = lo; k < hi; ++k) {
    const uint64_t key = abs_key(z[k]);
    if (key > thr || (key == thr && r++ < take_eq)) ++sel;
  }
  const int sel_base = block_exscan<BT>(sel, sh.scan, &tot);
  int pos = sel_base;
  r = eq_base;
  for (int64_t k = lo; k < hi; ++k) {
    const uint64_t key = abs_key(z[k]);
    const bool s = key > thr || (key == thr && r++ < take_eq);
    f(k, s, s ? pos++ : -1);
  }
}

// Consensus average of row k and the breakpoint data of the vector (z,t)
// problem for it; adds d_k |wbar_k| to *s1 and raises *thmax to theta_k when finite.
__device__ __forceinline__ void consensus_row(const GlobalArgs& a, int k, double* s1, double* thmax,
                                              bool* bad) {
  const int n = a.n, N = a.N, C = a.C;
  const int64_t nc = (int64_t)n * C;
  double* wbar = a.work;
  double* zprev = a.work + nc;
  double* rv = a.work + 2 * nc;
  double* th = rv + n;
  double* c1 = th + n;
  double* c2 = c1 + n;
  const double aa = N * a.rho_c;
  double nrm2 = 0.0, w1 = 0.0;
  for (int c = 0; c < C; ++c) {
    const int64_t e = (int64_t)k * C + c;
    zprev[e] = a.z[e];
    double sacc = 0.0;
    for (int i = 0; i < N; ++i) sacc += a.x[(int64_t)i * nc + e] + a.u[(int64_t)i * nc + e];
    const double w = sacc / N;
    wbar[e] = w;
    nrm2 += w * w;
    w1 = w;
  }
  const double w = C == 1 ? w1 : sqrt(nrm2);
  *bad |= !isfinite(w);
  rv[k] = w;
  const double sg = w > 0.0 ? 1.0 : (w < 0.0 ? -1.0 : 0.0);
  const double d = 1.0 - sg * a.s[k];
  const double aw = fabs(w);
  c1[k] = d * aw;
  c2[k] = d * d / aa;
  const double t = d > 0.0 ? aa * aw / d : INFINITY;
  th[k] = t;
  *s1 += d * aw;
  if (t < INFINITY) *thmax = fmax(*thmax, t);
}

// One global step with a workgroup of BT threads, PS interior points per
// multisection round; shd holds (BT / 64) * (PSECT + 2) doubles of shared memory.
// With a.split the O(N n) parts run in their own many-workgroup kernels: the
// consensus pass before (this step then only adds its per-workgroup partial
// sums, a.gp[0 .. G) and maxima a.gp[G .. 2G)), and the u-update with the
// residuals after (this step then leaves t, v and z^T s - t in scal[0], scal[1],
// scal[6]).
template <int BT, int PS = PSECT>
__device__ void global_step(const GlobalArgs& a, double* shd, TopkShared<BT>& tks) {
  constexpr int GT = BT;
  const int n = a.n, N = a.N, C = a.C;
  const int64_t nc = (int64_t)n * C;
  const int tid = threadIdx.x;
  double* wbar = a.work;              // n x C
  double* zprev = a.work + nc;        // n x C
  double* rv = a.work + 2 * nc;       // per row: wbar (C = 1) or ||wbar_k|| (C > 1)
  double* th = rv + n;
  double* c1 = th + n;
  double* c2 = c1 + n;
  double* rz = c2 + n;                // per row of z: z_k (C = 1) or ||z_k|| (C > 1)
  const double aa = N * a.rho_c, rb = a.rho_b;
  const double v = a.scal[1];

  // consensus average and breakpoint data of the vector (z,t) problem
  double s1loc = 0.0, thmax = 0.0;
  if (a.split) {
    for (int g = tid; g < a.G; g += GT) {
      s1loc += a.gp[g];
      thmax = fmax(thmax, a.gp[a.G + g]);
    }
  } else {
    bool bad = false;
    for (int k = tid; k < n; k += GT) consensus_row(a, k, &s1loc, &thmax, &bad);
    if (bad) atomicExch(a.status, 1);
  }
  const double S1all = block_sum<BT>(s1loc, shd);
  const double hi0 = block_max<BT>(thmax, shd);

  double theta;
  if (v - S1all >= 0.0) {
    theta = 0.0;
  } else if (v + hi0 / rb < 0.0) {
    // root beyond the last breakpoint: only coordinates with d_k = 0 remain, adding 0
    theta = -v * rb;
  } else {
    // psi is continuous, increasing and concave (terms leave the sum as theta
    // passes their breakpoints), so Newton steps from a point left of the root
    // stay left of it and move monotonically to it; a step is the root of the
    // linear piece active right of the current point, theta' = (sum_A c1 - v) /
    // (1/rho_b + sum_A c2) with A = {k : theta_k > theta}, and it is exact once A
    // no longer changes.  Newton starts at theta = 0 (psi(0) < 0 here) or at the
    // previous root; if it has not settled after 32 steps, multisection finishes
    // the bracket from there.
    double lo = 0.0, hi = hi0;
    bool isolated = false;
    auto multisect = [&](int max_rounds) {
      for (int round = 0; round < max_rounds; ++round) {
        double acc[PS + 1];
        double pts[PS];
#pragma unroll
        for (int p = 0; p < PS; ++p) {
          pts[p] = lo + (hi - lo) * (double)(p + 1) / (double)(PS + 1);
          acc[p] = 0.0;
        }
        acc[PS] = 0.0;  // breakpoints strictly inside (lo, hi)
        for (int k = tid; k < n; k += GT) {
          const double t = th[k];
          const double ca = c1[k], cb = c2[k];
#pragma unroll
          for (int p = 0; p < PS; ++p)
            if (t > pts[p]) acc[p] += pts[p] * cb - ca;
          if (t > lo && t < hi) acc[PS] += 1.0;
        }
        block_sum_n<BT, PS + 1>(acc, shd);
        if (acc[PS] == 0.0) {
          isolated = true;
          return;
        }
        int p = 0;
        while (p < PS && v + pts[p] / rb + acc[p] < 0.0) ++p;
        const double nlo = p == 0 ? lo : pts[p - 1];
        const double nhi = p == PS ? hi : pts[p];
        if (nlo == lo && nhi == hi) {
          isolated = true;
          return;
        }
        lo = nlo;
        hi = nhi;
      }
    };
    // sums of c1, c2 and the count over {theta_k > x}
    auto active = [&](double x, double (&sm)[3]) {
      sm[0] = sm[1] = sm[2] = 0.0;
      for (int k = tid; k < n; k += GT) {
        if (th[k] > x) {
          sm[0] += c1[k];
          sm[1] += c2[k];
          sm[2] += 1.0;
        }
      }
      block_sum_n<BT, 3>(sm, shd);
    };
    multisect(0);
    bool done = false;
    if (!isolated) {
      double cur = lo, sm[3];
      // warm start from the previous outer iteration's root tw: if psi(tw) <= 0
      // Newton starts there (the root is the same exact value from any start
      // left of it); otherwise tw bounds the root from above
      const double tw = a.scal[7];
      bool warm = false;
      if (tw > 0.0 && tw < hi) {
        active(tw, sm);
        if (v + tw / rb + tw * sm[1] - sm[0] <= 0.0) {
          cur = lo = tw;
          warm = true;
        } else {
          hi = tw;
        }
      }
      if (!warm) active(cur, sm);
      for (int it = 0; it < 32 && !done; ++it) {
        double nx = (sm[0] - v) / (1.0 / rb + sm[1]);
        nx = fmin(fmax(nx, cur), hi);
        double sn[3];
        active(nx, sn);
        if (sn[2] == sm[2]) {
          theta = nx;
          done = true;
        } else {
          cur = nx;
          sm[0] = sn[0];
          sm[1] = sn[1];
          sm[2] = sn[2];
        }
      }
      if (!done) {
        lo = cur;
        multisect(200);
      }
    }
    if (!done) {
      // exact root on the linear piece whose active set is {theta_k >= hi}
      double sums[2] = {0.0, 0.0};
      for (int k = tid; k < n; k += GT) {
        if (th[k] >= hi) {
          sums[0] += c1[k];
          sums[1] += c2[k];
        }
      }
      block_sum_n<BT, 2>(sums, shd);
      theta = (sums[0] - v) / (1.0 / rb + sums[1]);
      theta = fmin(fmax(theta, lo), hi);
    }
  }
  if (tid == 0) a.scal[7] = theta;   // the next step's warm start
  // z(theta) per row; rows of the matrix variable are scaled copies of wbar_k
  double tl = 0.0;
  for (int k = tid; k < n; k += GT) {
    const double w = rv[k];
    double zk;
    if (theta == 0.0) {
      zk = w;
      tl += a.s[k] * w;
    } else {
      const double y = w + theta * a.s[k] / aa;
      const double mag = fabs(y) - theta / aa;
      zk = mag > 0.0 ? (y > 0.0 ? mag : -mag) : 0.0;
      tl += fabs(zk);
    }
    rz[k] = zk;
    if (C == 1) {
      a.z[k] = zk;
    } else {
      const double sc = w > 0.0 ? zk / w : 0.0;
      for (int c = 0; c < C; ++c) a.z[(int64_t)k * C + c] = wbar[(int64_t)k * C + c] * sc;
    }
  }
  double t = block_sum<BT>(tl, shd);
  if (theta == 0.0) t += v;
  __syncthreads();

  // s-step on the row values: T_kappa, M_kappa, s
  int take_eq;
  const uint64_t thr = topk_threshold<BT, double>(rz, n, a.kappa, tks, &take_eq);
  double mk = 0.0;
  {
    const int64_t chunk = (n + GT - 1) / GT;
    const int64_t lo = (int64_t)tid * chunk;
    const int64_t hi = lo + chunk < n ? lo + chunk : n;
    int eq = 0;
    for (int64_t k = lo; k < hi; ++k) eq += (abs_key(rz[k]) == thr);
    int tot;
    const int eq_base = block_exscan<BT>(eq, tks.scan, &tot);
    int r = eq_base;
    for (int64_t k = lo; k < hi; ++k) {
      const uint64_t key = abs_key(rz[k]);
      if (key > thr || (key == thr && r++ < take_eq)) mk += fabs(rz[k]);
    }
  }
  const double Mk = block_sum<BT>(mk, shd);
  const double tau = t - v;
  const double alpha = Mk > 0.0 ? fmin(fmax(tau / Mk, -1.0), 1.0) : 0.0;
  double gl = 0.0;
  topk_apply<BT, double>(rz, n, thr, take_eq, tks, [&](int64_t k, bool sel, int pos) {
    const double zk = rz[k];
    const double sk = sel ? alpha * (zk > 0.0 ? 1.0 : (zk < 0.0 ? -1.0 : 0.0)) : 0.0;
    a.s[k] = sk;
    gl += zk * sk;
    if (sel && pos < a.kappa) a.support[pos] = (int32_t)k;
  });
  const double g = block_sum<BT>(gl, shd) - t;
  const double vn = v + g;
  if (a.split) {
    if (tid == 0) {
      a.scal[0] = t;
      a.scal[1] = vn;
      a.scal[6] = g;
      if (!isfinite(t) || !isfinite(vn)) atomicExch(a.status, 1);
    }
    return;
  }

  // u-update and residuals (Frobenius norms for C > 1)
  double dz = 0.0;
  for (int64_t e = tid; e < nc; e += GT) {
    const double d = a.z[e] - zprev[e];
    dz += d * d;
  }
  const double dzs = block_sum<BT>(dz, shd);
  double pr = 0.0;
  for (int i = 0; i < N; ++i) {
    double pl = 0.0;
    for (int64_t e = tid; e < nc; e += GT) {
      const int64_t o = (int64_t)i * nc + e;
      const double d = a.x[o] - a.z[e];
      pl += d * d;
      a.u[o] += d;
    }
    pr += sqrt(block_sum<BT>(pl, shd));
  }
  if (tid == 0) {
    const double dr = sqrt((double)N) * a.rho_c * sqrt(dzs);
    const double br = fabs(g);
    const int it = (int)a.scal[5];
    a.scal[0] = t;
    a.scal[1] = vn;
    a.scal[2] = pr;
    a.scal[3] = dr;
    a.scal[4] = br;
    a.scal[5] = (double)(it + 1);
    if (it < a.hist_cap) {
      a.hist[3 * (int64_t)it + 0] = pr;
      a.hist[3 * (int64_t)it + 1] = dr;
      a.hist[3 * (int64_t)it + 2] = br;
    }
    if (!isfinite(t) || !isfinite(vn) || !isfinite(pr)) atomicExch(a.status, 1);
  }
}

}  // namespace bca
