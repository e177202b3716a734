// Multi-class (softmax) form of the fused A-streaming pass of Algorithm 2.
//
// With C classes the block predictions are m_i x C (A_ij X_ij), the omega-bar
// step is a C-dimensional prox per sample and A_i^T E is n x C.  Thread t owns
// the features t, t + NT, ..., and for each of them all C columns of X in
// registers; the per-row dots (R rows x C classes) are reduced across the
// workgroup, the softmax prox runs with a 16-lane group per row and a lane per
// class, and e_k (C values) is read back for the A_i^T E accumulation.  Tile partial sums of A_i^T E are
// formed in the arithmetic type and folded every FLUSH tiles into the
// workgroup's FP64 partial vector in global memory.
//
// Softmax prox (omega-bar step of Sec. 3.1 with l(q; y) = LSE(q) - q_y): with
// beta = rho_l / M minimise F(q) = LSE(q) - q_y + (beta/2)||q - M c||^2 by Newton
// steps whose Hessian diag(p) - p p^T + beta I is inverted by Sherman-Morrison
// (D = diag(p + beta)): H^-1 g = D^-1 g + D^-1 p (p^T D^-1 g) / (1 - p^T D^-1 p),
// with backtracking (Armijo on F, or a decrease of ||grad|| once F is flat to
// rounding) until ||grad|| <= 1e-14 (or the rounding level of beta (q - Mc) when
// that is higher); omega-bar = q / M.
#include "bca_internal.h"

namespace bca {

template <typename T>
__device__ __forceinline__ typename Traits<T>::acc_t load_scalar(const T* p);
template <>
__device__ __forceinline__ double load_scalar<double>(const double* p) { return *p; }
template <>
__device__ __forceinline__ float load_scalar<float>(const float* p) { return *p; }
template <>
__device__ __forceinline__ float load_scalar<bf16_t>(const bf16_t* p) {
  return __uint_as_float((uint32_t)p->bits << 16);
}

__device__ double lse_c(const double* q, int C) {
  double mx = q[0];
  for (int c = 1; c < C; ++c) mx = fmax(mx, q[c]);
  double s = 0.0;
  for (int c = 0; c < C; ++c) s += exp(q[c] - mx);
  return mx + log(s);
}

// The softmax prox runs with one 16-lane group of a wavefront per sample and one
// lane per class (lane = 16 r + c): every sum, maximum and exponential over the
// classes is a group operation, so a wavefront solves 4 samples at the cost of
// one.  act: c < C; valid: the group's sample exists.
// Group sums and maxima run on DPP within the 16-lane row (quad permutes, then
// the half-row and row mirrors); every lane of the group gets the same bits,
// since each step combines a pair of lanes that hold equal values in swapped order.
__device__ __forceinline__ double gsum16(double v) { return row16_sum_dpp(v); }
__device__ __forceinline__ double gmax16(double v) {
  v = fmax(v, dpp_f64<0xB1>(v));   // quad_perm [1,0,3,2]
  v = fmax(v, dpp_f64<0x4E>(v));   // quad_perm [2,3,0,1]
  v = fmax(v, dpp_f64<0x141>(v));  // row_half_mirror
  v = fmax(v, dpp_f64<0x140>(v));  // row_mirror
  return v;
}

struct LseGrad {
  double l, p, g, gn;
};

// log-sum-exp of the group's q, and this lane's probability and gradient entry
__device__ __forceinline__ LseGrad lse_grad16(double q, double q0, bool act, bool is_y, double beta) {
  LseGrad r;
  const double mx = gmax16(act ? q : -INFINITY);
  const double s = gsum16(act ? exp(q - mx) : 0.0);
  r.l = mx + log(s);
  r.p = act ? exp(q - r.l) : 0.0;
  r.g = act ? r.p - (is_y ? 1.0 : 0.0) + beta * (q - q0) : 0.0;
  r.gn = sqrt(gsum16(r.g * r.g));
  return r;
}

__device__ __forceinline__ double F16(double q, double q0, bool act, bool is_y, double beta) {
  const double mx = gmax16(act ? q : -INFINITY);
  const double s = gsum16(act ? exp(q - mx) : 0.0);
  const double qy = gsum16(is_y ? q : 0.0);
  const double r2 = gsum16(act ? (q - q0) * (q - q0) : 0.0);
  return mx + log(s) - qy + 0.5 * beta * r2;
}

// Prox of one sample (this lane's class): start at the previous omega-bar, stop
// at ||grad|| <= 1e-14 or the rounding level of beta (q - Mc) if higher; returns
// q_c / M.  F and the gradient at an accepted trial point are those of the next
// iterate, so they are carried over instead of being evaluated again.
__device__ double prox_softmax_group(double cvc, double wprev, bool act, bool is_y, bool valid, int M,
                                     double rho_l) {
  const double beta = rho_l / M;
  const double q0 = M * cvc;
  double q = M * wprev;
  const double qmax0 = gmax16(act ? fabs(q0) : 0.0);
  bool done = !valid;
  LseGrad lg = lse_grad16(q, q0, act, is_y, beta);
  double f0 = F16(q, q0, act, is_y, beta);
  for (int it = 0; it < 100; ++it) {
    const double qa = fmax(qmax0, gmax16(act ? fabs(q) : 0.0));
    if (!(lg.gn > 1e-14 + 8.0 * 2.220446049250313e-16 * beta * 2.0 * qa)) done = true;
    if (__ballot(!done) == 0) break;
    const double d = act ? 1.0 / (lg.p + beta) : 0.0;
    const double pDp = gsum16(lg.p * lg.p * d);
    const double pDg = gsum16(lg.p * lg.g * d);
    const double coef = pDg / (1.0 - pDp);
    const double st = act ? d * lg.g + d * lg.p * coef : 0.0;
    const double slope = gsum16(lg.g * st);
    double t = 1.0;
    bool acc = done;
    LseGrad gt = lg;
    double ft = f0;
    for (int ls = 0; ls < 60; ++ls) {
      const double qt = q - t * st;
      // every lane takes part in the group operations, accepted or not
      ft = F16(qt, q0, act, is_y, beta);
      gt = lse_grad16(qt, q0, act, is_y, beta);
      // Armijo decrease, or a gradient-norm decrease once F is flat to rounding
      if (!acc && (ft <= f0 - 1e-4 * t * slope || gt.gn < lg.gn)) acc = true;
      if (__ballot(!acc) == 0) break;
      if (!acc) t *= 0.5;
    }
    if (__ballot(!acc) != 0) {   // no trial accepted: the step is the last halving
      const double qt = q - t * st;
      ft = F16(qt, q0, act, is_y, beta);
      gt = lse_grad16(qt, q0, act, is_y, beta);
    }
    if (!done) {
      q = q - t * st;
      lg = gt;
      f0 = ft;
    }
  }
  return q / M;
}

// The pass runs as three kernels: the C-dimensional prox of a sample costs far
// more than streaming its row of A (n <= 2048), so it gets a kernel of its own
// with every wavefront busy (4 samples per wavefront), between a kernel that
// forms the sample-space averages and one that accumulates A_i^T E.  A is read
// twice per inner iteration; both reads are cheap next to the prox.
//   dot_mc_kernel   a_k = (1/M) A_k X   (R rows per tile, reduced over the workgroup)
//   prox_mc_kernel  omega-bar, nu, e_k  (16-lane group per sample)
//   acc_mc_kernel   partial sums of A_i^T E per workgroup (same tiles and
//                   workgroups as dot_mc_kernel)
template <typename T, int NT, int NF, int R, int CC>
__global__ __launch_bounds__(NT) void dot_mc_kernel(StreamArgs a) {
  using acc = typename Traits<T>::acc_t;
  constexpr int NW = NT / 64;
  __shared__ double red[NW][R][CC];

  const int C = a.C;
  const int part = blockIdx.x / a.Gp;
  const int wg = blockIdx.x - part * a.Gp;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = a.n;

  const acc* xs = reinterpret_cast<const acc*>(a.xs) + (int64_t)part * a.ld * C;
  acc xr[NF][CC];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int k = tid + f * NT;
#pragma unroll
    for (int c = 0; c < CC; ++c) xr[f][c] = (k < n && c < C) ? xs[(int64_t)k * C + c] : acc(0);
  }
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld;
  const int64_t ntiles = (m + R - 1) / R;
  for (int64_t tile = wg; tile < ntiles; tile += a.Gp) {
    const int64_t rt = tile * R;
    acc v[R][NF];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = rt + r;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int k = tid + f * NT;
        v[r][f] = (row < m && k < n) ? load_scalar<T>(Ab + row * a.ld + k) : acc(0);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        acc d = acc(0);
#pragma unroll
        for (int f = 0; f < NF; ++f) d += v[r][f] * xr[f][c];
        const double s = wave_sum_dpp((double)d);
        if (lane == 0) red[wv][r][c] = s;
      }
    }
    __syncthreads();
    if (tid < R * CC) {
      const int r = tid / CC, c = tid % CC;
      const int64_t row = rt + r;
      if (row < m && c < C) {
        double sacc = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sacc += red[w][r][c];
        a.rowbuf[(r0 + row) * C + c] = sacc * a.inv_M;
      }
    }
    __syncthreads();
  }
}

// One wavefront per 4 samples: 16-lane group r takes sample 4 w + r, lane c of
// it class c.  In: rowbuf = a (averages); out: rowbuf = e.
__global__ __launch_bounds__(256) void prox_mc_kernel(StreamArgs a) {
  const int C = a.C;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int r = lane >> 4, c = lane & 15;
  const int64_t gr = ((int64_t)blockIdx.x * 4 + wv) * 4 + r;
  const bool valid = gr < a.m_total;
  const bool act = valid && c < C;
  const int64_t o = (valid ? gr : 0) * C + c;
  const double av = act ? a.rowbuf[o] : 0.0;
  const double nu0 = act ? a.nu[o] : 0.0;
  const double om0 = act ? a.omega[o] : 0.0;
  double e = 0.0;
  if (a.mode == 0) {
    const bool is_y = act && a.y[valid ? gr : 0] == c;
    const double om = prox_softmax_group(av + nu0, om0, act, is_y, valid, a.M, a.rho_l);
    if (act) {
      const double nu = nu0 + av - om;
      a.omega[o] = om;
      a.nu[o] = nu;
      e = om - av - nu;
    }
  } else if (act) {
    e = om0 - av - nu0;
  }
  if (act) a.rowbuf[o] = e;
}

template <typename T, int NT, int NF, int R, int CC>
__global__ __launch_bounds__(NT) void acc_mc_kernel(StreamArgs a) {
  using acc = typename Traits<T>::acc_t;
  constexpr int FLUSH = 16;
  const int C = a.C;
  const int part = blockIdx.x / a.Gp;
  const int wg = blockIdx.x - part * a.Gp;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int tid = threadIdx.x;
  const int n = a.n;

  double* gp = a.gpart + ((int64_t)part * a.Gp + wg) * a.ld * C;
  bool first = true;  // the first flush writes the partial sums, later ones add
  acc gt[NF][CC];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int c = 0; c < CC; ++c) gt[f][c] = acc(0);

  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld;
  const int64_t ntiles = (m + R - 1) / R;
  int since_flush = 0;
  for (int64_t tile = wg; tile < ntiles; tile += a.Gp) {
    const int64_t rt = tile * R;
    acc v[R][NF];
    double er[R][CC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = rt + r;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int k = tid + f * NT;
        v[r][f] = (row < m && k < n) ? load_scalar<T>(Ab + row * a.ld + k) : acc(0);
      }
#pragma unroll
      for (int c = 0; c < CC; ++c) er[r][c] = (row < m && c < C) ? a.rowbuf[(r0 + row) * C + c] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const acc e = (acc)er[r][c];
#pragma unroll
        for (int f = 0; f < NF; ++f) gt[f][c] += e * v[r][f];
      }
    if (++since_flush == FLUSH) {
      since_flush = 0;
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        const int k = tid + f * NT;
        if (k < n) {
#pragma unroll
          for (int c = 0; c < CC; ++c)
            if (c < C) {
              double* q = gp + (int64_t)k * C + c;
              *q = first ? (double)gt[f][c] : *q + (double)gt[f][c];
            }
        }
#pragma unroll
        for (int c = 0; c < CC; ++c) gt[f][c] = acc(0);
      }
      first = false;
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int k = tid + f * NT;
    if (k < n) {
#pragma unroll
      for (int c = 0; c < CC; ++c)
        if (c < C) {
          double* q = gp + (int64_t)k * C + c;
          *q = first ? (double)gt[f][c] : *q + (double)gt[f][c];
        }
    }
  }
}

// MFMA forms of the two streaming kernels, FP32 and BF16 storage (FP64 storage
// keeps the kernels above).  Both products are dense contractions with C <= 16
// columns: A_i X (m_i x n times n x C) and A_i^T E (n x m_i times m_i x C).  On
// v_mfma_f32_16x16x4f32 the contraction runs inside the matrix core, so the
// per-row cross-lane sums of the kernels above (C wave reductions per row) go
// away, and every lane reads 8 consecutive elements of a row per step.
// Operand layout of the instruction (lane l): A-side element (i = l % 16,
// k = l / 16), B-side element (k = l / 16, j = l % 16); result element v of lane l
// at (i = 4 (l / 16) + v, j = l % 16).  Lane l's 8 consecutive elements feed 8
// instructions (element u to instruction u), which is a fixed permutation of the
// contraction index.  FP32 products are summed in FP32 over at most 64 features
// (dot) or 16 samples (A^T E) and then in FP64.
typedef float mc_f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void load8(const float* p, float (&o)[8]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 4);
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
  o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
}
__device__ __forceinline__ void load8(const bf16_t* p, float (&o)[8]) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  o[0] = bf16_lo(v.x); o[1] = bf16_hi(v.x); o[2] = bf16_lo(v.y); o[3] = bf16_hi(v.y);
  o[4] = bf16_lo(v.z); o[5] = bf16_hi(v.z); o[6] = bf16_lo(v.w); o[7] = bf16_hi(v.w);
}

// a_k = (1/M) A_k X for a 16-row tile per workgroup: i = row, j = class, k =
// feature.  The row is cut into steps of 32 features (lane group g takes features
// 32 s + 8 g .. + 7); wave w takes steps s = w, w + W, ... (NS of them) and keeps
// its X operands in registers for the whole kernel; the W partial tiles are summed
// in wave order through LDS (double-buffered: one barrier per tile).
template <typename T, int W, int NS>
__global__ __launch_bounds__(64 * W) void dot_mfma_kernel(StreamArgs a) {
  __shared__ double red[2][W][4][64];
  const int C = a.C;
  const int part = blockIdx.x / a.Gd;
  const int wg = blockIdx.x - part * a.Gd;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int nsteps = (a.n + 31) >> 5;
  const float* xs = reinterpret_cast<const float*>(a.xs) + (int64_t)part * a.ld * C;
  float xb[NS][8];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const int st = wv + W * q;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int k = 32 * st + 8 * g + u;
      xb[q][u] = (st < nsteps && k < a.n && j < C) ? xs[(int64_t)k * C + j] : 0.f;
    }
  }
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld + 8 * g;
  const int64_t ntiles = (m + 15) >> 4;
  int buf = 0;
  for (int64_t tile = wg; tile < ntiles; tile += a.Gd) {
    const T* rp = Ab + min(tile * 16 + j, m - 1) * a.ld;
    float av[NS][8];
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      if (wv + W * q < nsteps) {
        load8(rp + 32 * (wv + W * q), av[q]);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) av[q][u] = 0.f;
      }
    }
    mc_f4 acc = {0.f, 0.f, 0.f, 0.f};
    double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      if (wv + W * q < nsteps) {
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[q][u], xb[q][u], acc, 0, 0, 0);
      }
      if ((q & 1) || q == NS - 1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          d[v] += (double)acc[v];
          acc[v] = 0.f;
        }
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) red[buf][wv][v][lane] = d[v];
    __syncthreads();
    if (threadIdx.x < 256) {
      const int L = threadIdx.x & 63, v = threadIdx.x >> 6;
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < W; ++w) sum += red[buf][w][v][L];
      const int64_t row = tile * 16 + 4 * (L >> 4) + v;
      const int c = L & 15;
      if (row < m && c < C) a.rowbuf[(r0 + row) * C + c] = sum * a.inv_M;
    }
    buf ^= 1;
  }
}

// Partial sums of A_i^T E: workgroup (partition, row range, strip of kMcStrip
// features), i = feature, j = class, k = sample.  Lane l reads features
// f0 + 8 (l % 16) .. + 7 of sample 4 t + l / 16, so a 4-sample step is 4 rows of
// 512 contiguous bytes (FP32); instruction u's output element v of lane l is
// feature f0 + 8 (4 (l / 16) + v) + u, class l % 16.  The four wavefronts split the
// range's steps (wave w takes t = w, w + 4, ...) and their sums are added in wave
// order through LDS into the partial sum of the range.
template <typename T>
__global__ __launch_bounds__(256) void acc_mfma_kernel(StreamArgs a) {
  constexpr int W = 4;
  __shared__ double sh[32][64];
  const int C = a.C;
  const int nstrips = (a.n + kMcStrip - 1) / kMcStrip;
  int bi = blockIdx.x;
  const int strip = bi % nstrips;
  bi /= nstrips;
  const int wg = bi % a.Gp;
  const int part = bi / a.Gp;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int g = lane >> 4, i = lane & 15;
  const int64_t nst = (m + 3) >> 2;
  const int64_t per = (nst + a.Gp - 1) / a.Gp;
  const int64_t s0 = wg * per, s1 = min(nst, s0 + per);
  const int f0 = strip * kMcStrip + 8 * i;
  const bool fin = f0 < a.n;
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld + (fin ? f0 : 0);
  const double* E = a.rowbuf + r0 * C;
  mc_f4 acc[8];
  double dacc[8][4];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    acc[u] = mc_f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < 4; ++v) dacc[u][v] = 0.0;
  }
  // four steps per round, their loads issued together
  for (int64_t st = s0 + wv; st < s1; st += 4 * W) {
    float av[4][8], e[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int64_t sb = st + (int64_t)b * W;
      const int64_t smp = sb * 4 + g;
      const bool ok = sb < s1 && smp < m;
      if (sb < s1 && fin) {
        load8(Ab + min(smp, m - 1) * a.ld, av[b]);
      } else {
#pragma unroll
        for (int u = 0; u < 8; ++u) av[b][u] = 0.f;
      }
      e[b] = (ok && i < C) ? (float)E[smp * C + i] : 0.f;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[b][u], e[b], acc[u], 0, 0, 0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        dacc[u][v] += (double)acc[u][v];
        acc[u][v] = 0.f;
      }
  }
  for (int w = 0; w < W; ++w) {
    if (wv == w) {
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) sh[u * 4 + v][lane] = w == 0 ? dacc[u][v] : sh[u * 4 + v][lane] + dacc[u][v];
    }
    __syncthreads();
  }
  if (wv == 0) {
    double* gp = a.gpart + ((int64_t)part * a.Gp + wg) * a.ld * C;
    const int c = lane & 15;
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int f = strip * kMcStrip + 8 * (4 * g + v) + u;
        if (f < a.n && c < C) gp[(int64_t)f * C + c] = sh[u * 4 + v][lane];
      }
  }
}

template <typename T>
static void mc_mfma_launch(const StreamArgs& a, hipStream_t s) {
  const int nsteps = (a.n + 31) >> 5;
  const dim3 gd(a.N * a.Gd);
  if (nsteps <= 4) hipLaunchKernelGGL((dot_mfma_kernel<T, 4, 1>), gd, dim3(256), 0, s, a);
  else if (nsteps <= 8) hipLaunchKernelGGL((dot_mfma_kernel<T, 4, 2>), gd, dim3(256), 0, s, a);
  else if (nsteps <= 16) hipLaunchKernelGGL((dot_mfma_kernel<T, 4, 4>), gd, dim3(256), 0, s, a);
  else if (nsteps <= 32) hipLaunchKernelGGL((dot_mfma_kernel<T, 4, 8>), gd, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((dot_mfma_kernel<T, 8, 8>), gd, dim3(512), 0, s, a);
  const unsigned waves = (unsigned)((a.m_total + 3) / 4);
  hipLaunchKernelGGL(prox_mc_kernel, dim3((waves + 3) / 4), dim3(256), 0, s, a);
  const int nstrips = (a.n + kMcStrip - 1) / kMcStrip;
  hipLaunchKernelGGL(acc_mfma_kernel<T>, dim3(a.N * a.Gp * nstrips), dim3(256), 0, s, a);
}

// Objective pass for C classes: per-workgroup partial sums of LSE(q_k) - q_{k, y_k}.
template <typename T, int NT, int NF, int CC>
__global__ __launch_bounds__(NT) void objective_mc_kernel(ObjArgs a) {
  using acc = typename Traits<T>::acc_t;
  constexpr int NW = NT / 64;
  __shared__ double red[NW][CC];
  const int C = a.C;
  const int part = blockIdx.x / a.Gp;
  const int wg = blockIdx.x - part * a.Gp;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int n = a.n;
  const acc* xs = reinterpret_cast<const acc*>(a.xs);
  acc xr[NF][CC];
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int k = tid + f * NT;
#pragma unroll
    for (int c = 0; c < CC; ++c) xr[f][c] = (k < n && c < C) ? xs[(int64_t)k * C + c] : acc(0);
  }
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld;
  double lsum = 0.0;
  for (int64_t row = wg; row < m; row += a.Gp) {
    acc v[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int k = tid + f * NT;
      v[f] = k < n ? load_scalar<T>(Ab + row * a.ld + k) : acc(0);
    }
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      acc d = acc(0);
#pragma unroll
      for (int f = 0; f < NF; ++f) d += v[f] * xr[f][c];
      const double s = wave_sum((double)d);
      if (lane == 0) red[wv][c] = s;
    }
    __syncthreads();
    if (tid == 0) {
      double q[CC];
      for (int c = 0; c < C; ++c) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += red[w][c];
        q[c] = s;
      }
      lsum += lse_c(q, C) - q[a.y[r0 + row]];
    }
    __syncthreads();
  }
  if (tid == 0) a.partial[blockIdx.x] = lsum;
}

// Supported multi-class shapes: C <= 16, n <= 2048 (features per thread NF <= 4
// with up to 512 threads).
bool mc_supported(int n, int C) { return C >= 2 && C <= 16 && n <= 2048; }

static void mc_shape(int n, int* nt, int* nf) {
  *nt = n <= 1024 ? 256 : 512;
  int f = (n + *nt - 1) / *nt;
  *nf = f <= 1 ? 1 : (f <= 2 ? 2 : 4);
}

template <typename T, int CC>
static void mc_launch(const StreamArgs& a, hipStream_t s) {
  int nt, nf;
  mc_shape(a.n, &nt, &nf);
  dim3 grid(a.N * a.Gp);
#define BCA_MC(K_, NT_, NF_) hipLaunchKernelGGL((K_<T, NT_, NF_, 4, CC>), grid, dim3(NT_), 0, s, a)
#define BCA_MC_ALL(K_)                    \
  if (nt == 256) {                        \
    if (nf == 1) BCA_MC(K_, 256, 1);      \
    else if (nf == 2) BCA_MC(K_, 256, 2); \
    else BCA_MC(K_, 256, 4);              \
  } else {                                \
    if (nf == 1) BCA_MC(K_, 512, 1);      \
    else if (nf == 2) BCA_MC(K_, 512, 2); \
    else BCA_MC(K_, 512, 4);              \
  }
  BCA_MC_ALL(dot_mc_kernel)
  const unsigned waves = (unsigned)((a.m_total + 3) / 4);
  hipLaunchKernelGGL(prox_mc_kernel, dim3((waves + 3) / 4), dim3(256), 0, s, a);
  BCA_MC_ALL(acc_mc_kernel)
#undef BCA_MC_ALL
#undef BCA_MC
}

template <typename T, int CC>
static int mc_occ(int n) {
  int nt, nf;
  mc_shape(n, &nt, &nf);
  int b1 = 0, b2 = 0;
#define BCA_OCC2(NT_, NF_)                                                                     \
  do {                                                                                         \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b1, dot_mc_kernel<T, NT_, NF_, 4, CC>, NT_, 0) != hipSuccess) b1 = 1; \
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b2, acc_mc_kernel<T, NT_, NF_, 4, CC>, NT_, 0) != hipSuccess) b2 = 1; \
  } while (0)
  if (nt == 256) {
    if (nf == 1) BCA_OCC2(256, 1);
    else if (nf == 2) BCA_OCC2(256, 2);
    else BCA_OCC2(256, 4);
  } else {
    if (nf == 1) BCA_OCC2(512, 1);
    else if (nf == 2) BCA_OCC2(512, 2);
    else BCA_OCC2(512, 4);
  }
#undef BCA_OCC2
  const int b = b1 < b2 ? b1 : b2;
  return b < 1 ? 1 : b;
}

template <typename T>
static int mc_occ_dispatch(int n, int C) {
  if (C <= 4) return mc_occ<T, 4>(n);
  if (C <= 10) return mc_occ<T, 10>(n);
  return mc_occ<T, 16>(n);
}

int mc_occupancy_workgroups(int dtype, int n, int C) {
  switch (dtype) {
    case BCA_F64: return mc_occ_dispatch<double>(n, C);
    case BCA_F32: return mc_occ_dispatch<float>(n, C);
    default: return mc_occ_dispatch<bf16_t>(n, C);
  }
}

template <typename T, int CC>
static void mc_obj_launch(const ObjArgs& a, hipStream_t s) {
  int nt, nf;
  mc_shape(a.n, &nt, &nf);
  dim3 grid(a.N * a.Gp);
#define BCA_MO(NT_, NF_) hipLaunchKernelGGL((objective_mc_kernel<T, NT_, NF_, CC>), grid, dim3(NT_), 0, s, a)
  if (nt == 256) {
    if (nf == 1) BCA_MO(256, 1);
    else if (nf == 2) BCA_MO(256, 2);
    else BCA_MO(256, 4);
  } else {
    if (nf == 1) BCA_MO(512, 1);
    else if (nf == 2) BCA_MO(512, 2);
    else BCA_MO(512, 4);
  }
#undef BCA_MO
}

template <typename T>
static void mc_dispatch(const StreamArgs& a, hipStream_t s) {
  if (a.C <= 4) mc_launch<T, 4>(a, s);
  else if (a.C <= 10) mc_launch<T, 10>(a, s);
  else mc_launch<T, 16>(a, s);
}

template <typename T>
static void mc_obj_dispatch(const ObjArgs& a, hipStream_t s) {
  if (a.C <= 4) mc_obj_launch<T, 4>(a, s);
  else if (a.C <= 10) mc_obj_launch<T, 10>(a, s);
  else mc_obj_launch<T, 16>(a, s);
}

hipError_t launch_stream_mc(const StreamArgs& a, int dtype, hipStream_t s) {
  if (!mc_supported(a.n, a.C)) return hipErrorInvalidValue;
  switch (dtype) {
    case BCA_F64: mc_dispatch<double>(a, s); break;
    case BCA_F32: mc_mfma_launch<float>(a, s); break;
    default: mc_mfma_launch<bf16_t>(a, s); break;
  }
  return hipGetLastError();
}

hipError_t launch_objective_mc(const ObjArgs& a, int dtype, hipStream_t s) {
  if (!mc_supported(a.n, a.C)) return hipErrorInvalidValue;
  switch (dtype) {
    case BCA_F64: mc_obj_dispatch<double>(a, s); break;
    case BCA_F32: mc_obj_dispatch<float>(a, s); break;
    default: mc_obj_dispatch<bf16_t>(a, s); break;
  }
  return hipGetLastError();
}

}  // namespace bca
