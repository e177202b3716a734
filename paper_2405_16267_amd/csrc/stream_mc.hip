// Multi-class (softmax) form of the fused A-streaming pass of Algorithm 2.
//
// With C classes the block predictions are m_i x C (A_ij X_ij), the omega-bar
// step is a C-dimensional prox per sample and A_i^T E is n x C.  Thread t owns
// the features t, t + NT, ..., and for each of them all C columns of X in
// registers; the per-row dots (R rows x C classes) are reduced across the
// workgroup, one thread per row runs the softmax prox, and e_k (C values) is
// broadcast back for the A_i^T E accumulation.  Tile partial sums of A_i^T E are
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

// F(q) and, if p/g are given, softmax probabilities and gradient.
__device__ double softmax_F(const double* q, const double* q0, int y, double beta, int C) {
  double f = lse_c(q, C) - q[y];
  double r = 0.0;
  for (int c = 0; c < C; ++c) r += (q[c] - q0[c]) * (q[c] - q0[c]);
  return f + 0.5 * beta * r;
}

__device__ double softmax_grad(const double* q, const double* q0, int y, double beta, int C,
                               double* p, double* g) {
  const double l = lse_c(q, C);
  double gn = 0.0;
  for (int c = 0; c < C; ++c) {
    p[c] = exp(q[c] - l);
    g[c] = p[c] - (c == y ? 1.0 : 0.0) + beta * (q[c] - q0[c]);
    gn += g[c] * g[c];
  }
  return sqrt(gn);
}

// scratch: 6 * C doubles (q0, q, p, g, step, trial); c: C values; w_prev (the
// previous omega-bar of the sample) seeds the iteration; result in w (C values)
__device__ void prox_softmax_row(const double* cvec, const double* w_prev, int y, int M,
                                 double rho_l, int C, double* scratch, double* w) {
  double* q0 = scratch;
  double* q = scratch + C;
  double* p = scratch + 2 * C;
  double* g = scratch + 3 * C;
  double* st = scratch + 4 * C;
  double* qt = scratch + 5 * C;
  const double beta = rho_l / M;
  for (int c = 0; c < C; ++c) {
    q0[c] = M * cvec[c];
    q[c] = M * w_prev[c];
  }
  // stop at ||grad|| <= 1e-14, or at the rounding level of beta (q - Mc) if higher
  double qmax = 0.0;
  for (int c = 0; c < C; ++c) qmax = fmax(qmax, fabs(q0[c]));
  for (int it = 0; it < 100; ++it) {
    const double gn = softmax_grad(q, q0, y, beta, C, p, g);
    double qa = qmax;
    for (int c = 0; c < C; ++c) qa = fmax(qa, fabs(q[c]));
    if (!(gn > 1e-14 + 8.0 * 2.220446049250313e-16 * beta * 2.0 * qa)) break;
    double pDp = 0.0, pDg = 0.0;
    for (int c = 0; c < C; ++c) {
      const double d = 1.0 / (p[c] + beta);
      pDp += p[c] * p[c] * d;
      pDg += p[c] * g[c] * d;
    }
    const double coef = pDg / (1.0 - pDp);
    double slope = 0.0;
    for (int c = 0; c < C; ++c) {
      const double d = 1.0 / (p[c] + beta);
      st[c] = d * g[c] + d * p[c] * coef;
      slope += g[c] * st[c];
    }
    const double f0 = softmax_F(q, q0, y, beta, C);
    double t = 1.0;
    for (int ls = 0; ls < 60; ++ls) {
      for (int c = 0; c < C; ++c) qt[c] = q[c] - t * st[c];
      if (softmax_F(qt, q0, y, beta, C) <= f0 - 1e-4 * t * slope) break;
      // gradient-norm decrease (F flat to rounding near the optimum)
      if (softmax_grad(qt, q0, y, beta, C, p, g) < gn) break;
      t *= 0.5;
    }
    for (int c = 0; c < C; ++c) q[c] = q[c] - t * st[c];
  }
  for (int c = 0; c < C; ++c) w[c] = q[c] / M;
}

template <typename T, int NT, int NF, int R, int CC>
__global__ __launch_bounds__(NT) void stream_mc_kernel(StreamArgs a) {
  using acc = typename Traits<T>::acc_t;
  constexpr int NW = NT / 64;
  constexpr int FLUSH = 16;
  __shared__ double red[NW][R][CC];
  __shared__ double e_sh[R][CC];
  __shared__ double scratch[R][7 * CC];

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
  double* gp = a.gpart + ((int64_t)part * a.Gp + wg) * a.ld * C;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int k = tid + f * NT;
    if (k < n)
      for (int c = 0; c < C; ++c) gp[(int64_t)k * C + c] = 0.0;
  }
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
        const double s = wave_sum((double)d);
        if (lane == 0) red[wv][r][c] = s;
      }
    }
    __syncthreads();
    if (tid < R) {
      const int r = tid;
      const int64_t row = rt + r;
      if (row < m) {
        const int64_t gr = r0 + row;
        double* cv = &scratch[r][6 * CC];   // c = a + nu (C values)
        double av[CC];
#pragma unroll
        for (int c = 0; c < CC; ++c) {
          double s = 0.0;
#pragma unroll
          for (int w = 0; w < NW; ++w) s += red[w][r][c];
          av[c] = s * a.inv_M;
        }
        if (a.mode == 0) {
          for (int c = 0; c < C; ++c) cv[c] = av[c] + a.nu[gr * C + c];
          double om[CC];
          prox_softmax_row(cv, a.omega + gr * C, a.y[gr], a.M, a.rho_l, C, &scratch[r][0], om);
          for (int c = 0; c < C; ++c) {
            const double nu = a.nu[gr * C + c] + av[c] - om[c];
            a.omega[gr * C + c] = om[c];
            a.nu[gr * C + c] = nu;
            e_sh[r][c] = om[c] - av[c] - nu;
          }
        } else {
          for (int c = 0; c < C; ++c) e_sh[r][c] = a.omega[gr * C + c] - av[c] - a.nu[gr * C + c];
        }
        for (int c = C; c < CC; ++c) e_sh[r][c] = 0.0;
      } else {
        for (int c = 0; c < CC; ++c) e_sh[r][c] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < CC; ++c) {
        const acc e = (acc)e_sh[r][c];
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
            if (c < C) gp[(int64_t)k * C + c] += (double)gt[f][c];
        }
#pragma unroll
        for (int c = 0; c < CC; ++c) gt[f][c] = acc(0);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    const int k = tid + f * NT;
    if (k < n) {
#pragma unroll
      for (int c = 0; c < CC; ++c)
        if (c < C) gp[(int64_t)k * C + c] += (double)gt[f][c];
    }
  }
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
#define BCA_MC(NT_, NF_) hipLaunchKernelGGL((stream_mc_kernel<T, NT_, NF_, 4, CC>), grid, dim3(NT_), 0, s, a)
  if (nt == 256) {
    if (nf == 1) BCA_MC(256, 1);
    else if (nf == 2) BCA_MC(256, 2);
    else BCA_MC(256, 4);
  } else {
    if (nf == 1) BCA_MC(512, 1);
    else if (nf == 2) BCA_MC(512, 2);
    else BCA_MC(512, 4);
  }
#undef BCA_MC
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
    case BCA_F32: mc_dispatch<float>(a, s); break;
    default: mc_dispatch<bf16_t>(a, s); break;
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
