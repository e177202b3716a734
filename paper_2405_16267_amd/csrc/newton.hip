// Exact x-update of the logistic loss (BCA_FLAG_EXACT_X with the logistic loss):
// every partition's x-subproblem of the ADMM iterations (Sec. 3) solved as a
// whole -- without the feature split of Sec. 3.1 -- by Newton's method:
//     phi_i(x) = sum_k log(1 + exp(-b_k a_k^T x)) + ||x||^2 / (2 N gamma)
//                + (rho_c / 2) ||x - z + u_i||^2,
//     g = A_i^T (-b sigmoid(-b q)) + s x - rho_c (z - u_i),   q = A_i x,
//     H = A_i^T diag(sigmoid(q) sigmoid(-q)) A_i + s I,        s = 1/(N gamma) + rho_c.
// Each Newton direction solves H d = -g by conjugate gradients preconditioned with
// the cached P_i = (A_i^T A_i / 4 + s I)^-1 (formed at finalize like the squared
// loss's exact factor; sigmoid(q) sigmoid(-q) <= 1/4, so H <= P_i^-1).  The
// products H p are the fused streaming pass (stream.hip, mode 3: row dot with p,
// weighted by the stored Hessian weight, accumulated into A_i^T); the gradient is
// the same pass in mode 2.  The step length is chosen by Armijo backtracking on
// phi over the sample-space values q_k + t a_k^T d, which the passes leave in row
// buffers, so no further pass over A is needed.
//
// CG stops once the preconditioned residual has fallen by the forcing factor
// eta_k = min(1/2, sqrt(|g_k| / |g_0|)) (|.| the P_i-norm, g_0 the gradient at the
// first Newton iteration of this x-update), floored at the working precision's
// tolerance: loose solves while far from the minimiser, tight ones near it, the
// inexact Newton method of Dembo, Eisenstat and Steihaug (superlinear).
//
// All partitions advance together; a partition whose Newton iteration (or CG)
// has ended is skipped by every kernel (flags in `done`).  Everything here is FP64.
#include "bca_internal.h"
#include "global_impl.h"
#include "symv_impl.h"

namespace bca {

constexpr int NTB = 1024;  // threads of the per-partition vector kernels

// z (the symmetric product's slots) of partition `part`, element i
__device__ __forceinline__ double nt_gather(const NewtonArgs& a, int part, int i) {
  const int T = (a.n + PT - 1) / PT;
  return symv_gather(a.ypart + (int64_t)part * a.tmax * a.tmax * PT, i, 0, 1, T);
}

__device__ __forceinline__ void nt_store_xs(const NewtonArgs& a, int part, int i, double v) {
  const int64_t o = (int64_t)part * a.ld + i;
  if (a.xs_f64)
    reinterpret_cast<double*>(a.xs)[o] = v;
  else
    reinterpret_cast<float*>(a.xs)[o] = (float)v;
}

// After the gradient pass and r = -g, z = P r: g, p = z, d = 0, rz = r^T z, the
// row values a_k^T d = 0, and the streaming copy of p for the first H p pass.
__global__ __launch_bounds__(NTB) void nt_start_kernel(NewtonArgs a) {
  __shared__ double sh[NTB / 64];
  const int part = blockIdx.x;
  int* dn = a.done + 2 * part;
  if (dn[0]) return;
  const int64_t o = (int64_t)part * a.n;
  double rz = 0.0;
  for (int i = threadIdx.x; i < a.n; i += NTB) {
    const double r = a.r[o + i];
    const double z = nt_gather(a, part, i);
    a.g[o + i] = -r;
    a.p[o + i] = z;
    a.d[o + i] = 0.0;
    rz += r * z;
    nt_store_xs(a, part, i, z);
  }
  const int64_t r0 = a.row_off[part], r1 = a.row_off[part + 1];
  for (int64_t k = r0 + threadIdx.x; k < r1; k += NTB) a.rowd[k] = 0.0;
  rz = block_sum<NTB>(rz, sh);
  if (threadIdx.x == 0) {
    double* sc = a.sc + NT_SCAL * part;
    sc[NT_RZ] = rz;
    sc[NT_RZ0] = rz;
    sc[NT_ALPHA] = 0.0;
    if (!(sc[NT_RZF] > 0.0)) sc[NT_RZF] = rz;   // first Newton iteration of this x-update
    const double f = rz > 0.0 ? sqrt(rz / sc[NT_RZF]) : 0.0;   // eta_k^2 = |g_k| / |g_0|
    sc[NT_ETA2] = fmax(a.eta2, fmin(0.25, f));
    dn[1] = !(rz > 0.0);   // g = 0: nothing to solve
  }
}

// alpha = r^T z / p^T H p; d += alpha p; r -= alpha H p (hp = H p from the pass)
__global__ __launch_bounds__(NTB) void nt_alpha_kernel(NewtonArgs a) {
  __shared__ double sh[NTB / 64];
  const int part = blockIdx.x;
  const int* dn = a.done + 2 * part;
  double* sc = a.sc + NT_SCAL * part;
  if (dn[0] || dn[1]) {
    if (threadIdx.x == 0) sc[NT_ALPHA] = 0.0;
    return;
  }
  const int64_t o = (int64_t)part * a.n;
  double php = 0.0;
  for (int i = threadIdx.x; i < a.n; i += NTB) php += a.p[o + i] * a.hp[o + i];
  php = block_sum<NTB>(php, sh);
  const double alpha = php > 0.0 ? sc[NT_RZ] / php : 0.0;
  for (int i = threadIdx.x; i < a.n; i += NTB) {
    a.d[o + i] += alpha * a.p[o + i];
    a.r[o + i] -= alpha * a.hp[o + i];
  }
  if (threadIdx.x == 0) sc[NT_ALPHA] = alpha;
}

// a_k^T d += alpha a_k^T p over the partition's rows (grid: row chunks x partitions)
__global__ __launch_bounds__(256) void nt_rowd_kernel(NewtonArgs a) {
  const int part = blockIdx.y;
  const double alpha = a.sc[NT_SCAL * part + NT_ALPHA];
  if (alpha == 0.0) return;
  const int64_t k = a.row_off[part] + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < a.row_off[part + 1]) a.rowd[k] += alpha * a.rowp[k];
}

// z = P r (slots); beta = r^T z / rz; p = z + beta p; CG ends once r^T z <= eta_k^2 rz0
__global__ __launch_bounds__(NTB) void nt_beta_kernel(NewtonArgs a) {
  __shared__ double sh[NTB / 64];
  const int part = blockIdx.x;
  int* dn = a.done + 2 * part;
  if (dn[0] || dn[1]) return;
  double* sc = a.sc + NT_SCAL * part;
  const int64_t o = (int64_t)part * a.n;
  double rz = 0.0;
  for (int i = threadIdx.x; i < a.n; i += NTB) rz += a.r[o + i] * nt_gather(a, part, i);
  rz = block_sum<NTB>(rz, sh);
  const double beta = sc[NT_RZ] > 0.0 ? rz / sc[NT_RZ] : 0.0;
  for (int i = threadIdx.x; i < a.n; i += NTB) {
    const double p = nt_gather(a, part, i) + beta * a.p[o + i];
    a.p[o + i] = p;
    nt_store_xs(a, part, i, p);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sc[NT_RZ] = rz;
    if (!(rz > sc[NT_ETA2] * sc[NT_RZ0])) dn[1] = 1;
  }
}

// Line search, rows: partial sums of sum_k log(1 + exp(-b_k (q_k + t_l a_k^T d)))
// for the trial steps t_l = 2^-l (l < NT_LS - 1) and t = 0 (last slot).
__global__ __launch_bounds__(256) void nt_ls_rows_kernel(NewtonArgs a) {
  __shared__ double sh[NT_LS * 4];
  const int part = blockIdx.y;
  if (a.done[2 * part]) return;
  const int64_t r0 = a.row_off[part], r1 = a.row_off[part + 1];
  double v[NT_LS];
#pragma unroll
  for (int l = 0; l < NT_LS; ++l) v[l] = 0.0;
  for (int64_t k = r0 + (int64_t)blockIdx.x * 256 + threadIdx.x; k < r1; k += (int64_t)gridDim.x * 256) {
    const double b = a.b[k], q = a.rowq[k], rd = a.rowd[k];
#pragma unroll
    for (int l = 0; l < NT_LS; ++l) {
      const double t = l == NT_LS - 1 ? 0.0 : ldexp(1.0, -l);
      const double u = -b * (q + t * rd);   // log(1 + exp(u)), overflow-safe
      v[l] += u > 0.0 ? u + log1p(exp(-u)) : log1p(exp(u));
    }
  }
  block_sum_n<256, NT_LS>(v, sh);
  if (threadIdx.x < NT_LS) {
    double out = 0.0;
#pragma unroll
    for (int l = 0; l < NT_LS; ++l)
      if (l == (int)threadIdx.x) out = v[l];
    a.lsp[((int64_t)part * gridDim.x + blockIdx.x) * NT_LS + threadIdx.x] = out;
  }
}

// Step choice and update: phi(x + t d) = L(t) + ||x + t d||^2 / (2 N gamma)
// + (rho_c / 2) ||x + t d - v||^2; the largest trial t with the Armijo decrease
// (none passes only when phi is flat to rounding, at the minimiser: then the
// smallest trial); x += t d; the Newton iteration ends when the step is below
// step_tol relative to x.
__global__ __launch_bounds__(NTB) void nt_update_kernel(NewtonArgs a, int ls_groups) {
  __shared__ double sh[(NTB / 64) * 6];
  __shared__ double tsel;
  const int part = blockIdx.x;
  int* dn = a.done + 2 * part;
  if (dn[0]) return;
  const int64_t o = (int64_t)part * a.n;
  double q[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // x.x, x.d, d.d, w.w, w.d, g.d  (w = x - v)
  for (int i = threadIdx.x; i < a.n; i += NTB) {
    const double x = a.x[o + i], d = a.d[o + i];
    const double w = x - (a.z[i] - a.u[o + i]);
    q[0] += x * x;
    q[1] += x * d;
    q[2] += d * d;
    q[3] += w * w;
    q[4] += w * d;
    q[5] += a.g[o + i] * d;
  }
  block_sum_n<NTB, 6>(q, sh);
  if (threadIdx.x == 0) {
    double L[NT_LS];
    for (int l = 0; l < NT_LS; ++l) {
      double s = 0.0;
      for (int w = 0; w < ls_groups; ++w) s += a.lsp[((int64_t)part * ls_groups + w) * NT_LS + l];
      L[l] = s;
    }
    auto quad = [&](double t) {
      return (q[0] + 2.0 * t * q[1] + t * t * q[2]) * a.inv2Ng +
             0.5 * a.rho_c * (q[3] + 2.0 * t * q[4] + t * t * q[2]);
    };
    const double f0 = L[NT_LS - 1] + quad(0.0);
    double t = ldexp(1.0, -(NT_LS - 2));
    bool found = false;
    for (int l = 0; l < NT_LS - 1 && !found; ++l) {
      const double tl = ldexp(1.0, -l);
      if (L[l] + quad(tl) <= f0 + 1e-4 * tl * q[5]) {
        t = tl;
        found = true;
      }
    }
    tsel = t;
  }
  __syncthreads();
  const double t = tsel;
  double dmax = 0.0, xmax = 0.0;
  for (int i = threadIdx.x; i < a.n; i += NTB) {
    const double xn = a.x[o + i] + t * a.d[o + i];
    a.x[o + i] = xn;
    dmax = fmax(dmax, fabs(t * a.d[o + i]));
    xmax = fmax(xmax, fabs(xn));
  }
  // maxima over the workgroup (order-free)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    dmax = fmax(dmax, __shfl_xor(dmax, off, 64));
    xmax = fmax(xmax, __shfl_xor(xmax, off, 64));
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = dmax;
    sh[(NTB / 64) + (threadIdx.x >> 6)] = xmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double dm = 0.0, xm = 0.0;
    for (int w = 0; w < NTB / 64; ++w) {
      dm = fmax(dm, sh[w]);
      xm = fmax(xm, sh[(NTB / 64) + w]);
    }
    if (dm <= a.step_tol * fmax(xm, 1e-300)) dn[0] = 1;
  }
}

// start of an x-update: flags cleared, the reference gradient norm unset
__global__ void nt_reset_kernel(int* done, double* sc, int N) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < 2 * N) done[k] = 0;
  if (k < N) sc[NT_SCAL * k + NT_RZF] = 0.0;
}

hipError_t launch_nt_reset(const NewtonArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(nt_reset_kernel, dim3((2 * a.N + 255) / 256), dim3(256), 0, s, a.done, a.sc, a.N);
  return hipGetLastError();
}

hipError_t launch_nt_start(const NewtonArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(nt_start_kernel, dim3(a.N), dim3(NTB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nt_cg_step(const NewtonArgs& a, int64_t max_rows, hipStream_t s) {
  hipLaunchKernelGGL(nt_alpha_kernel, dim3(a.N), dim3(NTB), 0, s, a);
  hipLaunchKernelGGL(nt_rowd_kernel, dim3((unsigned)((max_rows + 255) / 256), a.N), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nt_beta(const NewtonArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(nt_beta_kernel, dim3(a.N), dim3(NTB), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_nt_update(const NewtonArgs& a, int ls_groups, hipStream_t s) {
  hipLaunchKernelGGL(nt_ls_rows_kernel, dim3(ls_groups, a.N), dim3(256), 0, s, a);
  hipLaunchKernelGGL(nt_update_kernel, dim3(a.N), dim3(NTB), 0, s, a, ls_groups);
  return hipGetLastError();
}

}  // namespace bca
