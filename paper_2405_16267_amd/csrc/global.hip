// Global level of Algorithm 1 plus the node-level u-update.  For one problem
// the O(N n) consensus average and u-update with residuals run over many
// workgroups (consensus_kernel, uresid_kernel, gfinal_kernel) around one
// workgroup of 1024 threads for the O(n), latency-bound rest (global_kernel);
// the batched kernel runs all of it in one workgroup:
//   wbar = (1/N) sum_i (x_i + u_i)                         consensus average
//   (z, t) = argmin_{||z||_1 <= t} (a/2)||z - wbar||^2 + (rho_b/2)(s^T z - t + v)^2
//   s = clip((t - v)/M_kappa, -1, 1) sign(z) on T_kappa(z)  (s-step, Sec. 3)
//   v += z^T s - t;  u_i += x_i - z;  p_r, d_r, b_r          (Termination, Sec. 3)
// with a = N rho_c.  The (z, t) problem is strictly convex; from its KKT
// conditions z(theta) = S_{theta/a}(wbar + theta s / a) and theta >= 0 is the
// root of the increasing piecewise-linear
//   psi(theta) = v + theta / rho_b + sum_{k: theta_k > theta} (theta d_k^2 / a - d_k |wbar_k|),
//   d_k = 1 - sign(wbar_k) s_k,  theta_k = a |wbar_k| / d_k (breakpoints).
// psi is also concave, so Newton steps from theta = 0 reach the root exactly
// (each step is the root of the linear piece active right of the current
// point); multisection brackets it if Newton has not settled after 32 steps.
// T_kappa is a radix select on the bit patterns of |z_k| (FP64 bits with the
// sign cleared, so -0 == +0), ties resolved toward the lower index.
#include "global_impl.h"

namespace bca {

constexpr int GT = 1024;
constexpr int GW = GT / 64;

__global__ __launch_bounds__(GT) void global_kernel(GlobalArgs a) {
  __shared__ double shd[GW * (PSECT + 2)];
  __shared__ TopkShared<GT> tks;
  global_step<GT>(a, shd, tks);
}

// Split form, one problem: the O(N n) passes over many workgroups.
// consensus_kernel: one thread per row k; partial sum of d_k |wbar_k| and
// maximum finite breakpoint per workgroup into gp[g], gp[G + g].
__global__ __launch_bounds__(256) void consensus_kernel(GlobalArgs a) {
  __shared__ double shd[4];
  const int k = blockIdx.x * 256 + threadIdx.x;
  double s1 = 0.0, thm = 0.0;
  bool bad = false;
  if (k < a.n) consensus_row(a, k, &s1, &thm, &bad);
  if (bad) atomicExch(a.status, 1);
  s1 = block_sum<256>(s1, shd);
  thm = block_max<256>(thm, shd);
  if (threadIdx.x == 0) {
    a.gp[blockIdx.x] = s1;
    a.gp[a.G + blockIdx.x] = thm;
  }
}

// uresid_kernel: grid (G2, N + 1).  Row i < N: u_i += x_i - z and the partial
// sum of |x_i - z|^2 into gp[2G + i G2 + g]; row N: the partial sum of
// |z - z_prev|^2 into gp[2G + N G2 + g].
__global__ __launch_bounds__(256) void uresid_kernel(GlobalArgs a) {
  __shared__ double shd[4];
  const int i = blockIdx.y;
  const int64_t nc = (int64_t)a.n * a.C;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double acc = 0.0;
  if (e < nc) {
    if (i < a.N) {
      const int64_t o = (int64_t)i * nc + e;
      const double d = a.x[o] - a.z[e];
      acc = d * d;
      a.u[o] += d;
    } else {
      const double d = a.z[e] - a.work[nc + e];   // z_prev, saved by the consensus pass
      acc = d * d;
    }
  }
  acc = block_sum<256>(acc, shd);
  if (threadIdx.x == 0) a.gp[2 * (int64_t)a.G + (int64_t)i * a.G2 + blockIdx.x] = acc;
}

// gfinal_kernel: one workgroup; residuals from the partial sums in a fixed order.
__global__ __launch_bounds__(256) void gfinal_kernel(GlobalArgs a) {
  __shared__ double shd[4];
  const double* p = a.gp + 2 * (int64_t)a.G;
  double pr = 0.0;
  for (int i = 0; i < a.N; ++i) {
    double pl = 0.0;
    for (int g = threadIdx.x; g < a.G2; g += 256) pl += p[(int64_t)i * a.G2 + g];
    pr += sqrt(block_sum<256>(pl, shd));
  }
  double dz = 0.0;
  for (int g = threadIdx.x; g < a.G2; g += 256) dz += p[(int64_t)a.N * a.G2 + g];
  const double dzs = block_sum<256>(dz, shd);
  if (threadIdx.x == 0) {
    const double dr = sqrt((double)a.N) * a.rho_c * sqrt(dzs);
    const double br = fabs(a.scal[6]);
    const int it = (int)a.scal[5];
    a.scal[2] = pr;
    a.scal[3] = dr;
    a.scal[4] = br;
    a.scal[5] = (double)(it + 1);
    if (it < a.hist_cap) {
      a.hist[3 * (int64_t)it + 0] = pr;
      a.hist[3 * (int64_t)it + 1] = dr;
      a.hist[3 * (int64_t)it + 2] = br;
    }
    if (!isfinite(pr)) atomicExch(a.status, 1);
  }
}

hipError_t launch_global(const GlobalArgs& a, hipStream_t s) {
  if (a.C < 1) return hipErrorInvalidValue;
  if (!a.split) {
    hipLaunchKernelGGL(global_kernel, dim3(1), dim3(GT), 0, s, a);
    return hipGetLastError();
  }
  if (a.G != global_groups(a.n) || a.G2 != global_groups2(a.n, a.C) || !a.gp)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(consensus_kernel, dim3(a.G), dim3(256), 0, s, a);
  hipLaunchKernelGGL(global_kernel, dim3(1), dim3(GT), 0, s, a);
  hipLaunchKernelGGL(uresid_kernel, dim3(a.G2, a.N + 1), dim3(256), 0, s, a);
  hipLaunchKernelGGL(gfinal_kernel, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

template <typename Z>
__global__ __launch_bounds__(GT) void topk_kernel(const Z* z, int64_t n, int kappa, int32_t* idx) {
  __shared__ TopkShared<GT> tks;
  int take_eq;
  const uint64_t thr = topk_threshold<GT, Z>(z, n, kappa, tks, &take_eq);
  topk_apply<GT, Z>(z, n, thr, take_eq, tks, [&](int64_t k, bool sel, int pos) {
    if (sel && pos < kappa) idx[pos] = (int32_t)k;
  });
}

hipError_t launch_topk(const void* z, int f64, int64_t n, int kappa, int32_t* idx, double* work,
                       hipStream_t s) {
  (void)work;
  if (f64)
    hipLaunchKernelGGL(topk_kernel<double>, dim3(1), dim3(GT), 0, s, (const double*)z, n, kappa, idx);
  else
    hipLaunchKernelGGL(topk_kernel<float>, dim3(1), dim3(GT), 0, s, (const float*)z, n, kappa, idx);
  return hipGetLastError();
}

// T_kappa of the current z: row values (z_k, or ||z_k|| for C > 1) then the radix select.
__global__ __launch_bounds__(GT) void support_kernel(const double* z, int n, int C, int kappa,
                                                     int32_t* idx, double* rv) {
  __shared__ TopkShared<GT> tks;
  for (int k = threadIdx.x; k < n; k += GT) {
    if (C == 1) {
      rv[k] = z[k];
    } else {
      double s = 0.0;
      for (int c = 0; c < C; ++c) s += z[(int64_t)k * C + c] * z[(int64_t)k * C + c];
      rv[k] = sqrt(s);
    }
  }
  __syncthreads();
  int take_eq;
  const uint64_t thr = topk_threshold<GT, double>(rv, n, kappa, tks, &take_eq);
  topk_apply<GT, double>(rv, n, thr, take_eq, tks, [&](int64_t k, bool sel, int pos) {
    if (sel && pos < kappa) idx[pos] = (int32_t)k;
  });
}

hipError_t launch_support(const double* z, int n, int C, int kappa, int32_t* idx, double* work,
                          hipStream_t s) {
  hipLaunchKernelGGL(support_kernel, dim3(1), dim3(GT), 0, s, z, n, C, kappa, idx, work);
  return hipGetLastError();
}

// ------------------------------------------------------------------ input checks
template <typename T>
__global__ void check_kernel(const T* p, int64_t count, int* flag) {
  int bad = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    bad |= !isfinite((double)p[k]);
  if (bad) atomicExch(flag, 1);
}

__global__ void check_bf16_kernel(const uint16_t* p, int64_t count, int* flag) {
  int bad = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    bad |= ((p[k] & 0x7F80u) == 0x7F80u);
  if (bad) atomicExch(flag, 1);
}

hipError_t launch_check(const void* p, int dtype, int64_t count, int* flag, hipStream_t s) {
  dim3 g(1024), b(256);
  switch (dtype) {
    case BCA_F64: hipLaunchKernelGGL(check_kernel<double>, g, b, 0, s, (const double*)p, count, flag); break;
    case BCA_F32: hipLaunchKernelGGL(check_kernel<float>, g, b, 0, s, (const float*)p, count, flag); break;
    default: hipLaunchKernelGGL(check_bf16_kernel, g, b, 0, s, (const uint16_t*)p, count, flag); break;
  }
  return hipGetLastError();
}

__global__ void check_labels_kernel(const int32_t* y, int64_t count, int C, int* flag) {
  int bad = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    bad |= (y[k] < 0 || y[k] >= C);
  if (bad) atomicExch(flag, 1);
}

hipError_t launch_check_labels(const int32_t* y, int64_t count, int C, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(check_labels_kernel, dim3(256), dim3(256), 0, s, y, count, C, flag);
  return hipGetLastError();
}

__global__ void check_signs_kernel(const double* b, int64_t count, int* flag) {
  int bad = 0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
       k += (int64_t)gridDim.x * blockDim.x)
    bad |= !(b[k] == 1.0 || b[k] == -1.0);
  if (bad) atomicExch(flag, 1);
}

hipError_t launch_check_signs(const double* b, int64_t count, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(check_signs_kernel, dim3(256), dim3(256), 0, s, b, count, flag);
  return hipGetLastError();
}

}  // namespace bca
