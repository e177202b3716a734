// Sample-space (Woodbury) form of the x_ij-step of Sec. 3.1, for feature blocks
// wider than their partition is tall (m_i < n_j).
//
// The x_ij-step solves K_ij x = rho_l A_ij^T d + rho_c w with
// K_ij = rho_l A_ij^T A_ij + shift I, d = p_ij + e and w = z_j - u_ij.  By the
// matrix inversion lemma K_ij^-1 A_ij^T = A_ij^T S_ij^-1 with
// S_ij = rho_l A_ij A_ij^T + shift I (m_i x m_i), and rho_l A A^T S^-1 =
// I - shift S^-1, so the new block prediction p+ = A_ij x+ is
//     p+ = d - shift S^-1 d + rho_c h,   h = S^-1 A_ij w,
// and the new coefficients are x+ = (rho_l / shift) A_ij^T (d - p+) +
// (rho_c / shift) w.  w changes only in the global step, so one outer iteration
// is: one pass over A for A_ij w and p_ij = A_ij x_ij (wgemv_n), the product
// S^-1 A_ij w (wgather) and d = p_ij + e from the stored omega-bar and nu
// (wupdate, mode 1: the block predictions are re-derived from x at every outer
// iteration, so the iterates are a function of the state a checkpoint holds);
// K_in inner iterations that never touch A (one symmetric product with the
// cached S_ij^-1 per block, then wupdate: p+, the sample-space average, the
// omega-bar prox, the nu update and the next d); one pass over A for x+
// (wgemv_t).  Bytes per inner iteration: the m_i^2 / 2 stored entries of S_ij^-1
// per block instead of a pass over A and the n_j^2 / 2 entries of K_ij^-1.
//
//   rowgram_kernel  S_ij = rho_l A_ij A_ij^T + shift I, 64 x 64 lower tiles,
//                   FP64 sums of exact products (the form does not correct
//                   rounding in S_ij later, unlike the incremental x-step)
//   wgemv_n_kernel  A_ij w_j and A_ij x_ij per row and block, one workgroup per
//                   8 rows
//   wgemv_t_kernel  partial sums of A_ij^T r over row chunks, one thread per
//                   column; wxred_kernel adds them in a fixed order
//   wgather_kernel  h = S^-1 (A w) from the symmetric product's slots
//   wupdate_kernel  one thread per sample
#include "bca_internal.h"
#include "prox_impl.h"
#include "symv_impl.h"

namespace bca {

__device__ __forceinline__ double elem(const double* p) { return *p; }
__device__ __forceinline__ double elem(const float* p) { return (double)*p; }
__device__ __forceinline__ double elem(const bf16_t* p) { return (double)__uint_as_float((uint32_t)p->bits << 16); }

template <typename T>
__global__ __launch_bounds__(256) void rowgram_kernel(WoodArgs a) {
  constexpr int KC = 32;
  __shared__ double sI[64][KC + 1];
  __shared__ double sJ[64][KC + 1];
  const int bid = blockIdx.y;
  const int part = bid / a.M, blk = bid - part * a.M;
  const int c0 = a.col_off[blk];
  const int nj = a.col_off[blk + 1] - c0;
  const int T_ = (a.mw + 63) / 64;
  int ti, tj;
  tri_tile(blockIdx.x, &ti, &tj);
  if (ti >= T_) return;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld + c0;
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  double acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
  for (int k0 = 0; k0 < nj; k0 += KC) {
    for (int idx = tid; idx < 64 * KC; idx += 256) {
      const int rr = idx / KC, kk = idx % KC;
      const int col = k0 + kk;
      const int64_t ri = (int64_t)ti * 64 + rr, rj = (int64_t)tj * 64 + rr;
      sI[rr][kk] = (ri < m && col < nj) ? elem(Ab + ri * a.ld + col) : 0.0;
      sJ[rr][kk] = (rj < m && col < nj) ? elem(Ab + rj * a.ld + col) : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < KC; ++kk) {
      double ai[4], bj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) ai[u] = sI[tr + 16 * u][kk];
#pragma unroll
      for (int v = 0; v < 4; ++v) bj[v] = sJ[tc + 16 * v][kk];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] += ai[u] * bj[v];
    }
    __syncthreads();
  }
  double* K = a.kbuf + a.kmat_off[bid];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = ti * 64 + tr + 16 * u, col = tj * 64 + tc + 16 * v;
      if (row < a.mw && col < a.mw && row >= col)
        K[(int64_t)row * a.mw + col] = a.rho_l * acc[u][v] + (row == col ? a.shift : 0.0);
    }
}

// wt = A_ij (z_j - u_ij) and wr = A_ij x_ij in one pass.  A workgroup takes WR
// rows; its 256 threads stride over the columns, so each element of z, u and x
// is fetched once for all WR rows (with fewer rows per fetch the kernel is bound
// by those cached FP64 reads, not by A).  Row sums: DPP inside each wavefront,
// then the four wavefronts in a fixed order.
constexpr int WR = 8;
template <typename T>
__global__ __launch_bounds__(256) void wgemv_n_kernel(WoodArgs a) {
  __shared__ double red[4][2 * WR];
  const int part = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rb = blockIdx.x * WR;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int nr = (int)max((int64_t)0, min((int64_t)WR, m - rb));   // tile rows with data
  const T* A0 = reinterpret_cast<const T*>(a.A) + (r0 + rb) * a.ld;
  const double* xp = a.x + (int64_t)part * a.n;
  const double* up = a.u + (int64_t)part * a.n;
  for (int j = 0; j < a.M; ++j) {
    const int c0 = a.col_off[j], c1 = a.col_off[j + 1];
    double sw[WR], sx[WR];
#pragma unroll
    for (int q = 0; q < WR; ++q) sw[q] = sx[q] = 0.0;
    // branch-free loads: rows past the partition's end read its last row and
    // count zero times
    if (nr > 0) {
      const T* rp[WR];
      double keep[WR];
#pragma unroll
      for (int q = 0; q < WR; ++q) {
        rp[q] = A0 + (int64_t)min(q, nr - 1) * a.ld;
        keep[q] = q < nr ? 1.0 : 0.0;
      }
#pragma unroll 2
      for (int k = c0 + tid; k < c1; k += 256) {
        const double v = a.z[k] - up[k], xv = xp[k];
        double e[WR];
#pragma unroll
        for (int q = 0; q < WR; ++q) e[q] = elem(rp[q] + k);
#pragma unroll
        for (int q = 0; q < WR; ++q) {
          const double eq = e[q] * keep[q];
          sw[q] += eq * v;
          sx[q] += eq * xv;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < WR; ++q) {
      sw[q] = wave_sum_dpp(sw[q]);
      sx[q] = wave_sum_dpp(sx[q]);
    }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < WR; ++q) {
        red[wv][q] = sw[q];
        red[wv][WR + q] = sx[q];
      }
    }
    __syncthreads();
    if (tid < 2 * WR) {
      const int q = tid % WR;
      const double v = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
      if (rb + q < a.mw) {
        const int64_t o = ((int64_t)part * a.M + j) * a.mw + rb + q;
        (tid < WR ? a.wt : a.wr)[o] = v;
      }
    }
    __syncthreads();
  }
}

// grid (column groups of 256, row chunks Gw, partitions)
template <typename T>
__global__ __launch_bounds__(256) void wgemv_t_kernel(WoodArgs a) {
  const int part = blockIdx.z, g = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  int j = 0;
  while (j + 1 < a.M && a.col_off[j + 1] <= k) ++j;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int64_t chunk = (m + a.Gw - 1) / a.Gw;
  const int64_t rb = (int64_t)g * chunk, re = min(m, rb + chunk);
  const T* Ak = reinterpret_cast<const T*>(a.A) + r0 * a.ld + k;
  const double* rv = a.wr + ((int64_t)part * a.M + j) * a.mw;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t r = rb;
  for (; r + 4 <= re; r += 4) {
    s0 += elem(Ak + r * a.ld) * rv[r];
    s1 += elem(Ak + (r + 1) * a.ld) * rv[r + 1];
    s2 += elem(Ak + (r + 2) * a.ld) * rv[r + 2];
    s3 += elem(Ak + (r + 3) * a.ld) * rv[r + 3];
  }
  for (; r < re; ++r) s0 += elem(Ak + r * a.ld) * rv[r];
  a.gpart[((int64_t)part * a.Gp + g) * a.ld + k] = (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(256) void wxred_kernel(WoodArgs a) {
  const int part = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  const double* gp = a.gpart + (int64_t)part * a.Gp * a.ld + k;
  double s = 0.0;
  for (int g = 0; g < a.Gw; ++g) s += gp[(int64_t)g * a.ld];
  const int64_t o = (int64_t)part * a.n + k;
  a.x[o] = (a.rho_l / a.shift) * s + (a.rho_c / a.shift) * (a.z[k] - a.u[o]);
}

__global__ __launch_bounds__(256) void wgather_kernel(WoodArgs a) {
  const int bid = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  if (r >= a.mw) return;
  const int T = (a.mw + PT - 1) / PT;
  a.wh[(int64_t)bid * a.mw + r] = symv_gather(a.ypart + (int64_t)bid * T * T * PT, r, 0, 1, T);
}

__global__ __launch_bounds__(256) void wupdate_kernel(WoodArgs a) {
  const int part = blockIdx.y;
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  if (r >= m) return;
  const int T = (a.mw + PT - 1) / PT;
  const int64_t gr = r0 + r;
  double sum = 0.0;
  for (int j = 0; j < a.M; ++j) {
    const int64_t o = ((int64_t)part * a.M + j) * a.mw + r;
    if (a.mode == 0) {
      const double y = symv_gather(a.ypart + ((int64_t)part * a.M + j) * T * T * PT, r, 0, 1, T);
      const double p = a.wd[o] - a.shift * y + a.rho_c * a.wh[o];
      a.wr[o] = p;
      sum += p;
    } else {
      sum += a.wr[o];
    }
  }
  const double av = sum * a.inv_M;
  double nu = a.nu[gr], e;
  if (a.mode == 0) {
    const double om = prox_scalar(a.loss, av + nu, a.b[gr], a.M, a.rho_l,
                                  a.loss == BCA_LOSS_SQUARED ? 0.0 : a.omega[gr]);
    nu = nu + av - om;
    a.omega[gr] = om;
    a.nu[gr] = nu;
    e = om - av - nu;
  } else {
    e = a.omega[gr] - av - nu;
  }
  for (int j = 0; j < a.M; ++j) {
    const int64_t o = ((int64_t)part * a.M + j) * a.mw + r;
    if (a.mode == 0) {
      const double p = a.wr[o];
      a.wr[o] = a.wd[o] - p;
      a.wd[o] = p + e;
    } else {
      a.wd[o] = a.wr[o] + e;
    }
  }
}

template <typename T>
static hipError_t rowgram_t(const WoodArgs& a, hipStream_t s) {
  const int64_t T_ = (a.mw + 63) / 64;
  dim3 g((unsigned)(T_ * (T_ + 1) / 2), a.N * a.M);
  hipLaunchKernelGGL(rowgram_kernel<T>, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_rowgram(const WoodArgs& a, int dtype, hipStream_t s) {
  if (dtype == BCA_F64) return rowgram_t<double>(a, s);
  if (dtype == BCA_F32) return rowgram_t<float>(a, s);
  return rowgram_t<bf16_t>(a, s);
}

hipError_t launch_wgemv_n(const WoodArgs& a, int dtype, hipStream_t s) {
  dim3 g((unsigned)((a.mw + WR - 1) / WR), a.N);
  if (dtype == BCA_F64)
    hipLaunchKernelGGL(wgemv_n_kernel<double>, g, dim3(256), 0, s, a);
  else if (dtype == BCA_F32)
    hipLaunchKernelGGL(wgemv_n_kernel<float>, g, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(wgemv_n_kernel<bf16_t>, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wgemv_t(const WoodArgs& a, int dtype, hipStream_t s) {
  if (a.Gw < 1 || a.Gw > a.Gp) return hipErrorInvalidValue;
  dim3 g((unsigned)((a.n + 255) / 256), a.Gw, a.N);
  if (dtype == BCA_F64)
    hipLaunchKernelGGL(wgemv_t_kernel<double>, g, dim3(256), 0, s, a);
  else if (dtype == BCA_F32)
    hipLaunchKernelGGL(wgemv_t_kernel<float>, g, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(wgemv_t_kernel<bf16_t>, g, dim3(256), 0, s, a);
  dim3 g2((unsigned)((a.n + 255) / 256), a.N);
  hipLaunchKernelGGL(wxred_kernel, g2, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wgather(const WoodArgs& a, hipStream_t s) {
  dim3 g((unsigned)((a.mw + 255) / 256), a.N * a.M);
  hipLaunchKernelGGL(wgather_kernel, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_wupdate(const WoodArgs& a, hipStream_t s) {
  dim3 g((unsigned)((a.mw + 255) / 256), a.N);
  hipLaunchKernelGGL(wupdate_kernel, g, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace bca
