// x_ij-step of Sec. 3.1 (the M parallel regularised least-squares problems).
//
// The paper's update is x_ij <- K_ij^-1 (rho_l A_ij^T (p_ij + e) + rho_c (z_j - u_ij))
// with p_ij = A_ij x_ij and K_ij = rho_l G_ij + shift I, G_ij = A_ij^T A_ij,
// shift = 1/(N gamma) + rho_c.  Since A_ij^T p_ij = G_ij x_ij and
// K_ij^-1 rho_l G_ij = I - shift K_ij^-1, the same update reads
//     x_ij <- x_ij + K_ij^-1 (rho_l A_ij^T e + rho_c (z_j - u_ij) - shift x_ij),
// which needs only the streamed A_i^T e (no second pass over A) and whose fixed
// point does not depend on rounding in G_ij.  K_ij^-1 = W_ij^T W_ij with the
// cached inverse Cholesky factor W_ij = L_ij^-1, so the two triangular solves
// are two triangular matrix-vector products:
//   reduce_rhs_kernel  rhs = rho_l sum_w gpart[w] + rho_c (z - u) - shift x  (FP64,
//                      fixed summation order over the streaming workgroups)
//   trmv_kernel<0>     y = W rhs            (packed rows of W)
//   trmv_kernel<1>     x += W^T y, and the streaming copy of x
#include "bca_internal.h"

namespace bca {

__global__ __launch_bounds__(256) void reduce_rhs_kernel(SolveArgs a) {
  // one thread per element (k, c) of the n x C block vector, flat index k C + c
  const int part = blockIdx.y;
  const int64_t nc = (int64_t)a.n * a.C;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= nc) return;
  const int64_t stride = a.ld * a.C;
  const double* g = a.gpart + (int64_t)part * a.Gp * stride + k;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int w = 0;
  for (; w + 4 <= a.Gp; w += 4) {
    s0 += g[(int64_t)w * stride];
    s1 += g[(int64_t)(w + 1) * stride];
    s2 += g[(int64_t)(w + 2) * stride];
    s3 += g[(int64_t)(w + 3) * stride];
  }
  for (; w < a.Gp; ++w) s0 += g[(int64_t)w * stride];
  const double ate = (s0 + s1) + (s2 + s3);
  const int64_t o = (int64_t)part * nc + k;
  a.rhs[o] = a.rho_l * ate + a.rho_c * (a.z[k] - a.u[o]) - a.shift * a.x[o];
}

// One wavefront per pair of rows (q, nj - 1 - q) of a triangular block, so every
// wave reads about nj + 1 factor entries; each factor entry is applied to all C
// right-hand sides (the block vectors are n x C, feature-major).
//   TRANS = 0: row r of W, entries W[r, 0..r] at wr + r (r + 1) / 2, times in[0..r].
//   TRANS = 1: row c of W^T, entries W[c..nj-1, c] at wc + c nj - c (c - 1) / 2,
//              times in[c..nj-1]; the result is added to x.
template <int TRANS, int CC>
__global__ __launch_bounds__(256) void trmv_kernel(SolveArgs a, const double* in, double* out) {
  const int bid = blockIdx.y;
  const int part = bid / a.M, blk = bid - part * a.M;
  const int c0 = a.col_off[blk];
  const int nj = a.col_off[blk + 1] - c0;
  const int pairs = (nj + 1) / 2;
  const int lane = threadIdx.x & 63;
  const int pr = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (pr >= pairs) return;
  const int C = CC == 1 ? 1 : a.C;
  const double* F = (TRANS ? a.wc : a.wr) + a.fac_off[bid];
  const double* v = in + ((int64_t)part * a.n + c0) * C;
  for (int h = 0; h < 2; ++h) {
    const int r = h == 0 ? pr : nj - 1 - pr;
    if (h == 1 && r == pr) break;
    int64_t off;
    int st, len;
    if (!TRANS) {
      off = (int64_t)r * (r + 1) / 2;
      st = 0;
      len = r + 1;
    } else {
      off = (int64_t)r * nj - (int64_t)r * (r - 1) / 2;
      st = r;
      len = nj - r;
    }
    const double* f = F + off;
    double tot[CC];
    if (CC == 1) {
      const double* vv = v + st;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int e = lane;
      for (; e + 192 < len; e += 256) {
        s0 += f[e] * vv[e];
        s1 += f[e + 64] * vv[e + 64];
        s2 += f[e + 128] * vv[e + 128];
        s3 += f[e + 192] * vv[e + 192];
      }
      for (; e < len; e += 64) s0 += f[e] * vv[e];
      tot[0] = wave_sum((s0 + s1) + (s2 + s3));
    } else {
      double sc[CC];
#pragma unroll
      for (int c = 0; c < CC; ++c) sc[c] = 0.0;
      for (int e = lane; e < len; e += 64) {
        const double fe = f[e];
        const double* vv = v + (int64_t)(st + e) * C;
#pragma unroll
        for (int c = 0; c < CC; ++c)
          if (c < C) sc[c] += fe * vv[c];
      }
#pragma unroll
      for (int c = 0; c < CC; ++c) tot[c] = wave_sum(sc[c]);
    }
    if (lane == 0) {
      for (int c = 0; c < C; ++c) {
        const int64_t o = ((int64_t)part * a.n + c0 + r) * C + c;
        if (!TRANS) {
          out[o] = tot[c];
        } else {
          const double xn = a.x[o] + tot[c];
          a.xw[o] = xn;
          const int64_t so = (int64_t)part * a.ld * C + (int64_t)(c0 + r) * C + c;
          if (a.xs_f64)
            reinterpret_cast<double*>(a.xs)[so] = xn;
          else
            reinterpret_cast<float*>(a.xs)[so] = (float)xn;
        }
      }
    }
  }
}

template <int CC>
static void trmv_pair(const SolveArgs& a, hipStream_t s) {
  const int pairs = (a.nj_max + 1) / 2;
  dim3 g2((pairs + 3) / 4, a.N * a.M);
  hipLaunchKernelGGL((trmv_kernel<0, CC>), g2, dim3(256), 0, s, a, (const double*)a.rhs, a.tmp);
  hipLaunchKernelGGL((trmv_kernel<1, CC>), g2, dim3(256), 0, s, a, (const double*)a.tmp, (double*)nullptr);
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  if (a.C < 1 || a.C > 16) return hipErrorInvalidValue;
  dim3 g1((unsigned)(((int64_t)a.n * a.C + 255) / 256), a.N);
  hipLaunchKernelGGL(reduce_rhs_kernel, g1, dim3(256), 0, s, a);
  if (a.C == 1) trmv_pair<1>(a, s);
  else if (a.C <= 4) trmv_pair<4>(a, s);
  else if (a.C <= 10) trmv_pair<10>(a, s);
  else trmv_pair<16>(a, s);
  return hipGetLastError();
}

__global__ void make_xs_kernel(const double* x, void* xs, int xs_f64, int n, int C, int64_t ld) {
  const int part = blockIdx.y;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= ld * C) return;
  const double v = (k < (int64_t)n * C) ? x[(int64_t)part * n * C + k] : 0.0;
  if (xs_f64)
    reinterpret_cast<double*>(xs)[(int64_t)part * ld * C + k] = v;
  else
    reinterpret_cast<float*>(xs)[(int64_t)part * ld * C + k] = (float)v;
}

hipError_t launch_make_xs(const double* x, void* xs, int xs_f64, int N, int n, int C, int64_t ld,
                          hipStream_t s) {
  dim3 g((unsigned)((ld * C + 255) / 256), N);
  hipLaunchKernelGGL(make_xs_kernel, g, dim3(256), 0, s, x, xs, xs_f64, n, C, ld);
  return hipGetLastError();
}

}  // namespace bca
