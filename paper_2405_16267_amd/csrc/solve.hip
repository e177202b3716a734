// x_ij-step of Sec. 3.1 (the M parallel regularised least-squares problems).
//
// The paper's update is x_ij <- K_ij^-1 (rho_l A_ij^T (p_ij + e) + rho_c (z_j - u_ij))
// with p_ij = A_ij x_ij and K_ij = rho_l G_ij + shift I, G_ij = A_ij^T A_ij,
// shift = 1/(N gamma) + rho_c.  Since A_ij^T p_ij = G_ij x_ij and
// K_ij^-1 rho_l G_ij = I - shift K_ij^-1, the same update reads
//     x_ij <- x_ij + K_ij^-1 (rho_l A_ij^T e + rho_c (z_j - u_ij) - shift x_ij),
// which needs only the streamed A_i^T e (no second pass over A) and whose fixed
// point does not depend on rounding in G_ij.  K_ij^-1 = P_ij is cached (FP64,
// tiled lower block triangle), so the solve is one symmetric matrix-vector
// product that reads each stored entry once:
//   reduce_rhs_kernel  rhs = rho_l sum_w gpart[w] + rho_c (z - u) - shift x  (FP64,
//                      fixed summation order over the streaming workgroups)
//   symv_kernel        one wavefront per tile of P_ij: its row and column
//                      contributions to y = P_ij rhs, each into its own slot
//   xupd_kernel        x += y (slots summed in a fixed order), and the streaming
//                      copy of x
#include "bca_internal.h"
#include "symv_impl.h"

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

template <bool NTL>
__global__ __launch_bounds__(256) void symv_kernel(SolveArgs a) {
  const int bid = blockIdx.y;
  const int part = bid / a.M, blk = bid - part * a.M;
  const int c0 = a.col_off[blk];
  const int nj = a.col_off[blk + 1] - c0;
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (t >= ptile_count(nj)) return;
  int I, J;
  tri_tile(t, &I, &J);
  const int T = (nj + PT - 1) / PT, tmax = (a.nj_max + PT - 1) / PT;
  // with C right-hand sides, the grid's z index takes one of them, so that the C
  // products of a tile run in parallel (the tile is read C times, mostly from cache)
  const int cb = a.C > 1 ? (int)blockIdx.z : 0, ce = a.C > 1 ? cb + 1 : 1;
  symv_tile<NTL>(a.kinv + a.fac_off[bid] + (int64_t)t * PT_ELEMS, a.rhs + ((int64_t)part * a.n + c0) * a.C,
            nj, a.C, I, J, T, a.ypart + (int64_t)bid * tmax * tmax * PT * a.C, cb, ce);
}

// one thread per element (i, c) of the block's n_j x C vector; ASSIGN: x = y
// (the exact x-update) instead of x += y
template <bool ASSIGN>
__global__ __launch_bounds__(256) void xupd_kernel(SolveArgs a) {
  const int bid = blockIdx.y;
  const int part = bid / a.M, blk = bid - part * a.M;
  const int c0 = a.col_off[blk];
  const int nj = a.col_off[blk + 1] - c0;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= (int64_t)nj * a.C) return;
  const int i = (int)(k / a.C), c = (int)(k - (int64_t)i * a.C);
  const int T = (nj + PT - 1) / PT, tmax = (a.nj_max + PT - 1) / PT;
  const double y = symv_gather(a.ypart + (int64_t)bid * tmax * tmax * PT * a.C, i, c, a.C, T);
  const int64_t o = ((int64_t)part * a.n + c0 + i) * a.C + c;
  const double xn = ASSIGN ? y : a.x[o] + y;
  a.xw[o] = xn;
  const int64_t so = (int64_t)part * a.ld * a.C + (int64_t)(c0 + i) * a.C + c;
  if (a.xs_f64)
    reinterpret_cast<double*>(a.xs)[so] = xn;
  else
    reinterpret_cast<float*>(a.xs)[so] = (float)xn;
}

// The symmetric products of all blocks.  ntl: tiles beyond 1 GB in all are read
// with nontemporal loads.  Only the exact x-update asks for it: there nothing but
// these products touches HBM (6.4 GB of tiles at 16 x 10,000: 1.29 -> 1.19 ms),
// while with Algorithm 2's streaming pass between the products the nontemporal
// tiles made that pass slower (FP32 at 16 x 100,000 x 10,000: 9.25 -> 9.84 ms
// per launch, measured A/B in one job) and 220 MB of tiles read faster with
// ordinary loads.
static void symv_launch(const SolveArgs& a, hipStream_t s, bool ntl) {
  const int64_t tiles = ptile_count(a.nj_max);
  dim3 g2((unsigned)((tiles + 3) / 4), a.N * a.M, a.C > 1 ? a.C : 1);
  const double bytes = (double)tiles * PT_ELEMS * 8.0 * a.N * a.M;
  if (ntl && bytes > (double)(1ll << 30))
    hipLaunchKernelGGL(symv_kernel<true>, g2, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(symv_kernel<false>, g2, dim3(256), 0, s, a);
}

hipError_t launch_solve(const SolveArgs& a, hipStream_t s) {
  if (a.C < 1 || a.C > 16) return hipErrorInvalidValue;
  dim3 g1((unsigned)(((int64_t)a.n * a.C + 255) / 256), a.N);
  hipLaunchKernelGGL(reduce_rhs_kernel, g1, dim3(256), 0, s, a);
  symv_launch(a, s, false);
  dim3 g3((unsigned)(((int64_t)a.nj_max * a.C + 255) / 256), a.N * a.M);
  hipLaunchKernelGGL(xupd_kernel<false>, g3, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_symv(const SolveArgs& a, hipStream_t s) {
  if (a.C < 1 || a.C > 16) return hipErrorInvalidValue;
  symv_launch(a, s, false);
  return hipGetLastError();
}

hipError_t launch_reduce_rhs(const SolveArgs& a, hipStream_t s) {
  if (a.C < 1 || a.C > 16) return hipErrorInvalidValue;
  dim3 g1((unsigned)(((int64_t)a.n * a.C + 255) / 256), a.N);
  hipLaunchKernelGGL(reduce_rhs_kernel, g1, dim3(256), 0, s, a);
  return hipGetLastError();
}

// Exact x-update of the squared loss: rhs = 2 A_i^T b_i + rho_c (z - u_i) (the
// first term streamed once at setup), then x = P_i rhs with the same symmetric
// product as the inner loop's solve.
__global__ __launch_bounds__(256) void exact_rhs_kernel(SolveArgs a) {
  const int part = blockIdx.y;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  const int64_t o = (int64_t)part * a.n + k;
  a.rhs[o] = a.atb[o] + a.rho_c * (a.z[k] - a.u[o]);
}

hipError_t launch_solve_exact(const SolveArgs& a, hipStream_t s) {
  if (a.C != 1 || a.M != 1) return hipErrorInvalidValue;
  dim3 g1((unsigned)((a.n + 255) / 256), a.N);
  hipLaunchKernelGGL(exact_rhs_kernel, g1, dim3(256), 0, s, a);
  symv_launch(a, s, true);
  dim3 g3((unsigned)((a.nj_max + 255) / 256), a.N * a.M);
  hipLaunchKernelGGL(xupd_kernel<true>, g3, dim3(256), 0, s, a);
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
