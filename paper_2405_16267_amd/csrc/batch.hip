// Batched form: many independent Bi-cADMM problems of different sizes advanced
// together in ONE persistent (cooperative) launch.
//
// Every outer iteration of every problem is the same sequence of phases as the
// one-problem path (Algorithm 2's K_in inner iterations, then the global step
// of Algorithm 1), but here each phase is a list of independent work items
// spanning all problems:
//   SOLVE   item (problem, partition, block): the FP64 reduction of that block's
//           A^T e partial sums into the right-hand side, then the two triangular
//           products with the cached inverse factor (x_ij-step);
//   STREAM  item (problem, partition, row chunk): the fused A-streaming pass over
//           a chunk of rows, one wavefront per row tile (block predictions,
//           sample-space average, omega-bar prox, nu update, e, partial A^T e);
//   GLOBAL  item (problem): consensus average, exact (z,t) step, top-kappa
//           s-step, v and u updates, residuals.
// The workgroups of the persistent grid claim items of the current phase with an
// atomic counter (largest items first) and meet at a grid barrier between
// phases.  A problem's results depend only on its own items (fixed reduction
// orders inside each item, tile shape chosen per problem shape, never per
// batch), so a problem computes the same bits alone and inside any batch.
//
// Stream tile shapes: chunks per lane NC (a row of nvec 16-byte chunks is read by
// one wavefront, NC = ceil(nvec / 64) rounded up to 1, 2, 4 or 8) and rows per
// wave tile R in {1, 2, 4} with R NC <= 8, which bounds the kernel's register
// footprint; rows per item is a runtime parameter.
// The shape of each problem is picked by the autotuner in bca_api.hip.
#include <hip/hip_cooperative_groups.h>

#include "bca_internal.h"
#include "global_impl.h"
#include "prox_impl.h"

namespace bca {

namespace cg = cooperative_groups;

constexpr int BT = 256;
constexpr int BW = BT / 64;
constexpr int NJ_MAX = 1024;  // largest block width of a batched problem

constexpr int kShapes = 9;
static const int kShapeNC[kShapes] = {1, 1, 1, 2, 2, 2, 4, 4, 8};
static const int kShapeR[kShapes] = {1, 2, 4, 1, 2, 4, 1, 2, 1};

int batch_max_nvec() { return 64 * 8; }

int batch_shape_code(int nvec, int R) {
  int nc = 1;
  while (nc < 8 && 64 * nc < nvec) nc *= 2;
  if (64 * nc < nvec) return -1;
  for (int c = 0; c < kShapes; ++c)
    if (kShapeNC[c] == nc && kShapeR[c] == R) return c;
  return -1;
}

// LG: the widest FP32 shape (32 columns per lane) keeps its FP64 partial sums of
// A^T e in LDS (lg, 32 x BT doubles) instead of 64 registers, which would
// otherwise set the register budget of the whole persistent kernel.
template <typename T, int NC, int R>
__device__ void stream_item(const BatchInst& I, int part, int chunk, int mode, double* lg) {
  using TR = Traits<T>;
  using V = typename TR::vec_t;
  using acc = typename TR::acc_t;
  constexpr int VEC = TR::VEC;
  constexpr bool LG = NC * VEC == 32;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t r0 = I.row_off[part];
  const int64_t m = I.row_off[part + 1] - r0;
  const int64_t lo = (int64_t)chunk * I.rows_per_item;
  const int64_t hi = lo + I.rows_per_item < m ? lo + I.rows_per_item : m;
  const acc* xs = reinterpret_cast<const acc*>(I.xs) + (int64_t)part * I.ld;
  acc xr[NC][VEC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = lane + 64 * q;
#pragma unroll
    for (int e = 0; e < VEC; ++e) xr[q][e] = k < I.nvec ? xs[k * VEC + e] : acc(0);
  }
  double g[LG ? 1 : NC][LG ? 1 : VEC];
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      if constexpr (LG)
        lg[(q * VEC + e) * BT + threadIdx.x] = 0.0;
      else
        g[q][e] = 0.0;
    }
  const T* Ab = reinterpret_cast<const T*>(I.A) + r0 * I.ld;
  for (int64_t rt = lo + (int64_t)wv * R; rt < hi; rt += (int64_t)BW * R) {
    V v[R][NC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = rt + r;
      const V* rp = reinterpret_cast<const V*>(Ab + row * I.ld);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int k = lane + 64 * q;
        v[r][q] = (row < hi && k < I.nvec) ? rp[k] : vzero<V>();
      }
    }
    double mine = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc d = acc(0);
#pragma unroll
      for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) d += vget(v[r][q], e) * xr[q][e];
      const double s = wave_sum((double)d);
      if (lane == r) mine = s;
    }
    double e = 0.0;
    const int64_t row = rt + lane;
    if (lane < R && row < hi) {
      const int64_t gr = r0 + row;
      const double av = mine * I.inv_M;
      double nu = I.nu[gr];
      if (mode == 0) {
        const double om = prox_scalar(I.loss, av + nu, I.b[gr], I.M, I.rho_l,
                                      I.loss == BCA_LOSS_SQUARED ? 0.0 : I.omega[gr]);
        nu = nu + av - om;
        I.omega[gr] = om;
        I.nu[gr] = nu;
        e = om - av - nu;
      } else {
        e = I.omega[gr] - av - nu;
      }
    }
    acc er[R];
#pragma unroll
    for (int r = 0; r < R; ++r) er[r] = (acc)__shfl(e, r, 64);
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        acc t = acc(0);
#pragma unroll
        for (int r = 0; r < R; ++r) t += er[r] * vget(v[r][q], c);
        if constexpr (LG)
          lg[(q * VEC + c) * BT + threadIdx.x] += (double)t;
        else
          g[q][c] += (double)t;
      }
  }
  double* gp = I.gpart + (((int64_t)part * I.items_per_part + chunk) * BW + wv) * I.ld;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = lane + 64 * q;
    if (k < I.nvec) {
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        if constexpr (LG)
          gp[k * VEC + c] = lg[(q * VEC + c) * BT + threadIdx.x];
        else
          gp[k * VEC + c] = g[q][c];
      }
    }
  }
}

template <typename T>
__device__ void stream_item_dispatch(const BatchInst& I, int part, int chunk, int mode, double* lg) {
  switch (I.shape) {
    case 0: stream_item<T, 1, 1>(I, part, chunk, mode, lg); break;
    case 1: stream_item<T, 1, 2>(I, part, chunk, mode, lg); break;
    case 2: stream_item<T, 1, 4>(I, part, chunk, mode, lg); break;
    case 3: stream_item<T, 2, 1>(I, part, chunk, mode, lg); break;
    case 4: stream_item<T, 2, 2>(I, part, chunk, mode, lg); break;
    case 5: stream_item<T, 2, 4>(I, part, chunk, mode, lg); break;
    case 6: stream_item<T, 4, 1>(I, part, chunk, mode, lg); break;
    case 7: stream_item<T, 4, 2>(I, part, chunk, mode, lg); break;
    default: stream_item<T, 8, 1>(I, part, chunk, mode, lg); break;
  }
}

// x_ij-step of one block: rhs = rho_l sum_w gpart_w + rho_c (z - u) - shift x,
// y = W rhs, x += W^T y (W = L^-1, packed rows / packed columns).
__device__ __noinline__ void solve_item(const BatchInst& I, int part, int blk, double* rs, double* ys) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c0 = I.col_off[blk];
  const int nj = I.col_off[blk + 1] - c0;
  const int P = I.items_per_part * BW;
  const double* gb = I.gpart + (int64_t)part * P * I.ld;
  for (int c = tid; c < nj; c += BT) {
    const int k = c0 + c;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int w = 0;
    for (; w + 4 <= P; w += 4) {
      s0 += gb[(int64_t)w * I.ld + k];
      s1 += gb[(int64_t)(w + 1) * I.ld + k];
      s2 += gb[(int64_t)(w + 2) * I.ld + k];
      s3 += gb[(int64_t)(w + 3) * I.ld + k];
    }
    for (; w < P; ++w) s0 += gb[(int64_t)w * I.ld + k];
    const int64_t o = (int64_t)part * I.n + k;
    rs[c] = I.rho_l * ((s0 + s1) + (s2 + s3)) + I.rho_c * (I.z[k] - I.u[o]) - I.shift * I.x[o];
  }
  __syncthreads();
  const int64_t fo = I.fac_off[part * I.M + blk];
  const int pairs = (nj + 1) / 2;
  for (int tr = 0; tr < 2; ++tr) {
    const double* F = (tr == 0 ? I.wr : I.wc) + fo;
    const double* vin = tr == 0 ? rs : ys;
    for (int pr = wv; pr < pairs; pr += BW) {
      for (int h = 0; h < 2; ++h) {
        const int r = h == 0 ? pr : nj - 1 - pr;
        if (h == 1 && r == pr) break;
        int64_t off;
        int st, len;
        if (tr == 0) {
          off = (int64_t)r * (r + 1) / 2;
          st = 0;
          len = r + 1;
        } else {
          off = (int64_t)r * nj - (int64_t)r * (r - 1) / 2;
          st = r;
          len = nj - r;
        }
        const double* f = F + off;
        double s0 = 0.0, s1 = 0.0;
        int e = lane;
        for (; e + 64 < len; e += 128) {
          s0 += f[e] * vin[st + e];
          s1 += f[e + 64] * vin[st + e + 64];
        }
        if (e < len) s0 += f[e] * vin[st + e];
        const double tot = wave_sum(s0 + s1);
        if (lane == 0) {
          if (tr == 0) {
            ys[r] = tot;
          } else {
            const int64_t o = (int64_t)part * I.n + c0 + r;
            const double xn = I.x[o] + tot;
            I.x[o] = xn;
            const int64_t so = (int64_t)part * I.ld + c0 + r;
            if (I.dtype == BCA_F64)
              reinterpret_cast<double*>(I.xs)[so] = xn;
            else
              reinterpret_cast<float*>(I.xs)[so] = (float)xn;
          }
        }
      }
    }
    __syncthreads();
  }
}

// Out of line, with 7 multisection points per round, so that the global step's
// registers do not add to those of the streaming items.
__device__ __noinline__ void global_step_batched(const GlobalArgs& g, double* shd,
                                                 TopkShared<BT>& tks) {
  global_step<BT, 7>(g, shd, tks);
}

__device__ GlobalArgs global_args_of(const BatchInst& I) {
  GlobalArgs g;
  g.x = I.x;
  g.u = I.u;
  g.z = I.z;
  g.s = I.s;
  g.scal = I.scal;
  g.hist = I.hist;
  g.support = I.support;
  g.work = I.work;
  g.status = I.status;
  g.N = I.N;
  g.n = I.n;
  g.C = 1;
  g.kappa = I.kappa;
  g.hist_cap = I.hist_cap;
  g.rho_c = I.rho_c;
  g.rho_b = I.rho_b;
  return g;
}

// Two workgroups per CU: at most 256 registers per lane (VGPRs and AGPRs).
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(2))) void batch_kernel(BatchArgs ba) {
  // the solve phase's right-hand side and intermediate vector, and the widest
  // stream shape's partial sums, use the same LDS (phases never overlap)
  __shared__ double big[2 * NJ_MAX > 32 * BT ? 2 * NJ_MAX : 32 * BT];
  double* rs = big;
  double* ys = big + NJ_MAX;
  __shared__ double shd[BW * (PSECT + 2)];
  __shared__ TopkShared<BT> tks;
  __shared__ int item_sh;
  cg::grid_group grid = cg::this_grid();
  int phase = 0;

  // claims the next item of the current phase (all threads get the same index)
  auto claim = [&]() {
    if (threadIdx.x == 0) item_sh = (int)atomicAdd(&ba.counters[phase], 1u);
    __syncthreads();
    const int it = item_sh;
    __syncthreads();
    return it;
  };
  auto run_stream = [&](const BatchItem* items, int count, int mode, int k_inner, int o) {
    for (int it = claim(); it < count; it = claim()) {
      const BatchItem w = items[it];
      const BatchInst& I = ba.inst[w.inst];
      if (mode == 0 && (o >= I.outer || k_inner >= I.inner_iters)) continue;
      if (I.dtype == BCA_F64)
        stream_item_dispatch<double>(I, w.a, w.b, mode, big);
      else
        stream_item_dispatch<float>(I, w.a, w.b, mode, big);
    }
    ++phase;
  };

  if (ba.n_prime > 0) {
    run_stream(ba.prime_items, ba.n_prime, 1, 0, 0);
    if (ba.stream_only) return;
    grid.sync();
  }
  for (int o = 0; o < ba.outer; ++o) {
    for (int k = 0; k < ba.inner_max; ++k) {
      for (int it = claim(); it < ba.n_solve; it = claim()) {
        const BatchItem w = ba.solve_items[it];
        const BatchInst& I = ba.inst[w.inst];
        if (o >= I.outer || k >= I.inner_iters) continue;
        solve_item(I, w.a, w.b, rs, ys);
      }
      ++phase;
      grid.sync();
      run_stream(ba.stream_items, ba.n_stream, 0, k, o);
      grid.sync();
    }
    for (int it = claim(); it < ba.count; it = claim()) {
      const BatchInst& I = ba.inst[it];
      if (o >= I.outer) continue;
      global_step_batched(global_args_of(I), shd, tks);
      __syncthreads();
    }
    ++phase;
    grid.sync();
  }
}

int batch_grid_size() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
  cus = prop.multiProcessorCount;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, batch_kernel, BT, 0) != hipSuccess) return 0;
  return per * cus;
}

hipError_t launch_batch(const BatchArgs& a, int grid, hipStream_t s) {
  BatchArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(batch_kernel), dim3(grid), dim3(BT),
                                    params, 0, s);
}

}  // namespace bca
