// A-streaming pass of the node-level loop (Algorithm 2, Sec. 3.1), fused so that
// A is read from HBM once per inner iteration.
//
// For a partition i the x_ij-step needs rho_l A_ij^T (p_ij + e) with
// p_ij = A_ij x_ij and e = omega-bar - a - nu.  Because A_ij^T p_ij = G_ij x_ij
// with the cached Gram G_ij, only A_i^T e has to be streamed.  e is row-local
// (sample k only needs a_k, omega-bar_k, nu_k), so a workgroup that holds a tile
// of R full rows of A_i in registers can, in one pass:
//   1. form a_k = (1/M) sum_j A_ij,k x_ij        (block matvecs + average),
//   2. apply the per-sample omega-bar prox at c_k = a_k + nu_k,
//   3. update nu_k += a_k - omega-bar_k,
//   4. form e_k = omega-bar_k - a_k - nu_k,
//   5. accumulate e_k A_i,k into its partial sum of A_i^T e.
// The partial sums (one n-vector per workgroup) are reduced in a fixed order by
// the solve pass, so results are bitwise reproducible.
//
// Layout: thread t of the workgroup owns the 16-byte column chunks
// t, t + NT, t + 2 NT, ... of every row; a row of n elements is NC chunks per
// thread.  Products are formed in the arithmetic type of the storage (FP64 for
// FP64 A, FP32 for FP32 and BF16 A); every sum longer than one thread's chunk
// (across lanes, waves and row tiles) is carried in FP64.
#include <cstdlib>

#include "bca_internal.h"
#include "prox_impl.h"

namespace bca {

// XL: keep the thread's slice of x in LDS instead of registers (BF16 rows carry
// 8 columns per 16-byte chunk, so x and the FP64 sums would otherwise take
// 3 registers per streamed byte and cut the workgroups per CU).
template <typename T, int NT, int NC, int R, bool XL, bool PF>
__global__ __launch_bounds__(NT) void stream_kernel(StreamArgs a) {
  using TR = Traits<T>;
  using V = typename TR::vec_t;
  using acc = typename TR::acc_t;
  constexpr int VEC = TR::VEC;
  constexpr int NW = NT / 64;
  __shared__ double red[NW][R];
  __shared__ double e_sh[R];
  __shared__ acc xsh[XL ? NC * VEC : 1][XL ? NT : 1];

  const int part = blockIdx.x / a.Gp;
  const int wg = blockIdx.x - part * a.Gp;
  if (a.part_done && (a.part_done[2 * part] || (a.mode == 3 && a.part_done[2 * part + 1])))
    return;   // Newton passes: this partition's iteration (or its CG solve) has ended
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  const acc* xs = reinterpret_cast<const acc*>(a.xs) + (int64_t)part * a.ld;
  acc xr[XL ? 1 : NC][XL ? 1 : VEC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = tid + q * NT;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const acc xv = (k < a.nvec) ? xs[k * VEC + e] : acc(0);
      if constexpr (XL)
        xsh[q * VEC + e][tid] = xv;  // each thread reads back only its own slots
      else
        xr[q][e] = xv;
    }
  }
  double g[NC][VEC];
#pragma unroll
  for (int q = 0; q < NC; ++q)
#pragma unroll
    for (int e = 0; e < VEC; ++e) g[q][e] = 0.0;

  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld;
  const int64_t ntiles = (m + R - 1) / R;
  // Loads never branch: a row past the partition's end re-reads its last row and
  // a chunk past the row's end re-reads its last chunk.  Neither changes a
  // result: x is zero on the padded chunks (no dot contribution, no partial sum
  // written out) and e is zero on the padded rows (no A^T e contribution).
  int kc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) kc[q] = min(tid + q * NT, a.nvec - 1);
  auto load_tile = [&](V (&dst)[R][NC], int64_t t) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = min(t * R + r, m - 1);
      const V* rp = reinterpret_cast<const V*>(Ab + row * a.ld);
#pragma unroll
      for (int q = 0; q < NC; ++q) dst[r][q] = load_stream(rp + kc[q]);
    }
  };
  V v[R][NC];
  if constexpr (PF) {
    if (wg < ntiles) load_tile(v, wg);
  }
  for (int64_t tile = wg; tile < ntiles; tile += a.Gp) {
    const int64_t rt = tile * R;
    // PF: the next tile's loads are issued before this tile's arithmetic and
    // barriers, so HBM stays busy while the workgroup computes
    V vn[PF ? R : 1][PF ? NC : 1];
    if constexpr (PF) {
      if (tile + a.Gp < ntiles) load_tile(vn, tile + a.Gp);
    } else {
      load_tile(v, tile);
    }
    // 1. partial dots of each row with x
    double dd[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc d = acc(0);
#pragma unroll
      for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          if constexpr (XL)
            d += vget(v[r][q], e) * xsh[q * VEC + e][tid];
          else
            d += vget(v[r][q], e) * xr[q][e];
        }
      // BF16 (heavier per-chunk arithmetic): DPP lane moves and four read-outs
      // instead of six LDS permutes, +4 % on the streaming pass; for FP32 rows
      // the permutes measured slightly faster
      dd[r] = VEC == 8 ? wave_sum_dpp((double)d) : wave_sum((double)d);
    }
    if (lane == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) red[wv][r] = dd[r];
    }
    __syncthreads();
    // 2-4. average, prox, nu update, e (one thread per row of the tile)
    if (tid < R) {
      const int r = tid;
      const int64_t row = rt + r;
      double e = 0.0;
      if (row < m) {
        double sacc = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) sacc += red[w][r];
        const double av = sacc * a.inv_M;
        const int64_t gr = r0 + row;
        if (a.mode == 0) {
          double nu = a.nu[gr];
          const double om = prox_scalar(a.loss, av + nu, a.b[gr], a.M, a.rho_l,
                                        a.loss == BCA_LOSS_SQUARED ? 0.0 : a.omega[gr]);
          nu = nu + av - om;
          a.omega[gr] = om;
          a.nu[gr] = nu;
          e = om - av - nu;
        } else if (a.mode == 1) {
          e = a.omega[gr] - av - a.nu[gr];
        } else if (a.mode == 2) {
          // Newton gradient pass of the logistic exact x-update (one block, so av =
          // a_k^T x): loss derivative, Hessian weight to omega, q_k to nu
          const double b = a.b[gr];
          const double sg = 1.0 / (1.0 + exp(b * av));   // sigmoid(-b q)
          e = -b * sg;
          a.omega[gr] = sg * (1.0 - sg);
          a.nu[gr] = av;
        } else {
          // Hessian-vector pass (av = a_k^T p): weighted by the stored Hessian weight,
          // a_k^T p to nu
          e = a.omega[gr] * av;
          a.nu[gr] = av;
        }
      }
      e_sh[r] = e;
    }
    __syncthreads();
    // 5. accumulate e_k A_k (R products in the arithmetic type, then FP64)
    if constexpr (VEC == 8) {
      // BF16: widen the tile again here rather than keeping the 8 R NC widened
      // values of step 1 alive across the barriers (the empty asm hides the
      // raw words' values from the compiler, so the earlier widening is dead)
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < NC; ++q)
          asm volatile("" : "+v"(v[r][q].x), "+v"(v[r][q].y), "+v"(v[r][q].z), "+v"(v[r][q].w));
    }
    acc er[R];
#pragma unroll
    for (int r = 0; r < R; ++r) er[r] = (acc)e_sh[r];
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        acc t = acc(0);
#pragma unroll
        for (int r = 0; r < R; ++r) t += er[r] * vget(v[r][q], e);
        g[q][e] += (double)t;
      }
    if constexpr (PF) {
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < NC; ++q) v[r][q] = vn[r][q];
    }
  }
  double* gp = a.gpart + ((int64_t)part * a.Gp + wg) * a.ld;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = tid + q * NT;
    if (k < a.nvec) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) gp[k * VEC + e] = g[q][e];
    }
  }
}

// Objective pass: per-workgroup partial sums of l(A_k xhat; b_k).
template <typename T, int NT, int NC>
__global__ __launch_bounds__(NT) void objective_kernel(ObjArgs a) {
  using TR = Traits<T>;
  using V = typename TR::vec_t;
  using acc = typename TR::acc_t;
  constexpr int VEC = TR::VEC;
  constexpr int NW = NT / 64;
  __shared__ double red[NW];
  const int part = blockIdx.x / a.Gp;
  const int wg = blockIdx.x - part * a.Gp;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const acc* xs = reinterpret_cast<const acc*>(a.xs);
  acc xr[NC][VEC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = tid + q * NT;
#pragma unroll
    for (int e = 0; e < VEC; ++e) xr[q][e] = (k < a.nvec) ? xs[k * VEC + e] : acc(0);
  }
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld;
  double lsum = 0.0;  // meaningful on thread 0
  for (int64_t row = wg; row < m; row += a.Gp) {
    const V* rp = reinterpret_cast<const V*>(Ab + row * a.ld);
    acc d = acc(0);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int k = tid + q * NT;
      const V v = (k < a.nvec) ? rp[k] : vzero<V>();
#pragma unroll
      for (int e = 0; e < VEC; ++e) d += vget(v, e) * xr[q][e];
    }
    const double dw = wave_sum((double)d);
    if (lane == 0) red[wv] = dw;
    __syncthreads();
    if (tid == 0) {
      double qv = 0.0;
      for (int w = 0; w < NW; ++w) qv += red[w];
      const double b = a.b[r0 + row];
      if (a.loss == BCA_LOSS_SQUARED) {
        lsum += (qv - b) * (qv - b);
      } else if (a.loss == BCA_LOSS_HINGE) {
        lsum += fmax(0.0, 1.0 - b * qv);
      } else {
        const double t = -b * qv;  // log(1 + exp(t)), overflow-safe
        lsum += t > 0 ? t + log1p(exp(-t)) : log1p(exp(t));
      }
    }
    __syncthreads();
  }
  if (tid == 0) a.partial[blockIdx.x] = lsum;
}

// Launch shape of the streaming pass for rows of nvec 16-byte chunks: threads per
// workgroup, chunks per thread and rows per tile.  Up to `maxc` chunks per
// thread with 256 threads, then 512 threads (still up to 256 VGPRs per lane),
// then 1024, at most 8 chunks per thread (stream_max_chunks): FP32/FP64 rows
// maxc 6, BF16 rows (8 columns per chunk, so x and the FP64 sums take more
// registers per streamed byte, and the next tile is prefetched) maxc 4; 4 rows
// per tile.  BF16 rows of 1,025-1,344 chunks take 448 threads x 3 chunks.
struct StreamShape {
  int nt, nc, r;
};

template <typename T>
static StreamShape stream_shape(int nvec) {
  StreamShape sh;
  sh.r = 4;
  const int maxc = Traits<T>::VEC == 8 ? 4 : 6;
  if (nvec <= maxc * 256) {
    sh.nt = 256;
  } else if (nvec <= maxc * 512) {
    sh.nt = 512;
  } else {
    sh.nt = 1024;
  }
  int c = (nvec + sh.nt - 1) / sh.nt;
  if (c == 7) c = 8;
  sh.nc = c < 1 ? 1 : c;
  // BF16 rows of 1,025-1,344 chunks: 448 threads x 3 chunks leave fewer idle
  // chunk slots than 512 x 3 (10,000-column rows: 5.99 against 5.86 TB/s)
  if (Traits<T>::VEC == 8 && sh.nt == 512 && sh.nc == 3 && nvec <= 3 * 448) sh.nt = 448;
  return sh;
}

template <typename T>
constexpr bool use_pf() {
  return Traits<T>::VEC == 8;
}

template <typename T, int NT, int NC>
constexpr bool use_xl() {
  return Traits<T>::VEC == 8 && NC * Traits<T>::VEC * NT * 4 <= 128 * 1024;
}

// Calls F::template run<NT, NC, R>() for the shape (R = 4; sh.nc <= 8, which
// bca_create guarantees through stream_max_chunks).
template <typename T, typename F>
static auto with_shape(const StreamShape& sh, F f) {
#define BCA_NC(NT_, R_)                                  \
  switch (sh.nc) {                                       \
    case 1: return f.template run<NT_, 1, R_>();         \
    case 2: return f.template run<NT_, 2, R_>();         \
    case 3: return f.template run<NT_, 3, R_>();         \
    case 4: return f.template run<NT_, 4, R_>();         \
    case 5: return f.template run<NT_, 5, R_>();         \
    case 6: return f.template run<NT_, 6, R_>();         \
    default: return f.template run<NT_, 8, R_>();        \
  }
  if (sh.nt == 256) BCA_NC(256, 4)
  if constexpr (Traits<T>::VEC == 8) {
    if (sh.nt == 448) return f.template run<448, 3, 4>();
  }
  if (sh.nt == 512) BCA_NC(512, 4)
  BCA_NC(1024, 4)
#undef BCA_NC
}

template <typename T>
struct StreamLaunch {
  const StreamArgs& a;
  hipStream_t s;
  template <int NT, int NC, int R>
  hipError_t run() const {
    hipLaunchKernelGGL((stream_kernel<T, NT, NC, R, use_xl<T, NT, NC>(), use_pf<T>()>), dim3(a.N * a.Gp), dim3(NT), 0,
                       s, a);
    return hipGetLastError();
  }
};

template <typename T>
struct StreamOcc {
  template <int NT, int NC, int R>
  int run() const {
    int blocks = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &blocks, stream_kernel<T, NT, NC, R, use_xl<T, NT, NC>(), use_pf<T>()>, NT, 0);
    return (e != hipSuccess || blocks < 1) ? 1 : blocks;
  }
};

template <typename T>
static hipError_t stream_dispatch(const StreamArgs& a, hipStream_t s) {
  if (a.nvec < 1 || a.nvec > kStreamMaxVec) return hipErrorInvalidValue;
  return with_shape<T>(stream_shape<T>(a.nvec), StreamLaunch<T>{a, s});
}

hipError_t launch_stream(const StreamArgs& a, int dtype, hipStream_t s) {
  if (a.C != 1) return launch_stream_mc(a, dtype, s);
  switch (dtype) {
    case BCA_F64: return stream_dispatch<double>(a, s);
    case BCA_F32: return stream_dispatch<float>(a, s);
    default: return stream_dispatch<bf16_t>(a, s);
  }
}

template <typename T>
static int occ_one(int nvec) {
  return with_shape<T>(stream_shape<T>(nvec), StreamOcc<T>{});
}

int stream_occupancy_workgroups(int dtype, int nvec, int C) {
  (void)C;
  switch (dtype) {
    case BCA_F64: return occ_one<double>(nvec);
    case BCA_F32: return occ_one<float>(nvec);
    default: return occ_one<bf16_t>(nvec);
  }
}

template <typename T>
static hipError_t objective_dispatch(const ObjArgs& a, hipStream_t s) {
  if (a.nvec < 1 || a.nvec > kStreamMaxVec) return hipErrorInvalidValue;
  const StreamShape sh = stream_shape<T>(a.nvec);
  const int nt = sh.nt, nc = sh.nc;
  dim3 grid(a.N * a.Gp);
#define BCA_OBJ(NT_, NC_) hipLaunchKernelGGL((objective_kernel<T, NT_, NC_>), grid, dim3(NT_), 0, s, a)
  if (nt == 256) {
    switch (nc) {
      case 1: BCA_OBJ(256, 1); break;
      case 2: BCA_OBJ(256, 2); break;
      case 3: BCA_OBJ(256, 3); break;
      case 4: BCA_OBJ(256, 4); break;
      case 5: BCA_OBJ(256, 5); break;
      case 6: BCA_OBJ(256, 6); break;
      default: BCA_OBJ(256, 8); break;
    }
  } else if (nt == 512 || nt == 448) {  // 448: the BF16 shape of 1,025-1,344 chunks
    switch (nc) {
      case 1: BCA_OBJ(512, 1); break;
      case 2: BCA_OBJ(512, 2); break;
      case 3: BCA_OBJ(512, 3); break;
      case 4: BCA_OBJ(512, 4); break;
      case 5: BCA_OBJ(512, 5); break;
      case 6: BCA_OBJ(512, 6); break;
      default: BCA_OBJ(512, 8); break;
    }
  } else {
    switch (nc) {
      case 1: BCA_OBJ(1024, 1); break;
      case 2: BCA_OBJ(1024, 2); break;
      case 3: BCA_OBJ(1024, 3); break;
      case 4: BCA_OBJ(1024, 4); break;
      case 5: BCA_OBJ(1024, 5); break;
      case 6: BCA_OBJ(1024, 6); break;
      default: BCA_OBJ(1024, 8); break;
    }
  }
#undef BCA_OBJ
  return hipGetLastError();
}

hipError_t launch_objective(const ObjArgs& a, int dtype, hipStream_t s) {
  if (a.C != 1) return launch_objective_mc(a, dtype, s);
  switch (dtype) {
    case BCA_F64: return objective_dispatch<double>(a, s);
    case BCA_F32: return objective_dispatch<float>(a, s);
    default: return objective_dispatch<bf16_t>(a, s);
  }
}

}  // namespace bca
