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
#include "bca_internal.h"
#include "prox_impl.h"

namespace bca {

// LACC: keep the FP64 partial sums of A^T e in LDS instead of registers (for
// 8-element BF16 chunks, whose register footprint would otherwise halve occupancy).
template <typename T, int NT, int NC, int R, bool LACC>
__global__ __launch_bounds__(NT) void stream_kernel(StreamArgs a) {
  using TR = Traits<T>;
  using V = typename TR::vec_t;
  using acc = typename TR::acc_t;
  constexpr int VEC = TR::VEC;
  constexpr int NW = NT / 64;
  __shared__ double red[NW][R];
  __shared__ double e_sh[R];
  __shared__ double gsh[LACC ? NC * VEC : 1][LACC ? NT : 1];

  const int part = blockIdx.x / a.Gp;
  const int wg = blockIdx.x - part * a.Gp;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  const acc* xs = reinterpret_cast<const acc*>(a.xs) + (int64_t)part * a.ld;
  acc xr[NC][VEC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = tid + q * NT;
#pragma unroll
    for (int e = 0; e < VEC; ++e) xr[q][e] = (k < a.nvec) ? xs[k * VEC + e] : acc(0);
  }
  double g[LACC ? 1 : NC][LACC ? 1 : VEC];
  if constexpr (LACC) {
#pragma unroll
    for (int q = 0; q < NC * VEC; ++q) gsh[q][tid] = 0.0;
  } else {
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int e = 0; e < VEC; ++e) g[q][e] = 0.0;
  }

  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld;
  const int64_t ntiles = (m + R - 1) / R;
  for (int64_t tile = wg; tile < ntiles; tile += a.Gp) {
    const int64_t rt = tile * R;
    V v[R][NC];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = rt + r;
      const V* rp = reinterpret_cast<const V*>(Ab + row * a.ld);
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int k = tid + q * NT;
        v[r][q] = (row < m && k < a.nvec) ? rp[k] : vzero<V>();
      }
    }
    // 1. partial dots of each row with x
    double dd[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc d = acc(0);
#pragma unroll
      for (int q = 0; q < NC; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) d += vget(v[r][q], e) * xr[q][e];
      dd[r] = wave_sum((double)d);
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
        double nu = a.nu[gr];
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
      }
      e_sh[r] = e;
    }
    __syncthreads();
    // 5. accumulate e_k A_k (R products in the arithmetic type, then FP64)
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
        if constexpr (LACC)
          gsh[q * VEC + e][tid] += (double)t;
        else
          g[q][e] += (double)t;
      }
  }
  double* gp = a.gpart + ((int64_t)part * a.Gp + wg) * a.ld;
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = tid + q * NT;
    if (k < a.nvec) {
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        if constexpr (LACC)
          gp[k * VEC + e] = gsh[q * VEC + e][tid];
        else
          gp[k * VEC + e] = g[q][e];
      }
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
      } else {
        const double t = -b * qv;  // log(1 + exp(t)), overflow-safe
        lsum += t > 0 ? t + log1p(exp(-t)) : log1p(exp(t));
      }
    }
    __syncthreads();
  }
  if (tid == 0) a.partial[blockIdx.x] = lsum;
}

#define BCA_STREAM_NC_CASES(T, NT, RT)                                                           \
  switch (nc) {                                                                                   \
    case 1: hipLaunchKernelGGL((stream_kernel<T, NT, 1, RT, use_lacc<T, NT, 1>()>), grid, dim3(NT), 0, s, a); break;    \
    case 2: hipLaunchKernelGGL((stream_kernel<T, NT, 2, RT, use_lacc<T, NT, 2>()>), grid, dim3(NT), 0, s, a); break;    \
    case 3: hipLaunchKernelGGL((stream_kernel<T, NT, 3, RT, use_lacc<T, NT, 3>()>), grid, dim3(NT), 0, s, a); break;    \
    case 4: hipLaunchKernelGGL((stream_kernel<T, NT, 4, RT, use_lacc<T, NT, 4>()>), grid, dim3(NT), 0, s, a); break;    \
    case 5: hipLaunchKernelGGL((stream_kernel<T, NT, 5, RT, use_lacc<T, NT, 5>()>), grid, dim3(NT), 0, s, a); break;    \
    case 6: hipLaunchKernelGGL((stream_kernel<T, NT, 6, RT, use_lacc<T, NT, 6>()>), grid, dim3(NT), 0, s, a); break;    \
    default: hipLaunchKernelGGL((stream_kernel<T, NT, 8, RT, use_lacc<T, NT, 8>()>), grid, dim3(NT), 0, s, a); break;   \
  }

// Threads per workgroup and 16-byte chunks per thread for a row of nvec chunks:
// up to 6 chunks per thread with 256 threads, then 512 threads (still up to 256
// VGPRs per lane), then 1024.
static void stream_shape(int nvec, int* nt, int* nc) {
  if (nvec <= 6 * 256) {
    *nt = 256;
  } else if (nvec <= 6 * 512) {
    *nt = 512;
  } else {
    *nt = 1024;
  }
  int c = (nvec + *nt - 1) / *nt;
  if (c == 7) c = 8;
  *nc = c < 1 ? 1 : c;
}

// Rows per tile and where the FP64 partial sums live (LDS for BF16 when they fit
// in 96 KB, so that a CU still holds more than one workgroup).
template <typename T>
struct StreamRows {
  static constexpr int R = 4;
  static constexpr bool LACC = false;
};
template <>
struct StreamRows<bf16_t> {
  static constexpr int R = 2;
  static constexpr bool LACC = true;
};

template <typename T, int NT, int NC>
constexpr bool use_lacc() {
  return StreamRows<T>::LACC && NC * Traits<T>::VEC * NT * 8 <= 96 * 1024;
}

template <typename T>
static hipError_t stream_dispatch(const StreamArgs& a, hipStream_t s) {
  constexpr int RT = StreamRows<T>::R;
  int nt, nc;
  stream_shape(a.nvec, &nt, &nc);
  if (nc > 8) return hipErrorInvalidValue;
  dim3 grid(a.N * a.Gp);
  if (nt == 256) {
    BCA_STREAM_NC_CASES(T, 256, RT)
  } else if (nt == 512) {
    BCA_STREAM_NC_CASES(T, 512, RT)
  } else {
    BCA_STREAM_NC_CASES(T, 1024, RT)
  }
  return hipGetLastError();
}

hipError_t launch_stream(const StreamArgs& a, int dtype, hipStream_t s) {
  if (a.C != 1) return launch_stream_mc(a, dtype, s);
  switch (dtype) {
    case BCA_F64: return stream_dispatch<double>(a, s);
    case BCA_F32: return stream_dispatch<float>(a, s);
    default: return stream_dispatch<bf16_t>(a, s);
  }
}

template <typename T, int NT>
static int occ_nt(int nc) {
  constexpr int RT = StreamRows<T>::R;
  int blocks = 0;
  hipError_t e = hipSuccess;
#define BCA_OCC(NC_) \
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, stream_kernel<T, NT, NC_, RT, use_lacc<T, NT, NC_>()>, NT, 0)
  switch (nc) {
    case 1: BCA_OCC(1); break;
    case 2: BCA_OCC(2); break;
    case 3: BCA_OCC(3); break;
    case 4: BCA_OCC(4); break;
    case 5: BCA_OCC(5); break;
    case 6: BCA_OCC(6); break;
    default: BCA_OCC(8); break;
  }
#undef BCA_OCC
  if (e != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

template <typename T>
static int occ_one(int nvec) {
  int nt, nc;
  stream_shape(nvec, &nt, &nc);
  if (nt == 256) return occ_nt<T, 256>(nc);
  if (nt == 512) return occ_nt<T, 512>(nc);
  return occ_nt<T, 1024>(nc);
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
  int nt, nc;
  stream_shape(a.nvec, &nt, &nc);
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
  } else if (nt == 512) {
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
