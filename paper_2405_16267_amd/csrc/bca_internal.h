// Internal declarations of the Bi-cADMM HIP library: storage traits, kernel
// argument blocks and the host-side launchers each kernel file provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "bca.h"

namespace bca {

// BF16 storage tag: the upper 16 bits of an IEEE binary32.
struct bf16_t {
  uint16_t bits;
};

// Per storage type: 16-byte vector used to stream A, elements per vector,
// arithmetic type of the products (and of the streaming copy of x).
template <typename T>
struct Traits;
template <>
struct Traits<double> {
  using vec_t = double2;
  using acc_t = double;
  static constexpr int VEC = 2;
};
template <>
struct Traits<float> {
  using vec_t = float4;
  using acc_t = float;
  static constexpr int VEC = 4;
};
template <>
struct Traits<bf16_t> {
  using vec_t = uint4;
  using acc_t = float;
  static constexpr int VEC = 8;
};

__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Element e of a 16-byte vector, as the arithmetic type.
__device__ __forceinline__ double vget(const double2& v, int e) { return e == 0 ? v.x : v.y; }
__device__ __forceinline__ float vget(const float4& v, int e) {
  return e == 0 ? v.x : (e == 1 ? v.y : (e == 2 ? v.z : v.w));
}
__device__ __forceinline__ float vget(const uint4& v, int e) {
  uint32_t w = (e >> 1) == 0 ? v.x : ((e >> 1) == 1 ? v.y : ((e >> 1) == 2 ? v.z : v.w));
  return (e & 1) ? bf16_hi(w) : bf16_lo(w);
}

template <typename V>
__device__ __forceinline__ V vzero();
template <>
__device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }
template <>
__device__ __forceinline__ float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <>
__device__ __forceinline__ uint4 vzero<uint4>() { return make_uint4(0u, 0u, 0u, 0u); }

// Streaming 16-byte load that bypasses cache retention (A is read once per pass
// and never reused within it).
template <typename V>
__device__ __forceinline__ V load_stream(const V* p) {
  static_assert(sizeof(V) == 16, "16-byte vectors only");
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 t = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  V v;
  __builtin_memcpy(&v, &t, 16);
  return v;
}

// Sum over the 64 lanes of a wavefront (every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
// Sum over the 64 lanes with DPP lane moves inside each row of 16 lanes (xor 1,
// xor 2, half mirror, mirror: every lane of a row ends with the row's sum) and
// the four row sums read out and added in a fixed order; the same total in
// every lane, with far less latency than four-byte permutes through LDS.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// Sum over each row of 16 lanes (every lane of the row gets its row's sum).
__device__ __forceinline__ double row16_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  auto lane_val = [&](int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
  };
  return (lane_val(0) + lane_val(16)) + (lane_val(32) + lane_val(48));
}
__device__ __forceinline__ int wave_sum_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ------------------------------------------------------------------ kernels
// One pass over A per inner iteration (Algorithm 2): block predictions,
// sample-space average, omega-bar prox, nu update, e = omega - a - nu, and the
// per-workgroup partial sums of A^T e for the next x_ij-step.
struct StreamArgs {
  const void* A;           // all partitions, row-major, m_total x ld
  int64_t ld;              // row stride (elements)
  const int64_t* row_off;  // N + 1 row offsets (device)
  const double* b;         // m_total targets / labels
  const int32_t* y;        // m_total class ids (softmax)
  double* omega;           // m_total x C
  double* nu;              // m_total x C
  const void* xs;          // N x ld x C streaming copy of x (FP64 or FP32)
  double* gpart;           // N x Gp x ld x C partial sums of A^T e
  double* rowbuf;          // m_total x C (C > 1): sample-space averages, then e
  int64_t m_total;
  int N, Gp, nvec, n, M, C, loss;
  int Gd;                  // C > 1, FP32 / BF16 storage: workgroups per partition of the
                           // sample-space average kernel (16-row tiles, no partial sums)
  double inv_M, rho_l;
  int mode;                // 0: inner iteration; 1: prime (e from stored state, no prox);
                           // 2, 3: gradient and Hessian-vector passes of the logistic
                           // exact x-update (Newton-CG, newton.hip)
  const int* part_done;    // modes 2, 3 (or null): N x 2 flags, Newton ended / CG ended;
                           // a partition with either set (mode 3) or the first (mode 2) is skipped
};

// Objective: per-workgroup partial loss sums of l(A_i xhat; b_i).
struct ObjArgs {
  const void* A;
  int64_t ld;
  const int64_t* row_off;
  const double* b;
  const int32_t* y;
  const void* xs;          // x_hat streaming copy, ld x C (shared by all partitions)
  double* partial;         // N x Gp
  int N, Gp, nvec, n, C, loss;
};

struct Problem;  // host-side problem (bca_api.hip)

// Later work of the problem goes to stream s (the work queued on its current
// stream is waited for first); used by the serving form, which finalizes admitted
// requests on a stream of their own.
int set_problem_stream(bca_problem P, hipStream_t s);

// Launchers (host side).  Each returns hipSuccess or the launch error.
hipError_t launch_stream(const StreamArgs& a, int dtype, hipStream_t s);
// Resident workgroups per CU of the multi-class streaming kernels (C > 1).
int mc_occupancy_workgroups(int dtype, int n, int C);
// C > 1 with FP32 / BF16 storage: the streaming pass runs on MFMA (stream_mc.hip);
// its A^T E kernel covers 128 features per workgroup.
inline bool mc_uses_mfma(int dtype) { return dtype != BCA_F64; }
constexpr int kMcStrip = 128;
hipError_t launch_objective(const ObjArgs& a, int dtype, hipStream_t s);
// C > 1 (softmax) forms of the two passes (stream_mc.hip)
bool mc_supported(int n, int C);
hipError_t launch_stream_mc(const StreamArgs& a, int dtype, hipStream_t s);
hipError_t launch_objective_mc(const ObjArgs& a, int dtype, hipStream_t s);
int stream_occupancy_workgroups(int dtype, int nvec, int C);   // resident workgroups per CU
// Widest row of the one-class streaming and objective passes, in 16-byte chunks:
// 1,024 threads x 8 chunks (n <= 16,384 FP64, 32,768 FP32, 65,536 BF16).
constexpr int kStreamMaxVec = 1024 * 8;

struct GramArgs {
  const void* A;
  int64_t ld;
  const int64_t* row_off;  // N + 1
  const int32_t* col_off;  // M + 1
  const int64_t* kmat_off; // N*M offsets (doubles) of each K_ij in kbuf
  double* kbuf;            // K_ij dense n_j x n_j row-major (lower part written)
  int N, M, tiles_max;     // tiles_max = ceil(max n_j / 64)
  double rho_l, shift;     // K = rho_l G + shift I
};
hipError_t launch_gram(const GramArgs& a, int dtype, hipStream_t s);
// Zero bytes allocated past the last row of A (reads of whole 16-byte pieces there).
constexpr size_t kATailBytes = 256;

// Tiled inverse P_ij = K_ij^-1 (FP64), the operator of the x_ij-step.  Block
// (i, j) holds the 64 x 64 tiles (I, J), I >= J, of the lower block triangle of
// P_ij (T = ceil(n_j / 64) tiles per side), tile t = I (I + 1) / 2 + J at
// kinv + fac_off[i M + j] + t * 4096; diagonal tiles are stored in full and
// entries outside n_j x n_j are zero.  Inside a tile, element (row, col) sits at
// ptile_pos(row, col): lane l of a wavefront reads rows 16 q + 2 (l / 8) + {0, 1}
// and columns 8 (l % 8) .. 8 (l % 8) + 7 of row chunk q with 8 coalesced 16-byte
// loads (vector k = 4 (row % 2) + (col % 8) / 2 of the chunk).
constexpr int PT = 64;
constexpr int PT_ELEMS = PT * PT;
__host__ __device__ __forceinline__ int ptile_pos(int row, int col) {
  const int q = row >> 4, l = 8 * ((row & 15) >> 1) + (col >> 3);
  const int k = 4 * (row & 1) + ((col & 7) >> 1);
  return ((q * 8 + k) * 64 + l) * 2 + (col & 1);
}
__host__ __device__ __forceinline__ int64_t ptile_count(int nj) {
  const int64_t T = (nj + PT - 1) / PT;
  return T * (T + 1) / 2;
}
// Lower-triangular tile index t -> (ti, tj), ti >= tj.
__device__ __forceinline__ void tri_tile(int t, int* ti, int* tj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  *ti = i;
  *tj = t - i * (i + 1) / 2;
}

struct FactorArgs {
  double* kbuf;            // in: K_ij (lower); out: L_ij (lower)
  double* wbuf;            // out: W_ij = L_ij^-1 dense (lower, upper part zero)
  const int64_t* kmat_off; // N*M
  const int32_t* col_off;  // M + 1
  double* kinv;            // out: tiled P_ij = W_ij^T W_ij
  const int64_t* fac_off;  // N*M offsets (doubles) into kinv
  int* status;             // set nonzero if a pivot is not positive
  int N, M, nj_max;
};
hipError_t launch_cholesky(const FactorArgs& a, hipStream_t s);
hipError_t launch_inverse(const FactorArgs& a, hipStream_t s);
hipError_t launch_kinv(const FactorArgs& a, hipStream_t s);

struct SolveArgs {
  const double* gpart;     // N x Gp x ld x C
  int64_t ld;
  int Gp;
  const double* x;         // N x n x C
  double* xw;              // x updated in place (same as x)
  void* xs;                // streaming copy N x ld x C (FP32 or FP64)
  int xs_f64;
  const double* u;         // N x n x C
  const double* z;         // n x C
  double* rhs;             // N x n x C
  double* ypart;           // N*M blocks x (tmax x tmax slots x 64 x C) partial products
  const double* kinv;      // tiled P_ij
  const int64_t* fac_off;  // N*M
  const int32_t* col_off;  // M + 1
  const double* atb;       // exact x-update: N x n, 2 A_i^T b_i
  int N, M, n, C, nj_max;
  double rho_l, rho_c, shift;
};
hipError_t launch_solve(const SolveArgs& a, hipStream_t s);
// Only the symmetric product y = P_ij rhs_ij, into the slots at ypart.
hipError_t launch_symv(const SolveArgs& a, hipStream_t s);
// rhs = rho_l sum_w gpart[w] + rho_c (z - u) - shift x only.
hipError_t launch_reduce_rhs(const SolveArgs& a, hipStream_t s);
// Exact x-update (squared loss, one block per partition): x = P (atb + rho_c (z - u)).
hipError_t launch_solve_exact(const SolveArgs& a, hipStream_t s);

// Exact x-update of the logistic loss (newton.hip): Newton's method on every
// partition's whole x-subproblem, conjugate gradients for the Newton direction.
constexpr int NT_LS = 17;     // line-search trial steps 2^-l (l < 16) and 0
constexpr int NT_SCAL = 8;    // per-partition scalars
enum { NT_RZ = 0, NT_RZ0 = 1, NT_ALPHA = 2, NT_RZF = 3, NT_ETA2 = 4 };
struct NewtonArgs {
  int N, n, tmax;
  int64_t ld;
  const int64_t* row_off;  // N + 1
  const double* b;         // labels
  double* x;               // N x n
  const double* z;         // n
  const double* u;         // N x n
  double *r, *p, *hp, *d, *g;      // N x n: CG residual, direction, H p, Newton step, gradient
  double *rowq, *rowp, *rowd;      // m_total: a_k^T x, a_k^T p, a_k^T d
  void* xs;                // streaming copy (of p during CG)
  int xs_f64;
  const double* ypart;     // slots of the symmetric product with P_i
  double* sc;              // N x NT_SCAL
  double* lsp;             // N x line-search workgroups x NT_LS
  int* done;               // N x 2: Newton ended, CG ended
  double rho_c, inv2Ng, eta2, step_tol;
};
hipError_t launch_nt_reset(const NewtonArgs& a, hipStream_t s);
hipError_t launch_nt_start(const NewtonArgs& a, hipStream_t s);
hipError_t launch_nt_cg_step(const NewtonArgs& a, int64_t max_rows, hipStream_t s);
hipError_t launch_nt_beta(const NewtonArgs& a, hipStream_t s);
hipError_t launch_nt_update(const NewtonArgs& a, int ls_groups, hipStream_t s);

struct GlobalArgs {
  double* x;               // N x n x C
  double* u;               // N x n x C
  double* z;               // n x C
  double* s;               // n
  double* scal;            // [0] t, [1] v, [2] pr, [3] dr, [4] br, [5] iter (as double),
                           // [6] z^T s - t (split form), [7] last root theta of the (z,t) step
  double* hist;            // hist_cap x 3
  int32_t* support;        // kappa
  double* work;            // scratch: (2 C + 5) n doubles
  int* status;             // nonzero on NaN/Inf
  int N, n, C, kappa, hist_cap;
  double rho_c, rho_b;
  // split form (one problem): per-workgroup partial sums of the consensus pass
  // (2 G) and of the u-update / residual pass ((N + 1) G2); 0 in the batched form
  double* gp;
  int split, G, G2;
};
// Workgroups of the consensus pass and of the u-update pass of the split form.
inline int global_groups(int n) { return (n + 255) / 256; }
inline int global_groups2(int n, int C) { return (int)(((int64_t)n * C + 255) / 256); }
hipError_t launch_global(const GlobalArgs& a, hipStream_t s);

hipError_t launch_topk(const void* z, int f64, int64_t n, int kappa, int32_t* idx, double* work,
                       hipStream_t s);
// T_kappa of z (rows by Euclidean norm when C > 1); work holds n doubles.
hipError_t launch_support(const double* z, int n, int C, int kappa, int32_t* idx, double* work,
                          hipStream_t s);

// ------------------------------------------------------------------ sample-space x_ij-step
// Woodbury form of the x_ij-step for blocks with fewer rows than columns
// (m_i < n_j): with S_ij = shift I + rho_l A_ij A_ij^T (m_i x m_i), the update
// x+ = K_ij^-1 (rho_l A_ij^T d_ij + rho_c w_j), w_j = z_j - u_ij, maps the block
// prediction p_ij = A_ij x_ij to
//     p+ = d - shift S^-1 d + rho_c S^-1 A_ij w_j,
// and after the last inner iteration x+ = (rho_l / shift) A_ij^T (d - p+) +
// (rho_c / shift) w_j.  Sample-space vectors are N x M x mw doubles (block (i, j)
// at (i M + j) mw, rows past m_i zero), mw = max_i m_i.
struct WoodArgs {
  const void* A;
  int64_t ld;
  const int64_t* row_off;  // N + 1
  const int32_t* col_off;  // M + 1 (feature blocks)
  const double* b;
  double* omega;
  double* nu;
  double* x;               // N x n
  const double* u;         // N x n
  const double* z;         // n
  double* wt;              // A_ij w_j
  double* wh;              // S^-1 A_ij w_j
  double* wd;              // d_ij = p_ij + e
  double* wr;              // A_ij x_ij, then d_ij - p+_ij of the last inner iteration
  const double* ypart;     // slots of the sample-space symmetric products
  double* gpart;           // N x Gp x ld partial sums of A^T r
  double* kbuf;            // setup: dense S_ij, mw x mw each, at kmat_off
  const int64_t* kmat_off; // N*M
  int N, M, n, mw, Gp, Gw, loss, mode;
  double rho_l, rho_c, shift, inv_M;
};
// S_ij = rho_l A_ij A_ij^T + shift I (lower part, FP64 sums), padded rows: shift I.
hipError_t launch_rowgram(const WoodArgs& a, int dtype, hipStream_t s);
// wt = A_ij (z_j - u_ij) and wr = A_ij x_ij, one pass over A.
hipError_t launch_wgemv_n(const WoodArgs& a, int dtype, hipStream_t s);
// x = (rho_l / shift) A_ij^T wr + (rho_c / shift)(z - u), one pass over A.
hipError_t launch_wgemv_t(const WoodArgs& a, int dtype, hipStream_t s);
// wh = the gathered symmetric product (after symv of wt).
hipError_t launch_wgather(const WoodArgs& a, hipStream_t s);
// mode 0: one inner iteration from the gathered S^-1 d; mode 1: d = wr + e, e
// from the stored omega-bar and nu.
hipError_t launch_wupdate(const WoodArgs& a, hipStream_t s);

// ------------------------------------------------------------------ batched form
// Device-side descriptor of one problem of a batch (all pointers are that
// problem's own device buffers).
struct BatchInst {
  const void* A;
  int64_t ld;
  const int64_t* row_off;
  const double* b;
  double* omega;
  double* nu;
  void* xs;                // N x ld streaming copy of x (FP32 or FP64)
  double* x;
  double* u;
  double* z;
  double* s;
  double* scal;
  double* hist;
  int32_t* support;
  double* work;
  int* status;
  double* gpart;           // N x (items_per_part * 4) x ld wave partials of A^T e
  double* rhs;             // N x n right-hand sides of the x_ij-step
  double* ypart;           // N*M blocks x (tmax x tmax slots x 64) partial products
  const double* kinv;      // tiled P_ij = K_ij^-1
  const int64_t* fac_off;
  const int32_t* col_off;
  int N, M, n, kappa, loss, dtype, nvec, hist_cap, inner_iters, tmax;
  int rows_per_item, items_per_part, shape;   // stream tile shape (see batch.hip)
  int outer;               // outer iterations this launch runs for the problem
  double rho_l, rho_c, rho_b, shift, inv_M;
};

struct BatchItem {
  int inst, a, b, c, d;
};

struct BatchArgs {
  const BatchInst* inst;
  int count;
  const BatchItem* rhs_items;      // (inst, partition, block), largest first
  int n_rhs;
  const BatchItem* symv_items;     // (inst, partition, block, first tile, end tile)
  int n_symv;
  const BatchItem* xupd_items;     // (inst, partition, block)
  int n_xupd;
  const BatchItem* stream_items;   // (inst, partition, chunk), largest first
  int n_stream;
  const BatchItem* prime_items;    // stream items of problems whose partial sums are stale
  int n_prime;
  int outer, inner_max;
  unsigned int* counters;          // 8 work counters per phase (one per group of
                                   // workgroups), zeroed before the launch
  unsigned int* bar;               // grid barrier words (kBatchBarWords), zeroed before the launch
  unsigned long long* stamps;      // phase tracing (or null): workgroup 0 stores the 100 MHz
                                   // real-time counter at the start and after every grid barrier
  int stream_only;                 // 1: run only the prime phase (tile-shape timing)
};
constexpr int kBatchCounterGroups = 8;
constexpr int kBatchBarWords = 320;
hipError_t launch_batch(const BatchArgs& a, int grid, hipStream_t s);
hipError_t launch_zero_u32(unsigned int* p, int count, hipStream_t s);   // p[0..count) = 0
int batch_grid_size();            // co-resident workgroups of the batched kernel
int batch_shape_code(int nvec, int R);  // -1 if the (chunks per lane, rows per tile) pair is not built
int batch_max_nvec();

// Non-finite scan of a device buffer of `count` elements (dtype BCA_*), plus an
// optional label range check; sets *flag nonzero if anything is off.
hipError_t launch_check(const void* p, int dtype, int64_t count, int* flag, hipStream_t s);
hipError_t launch_check_labels(const int32_t* y, int64_t count, int C, int* flag, hipStream_t s);
hipError_t launch_check_signs(const double* b, int64_t count, int* flag, hipStream_t s);

// Streaming copy of x: xs[i][k*C + c] = x[i][k*C + c] for k < n, in FP64 or FP32.
hipError_t launch_make_xs(const double* x, void* xs, int xs_f64, int N, int n, int C, int64_t ld,
                          hipStream_t s);

}  // namespace bca
