// One-time setup of the x_ij-step of Sec. 3.1: the ridge problem of every
// feature block is K_ij x = rhs with
//     K_ij = rho_l A_ij^T A_ij + (1/(N gamma) + rho_c) I.
// Its Cholesky factor L_ij, the inverse factor W_ij = L_ij^-1 and from it the
// inverse P_ij = K_ij^-1 = W_ij^T W_ij are computed here once in FP64; the
// iterations then apply P_ij as one symmetric matrix-vector product per block,
// which reads each stored entry once (the two triangular solves with L_ij would
// be sequential, and two triangular products with W_ij read twice the bytes).
//
//   gram_kernel / gram128_kernel
//                    G_ij = A_ij^T A_ij on MFMA (FP64, FP32 or BF16 inputs,
//                    FP64/FP32 accumulation), lower tiles, epilogue writes K_ij
//                    in FP64.
//   chol_*_kernel    right-looking blocked Cholesky (32-wide panels) of all
//                    blocks at once, FP64.
//   inv_*_kernel     W_ij = L_ij^-1 right-looking by 64-row blocks, FP64.
//   kinv_kernel      P_ij = W_ij^T W_ij on FP64 MFMA, written as the tiled
//                    symmetric layout the solve reads (64 x 64 tiles of the
//                    lower block triangle, diagonal tiles in full).
#include "bca_internal.h"

namespace bca {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------------------------ Gram
// Linear work-group id remapped so that each of the 8 XCDs (work-groups are
// dispatched to them round-robin by linear id) takes one contiguous range of the
// grid's work: neighbouring tiles, which share operand panels, then run on the
// same XCD and meet in its L2.  A bijection on [0, total).
__device__ __forceinline__ int xcd_remap(int id, int total) {
  constexpr int X = 8;
  const int xcd = id % X, slot = id / X;
  const int q = total / X, r = total % X;
  return xcd < r ? xcd * (q + 1) + slot : r * (q + 1) + (xcd - r) * q + slot;
}

// MFMA shapes: 16x16 output per instruction, K_STEP contraction rows per
// instruction.  Operand layout (lane l): A-side element (i = l % 16,
// k = K_PER_LANE * (l / 16) + e), B-side element (k likewise, j = l % 16).
// Result element v of lane l is at column l % 16 and row out_row(l, v):
// 4 (l / 16) + v for the FP32-accumulating shapes, l / 16 + 4 v for FP64
// (both measured on gfx950).
template <typename T>
struct GramMfma;

template <>
struct GramMfma<float> {
  using lds_t = float;
  using acc_t = floatx4;
  static constexpr int KB = 16;       // rows per LDS chunk
  static constexpr int K_STEP = 4;    // contraction rows per MFMA
  static constexpr int K_PER_LANE = 1;
  static constexpr int PAD = 1;
  __device__ static lds_t load(const float* p) { return *p; }
  __device__ static void mma(acc_t& c, const lds_t* a, const lds_t* b) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b[0], c, 0, 0, 0);
  }
  __device__ static double out(const acc_t& c, int v) { return (double)c[v]; }
  __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

template <>
struct GramMfma<double> {
  using lds_t = double;
  using acc_t = doublex4;
  static constexpr int KB = 16;
  static constexpr int K_STEP = 4;
  static constexpr int K_PER_LANE = 1;
  static constexpr int PAD = 1;
  __device__ static lds_t load(const double* p) { return *p; }
  __device__ static void mma(acc_t& c, const lds_t* a, const lds_t* b) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
  }
  __device__ static double out(const acc_t& c, int v) { return c[v]; }
  __device__ static int out_row(int lane, int v) { return (lane >> 4) + 4 * v; }
};

template <>
struct GramMfma<bf16_t> {
  using lds_t = __bf16;
  using acc_t = floatx4;
  static constexpr int KB = 32;
  static constexpr int K_STEP = 32;
  static constexpr int K_PER_LANE = 8;
  static constexpr int PAD = 8;  // keeps 16-byte alignment of each LDS row
  __device__ static lds_t load(const bf16_t* p) { return __builtin_bit_cast(__bf16, p->bits); }
  __device__ static void mma(acc_t& c, const lds_t* a, const lds_t* b) {
    bf16x8 va = *reinterpret_cast<const bf16x8*>(a);
    bf16x8 vb = *reinterpret_cast<const bf16x8*>(b);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, c, 0, 0, 0);
  }
  __device__ static double out(const acc_t& c, int v) { return (double)c[v]; }
  __device__ static int out_row(int lane, int v) { return 4 * (lane >> 4) + v; }
};

// 64x64 output tile per workgroup of 256 threads; wave w computes the 32x32
// quadrant (w / 2, w % 2) as 2 x 2 MFMA tiles.  LDS holds the two 64-column
// panels of a KB-row chunk, transposed (column-major) so each lane's operand
// run along the contraction index is contiguous.
template <typename T>
__global__ __launch_bounds__(256) void gram_kernel(GramArgs a) {
  using MF = GramMfma<T>;
  using L = typename MF::lds_t;
  constexpr int KB = MF::KB;
  constexpr int LS = KB + MF::PAD;
  __shared__ __attribute__((aligned(16))) L sI[64 * LS];
  __shared__ __attribute__((aligned(16))) L sJ[64 * LS];

  const int bid = blockIdx.y;
  const int part = bid / a.M, blk = bid - part * a.M;
  const int c0 = a.col_off[blk];
  const int nj = a.col_off[blk + 1] - c0;
  const int T_ = (nj + 63) / 64;
  int ti, tj;
  tri_tile(blockIdx.x, &ti, &tj);
  if (ti >= T_) return;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld + c0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const bool diag = (ti == tj);

  typename MF::acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = 0;

  for (int64_t k0 = 0; k0 < m; k0 += KB) {
    // stage: sI[c][k] = A[k0 + k][ti*64 + c], sJ likewise for tj
    for (int idx = tid; idx < KB * 64; idx += 256) {
      const int k = idx >> 6, c = idx & 63;
      const int64_t row = k0 + k;
      const int ci = ti * 64 + c, cj = tj * 64 + c;
      L vi = L(0), vj = L(0);
      if (row < m) {
        if (ci < nj) vi = MF::load(Ab + row * a.ld + ci);
        if (!diag && cj < nj) vj = MF::load(Ab + row * a.ld + cj);
      }
      sI[c * LS + k] = vi;
      if (!diag) sJ[c * LS + k] = vj;
    }
    __syncthreads();
    const L* pJ = diag ? sI : sJ;
#pragma unroll
    for (int ks = 0; ks < KB; ks += MF::K_STEP) {
      const int kk = ks + MF::K_PER_LANE * (lane >> 4);
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const L* pa = sI + (wr * 32 + x * 16 + (lane & 15)) * LS + kk;
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const L* pb = pJ + (wc * 32 + y * 16 + (lane & 15)) * LS + kk;
          MF::mma(acc[x][y], pa, pb);
        }
      }
    }
    __syncthreads();
  }
  double* K = a.kbuf + a.kmat_off[bid];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 64 + wr * 32 + x * 16 + MF::out_row(lane, v);
        const int col = tj * 64 + wc * 32 + y * 16 + (lane & 15);
        if (row < nj && col < nj && row >= col) {
          double g = MF::out(acc[x][y], v);
          K[(int64_t)row * nj + col] = a.rho_l * g + (row == col ? a.shift : 0.0);
        }
      }
}

// FP32 / BF16 Gram with 128 x 128 output tiles (4 wavefronts of 64 x 64, each a
// 4 x 4 grid of 16 x 16 MFMA tiles) and double-buffered LDS: while the MFMAs run
// on one KB-row chunk, the next chunk is loaded from HBM into registers.  LDS
// holds the panels row-major, exactly as in HBM (16-byte stores, no transpose);
// since G = sum_k a_k a_k^T may take its rows in any order, the 8 contraction
// rows of lane group g = lane / 16 in a BF16 MFMA are rows g, g + 4, ..., g + 28
// of the 32-row step.  The four 16 x 16 subtiles of a wavefront's 64 columns are
// interleaved (subtile x holds columns 4 i + x), so a lane reads its four
// operands' columns at once: 8-byte reads of 4 columns per row (BF16), one
// 16-byte read (FP32).
template <typename T>
struct Gram2;
template <>
struct Gram2<float> {
  using lds_t = float;
  using vec_t = float4;
  using op_t = float;
  static constexpr int KB = 32;         // rows per chunk
  static constexpr int K_STEP = 4;      // contraction rows per MFMA
  static constexpr int EPV = 4;         // elements per 16-byte load
  // operands of the four interleaved subtiles (columns c4 + x, x = 0..3) for
  // lane group g of the K_STEP-row step at row ks: one 16-byte LDS read
  __device__ static void operands4(const float* p, int ks, int g, int c4, int ls, float (&op)[4]) {
    const float4 v = *reinterpret_cast<const float4*>(p + (ks + g) * ls + c4);
    op[0] = v.x;
    op[1] = v.y;
    op[2] = v.z;
    op[3] = v.w;
  }
  __device__ static void mma(floatx4& acc, float a, float b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
};
template <>
struct Gram2<bf16_t> {
  using lds_t = uint16_t;
  using vec_t = uint4;
  using op_t = bf16x8;
  static constexpr int KB = 64;
  static constexpr int K_STEP = 32;
  static constexpr int EPV = 8;
  // rows ks + g + 4 e (e = 0..7) of columns c4 .. c4 + 3: eight 8-byte LDS reads,
  // then byte permutes put column x of rows (2p, 2p + 1) in dword p of operand x
  __device__ static void operands4(const uint16_t* p, int ks, int g, int c4, int ls, bf16x8 (&op)[4]) {
    uint2 r[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) r[e] = *reinterpret_cast<const uint2*>(p + (ks + g + 4 * e) * ls + c4);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      uint32_t w[4];
      const uint32_t sel = (x & 1) ? 0x07060302u : 0x05040100u;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t lo = (x < 2) ? r[2 * q].x : r[2 * q].y;
        const uint32_t hi = (x < 2) ? r[2 * q + 1].x : r[2 * q + 1].y;
        w[q] = __builtin_amdgcn_perm(hi, lo, sel);
      }
      __builtin_memcpy(&op[x], w, sizeof(w));
    }
  }
  __device__ static void mma(floatx4& acc, const bf16x8& a, const bf16x8& b) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
};

template <typename T>
__global__ __launch_bounds__(256) void gram128_kernel(GramArgs a) {
  using G = Gram2<T>;
  using L = typename G::lds_t;
  using V = typename G::vec_t;
  constexpr int KB = G::KB;
  constexpr int LS = 128 + 16;                    // LDS row stride (elements)
  constexpr int VPR = 128 / G::EPV;               // 16-byte vectors per panel row
  constexpr int NV = KB * VPR / 256;              // vectors per thread per panel and chunk
  __shared__ __attribute__((aligned(16))) L lds[2][2][KB * LS];   // [buffer][panel I/J]

  // XCD-aware order: an XCD takes consecutive tiles of the lower triangle, which
  // share their row and column panels
  const int lin = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bid = lin / gridDim.x;
  const int part = bid / a.M, blk = bid - part * a.M;
  const int c0 = a.col_off[blk];
  const int nj = a.col_off[blk + 1] - c0;
  const int T_ = (nj + 127) / 128;
  int ti, tj;
  tri_tile(lin - bid * gridDim.x, &ti, &tj);
  if (ti >= T_) return;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const T* Ab = reinterpret_cast<const T*>(a.A) + r0 * a.ld + c0;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const bool diag = (ti == tj);

  floatx4 acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = floatx4{0.f, 0.f, 0.f, 0.f};

  // rows start at multiples of ld (a multiple of 64 elements), so the alignment
  // of every vector of the block follows from its first column
  const bool align16 = (c0 % G::EPV) == 0;
  const bool align4 = ((c0 * (int)sizeof(T)) % 4) == 0;
  // staging: vector q of this thread covers chunk row k = idx / VPR, columns
  // EPV * (idx % VPR) .. + EPV - 1 of the panel (idx = tid + 256 q)
  V stg[2][NV];
  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int pnl = 0; pnl < 2; ++pnl) {
      if (pnl == 1 && diag) break;
      const int tcol = (pnl == 0 ? ti : tj) * 128;
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int idx = tid + 256 * q;
        const int k = idx / VPR, cv = idx % VPR;
        const int64_t row = k0 + k;
        const int col = tcol + G::EPV * cv;
        V v;
        __builtin_memset(&v, 0, sizeof(v));
        if (row < m) {
          const T* src = Ab + row * a.ld + col;
          if (col + G::EPV <= nj && align16) {
            v = *reinterpret_cast<const V*>(src);
          } else if (col + G::EPV <= nj && align4) {
            // block start not 16-byte aligned: four dword loads
            uint32_t w[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) w[i] = reinterpret_cast<const uint32_t*>(src)[i];
            __builtin_memcpy(&v, w, sizeof(v));
          } else {
            L tmp[G::EPV];
#pragma unroll
            for (int e = 0; e < G::EPV; ++e) tmp[e] = L(0);
            for (int e = 0; e < G::EPV; ++e)
              if (col + e < nj) tmp[e] = __builtin_bit_cast(L, src[e]);
            __builtin_memcpy(&v, tmp, sizeof(v));
          }
        }
        stg[pnl][q] = v;
      }
    }
  };
  auto store_chunk = [&](int buf) {
#pragma unroll
    for (int pnl = 0; pnl < 2; ++pnl) {
      if (pnl == 1 && diag) break;
      L* dst = lds[buf][pnl];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const int idx = tid + 256 * q;
        const int k = idx / VPR, cv = idx % VPR;
        *reinterpret_cast<V*>(dst + k * LS + G::EPV * cv) = stg[pnl][q];
      }
    }
  };

  const int64_t nchunks = (m + KB - 1) / KB;
  load_chunk(0);
  store_chunk(0);
  __syncthreads();
  const int g = lane >> 4, cl = lane & 15;
  for (int64_t ch = 0; ch < nchunks; ++ch) {
    const int buf = (int)(ch & 1);
    if (ch + 1 < nchunks) load_chunk((ch + 1) * KB);
    const L* pI = lds[buf][0];
    const L* pJ = diag ? lds[buf][0] : lds[buf][1];
#pragma unroll
    for (int ks = 0; ks < KB; ks += G::K_STEP) {
      // subtile x of a wavefront's 64 columns holds columns 4 i + x (i = 0..15),
      // so one lane's four operands are four adjacent LDS columns
      typename G::op_t opa[4], opb[4];
      G::operands4(pI, ks, g, wr * 64 + 4 * cl, LS, opa);
      G::operands4(pJ, ks, g, wc * 64 + 4 * cl, LS, opb);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y) G::mma(acc[x][y], opa[x], opb[y]);
    }
    if (ch + 1 < nchunks) store_chunk(buf ^ 1);
    __syncthreads();
  }
  double* K = a.kbuf + a.kmat_off[bid];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * 128 + wr * 64 + 4 * (4 * (lane >> 4) + v) + x;
        const int col = tj * 128 + wc * 64 + 4 * (lane & 15) + y;
        if (row < nj && col < nj && row >= col) {
          const double gv = (double)acc[x][y][v];
          K[(int64_t)row * nj + col] = a.rho_l * gv + (row == col ? a.shift : 0.0);
        }
      }
}

// BF16 Gram with 256 x 256 output tiles, fed by LDS DMA.  8 wavefronts, each
// 128 x 64 outputs (an 8 x 4 grid of 16 x 16 tiles of v_mfma_f32_16x16x32_bf16,
// FP32 accumulation).  The two 256-column panels of the tile stream through LDS in
// 32-row stages, four stages deep: global_load_lds_dwordx4 writes each panel row
// into LDS as it sits in HBM (no registers, so three stages stay in flight while
// the MFMAs run on the fourth), and ds_read_b64_tr_b16 reads the MFMA operands --
// 8 consecutive rows of one column per lane -- transposed out of that row-major
// layout.  One barrier per stage.
//
// LDS layout of a stage: panel P (0 = I, 1 = J), row pair p = r / 2: 1 KB, lanes
// 0-31 of a DMA instruction fill row 2p, lanes 32-63 row 2p + 1.  Within a row the
// 16-byte pieces (8 columns) are XOR-swizzled by 4 (p & 1) + 2 (r & 1), so the four
// consecutive rows a group of 16 lanes reads transposed land in four different
// 32-byte slots of the 128-byte LDS bank period.
//
// Block starts that are not 16-byte aligned: each panel starts delta = c0 mod 8
// columns before its tile (delta columns of the previous block, or of this one),
// so every DMA source is a whole aligned piece; outputs whose shifted index falls
// outside [0, n_j) are dropped.  Pieces past the block's last column read a zero
// vector; a piece that straddles it reads up to 7 columns beyond (harmless: they
// only meet outputs that are dropped; A carries a zero tail for the last row).
namespace gdma {
constexpr int TILE = 256;
constexpr int KB = 32;                       // rows per stage
constexpr int STAGES = 4;
constexpr int STAGE_BYTES = 2 * KB * 512;    // two panels x KB rows x 512 bytes
constexpr int DMA_PER_WAVE = KB / 8;         // 16-byte DMA instructions per wavefront and stage
__device__ __forceinline__ int swz(int p, int h) { return 4 * (p & 1) + 2 * h; }
// byte offset in a stage of panel P, stage row r, panel column c (c % 4 == 0)
__device__ __forceinline__ int off(int P, int r, int c) {
  const int p = r >> 1, h = r & 1;
  return P * (KB * 512) + p * 1024 + 16 * (32 * h + ((c >> 3) ^ swz(p, h))) + 2 * (c & 7);
}
// s_waitcnt with vmcnt <= n (n < 64), expcnt and lgkmcnt unconstrained
constexpr int vmcnt(int n) { return (n & 15) | (((n >> 4) & 3) << 14) | (7 << 4) | (15 << 8); }
}  // namespace gdma

__device__ const uint32_t kGramZero[4] = {0u, 0u, 0u, 0u};

typedef short v4i16 __attribute__((ext_vector_type(4)));
#define BCA_LDS __attribute__((address_space(3)))

__global__ __launch_bounds__(512) void gram_dma_bf16_kernel(GramArgs a) {
  using namespace gdma;
  __shared__ __attribute__((aligned(16))) unsigned char smem[STAGES * STAGE_BYTES];

  const int lin = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const int bid = lin / gridDim.x;
  const int part = bid / a.M, blk = bid - part * a.M;
  const int c0 = a.col_off[blk];
  const int nj = a.col_off[blk + 1] - c0;
  const int delta = c0 & 7;
  const int T_ = (nj + delta + TILE - 1) / TILE;
  int ti, tj;
  tri_tile(lin - bid * gridDim.x, &ti, &tj);
  if (ti >= T_) return;
  const int64_t r0 = a.row_off[part];
  const int64_t m = a.row_off[part + 1] - r0;
  const uint16_t* Ab = reinterpret_cast<const uint16_t*>(a.A) + r0 * a.ld + (c0 - delta);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = wv >> 2, wc = wv & 3;
  const int64_t nch = (m + KB - 1) / KB;

  // stage ch: DMA instruction q = wv + 8 i (i < DMA_PER_WAVE) fills row pair q % 16 of
  // panel q / 16; lane l loads piece (l & 31) ^ swz of row 2p + l / 32
  auto issue = [&](int64_t ch) {
    unsigned char* st = smem + (int)(ch % STAGES) * STAGE_BYTES;
#pragma unroll
    for (int i = 0; i < DMA_PER_WAVE; ++i) {
      const int q = wv + 8 * i;
      const int P = q / (KB / 2), p = q % (KB / 2), h = lane >> 5;
      const int pc = (lane & 31) ^ swz(p, h);
      const int64_t row = ch * KB + 2 * p + h;
      const int col = (P ? tj : ti) * TILE + 8 * pc;    // shifted column of the piece
      const void* src = (row < m && col - delta < nj) ? (const void*)(Ab + row * a.ld + col)
                                                       : (const void*)kGramZero;
      const uint32_t dst = __builtin_amdgcn_readfirstlane(
          (uint32_t)(uintptr_t)(BCA_LDS void*)(st + P * (KB * 512) + p * 1024));
      // written out: the builtin form makes the compiler wait for all DMA before
      // every LDS read; this kernel waits for its own stages explicitly
      asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "s"(dst)
                   : "memory", "m0");
    }
  };

  floatx4 acc[8][4];
#pragma unroll
  for (int x = 0; x < 8; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = floatx4{0.f, 0.f, 0.f, 0.f};
  // a wavefront of a diagonal tile whose columns all lie above its rows has no output
  const bool idle = ti == tj && wc * 64 >= (wr + 1) * 128;
  const int s16 = lane & 15, g = lane >> 4;
  const int rA = 8 * g + (s16 >> 2);    // stage row of this lane's first transposed read
  const int cq = 4 * (s16 & 3);

  for (int d = 0; d < STAGES - 1; ++d)
    if (d < nch) issue(d);
  for (int64_t ch = 0; ch < nch; ++ch) {
    // this wavefront's DMA of stage ch is complete once at most the instructions of
    // the stages issued after it are outstanding
    const int64_t newer = nch - 1 - ch;
    if (newer >= 2) __builtin_amdgcn_s_waitcnt(vmcnt(2 * DMA_PER_WAVE));
    else if (newer == 1) __builtin_amdgcn_s_waitcnt(vmcnt(DMA_PER_WAVE));
    else __builtin_amdgcn_s_waitcnt(vmcnt(0));
    __syncthreads();   // stage ch complete for all wavefronts; stage ch - 1 fully read
    if (ch + STAGES - 1 < nch) issue(ch + STAGES - 1);
    if (idle) continue;
    const unsigned char* st = smem + (int)(ch % STAGES) * STAGE_BYTES;
    bf16x8 ob[4];
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int c = wc * 64 + 16 * y + cq;
      const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((BCA_LDS v4i16*)(st + off(1, rA, c)));
      const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((BCA_LDS v4i16*)(st + off(1, rA + 4, c)));
      const short t8[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      __builtin_memcpy(&ob[y], t8, 16);
    }
#pragma unroll
    for (int x = 0; x < 8; ++x) {
      const int c = wr * 128 + 16 * x + cq;
      const v4i16 lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16((BCA_LDS v4i16*)(st + off(0, rA, c)));
      const v4i16 hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16((BCA_LDS v4i16*)(st + off(0, rA + 4, c)));
      const short t8[8] = {lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
      bf16x8 oa;
      __builtin_memcpy(&oa, t8, 16);
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(oa, ob[y], acc[x][y], 0, 0, 0);
    }
  }
  if (idle) return;
  double* K = a.kbuf + a.kmat_off[bid];
#pragma unroll
  for (int x = 0; x < 8; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = ti * TILE + wr * 128 + 16 * x + 4 * g + v - delta;
        const int col = tj * TILE + wc * 64 + 16 * y + s16 - delta;
        if (col >= 0 && row < nj && row >= col) {
          const double gv = (double)acc[x][y][v];
          K[(int64_t)row * nj + col] = a.rho_l * gv + (row == col ? a.shift : 0.0);
        }
      }
}
#undef BCA_LDS

hipError_t launch_gram(const GramArgs& a, int dtype, hipStream_t s) {
  if (dtype == BCA_F64) {
    dim3 grid(a.tiles_max * (a.tiles_max + 1) / 2, a.N * a.M);
    hipLaunchKernelGGL(gram_kernel<double>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (dtype == BCA_F32) {
    const int t128 = (a.tiles_max + 1) / 2;   // tiles_max counts 64-column tiles
    dim3 grid(t128 * (t128 + 1) / 2, a.N * a.M);
    hipLaunchKernelGGL(gram128_kernel<float>, grid, dim3(256), 0, s, a);
  } else {
    // tiles_max counts 64-column tiles of the widest block; panels shift by up to 7 columns
    const int t256 = (a.tiles_max * 64 + 7 + 255) / 256;
    dim3 grid(t256 * (t256 + 1) / 2, a.N * a.M);
    hipLaunchKernelGGL(gram_dma_bf16_kernel, grid, dim3(512), 0, s, a);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ Cholesky
// Right-looking blocked Cholesky of all N M blocks at once, one 32-column panel
// per step and three launches per step so that every workgroup of the GPU
// takes part: the diagonal 32 x 32 block (one workgroup per matrix), the panel
// below it (one thread per row), and the trailing update of the lower 64 x 64
// tiles (one workgroup per tile and matrix).
constexpr int CHB = 32;

__global__ __launch_bounds__(256) void chol_diag_kernel(FactorArgs a, int k0) {
  __shared__ double D[CHB][CHB + 1];
  const int bid = blockIdx.x;
  const int blk = bid % a.M;
  const int n = a.col_off[blk + 1] - a.col_off[blk];
  if (k0 >= n) return;
  double* K = a.kbuf + a.kmat_off[bid];
  const int tid = threadIdx.x;
  const int kb = min(CHB, n - k0);
  for (int idx = tid; idx < CHB * CHB; idx += 256) {
    const int r = idx / CHB, c = idx % CHB;
    D[r][c] = (r < kb && c <= r) ? K[(int64_t)(k0 + r) * n + k0 + c] : 0.0;
  }
  __syncthreads();
  for (int p = 0; p < kb; ++p) {
    if (tid == 0) {
      double d = D[p][p];
      if (!(d > 0.0) || !isfinite(d)) {
        atomicExch(a.status, 1);
        d = 1.0;
      }
      D[p][p] = sqrt(d);
    }
    __syncthreads();
    if (tid > p && tid < kb) D[tid][p] /= D[p][p];
    __syncthreads();
    for (int idx = tid; idx < CHB * CHB; idx += 256) {
      const int r = idx / CHB, c = idx % CHB;
      if (c > p && r >= c && r < kb) D[r][c] -= D[r][p] * D[c][p];
    }
    __syncthreads();
  }
  for (int idx = tid; idx < CHB * CHB; idx += 256) {
    const int r = idx / CHB, c = idx % CHB;
    if (r < kb && c <= r) K[(int64_t)(k0 + r) * n + k0 + c] = D[r][c];
  }
}

// rows r >= k0 + 32: L[r, k0:k0+kb] = K[r, k0:k0+kb] D^-T (forward substitution)
__global__ __launch_bounds__(256) void chol_panel_kernel(FactorArgs a, int k0) {
  __shared__ double D[CHB][CHB + 1];
  const int bid = blockIdx.y;
  const int blk = bid % a.M;
  const int n = a.col_off[blk + 1] - a.col_off[blk];
  const int k1 = k0 + CHB;
  if (k1 >= n) return;
  const int r = k1 + blockIdx.x * 256 + threadIdx.x;
  if (k1 + blockIdx.x * 256 >= n) return;
  double* K = a.kbuf + a.kmat_off[bid];
  for (int idx = threadIdx.x; idx < CHB * CHB; idx += 256) {
    const int i = idx / CHB, j = idx % CHB;
    D[i][j] = j <= i ? K[(int64_t)(k0 + i) * n + k0 + j] : 0.0;
  }
  __syncthreads();
  if (r >= n) return;
  double x[CHB];
  double* row = K + (int64_t)r * n + k0;
#pragma unroll
  for (int p = 0; p < CHB; ++p) x[p] = row[p];
#pragma unroll
  for (int p = 0; p < CHB; ++p) {
    double v = x[p];
#pragma unroll
    for (int q = 0; q < p; ++q) v -= x[q] * D[p][q];
    x[p] = v / D[p][p];
  }
#pragma unroll
  for (int p = 0; p < CHB; ++p) row[p] = x[p];
}

// K[r, c] -= sum_p L[r, p] L[c, p] over the lower 64 x 64 tiles of the trailing part
__global__ __launch_bounds__(256) void chol_update_kernel(FactorArgs a, int k0) {
  __shared__ double P0[64][CHB + 1];
  __shared__ double P1[64][CHB + 1];
  const int bid = blockIdx.y;
  const int blk = bid % a.M;
  const int n = a.col_off[blk + 1] - a.col_off[blk];
  const int k1 = k0 + CHB;
  if (k1 >= n) return;
  const int nt = (n - k1 + 63) / 64;
  int ti, tj;
  tri_tile(blockIdx.x, &ti, &tj);
  if (ti >= nt) return;
  double* K = a.kbuf + a.kmat_off[bid];
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int idx = tid; idx < 64 * CHB; idx += 256) {
    const int r = idx / CHB, p = idx % CHB;
    const int gi = k1 + ti * 64 + r, gj = k1 + tj * 64 + r;
    P0[r][p] = gi < n ? K[(int64_t)gi * n + k0 + p] : 0.0;
    P1[r][p] = gj < n ? K[(int64_t)gj * n + k0 + p] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
#pragma unroll 8
  for (int p = 0; p < CHB; ++p) {
    double li[4], lj[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) li[x] = P0[ty + 16 * x][p];
#pragma unroll
    for (int y = 0; y < 4; ++y) lj[y] = P1[tx + 16 * y][p];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] += li[x] * lj[y];
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int gi = k1 + ti * 64 + ty + 16 * x, gj = k1 + tj * 64 + tx + 16 * y;
      if (gi < n && gj <= gi) K[(int64_t)gi * n + gj] -= acc[x][y];
    }
}

hipError_t launch_cholesky(const FactorArgs& a, hipStream_t s) {
  const int nm = a.N * a.M;
  for (int k0 = 0; k0 < a.nj_max; k0 += CHB) {
    hipLaunchKernelGGL(chol_diag_kernel, dim3(nm), dim3(256), 0, s, a, k0);
    const int rest = a.nj_max - k0 - CHB;
    if (rest <= 0) break;
    hipLaunchKernelGGL(chol_panel_kernel, dim3((rest + 255) / 256, nm), dim3(256), 0, s, a, k0);
    const int nt = (rest + 63) / 64;
    hipLaunchKernelGGL(chol_update_kernel, dim3(nt * (nt + 1) / 2, nm), dim3(256), 0, s, a, k0);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ inverse factor
// W = L^-1 by 64 x 64 blocks, right-looking over the block rows pb of W, all
// N M blocks at once:
//   inv_diag    W[b, b] = L[b, b]^-1 for every diagonal block (forward substitution,
//               one thread per column);
//   then for pb = 0, 1, ...:
//   inv_row     W[pb, kc] = -W[pb, pb] S[pb, kc] for kc < pb, where S[pb, kc] =
//               sum_{kc <= q < pb} L[pb, q] W[q, kc] has been accumulated in place;
//   inv_update  S[ib, kc] += L[ib, pb] W[pb, kc] for ib > pb, kc <= pb.
// Every launch works on independent 64 x 64 tiles, so the whole GPU takes part.
constexpr int IB = 64;

__device__ __forceinline__ void inv_matrix(const FactorArgs& a, int bid, int* n, const double** L, double** W) {
  const int blk = bid % a.M;
  *n = a.col_off[blk + 1] - a.col_off[blk];
  *L = a.kbuf + a.kmat_off[bid];
  *W = a.wbuf + a.kmat_off[bid];
}

__global__ __launch_bounds__(256) void inv_diag_kernel(FactorArgs a) {
  __shared__ double Ld[IB][IB + 1];
  __shared__ double X[IB][IB + 1];
  int n;
  const double* L;
  double* W;
  inv_matrix(a, blockIdx.y, &n, &L, &W);
  const int R0 = blockIdx.x * IB;
  if (R0 >= n) return;
  const int nr = min(IB, n - R0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < IB * IB; idx += 256) {
    const int r = idx / IB, q = idx % IB;
    Ld[r][q] = (r < nr && q <= r) ? L[(int64_t)(R0 + r) * n + R0 + q] : (q == r ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < IB) {
    const int c = tid;
    for (int r = 0; r < IB; ++r) {
      double v = (r == c) ? 1.0 : 0.0;
      for (int q = c; q < r; ++q) v -= Ld[r][q] * X[q][c];
      X[r][c] = r < c ? 0.0 : v / Ld[r][r];
    }
  }
  __syncthreads();
  for (int idx = tid; idx < IB * IB; idx += 256) {
    const int r = idx / IB, c = idx % IB;
    if (r < nr && c <= r) W[(int64_t)(R0 + r) * n + R0 + c] = X[r][c];
  }
}

__global__ __launch_bounds__(256) void inv_row_kernel(FactorArgs a, int pb) {
  __shared__ double D[IB][IB + 1];
  __shared__ double Sm[IB][IB + 1];
  int n;
  const double* L;
  double* W;
  inv_matrix(a, blockIdx.y, &n, &L, &W);
  const int R0 = pb * IB;
  const int kc = blockIdx.x;
  if (R0 >= n || kc >= pb) return;
  const int nr = min(IB, n - R0);
  const int C0 = kc * IB;
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int idx = tid; idx < IB * IB; idx += 256) {
    const int r = idx / IB, q = idx % IB;
    D[r][q] = (r < nr && q <= r) ? W[(int64_t)(R0 + r) * n + R0 + q] : 0.0;
    Sm[r][q] = r < nr ? W[(int64_t)(R0 + r) * n + C0 + q] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = 0.0;
  for (int q = 0; q < IB; ++q) {
    double dv[4], sv[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) dv[x] = D[ty + 16 * x][q];
#pragma unroll
    for (int y = 0; y < 4; ++y) sv[y] = Sm[q][tx + 16 * y];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] += dv[x] * sv[y];
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int r = ty + 16 * x, c = tx + 16 * y;
      if (r < nr) W[(int64_t)(R0 + r) * n + C0 + c] = -acc[x][y];
    }
}

__global__ __launch_bounds__(256) void inv_update_kernel(FactorArgs a, int pb) {
  __shared__ double Lt[IB][IB + 1];
  __shared__ double Wt[IB][IB + 1];
  int n;
  const double* L;
  double* W;
  inv_matrix(a, blockIdx.y, &n, &L, &W);
  const int nb = (n + IB - 1) / IB;
  const int ib = pb + 1 + blockIdx.x / (pb + 1);
  const int kc = blockIdx.x % (pb + 1);
  if (ib >= nb) return;
  const int R0 = ib * IB, P0 = pb * IB, C0 = kc * IB;
  const int nr = min(IB, n - R0);
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  for (int idx = tid; idx < IB * IB; idx += 256) {
    const int r = idx / IB, q = idx % IB;
    Lt[r][q] = r < nr ? L[(int64_t)(R0 + r) * n + P0 + q] : 0.0;
    Wt[r][q] = (kc < pb || q <= r) ? W[(int64_t)(P0 + r) * n + C0 + q] : 0.0;
  }
  __syncthreads();
  double acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int r = ty + 16 * x, c = tx + 16 * y;
      acc[x][y] = r < nr ? W[(int64_t)(R0 + r) * n + C0 + c] : 0.0;
    }
  for (int q = 0; q < IB; ++q) {
    double lv[4], wv[4];
#pragma unroll
    for (int x = 0; x < 4; ++x) lv[x] = Lt[ty + 16 * x][q];
#pragma unroll
    for (int y = 0; y < 4; ++y) wv[y] = Wt[q][tx + 16 * y];
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 4; ++y) acc[x][y] += lv[x] * wv[y];
  }
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) {
      const int r = ty + 16 * x, c = tx + 16 * y;
      if (r < nr) W[(int64_t)(R0 + r) * n + C0 + c] = acc[x][y];
    }
}

hipError_t launch_inverse(const FactorArgs& a, hipStream_t s) {
  const int nm = a.N * a.M;
  const int nb = (a.nj_max + IB - 1) / IB;
  hipLaunchKernelGGL(inv_diag_kernel, dim3(nb, nm), dim3(256), 0, s, a);
  for (int pb = 0; pb < nb; ++pb) {
    if (pb > 0) hipLaunchKernelGGL(inv_row_kernel, dim3(pb, nm), dim3(256), 0, s, a, pb);
    const int rest = nb - pb - 1;
    if (rest > 0) hipLaunchKernelGGL(inv_update_kernel, dim3(rest * (pb + 1), nm), dim3(256), 0, s, a, pb);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ P = W^T W
// Tile (I, J), I >= J, of P_ij: P[i][j] = sum_k W[k][i] W[k][j].  W is lower
// triangular, so rows k < 64 I (< every i of the tile) contribute nothing and the
// contraction runs over rows 64 I .. n_j - 1 only.  Same MFMA scheme as
// gram_kernel<double> (64 x 64 tile per workgroup, a 32 x 32 quadrant per
// wavefront, the two 64-column panels of a 16-row chunk staged transposed in LDS);
// the epilogue writes the whole tile, zeros outside n_j x n_j.
__global__ __launch_bounds__(256) void kinv_kernel(FactorArgs a) {
  using MF = GramMfma<double>;
  constexpr int KB = MF::KB;
  constexpr int LS = KB + MF::PAD;
  __shared__ double sI[64 * LS];
  __shared__ double sJ[64 * LS];
  const int bid = blockIdx.y;
  const int blk = bid % a.M;
  const int n = a.col_off[blk + 1] - a.col_off[blk];
  const int T_ = (n + PT - 1) / PT;
  int ti, tj;
  tri_tile(blockIdx.x, &ti, &tj);
  if (ti >= T_) return;
  const double* W = a.wbuf + a.kmat_off[bid];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const bool diag = (ti == tj);
  MF::acc_t acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[x][y][v] = 0.0;
  for (int k0 = ti * PT; k0 < n; k0 += KB) {
    for (int idx = tid; idx < KB * 64; idx += 256) {
      const int k = idx >> 6, c = idx & 63;
      const int row = k0 + k;
      const int ci = ti * PT + c, cj = tj * PT + c;
      double vi = 0.0, vj = 0.0;
      if (row < n) {
        if (ci < n) vi = W[(int64_t)row * n + ci];
        if (!diag && cj < n) vj = W[(int64_t)row * n + cj];
      }
      sI[c * LS + k] = vi;
      if (!diag) sJ[c * LS + k] = vj;
    }
    __syncthreads();
    const double* pJ = diag ? sI : sJ;
#pragma unroll
    for (int ks = 0; ks < KB; ks += MF::K_STEP) {
      const int kk = ks + MF::K_PER_LANE * (lane >> 4);
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const double* pa = sI + (wr * 32 + x * 16 + (lane & 15)) * LS + kk;
#pragma unroll
        for (int y = 0; y < 2; ++y) {
          const double* pb = pJ + (wc * 32 + y * 16 + (lane & 15)) * LS + kk;
          MF::mma(acc[x][y], pa, pb);
        }
      }
    }
    __syncthreads();
  }
  double* out = a.kinv + a.fac_off[bid] + (int64_t)blockIdx.x * PT_ELEMS;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = wr * 32 + x * 16 + MF::out_row(lane, v);
        const int col = wc * 32 + y * 16 + (lane & 15);
        const bool in = ti * PT + row < n && tj * PT + col < n;
        out[ptile_pos(row, col)] = in ? MF::out(acc[x][y], v) : 0.0;
      }
}

hipError_t launch_kinv(const FactorArgs& a, hipStream_t s) {
  const int T_ = (a.nj_max + PT - 1) / PT;
  dim3 grid(T_ * (T_ + 1) / 2, a.N * a.M);
  hipLaunchKernelGGL(kinv_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace bca
