// Batched form: many independent Bi-cADMM problems of different sizes advanced
// together in ONE persistent (cooperative) launch.
//
// Every outer iteration of every problem is the same sequence of phases as the
// one-problem path (Algorithm 2's K_in inner iterations, then the global step
// of Algorithm 1), but here each phase is a list of independent work items
// spanning all problems:
//   RHS     item (problem, partition, block, 64 columns): the FP64 reduction of
//           the A^T e partial sums into the right-hand side of the x_ij-step;
//   SYMV    item (problem, partition, block, tile range): one wavefront applies
//           tiles of the cached inverse P_ij = K_ij^-1 to r (symmetric product,
//           each stored tile read once), so a large block is shared by many
//           wavefronts;
//   XUPD    item (problem, partition, block, 64 rows): x += P_ij r from the
//           product's slots, in a fixed order, and the streaming copy of x;
//   STREAM  item (problem, partition, row chunk): the fused streaming pass over
//           a chunk of rows by one wavefront (block predictions, sample-space
//           average, omega-bar prox, nu update, e, partial A^T e of the chunk);
//   GLOBAL  item (problem): consensus average, exact (z,t) step, top-kappa
//           s-step, v and u updates, residuals.
// The wavefronts of the persistent grid take the items of the current phase
// (largest first: stream items through atomic counters, solve items
// round-robin; global items per workgroup through counters) and meet at a grid
// barrier between phases.  Both the counters and the barrier are split over
// eight groups of workgroups (blockIdx mod 8, the XCD a workgroup is dispatched
// to): a device-scope atomic on one address serialises every arrival, and with
// 512 workgroups (2,048 wavefronts) the cooperative-groups grid barrier took
// 50-70 us and one claim per wavefront on one counter about 20 us, against a few
// microseconds of work per phase for small problems.  A problem's results depend only on its own items
// (fixed reduction orders inside each item, tile shape chosen per problem shape,
// never per batch), so a problem computes the same bits alone and inside any
// batch.
//
// Stream tile shapes: chunks per lane NC (a row of nvec 16-byte chunks is read by
// one wavefront, NC = ceil(nvec / 64) rounded up to 1, 2, 4 or 8, or by a
// segment of 16 or 32 lanes for rows of at most 16 or 32 chunks) and rows per
// segment tile R in {1, 2, 4} with R NC <= 8 (and R = 8 for one-chunk rows, whose
// tiles are otherwise too small to keep enough bytes in flight), which bounds the
// kernel's register footprint; rows per item is a runtime parameter.
// The shape of each problem is picked by the autotuner in bca_api.hip.
#include "bca_internal.h"
#include "global_impl.h"
#include "prox_impl.h"
#include "symv_impl.h"

namespace bca {

constexpr int BT = 256;
constexpr int BW = BT / 64;

// Shapes (chunks per lane NC, rows per segment tile R, segments per wave S): a
// wavefront is split into S segments of 64 / S lanes, each streaming its own rows,
// so that rows of at most 16 or 32 chunks (short feature vectors) still keep
// every lane busy; S follows from the row length, R is tuned.
constexpr int kShapes = 18;
static const int kShapeNC[kShapes] = {1, 1, 1, 2, 2, 2, 4, 4, 8, 1, 1, 1, 1, 1, 1, 1, 1, 1};
static const int kShapeR[kShapes] = {1, 2, 4, 1, 2, 4, 1, 2, 1, 1, 2, 4, 1, 2, 4, 8, 8, 8};
static const int kShapeS[kShapes] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 4, 4, 4, 1, 2, 4};

int batch_max_nvec() { return 64 * 8; }

int batch_shape_code(int nvec, int R) {
  int nc = 1;
  while (nc < 8 && 64 * nc < nvec) nc *= 2;
  if (64 * nc < nvec) return -1;
  const int S = nc > 1 ? 1 : (nvec <= 16 ? 4 : (nvec <= 32 ? 2 : 1));
  for (int c = 0; c < kShapes; ++c)
    if (kShapeNC[c] == nc && kShapeR[c] == R && kShapeS[c] == S) return c;
  return -1;
}

// Item functions are called out of line, so their pointer arguments are generic:
// loads through them become FLAT instructions, which count on both the vector
// memory and the LDS counters, and waiting for one of them means waiting for all
// (lgkmcnt(0)).  The streaming item therefore casts its pointers to the global
// (and its LDS scratch to the local) address space, and copies the problem's
// fields to registers first: its own stores of omega-bar and nu could otherwise
// alias the BatchInst and make the compiler re-read those fields, with a wait for
// every load in flight, on each tile.
template <typename P>
using gptr = __attribute__((address_space(1))) P*;
template <typename P>
__device__ __forceinline__ gptr<P> glob(P* p) {
  return (gptr<P>)p;
}
typedef __attribute__((address_space(3))) double* lds_dptr;

template <typename V>
__device__ __forceinline__ V load_v(gptr<const V> p) {
  static_assert(sizeof(V) == 16, "16-byte vectors only");
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 t = *(gptr<const u32x4>)p;
  V v;
  __builtin_memcpy(&v, &t, 16);
  return v;
}

template <typename V>
__device__ __forceinline__ V load_nt(gptr<const V> p) {
  static_assert(sizeof(V) == 16, "16-byte vectors only");
  typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 t = __builtin_nontemporal_load((gptr<const u32x4>)p);
  V v;
  __builtin_memcpy(&v, &t, 16);
  return v;
}

// Sums over the wavefront of R (2, 4, 8) per-lane values at once (reduce-scatter):
// each halving step over lane bit 5, 4, 3 adds half of the remaining values to the
// partner lane's and keeps the upper half where the lane's bit is set, so that
// after log2 R steps the lane holds a partial of row lane >> (6 - log2 R); the
// remaining low bits are summed as in wave_sum_dpp.  Every lane of a group of
// 64 / R returns its row's total: about 40 instructions for 8 rows where 8 full
// wave sums take about 240.
template <int R>
__device__ __forceinline__ double rows_sum_scatter(double (&v)[R]) {
  constexpr int K = R == 2 ? 1 : (R == 4 ? 2 : 3);
  static_assert(R == 2 || R == 4 || R == 8, "2, 4 or 8 rows");
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < K; ++i) {
    const int half = R >> (i + 1);
#pragma unroll
    for (int j = 0; j < half; ++j) {
      double a = v[j], b = v[j + half];
      if (i == 0) {
        swap32(a, b);
        v[j] = a + b;
      } else if (i == 1) {
        swap16(a, b);
        v[j] = a + b;
      } else {
        const double pa = dpp_f64<0x128>(a), pb = dpp_f64<0x128>(b);   // lane ^ 8
        v[j] = (lane & 8) ? b + pb : a + pa;
      }
    }
  }
  double x = v[0];
  x += dpp_f64<0xB1>(x);    // quad_perm [1,0,3,2]
  x += dpp_f64<0x4E>(x);    // quad_perm [2,3,0,1]
  x += dpp_f64<0x141>(x);   // row_half_mirror
  if constexpr (K <= 2) x += dpp_f64<0x140>(x);   // row_mirror
  if constexpr (K <= 1) {
    double t = x;
    swap16(x, t);
    x = x + t;
  }
  return x;
}

// Tiles kept in flight per wavefront: a ring of D tile buffers, the load of tile
// t + D issued as soon as tile t is processed, so that D tiles (about 4 KB to
// 16 KB per wavefront) are in flight while one is processed; D shrinks as the tile
// grows to bound the registers (D R NC <= 16 chunks of 16 bytes per lane).
constexpr int stream_depth(int R, int NC) { return R * NC <= 2 ? 4 : (R * NC <= 4 ? 3 : 2); }

// LG: the widest FP32 shape (32 columns per lane) keeps its FP64 partial sums of
// A^T e in LDS (lg, 32 x BT doubles) instead of 64 registers, which would
// otherwise set the register budget of the whole persistent kernel.
template <typename T, int NC, int R, int S>
__device__ __noinline__ void stream_item(const BatchInst& I, int part, int chunk, int mode, double* lg_) {
  using TR = Traits<T>;
  using V = typename TR::vec_t;
  using acc = typename TR::acc_t;
  constexpr int VEC = TR::VEC;
  constexpr bool LG = NC * VEC == 32;
  constexpr int LSEG = 64 / S;  // lanes per segment
  constexpr int D = stream_depth(R, NC);
  const lds_dptr lg = (lds_dptr)lg_;
  const int lane = threadIdx.x & 63;
  const int sl = lane % LSEG, seg = lane / LSEG;
  // One-segment tiles of several rows reduce their row sums together
  // (rows_sum_scatter): row r's total is then in lanes r G .. r G + G - 1 (G =
  // 64 / R), and lane r G runs the row's prox; otherwise lane sl < R of the
  // segment runs row sl's.
  constexpr bool RS = S == 1 && R > 1;
  constexpr int G = 64 / R;
  const int myrow = RS ? lane / G : sl;              // the row this lane's values are for
  const bool leader = RS ? (lane % G) == 0 : sl < R;
  // the problem's fields, read once
  const int64_t ld = I.ld;
  const int nvec = I.nvec;
  const int64_t r0 = I.row_off[part];
  const int64_t m = I.row_off[part + 1] - r0;
  const int64_t rows_per_item = I.rows_per_item;
  const int items_per_part = I.items_per_part;
  const int loss = I.loss, M = I.M;
  const double rho_l = I.rho_l, inv_M = I.inv_M;
  const gptr<const double> bv = glob(I.b);
  const gptr<double> omv = glob(I.omega);
  const gptr<double> nuv = glob(I.nu);
  const gptr<const T> Ab = glob(reinterpret_cast<const T*>(I.A)) + r0 * ld;
  const gptr<const acc> xs = glob(reinterpret_cast<const acc*>(I.xs)) + (int64_t)part * ld;
  const gptr<double> gp = glob(I.gpart) + ((int64_t)part * items_per_part + chunk) * ld;
  const int64_t lo = (int64_t)chunk * rows_per_item;
  const int64_t hi = lo + rows_per_item < m ? lo + rows_per_item : m;
  // the lane's chunks of x, one 16-byte load each (rows of xs are 16-byte aligned:
  // ld is a multiple of 64 elements, and its columns past n are zero)
  acc xr[NC][VEC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const int k = sl + LSEG * q;
    V xv = vzero<V>();
    if (k < nvec) xv = load_v<V>((gptr<const V>)xs + k);
#pragma unroll
    for (int e = 0; e < VEC; ++e) xr[q][e] = vget(xv, e);
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
  // Branch-free loads (rows past the item's end re-read its last row, chunks past
  // the row's end its last chunk: x is zero there and e is zero on such rows).
  // byte offsets of the lane's chunks in a row
  uint32_t kb[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) kb[q] = 16u * (uint32_t)min(sl + LSEG * q, nvec - 1);
  // a wave tile is S R rows: segment s takes rows rt + s R .. rt + s R + R - 1; with
  // one segment the row is the same for the whole wavefront, and its address is
  // kept in scalar registers (a 64-bit address per lane and chunk would take 2 NC
  // vector registers per row in flight)
  auto load_tile = [&](V (&dst)[R][NC], int64_t t0) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int64_t row = min(t0 + seg * R + r, hi - 1);
      uint64_t base = (uint64_t)(Ab + row * ld);
      if constexpr (S == 1)
        base = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32) |
               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
#pragma unroll
      for (int q = 0; q < NC; ++q) dst[r][q] = load_nt<V>((gptr<const V>)(base + kb[q]));
    }
  };
  // Per-row values (b, omega-bar, nu) of a tile are loaded together with its A
  // rows: loads complete in issue order, so a row value loaded after later tiles'
  // loads would make the wavefront wait for those too.  The rows of a tile lie
  // beyond those of every earlier tile, so reading their omega-bar and nu before
  // the earlier tiles' stores is safe.
  struct RowVals {
    double b, om, nu;
  };
  auto load_rows = [&](int64_t t0) {
    // lanes past the segment's R rows read its last row (one address, unused)
    const int64_t gr = r0 + min(t0 + seg * R + min(myrow, R - 1), hi - 1);
    return RowVals{bv[gr], omv[gr], nuv[gr]};
  };
  // One tile: row sums of A x, the omega-bar/nu step of its rows, and e times
  // its rows added to the partial sums of A^T e.
  auto process = [&](const V (&v)[R][NC], const RowVals& rv, int64_t rt) {
    double mine = 0.0;
    if constexpr (RS) {
      double dv[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc d = acc(0);
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
          for (int e = 0; e < VEC; ++e) d += vget(v[r][q], e) * xr[q][e];
        dv[r] = (double)d;
      }
      mine = rows_sum_scatter<R>(dv);
    } else {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc d = acc(0);
#pragma unroll
        for (int q = 0; q < NC; ++q)
#pragma unroll
          for (int e = 0; e < VEC; ++e) d += vget(v[r][q], e) * xr[q][e];
        double sv = (double)d;
        if constexpr (S == 1) {
          sv = wave_sum_dpp(sv);
        } else {
          sv = row16_sum_dpp(sv);                          // 16-lane segments
          if constexpr (S == 2) sv += __shfl_xor(sv, 16, 64);  // 32-lane segments
        }
        if (sl == r) mine = sv;
      }
    }
    double e = 0.0;
    const int64_t row = rt + seg * R + myrow;
    if (leader && row < hi) {
      const int64_t gr = r0 + row;
      const double av = mine * inv_M;
      double nu = rv.nu;
      if (mode == 0) {
        const double om = prox_scalar(loss, av + nu, rv.b, M, rho_l,
                                      loss == BCA_LOSS_SQUARED ? 0.0 : rv.om);
        nu = nu + av - om;
        omv[gr] = om;
        nuv[gr] = nu;
        e = om - av - nu;
      } else {
        e = rv.om - av - nu;
      }
    }
    acc er[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (S == 1)
        er[r] = (acc)__hiloint2double(__builtin_amdgcn_readlane(__double2hiint(e), RS ? r * G : r),
                                      __builtin_amdgcn_readlane(__double2loint(e), RS ? r * G : r));
      else
        er[r] = (acc)__shfl(e, seg * LSEG + r, 64);
    }
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int c = 0; c < VEC; ++c) {
        acc t = acc(0);
#pragma unroll
        for (int r = 0; r < R; ++r) t += er[r] * vget(v[r][q], c);
        if constexpr (LG)   // an LDS add (the slot is this lane's own): no read back
          __hip_atomic_fetch_add(&lg[(q * VEC + c) * BT + threadIdx.x], (double)t, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WAVEFRONT);
        else
          g[q][c] += (double)t;
      }
  };
  // The ring's loads are unconditional (tiles past the item's end re-read its last
  // row, which the cache holds): a conditional load would make the compiler copy
  // the buffers between iterations, and each copy waits for its load.
  constexpr int64_t STEP = (int64_t)S * R;
  const int64_t ntiles = lo < hi ? (hi - lo + STEP - 1) / STEP : 0;
  if (ntiles > 0) {
    V buf[D][R][NC];
    RowVals rvb[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      load_tile(buf[d], lo + d * STEP);
      rvb[d] = load_rows(lo + d * STEP);
    }
    int64_t t = 0;
    for (; t + D <= ntiles; t += D) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        process(buf[d], rvb[d], lo + (t + d) * STEP);
        // the buffer's next loads stay after its last use (else they need
        // registers of their own)
        __builtin_amdgcn_sched_barrier(0);
        load_tile(buf[d], lo + (t + d + D) * STEP);
        rvb[d] = load_rows(lo + (t + d + D) * STEP);
      }
    }
#pragma unroll
    for (int d = 0; d < D - 1; ++d)
      if (t + d < ntiles) process(buf[d], rvb[d], lo + (t + d) * STEP);
  }
  // segments hold sums over different rows for the same columns: combine them
  if constexpr (S > 1 && !LG) {
#pragma unroll
    for (int q = 0; q < NC; ++q)
#pragma unroll
      for (int c = 0; c < VEC; ++c)
#pragma unroll
        for (int o = LSEG; o < 64; o <<= 1) g[q][c] += __shfl_xor(g[q][c], o, 64);
  }
  // the partial sums are written with nontemporal stores (read once, by the RHS
  // phase: measured 0.7 % faster than cached stores)
  if (seg == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int k = sl + LSEG * q;
      if (k < nvec) {
#pragma unroll
        for (int c = 0; c < VEC; ++c) {
          if constexpr (LG)
            __builtin_nontemporal_store((double)lg[(q * VEC + c) * BT + threadIdx.x], &gp[k * VEC + c]);
          else
            __builtin_nontemporal_store(g[q][c], &gp[k * VEC + c]);
        }
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void stream_item_dispatch(const BatchInst& I, int part, int chunk, int mode, double* lg) {
  switch (I.shape) {
    case 0: stream_item<T, 1, 1, 1>(I, part, chunk, mode, lg); break;
    case 1: stream_item<T, 1, 2, 1>(I, part, chunk, mode, lg); break;
    case 2: stream_item<T, 1, 4, 1>(I, part, chunk, mode, lg); break;
    case 3: stream_item<T, 2, 1, 1>(I, part, chunk, mode, lg); break;
    case 4: stream_item<T, 2, 2, 1>(I, part, chunk, mode, lg); break;
    case 5: stream_item<T, 2, 4, 1>(I, part, chunk, mode, lg); break;
    case 6: stream_item<T, 4, 1, 1>(I, part, chunk, mode, lg); break;
    case 7: stream_item<T, 4, 2, 1>(I, part, chunk, mode, lg); break;
    case 8: stream_item<T, 8, 1, 1>(I, part, chunk, mode, lg); break;
    case 9: stream_item<T, 1, 1, 2>(I, part, chunk, mode, lg); break;
    case 10: stream_item<T, 1, 2, 2>(I, part, chunk, mode, lg); break;
    case 11: stream_item<T, 1, 4, 2>(I, part, chunk, mode, lg); break;
    case 12: stream_item<T, 1, 1, 4>(I, part, chunk, mode, lg); break;
    case 13: stream_item<T, 1, 2, 4>(I, part, chunk, mode, lg); break;
    case 14: stream_item<T, 1, 4, 4>(I, part, chunk, mode, lg); break;
    case 15: stream_item<T, 1, 8, 1>(I, part, chunk, mode, lg); break;
    case 16: stream_item<T, 1, 8, 2>(I, part, chunk, mode, lg); break;
    default: stream_item<T, 1, 8, 4>(I, part, chunk, mode, lg); break;
  }
}

// x_ij-step of one block, in three phases of independent items, each claimed by
// one wavefront, so that a large block is spread over many wavefronts:
//   RHS  (partition, block, 64 columns): r = rho_l sum_w gpart_w + rho_c (z - u) - shift x;
//   SYMV (partition, block, tile range): slots of y = P_ij r (symv_impl.h);
//   XUPD (partition, block, 64-row slot row): x += y, y summed from the slots in a
//        fixed order.
// Wave-uniform values read from memory stay in vector registers unless the
// compiler is told they are uniform: these move them to scalar registers.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const uint64_t u = (uint64_t)v;
  return (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                   (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u));
}
__device__ __forceinline__ double uni(double v) {
  return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                          __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
template <typename P>
__device__ __forceinline__ gptr<P> uni(gptr<P> p) {
  return (gptr<P>)(uintptr_t)uni((int64_t)(uintptr_t)p);
}
template <typename P>
__device__ __forceinline__ gptr<P> uni_glob(P* p) {
  return uni(glob(p));
}
__device__ __forceinline__ BatchItem load_item(gptr<const BatchItem> p) {
  BatchItem w;
  w.inst = p->inst;
  w.a = p->a;
  w.b = p->b;
  w.c = p->c;
  w.d = p->d;
  return w;
}

// The RHS and XUPD phases: each wavefront takes two of its round-robin items at a
// time and moves them through their chains of dependent loads (item, problem
// descriptor, column offsets, then the data) step by step together, so that the
// two chains' latencies overlap; each item's arithmetic is that of one item alone.
// (Global-address-space pointers, as in the streaming item: generic pointers would
// make every load a FLAT load.)
struct RhsRef {
  bool on;
  int P, n, k;
  int64_t ld, o;
  double rho_l, rho_c, shift;
  gptr<const double> gb;
  gptr<double> rhs;
};

__device__ __noinline__ void rhs_phase(const BatchArgs& ba, int o, int k, int gwave, int nwaves) {
  const gptr<const BatchItem> items = uni_glob(ba.rhs_items);
  const gptr<const BatchInst> insts = uni_glob(ba.inst);
  const int n_items = uni(ba.n_rhs);
  const int lane = threadIdx.x & 63;
  for (int it0 = gwave; it0 < n_items; it0 += 2 * nwaves) {
    BatchItem w[2];
    bool take[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int it = it0 + j * nwaves;
      take[j] = it < n_items;
      if (take[j]) w[j] = load_item(items + it);
    }
    RhsRef d[2];
    gptr<const int32_t> colp[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      d[j].on = false;
      if (!take[j]) continue;
      const gptr<const BatchInst> I = insts + uni(w[j].inst);
      if (o >= uni(I->outer) || k >= uni(I->inner_iters)) continue;
      d[j].on = true;
      d[j].P = uni(I->items_per_part);
      d[j].ld = uni(I->ld);
      d[j].rho_l = uni(I->rho_l);
      d[j].rho_c = uni(I->rho_c);
      d[j].shift = uni(I->shift);
      d[j].n = uni(I->n);
      colp[j] = uni_glob(I->col_off) + uni(w[j].b);
    }
    double zk[2], uo[2], xo[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!d[j].on) continue;
      const gptr<const BatchInst> I = insts + uni(w[j].inst);
      const int c0 = uni(colp[j][0]);
      const int nj = uni(colp[j][1]) - c0;
      const int c = uni(w[j].c) + lane;
      const int part = uni(w[j].a);
      if (c >= nj) {
        d[j].on = false;
        continue;
      }
      d[j].k = c0 + c;
      d[j].o = (int64_t)part * d[j].n + d[j].k;
      d[j].gb = uni_glob(I->gpart) + (int64_t)part * d[j].P * d[j].ld + d[j].k;
      d[j].rhs = uni_glob(I->rhs);
      zk[j] = uni_glob(I->z)[d[j].k];
      uo[j] = uni_glob(I->u)[d[j].o];
      xo[j] = uni_glob(I->x)[d[j].o];
    }
    // partial w goes to s[w mod 8] in increasing w for w < P & ~7, the rest to s[0];
    // the partials are read once (nontemporal loads)
    double s[2][8];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int u = 0; u < 8; ++u) s[j][u] = 0.0;
    int P8[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) P8[j] = d[j].on ? (d[j].P & ~7) : 0;
    const int P8m = max(P8[0], P8[1]);
    for (int wv = 0; wv < P8m; wv += 16) {
      double v[2][16];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (wv + u < P8[j]) v[j][u] = __builtin_nontemporal_load(d[j].gb + (int64_t)(wv + u) * d[j].ld);
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int u = 0; u < 16; ++u)
          if (wv + u < P8[j]) s[j][u & 7] += v[j][u];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!d[j].on) continue;
      for (int wv = P8[j]; wv < d[j].P; ++wv) s[j][0] += d[j].gb[(int64_t)wv * d[j].ld];
      const double ate = ((s[j][0] + s[j][1]) + (s[j][2] + s[j][3])) +
                         ((s[j][4] + s[j][5]) + (s[j][6] + s[j][7]));
      d[j].rhs[d[j].o] = d[j].rho_l * ate + d[j].rho_c * (zk[j] - uo[j]) - d[j].shift * xo[j];
    }
  }
}

// Tiles [t0, t1) of block (part, blk), one after the other, by one wavefront
// (NTL: nontemporal tile loads).
template <bool NTL>
__device__ __forceinline__ void symv_item(const BatchInst& I, int part, int blk, int t0, int t1) {
  const int bid = part * I.M + blk;
  const int c0 = I.col_off[blk];
  const int nj = I.col_off[blk + 1] - c0;
  const int T = (nj + PT - 1) / PT;
  const double* P = I.kinv + I.fac_off[bid];
  const double* r = I.rhs + (int64_t)part * I.n + c0;
  double* ys = I.ypart + (int64_t)bid * I.tmax * I.tmax * PT;
  for (int t = t0; t < t1; ++t) {
    int ti, tj;
    tri_tile(t, &ti, &tj);
    symv_tile<NTL>(P + (int64_t)t * PT_ELEMS, r, nj, 1, ti, tj, T, ys);
  }
}

// XUPD: x += y over the 64 features of slot row R of block (part, blk), y summed
// from the row's T slots in the order of symv_gather (two alternating sums); the
// slots are loaded together first (T <= 16 for the blocks of the batched form,
// n_j <= 1024; larger T takes the rest one by one).  Two items at a time, as RHS.
struct XupdRef {
  bool on;
  bool f64;
  int T;
  int64_t o, so;
  gptr<double> x;
  gptr<void> xs;
  gptr<const double> p;
};

__device__ __noinline__ void xupd_phase(const BatchArgs& ba, int o, int k, int gwave, int nwaves) {
  const gptr<const BatchItem> items = uni_glob(ba.xupd_items);
  const gptr<const BatchInst> insts = uni_glob(ba.inst);
  const int n_items = uni(ba.n_xupd);
  const int lane = threadIdx.x & 63;
  constexpr int TU = 16;
  for (int it0 = gwave; it0 < n_items; it0 += 2 * nwaves) {
    BatchItem w[2];
    bool take[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int it = it0 + j * nwaves;
      take[j] = it < n_items;
      if (take[j]) w[j] = load_item(items + it);
    }
    XupdRef d[2];
    gptr<const int32_t> colp[2];
    int Mn[2], nn[2], ldn[2], tm[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      d[j].on = false;
      if (!take[j]) continue;
      const gptr<const BatchInst> I = insts + uni(w[j].inst);
      if (o >= uni(I->outer) || k >= uni(I->inner_iters)) continue;
      d[j].on = true;
      d[j].f64 = uni(I->dtype) == BCA_F64;
      Mn[j] = uni(I->M);
      nn[j] = uni(I->n);
      ldn[j] = (int)uni(I->ld);
      tm[j] = uni(I->tmax);
      colp[j] = uni_glob(I->col_off) + uni(w[j].b);
      d[j].x = uni_glob(I->x);
      d[j].xs = uni_glob(I->xs);
      d[j].p = uni_glob(I->ypart);
    }
    double xo[2], v[2][TU];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!d[j].on) continue;
      const int part = uni(w[j].a), blk = uni(w[j].b), R = uni(w[j].c);
      const int c0 = uni(colp[j][0]);
      const int nj = uni(colp[j][1]) - c0;
      const int i = R * PT + lane;
      if (i >= nj) {
        d[j].on = false;
        continue;
      }
      const int bid = part * Mn[j] + blk;
      d[j].T = (nj + PT - 1) / PT;
      d[j].o = (int64_t)part * nn[j] + c0 + i;
      d[j].so = (int64_t)part * ldn[j] + c0 + i;
      d[j].p = d[j].p + (int64_t)bid * tm[j] * tm[j] * PT + ((int64_t)(i >> 6) * d[j].T * PT + (i & 63));
      xo[j] = d[j].x[d[j].o];
#pragma unroll
      for (int S = 0; S < TU; ++S)
        if (S < d[j].T) v[j][S] = d[j].p[(int64_t)S * PT];
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (!d[j].on) continue;
      const int T = d[j].T;
      double y0 = 0.0, y1 = 0.0;
#pragma unroll
      for (int S = 0; S < TU; S += 2) {
        if (S + 2 <= T) {
          y0 += v[j][S];
          y1 += v[j][S + 1];
        } else if (S + 1 == T) {
          y0 += v[j][S];
        }
      }
      if (T > TU) {
        int S = TU;
        for (; S + 2 <= T; S += 2) {
          y0 += d[j].p[(int64_t)S * PT];
          y1 += d[j].p[(int64_t)(S + 1) * PT];
        }
        if (S < T) y0 += d[j].p[(int64_t)S * PT];
      }
      const double xn = xo[j] + (y0 + y1);
      d[j].x[d[j].o] = xn;
      if (d[j].f64)
        ((gptr<double>)d[j].xs)[d[j].so] = xn;
      else
        ((gptr<float>)d[j].xs)[d[j].so] = (float)xn;
    }
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
  g.gp = nullptr;   // the whole step in this workgroup
  g.split = 0;
  g.G = 0;
  g.G2 = 0;
  return g;
}

// One wavefront's share of a symmetric-product phase (items dealt round-robin).
// The item body is inlined and this function called once per phase: a call per
// item made every item pay the callee-saved register stores and loads of the
// call convention, in scratch memory (measured at 512 problems: 684 -> 603 us
// per phase).  (The streaming items keep one call per item: with their 36 shape
// bodies inlined into one function it spills in the item loop, 1.7 -> 2.4 ms.)
//
// A launch whose tiles far exceed the last-level cache (256 MB of Infinity Cache)
// reads them with nontemporal loads: cached, they evicted the phase's small reused
// data (r, and the slots that XUPD reads next) for no reuse of their own (512
// problems, 2.9 GB of tiles: SYMV 0.57 -> 0.53 ms, XUPD 0.048 -> 0.042 ms per inner
// iteration); a smaller set stays cached for the next inner iteration.  Items hold
// at most two 32 KB tiles.
constexpr int64_t kSymvNtlBytes = int64_t(128) << 20;

__device__ __noinline__ void symv_phase(const BatchArgs& ba, int o, int k, int gwave, int nwaves) {
  const bool ntl = (int64_t)ba.n_symv * 2 * PT_ELEMS * (int64_t)sizeof(double) > kSymvNtlBytes;
  for (int it = gwave; it < ba.n_symv; it += nwaves) {
    const BatchItem w = ba.symv_items[it];
    const BatchInst& I = ba.inst[w.inst];
    if (o >= I.outer || k >= I.inner_iters) continue;
    if (ntl)
      symv_item<true>(I, w.a, w.b, w.c, w.d);
    else
      symv_item<false>(I, w.a, w.b, w.c, w.d);
  }
}

// Grid barrier of the persistent launch (all workgroups are resident: the launch
// is cooperative).  Workgroup g arrives at the counter of its group g mod 8; the
// last arrival of a group adds the group to a second counter, and the last group
// publishes the barrier's number in a generation word that every workgroup polls.
// Counters only grow (barrier e completes a group at (e + 1) times its size), so
// no reset is needed within a launch; all start at zero.  Layout (32-bit words,
// each on its own 128-byte line): group counters at 32 x, x < 8; the group
// arrivals at 256; the generation at 288.  Visibility: every wavefront waits for
// its own memory operations; one release fence per workgroup (agent scope) writes
// the XCD's L2 back before a relaxed arrival; the last arrival of a group
// acquires the group's arrivals before adding the group to the second counter
// (acquire-release), the last group stores the generation (release); the others
// poll with relaxed loads (an acquiring load would invalidate the caches at every
// poll) and acquire once they see it.
constexpr int kGroups = kBatchCounterGroups;
static_assert(kBatchBarWords >= 289, "barrier words");

__device__ __forceinline__ void grid_barrier(unsigned int* bar, unsigned int& epoch) {
  __builtin_amdgcn_s_waitcnt(0);   // this wavefront's loads and stores are complete
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned int x = blockIdx.x % kGroups;
    const unsigned int nx = (gridDim.x + kGroups - 1 - x) / kGroups;   // workgroups in group x
    const unsigned int ng = gridDim.x < kGroups ? gridDim.x : kGroups;   // groups in use
    const unsigned int target = epoch + 1;
    const unsigned int old = __hip_atomic_fetch_add(&bar[32 * x], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == target * nx - 1) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const unsigned int g = __hip_atomic_fetch_add(&bar[256], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (g == target * ng - 1) __hip_atomic_store(&bar[288], target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    while (__hip_atomic_load(&bar[288], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
      __builtin_amdgcn_s_sleep(8);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
  epoch += 1;
}

// Two workgroups per CU: at most 256 registers per lane (VGPRs and AGPRs).
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(2))) void batch_kernel(BatchArgs ba) {
  // the widest stream shape's partial sums
  __shared__ double big[32 * BT];
  __shared__ double shd[BW * (PSECT + 2)];
  __shared__ TopkShared<BT> tks;
  __shared__ int item_sh;
  unsigned int epoch = 0;
  int phase = 0;
  // phase tracing: timestamp k is taken once barrier k - 1 has been passed
  auto stamp = [&]() {
    if (ba.stamps && blockIdx.x == 0 && threadIdx.x == 0) ba.stamps[epoch] = __builtin_amdgcn_s_memrealtime();
  };
  stamp();
  // the workgroup's group (of kGroups) for counters and barrier, and the group's size
  const int grp = blockIdx.x % kGroups;
  const int ngrp = (int)gridDim.x < kGroups ? (int)gridDim.x : kGroups;

  // Claims of a phase: group x takes items x, x + ngrp, x + 2 ngrp, ... from its
  // own counter (counters[kGroups * phase + x]).
  // claims the next item of the current phase (all threads get the same index)
  auto claim = [&]() {
    if (threadIdx.x == 0)
      item_sh = grp + ngrp * (int)atomicAdd(&ba.counters[kGroups * phase + grp], 1u);
    __syncthreads();
    const int it = item_sh;
    __syncthreads();
    return it;
  };
  // The items of the solve and stream phases go to single wavefronts (no
  // workgroup barrier between items, so the 8 wavefronts of a CU overlap their
  // per-item latencies).  Stream items, whose costs vary with the tile shape,
  // are claimed through the group counters; the many small solve items are dealt
  // round-robin over the wavefronts of the grid (largest first), since a claim
  // costs about as much as such an item and the claims of one counter serialise.
  const int gwave = blockIdx.x * BW + (threadIdx.x >> 6), nwaves = gridDim.x * BW;
  auto claim_wave = [&]() {
    int it = 0;
    if ((threadIdx.x & 63) == 0) it = (int)atomicAdd(&ba.counters[kGroups * phase + grp], 1u);
    return grp + ngrp * __shfl(it, 0, 64);
  };
  auto run_stream = [&](const BatchItem* items, int count, int mode, int k_inner, int o) {
    for (int it = claim_wave(); it < count; it = claim_wave()) {
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
    grid_barrier(ba.bar, epoch);
      stamp();
  }
  for (int o = 0; o < ba.outer; ++o) {
    for (int k = 0; k < ba.inner_max; ++k) {
      rhs_phase(ba, o, k, gwave, nwaves);
      ++phase;
      grid_barrier(ba.bar, epoch);
      stamp();
      symv_phase(ba, o, k, gwave, nwaves);
      ++phase;
      grid_barrier(ba.bar, epoch);
      stamp();
      xupd_phase(ba, o, k, gwave, nwaves);
      ++phase;
      grid_barrier(ba.bar, epoch);
      stamp();
      run_stream(ba.stream_items, ba.n_stream, 0, k, o);
      grid_barrier(ba.bar, epoch);
      stamp();
    }
    for (int it = claim(); it < ba.count; it = claim()) {
      const BatchInst& I = ba.inst[it];
      if (o >= I.outer) continue;
      global_step_batched(global_args_of(I), shd, tks);
      __syncthreads();
    }
    ++phase;
    grid_barrier(ba.bar, epoch);
      stamp();
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

__global__ void zero_u32_kernel(unsigned int* p, int count) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) p[k] = 0u;
}

hipError_t launch_zero_u32(unsigned int* p, int count, hipStream_t s) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(zero_u32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, p, count);
  return hipGetLastError();
}

// out[r] = the non-finite flag of problem r of a launch (one copy back for all).
__global__ void batch_status_kernel(const BatchInst* inst, int count, int* out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < count) out[r] = *inst[r].status;
}

hipError_t launch_batch_status(const BatchInst* inst, int count, int* out, hipStream_t s) {
  if (count < 1) return hipSuccess;
  hipLaunchKernelGGL(batch_status_kernel, dim3((count + 255) / 256), dim3(256), 0, s, inst, count, out);
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& a, int grid, hipStream_t s) {
  BatchArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(batch_kernel), dim3(grid), dim3(BT),
                                    params, 0, s);
}

}  // namespace bca
