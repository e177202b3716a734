// Symmetric product y = P r of the x_ij-step, one 64 x 64 tile per wavefront
// (shared by the one-problem solve and the batched kernel).
//
// P is stored as the tiles (I, J), I >= J, of its lower block triangle (layout in
// bca_internal.h).  An off-diagonal tile contributes P_IJ r_J to rows I and
// P_IJ^T r_I to rows J, so every stored entry is read once and used twice; a
// diagonal tile (stored in full) contributes P_II r_I.  Each contribution is a
// 64-vector written to its own slot, slot (R, S) = the part of y_R that comes
// from the tile pair of block rows R and S, so the final sum over S runs in a
// fixed order and the result is bitwise reproducible.
#pragma once

#include "bca_internal.h"

namespace bca {

typedef double symv_d2 __attribute__((ext_vector_type(2)));

// Lane exchanges of gfx950: after swap32(a, b) lanes 32-63 of a and lanes 0-31 of
// b have traded places; after swap16(a, b) the odd 16-lane rows of a and the even
// rows of b have.  In both, a + b is then, in every lane, the lane's own value of
// one of the pair plus its partner's (lane ^ 32, lane ^ 16) value of the same one:
// of a where the lane's bit (5, 4) is clear, of b where it is set.
__device__ __forceinline__ void swap32(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ void swap16(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a),
                                                   (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a),
                                                   (unsigned)__double2hiint(b), false, false);
  a = __hiloint2double((int)hi[0], (int)lo[0]);
  b = __hiloint2double((int)hi[1], (int)lo[1]);
}

// tile: this tile's 4096 doubles; r: the block's right-hand sides (n_j x C,
// feature-major); ys: the block's slots, slot (R, S) at ys + (R T + S) 64 C;
// right-hand sides cb .. ce - 1 (all C when ce < 0).
// Lane l = 8 a + b holds rows 16 q + 2 a + h (q < 4, h < 2) and columns
// 8 b .. 8 b + 7 of the tile.  Row sums are reduced over the 8 lanes of equal a
// (DPP), column sums over the 8 lanes of equal b.  NTL: nontemporal tile loads,
// for tile sets far larger than the last-level cache (smaller ones are partly
// still cached from the previous product).
template <bool NTL = false>
__device__ __forceinline__ void symv_tile(const double* __restrict__ tile, const double* __restrict__ r,
                                          int nj, int C, int I, int J, int T, double* __restrict__ ys,
                                          int cb = 0, int ce = -1) {
  const int lane = threadIdx.x & 63;
  const int a = lane >> 3, b = lane & 7;
  const bool diag = I == J;
  // rows and columns past n_j (the block's last tile row and column) are zero in
  // the stored tile: their 16-row bands (loads q) and this lane's 8 columns are
  // not read when they lie wholly past it
  const int rows = I == T - 1 ? nj - PT * I : PT;
  const bool cols = 8 * b < (J == T - 1 ? nj - PT * J : PT);
  symv_d2 p[4][8];
  const symv_d2* tp = reinterpret_cast<const symv_d2*>(tile) + lane;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (16 * q < rows && cols) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if constexpr (NTL)
          p[q][k] = __builtin_nontemporal_load(tp + (q * 8 + k) * 64);
        else
          p[q][k] = tp[(q * 8 + k) * 64];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) p[q][k] = symv_d2{0.0, 0.0};
    }
  }
  const int colJ = PT * J + 8 * b, rowI = PT * I + 2 * a;
  if (ce < 0) ce = C;
  for (int c = cb; c < ce; ++c) {
    // indices past n_j are clamped: the tile is zero there
    double rj[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) rj[e] = r[(int64_t)min(colJ + e, nj - 1) * C + c];
    double rs[8], cs[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) cs[e] = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double s = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          s += p[q][4 * h + v][0] * rj[2 * v];
          s += p[q][4 * h + v][1] * rj[2 * v + 1];
        }
        rs[2 * q + h] = s;
      }
      if (!diag) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const double ri = r[(int64_t)min(rowI + 16 * q + h, nj - 1) * C + c];
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            cs[2 * v] += p[q][4 * h + v][0] * ri;
            cs[2 * v + 1] += p[q][4 * h + v][1] * ri;
          }
        }
      }
    }
    // row sums: xor 1, xor 2, then the mirrored half of the 8-lane group
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      rs[e] += dpp_f64<0xB1>(rs[e]);
      rs[e] += dpp_f64<0x4E>(rs[e]);
      rs[e] += dpp_f64<0x141>(rs[e]);
    }
    // lane (a, b) writes row 16 (b / 2) + 2 a + b % 2, i.e. rs[b]
    double rv = rs[0];
#pragma unroll
    for (int e = 1; e < 8; ++e) rv = b == e ? rs[e] : rv;
    const int row = 16 * (b >> 1) + 2 * a + (b & 1);
    ys[(((int64_t)I * T + J) * PT + row) * C + c] = rv;
    if (!diag) {
      // column sums over a: xor 8 (rotate by 8 inside each row of 16 lanes), 16, 32
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        cs[e] += dpp_f64<0x128>(cs[e]);
        // + the lane ^ 16, then the lane ^ 32 value (lane swaps, not LDS permutes)
        double t = cs[e];
        swap16(cs[e], t);
        cs[e] = cs[e] + t;
        t = cs[e];
        swap32(cs[e], t);
        cs[e] = cs[e] + t;
      }
      // lane (a, b) writes column 8 b + a, i.e. cs[a]
      double cv = cs[0];
#pragma unroll
      for (int e = 1; e < 8; ++e) cv = a == e ? cs[e] : cv;
      ys[(((int64_t)J * T + I) * PT + 8 * b + a) * C + c] = cv;
    }
  }
}

// y_i = sum over S of slot (i / 64, S) entry i % 64, S = 0 .. T - 1 in order.
__device__ __forceinline__ double symv_gather(const double* __restrict__ ys, int i, int c, int C, int T) {
  const double* p = ys + ((int64_t)(i >> 6) * T * PT + (i & 63)) * C + c;
  double y0 = 0.0, y1 = 0.0;
  int S = 0;
  for (; S + 2 <= T; S += 2) {
    y0 += p[(int64_t)S * PT * C];
    y1 += p[(int64_t)(S + 1) * PT * C];
  }
  if (S < T) y0 += p[(int64_t)S * PT * C];
  return y0 + y1;
}

}  // namespace bca
