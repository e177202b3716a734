/*
 * Seeded synthetic inputs for the sparse-learning workloads (sample-partitioned
 * data matrices, planted sparse models, targets and labels).
 *
 * This file holds no arithmetic of the fitting method itself: it only draws
 * random numbers and applies the data recipes (i.i.d. or AR(1) Gaussian rows,
 * per-partition column normalisation, rounding to storage precisions, planted
 * targets).  Both the FP64 reference implementation and the GPU library are fed
 * from here.
 *
 * Random numbers come from Philox4x32-10, the counter-based generator of
 * Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as 1, 2, 3"
 * (SC 2011), written here from its published definition: ten rounds of
 *   (hi0,lo0) = M0 * c0,  (hi1,lo1) = M1 * c2,
 *   c' = (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
 * with the key bumped by the Weyl constants (W0, W1) between rounds.
 * Every value is addressed by (seed, stream, row, column), so any row can be
 * regenerated on its own.  Normals use the Box-Muller transform.
 */
#include <math.h>
#include <stdlib.h>
#include <stdint.h>
#include <string.h>

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

void bcd_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c0 = hi1 ^ c1 ^ k0;
    c1 = lo1;
    c2 = hi0 ^ c3 ^ k1;
    c3 = lo0;
    k0 += PHILOX_W0;
    k1 += PHILOX_W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Four words for (seed, stream, row, group-of-four-columns q). */
static inline void words4(uint64_t seed, uint32_t stream, uint64_t row, uint32_t q, uint32_t w[4]) {
  uint32_t ctr[4] = {q, (uint32_t)row, (uint32_t)(row >> 32), stream};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  bcd_philox4x32_10(ctr, key, w);
}

/* Uniform on the open interval (0, 1). */
static inline double u01(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

static const double TWO_PI = 6.283185307179586476925286766559;

/* Four standard normals from one Philox call: Box-Muller on (w0,w1) and (w2,w3). */
static inline void normals4(uint64_t seed, uint32_t stream, uint64_t row, uint32_t q, double z[4]) {
  uint32_t w[4];
  words4(seed, stream, row, q, w);
  for (int h = 0; h < 2; ++h) {
    double r = sqrt(-2.0 * log(u01(w[2 * h])));
    double th = TWO_PI * u01(w[2 * h + 1]);
    z[2 * h] = r * cos(th);
    z[2 * h + 1] = r * sin(th);
  }
}

/* out[r*ld + c] = N(0,1) draw at (seed, stream, row0 + r, c), c < n. */
void bcd_normal_matrix(uint64_t seed, uint32_t stream, int64_t m, int64_t n, int64_t row0,
                       double* out, int64_t ld) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r) {
    double* o = out + r * ld;
    for (int64_t q = 0; q * 4 < n; ++q) {
      double z[4];
      normals4(seed, stream, (uint64_t)(row0 + r), (uint32_t)q, z);
      for (int t = 0; t < 4 && q * 4 + t < n; ++t) o[q * 4 + t] = z[t];
    }
  }
}

/* out[k] = U(0,1) draw at (seed, stream, row, k0 + k). */
void bcd_uniform_vector(uint64_t seed, uint32_t stream, uint64_t row, int64_t k0, int64_t n,
                        double* out) {
#pragma omp parallel for schedule(static) if (n > 65536)
  for (int64_t k = 0; k < n; ++k) {
    uint32_t w[4];
    int64_t g = k0 + k;
    words4(seed, stream, row, (uint32_t)(g / 4), w);
    out[k] = u01(w[g % 4]);
  }
}

/* out[k] = N(0,1) draw at (seed, stream, row, k0 + k). */
void bcd_normal_vector(uint64_t seed, uint32_t stream, uint64_t row, int64_t k0, int64_t n,
                       double* out) {
#pragma omp parallel for schedule(static) if (n > 65536)
  for (int64_t k = 0; k < n; ++k) {
    double z[4];
    int64_t g = k0 + k;
    normals4(seed, stream, row, (uint32_t)(g / 4), z);
    out[k] = z[g % 4];
  }
}

/* AR(1) along each row, in place: a_0 = g_0, a_l = rho a_{l-1} + sqrt(1 - rho^2) g_l.
 * With i.i.d. N(0,1) input this gives rows with covariance rho^|i-j|. */
void bcd_ar1_rows(double* A, int64_t m, int64_t n, int64_t ld, double rho) {
  const double c = sqrt(1.0 - rho * rho);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r) {
    double* a = A + r * ld;
    for (int64_t l = 1; l < n; ++l) a[l] = rho * a[l - 1] + c * a[l];
  }
}

/* Scale every column of an m x n block to unit Euclidean norm (FP64 sums). */
void bcd_normalize_columns(double* A, int64_t m, int64_t n, int64_t ld) {
#pragma omp parallel for schedule(static)
  for (int64_t c0 = 0; c0 < n; c0 += 64) {
    int64_t c1 = c0 + 64 < n ? c0 + 64 : n;
    double ss[64];
    for (int64_t c = c0; c < c1; ++c) ss[c - c0] = 0.0;
    for (int64_t r = 0; r < m; ++r)
      for (int64_t c = c0; c < c1; ++c) ss[c - c0] += A[r * ld + c] * A[r * ld + c];
    for (int64_t c = c0; c < c1; ++c) ss[c - c0] = ss[c - c0] > 0 ? 1.0 / sqrt(ss[c - c0]) : 0.0;
    for (int64_t r = 0; r < m; ++r)
      for (int64_t c = c0; c < c1; ++c) A[r * ld + c] *= ss[c - c0];
  }
}

/* Round to FP32 (round-to-nearest-even by the host FPU), dense m x n. */
void bcd_to_f32(const double* in, int64_t m, int64_t n, int64_t ld_in, float* out, int64_t ld_out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int64_t c = 0; c < n; ++c) out[r * ld_out + c] = (float)in[r * ld_in + c];
}

/* FP32 -> BF16 bit pattern, round to nearest even (finite inputs). */
static inline uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return (uint16_t)(u >> 16);
}

void bcd_f32_to_bf16(const float* in, int64_t m, int64_t n, int64_t ld_in, uint16_t* out,
                     int64_t ld_out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int64_t c = 0; c < n; ++c) out[r * ld_out + c] = f32_to_bf16_rne(in[r * ld_in + c]);
}

/* Gaussian block straight to its storage precisions, without an FP64 copy:
 * out32[r*ld + c] = fp32(z(r, c) * s_c) and, if outbf is given, outbf = bf16 RNE of
 * that FP32 value, with z the N(0,1) draw at (seed, stream, row0 + r, c).
 * With normalize set, s_c = 1/||z(., c)||_2 (FP64 sums, column by column over
 * fixed 256-row chunks whose partial sums are added in chunk order, so the
 * result does not depend on the thread count); otherwise s_c = 1.  The rows are
 * drawn twice (once for the norms, once for the output), which the counter-based
 * generator makes exact. */
void bcd_gaussian_block(uint64_t seed, uint32_t stream, int64_t m, int64_t n, int64_t row0,
                        int normalize, float* out32, uint16_t* outbf, int64_t ld) {
  const int64_t CH = 256;
  const int64_t nch = (m + CH - 1) / CH;
  const int64_t nq = (n + 3) / 4;
  double* scale = (double*)malloc(sizeof(double) * (size_t)(nq * 4));
  for (int64_t c = 0; c < nq * 4; ++c) scale[c] = 1.0;
  if (normalize) {
    double* part = (double*)calloc((size_t)(nch * nq * 4), sizeof(double));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nch; ++k) {
      double* ps = part + k * nq * 4;
      const int64_t r1 = (k + 1) * CH < m ? (k + 1) * CH : m;
      for (int64_t r = k * CH; r < r1; ++r)
        for (int64_t q = 0; q < nq; ++q) {
          double z[4];
          normals4(seed, stream, (uint64_t)(row0 + r), (uint32_t)q, z);
          for (int t = 0; t < 4; ++t) ps[q * 4 + t] += z[t] * z[t];
        }
    }
    for (int64_t c = 0; c < n; ++c) {
      double ss = 0.0;
      for (int64_t k = 0; k < nch; ++k) ss += part[k * nq * 4 + c];
      scale[c] = ss > 0 ? 1.0 / sqrt(ss) : 0.0;
    }
    free(part);
  }
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r) {
    float* o = out32 + r * ld;
    uint16_t* ob = outbf ? outbf + r * ld : 0;
    for (int64_t q = 0; q < nq; ++q) {
      double z[4];
      normals4(seed, stream, (uint64_t)(row0 + r), (uint32_t)q, z);
      for (int t = 0; t < 4 && q * 4 + t < n; ++t) {
        const float f = (float)(z[t] * scale[q * 4 + t]);
        o[q * 4 + t] = f;
        if (ob) ob[q * 4 + t] = f32_to_bf16_rne(f);
      }
    }
  }
  free(scale);
}

void bcd_bf16_to_f64(const uint16_t* in, int64_t m, int64_t n, int64_t ld_in, double* out,
                     int64_t ld_out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r)
    for (int64_t c = 0; c < n; ++c) {
      uint32_t u = (uint32_t)in[r * ld_in + c] << 16;
      float f;
      memcpy(&f, &u, 4);
      out[r * ld_out + c] = (double)f;
    }
}

/* Planted linear predictor of a sparse model: out[r] = sum_t A[r, idx[t]] * val[t]
 * (FP32 storage of A read as exact values, FP64 sums). */
void bcd_sparse_predict_f32(const float* A, int64_t m, int64_t ld, const int64_t* idx,
                            const double* val, int64_t k, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r) {
    double s = 0.0;
    for (int64_t t = 0; t < k; ++t) s += (double)A[r * ld + idx[t]] * val[t];
    out[r] = s;
  }
}

void bcd_sparse_predict_f64(const double* A, int64_t m, int64_t ld, const int64_t* idx,
                            const double* val, int64_t k, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < m; ++r) {
    double s = 0.0;
    for (int64_t t = 0; t < k; ++t) s += A[r * ld + idx[t]] * val[t];
    out[r] = s;
  }
}
