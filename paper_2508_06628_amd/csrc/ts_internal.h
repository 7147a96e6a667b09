// Internal helpers shared by the HIP translation units of the library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>

#include "ts_api.h"

namespace ts {

constexpr int kWave = 64;

// ----------------------------------------------------------------------------- host helpers

#define TS_CHECK_ARG(cond)      \
  do {                          \
    if (!(cond)) return TS_E_INVALID; \
  } while (0)

#define TS_HIP(expr)                           \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return TS_E_HIP;     \
  } while (0)

#define TS_LAUNCH_CHECK()                        \
  do {                                           \
    if (hipPeekAtLastError() != hipSuccess) {    \
      (void)hipGetLastError();                   \
      return TS_E_HIP;                           \
    }                                            \
  } while (0)

inline int64_t stride_of(const ts_batch *b) { return b->stride > 0 ? b->stride : b->n_atoms; }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

inline hipStream_t as_stream(ts_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// Host-side validation of a batch; fills max_atoms (largest system).
int validate_batch(const ts_batch *b, bool need_vel, int64_t *max_atoms);
int validate_params(const ts_pair_params *pp);
int validate_list(const ts_batch *b, const ts_neighbor_list *nl, bool need_workspace = true);

// Compute units of the current device (cached per device; 256 when the query fails) and the LDS
// of one CU in bytes.
int device_cus();
constexpr int64_t kLdsBytes = 160 * 1024;

// ----------------------------------------------------------------------------- list entries

// List entry: j_local in bits 15..31 and each image component S_k + 16 in a 5-bit field, so that the
// unsigned order of entries is the lexicographic order of (j_local, S0, S1, S2).
__host__ __device__ inline uint32_t pack_entry(int j_local, int s0, int s1, int s2) {
  return ((uint32_t)j_local << 15) | ((uint32_t)(s0 + 16) << 10) | ((uint32_t)(s1 + 16) << 5) | (uint32_t)(s2 + 16);
}
__device__ inline int entry_j(uint32_t e) { return (int)(e >> 15); }
// The image shifts as exact doubles without a conversion instruction: for a field value u < 2^20
// the bit pattern 0x43300000:u is the double 2^52 + u, so S = u - 16 = that - (2^52 + 16).
__device__ inline double entry_sd(uint32_t field) {
  return __hiloint2double(0x43300000, (int)field) - 4503599627370512.0;
}
__device__ inline double entry_s0d(uint32_t e) { return entry_sd((e >> 10) & 31u); }
__device__ inline double entry_s1d(uint32_t e) { return entry_sd((e >> 5) & 31u); }
__device__ inline double entry_s2d(uint32_t e) { return entry_sd(e & 31u); }
__device__ inline int entry_s0(uint32_t e) { return (int)((e >> 10) & 31u) - 16; }
__device__ inline int entry_s1(uint32_t e) { return (int)((e >> 5) & 31u) - 16; }
__device__ inline int entry_s2(uint32_t e) { return (int)(e & 31u) - 16; }

// Row layout: entries come in blocks of kRowBlock per atom, block b of atom i at
// nbr[(b * stride + i) * kRowBlock ...] -- the kRowBlock lanes that share an atom read one
// contiguous 32-byte segment, and a wavefront writing one row writes contiguous segments.
constexpr int kRowBlock = 8;
__host__ __device__ inline int64_t row_index(int k, int64_t i, int64_t st) {
  return ((int64_t)(k >> 3) * st + i) * kRowBlock + (k & (kRowBlock - 1));
}

// Pair vector component d_c = (r_j,c - r_i,c) + S @ cell (column c), written with explicit fused
// multiply-adds so that every kernel evaluates it, and |d|^2, with the same rounding.
__device__ inline double shift_comp(double dr, double S0, double S1, double S2, double h0c, double h1c, double h2c) {
  return dr + fma(S2, h2c, fma(S1, h1c, S0 * h0c));
}
// Workgroups go to the 8 XCDs of the chip round-robin by workgroup number.  The renumbering
// b -> (b mod 8) * (grid / 8) + b / 8 hands XCD x the consecutive range [x grid/8, (x+1) grid/8), so
// workgroups that share data (those of one system) sit behind one L2.  It is a bijection of
// [0, grid) when grid is a multiple of 8.
constexpr int kXcds = 8;
__device__ inline int64_t xcd_order(int64_t b, int64_t grid) {
  return (b % kXcds) * (grid / kXcds) + b / kXcds;
}

__device__ inline double norm2(double dx, double dy, double dz) { return fma(dz, dz, fma(dy, dy, dx * dx)); }

// ----------------------------------------------------------------------------- pair tables

// Per species-pair coefficients prepared on the host (both precisions), passed by value.
//   LJ:    a = 4 eps sigma^12, b = 4 eps sigma^6          phi = a/r^12 - b/r^6
//   Morse: a = D, b = alpha, c = r0
//   SS:    a = eps, b = sigma_ij, c = 1/sigma_ij
//   shift: phi(r_c) when the energy is shifted (always for the shifted-force kinds), else 0.
//   Shifted-force kinds: fs = phi'(r_c), rc = r_c, dfs[k] = d phi'(r_c) / d raw[k].
struct PairCoef {
  double a, b, c, shift;
  double sig2;  // sigma_ij^2 (soft sphere mask), else +inf
  double raw[3];  // the caller's parameter triple (for parameter derivatives)
  double fs, rc;
  double dfs[3];
};
struct PairTable {
  PairCoef c[TS_MAX_SPECIES * TS_MAX_SPECIES];
  double cut2;
  int n_species;
  int kind;
};

PairTable make_table(const ts_pair_params *pp);

// The plain form a shifted-force kind truncates.
template <int KIND>
struct BaseKind {
  static constexpr int value = KIND == TS_LJ_SF ? TS_LJ : (KIND == TS_MORSE_SF ? TS_MORSE : KIND);
};

// Calls f(std::integral_constant<int, KIND>{}) for the run-time kind (one instantiation per kind).
template <typename F>
inline void with_kind(int kind, F &&f) {
  switch (kind) {
    case TS_LJ: f(std::integral_constant<int, TS_LJ>{}); break;
    case TS_MORSE: f(std::integral_constant<int, TS_MORSE>{}); break;
    case TS_SOFT_SPHERE: f(std::integral_constant<int, TS_SOFT_SPHERE>{}); break;
    case TS_LJ_SF: f(std::integral_constant<int, TS_LJ_SF>{}); break;
    default: f(std::integral_constant<int, TS_MORSE_SF>{}); break;
  }
}

// Visit the row entries k = lane, lane + TL, lane + 2 TL, ... (k < nn) of atom i in increasing k,
// with the loads of the next U entries in flight while the current U are processed (the entry
// load heads a dependent chain, so issuing it early hides most of its latency).  The visiting
// order is the plain loop's, so sums over the row round identically.
template <int TL, typename F>
__device__ inline void for_row(const uint32_t *__restrict__ nbr, int64_t st, int64_t i, int nn, int lane, F &&f) {
  constexpr int U = 4;
  uint32_t cur[U], nxt[U];
  // past the end of the row a lane reloads an entry of the row's first block (always allocated):
  // the loads carry no branch, so they stay in flight while the previous entries are evaluated
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int kk = lane + u * TL;
    cur[u] = nbr[row_index(kk < nn ? kk : (kk & (kRowBlock - 1)), i, st)];
  }
  for (int k = lane; k < nn; k += U * TL) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k + (U + u) * TL;
      nxt[u] = nbr[row_index(kk < nn ? kk : (kk & (kRowBlock - 1)), i, st)];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k + u * TL < nn) f(cur[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
  }
}

// Visit the same entries as for_row, U visits at a time: f(ent, ok) receives U consecutive entries
// of the lane (ok[u] false past the end of the row, where ent[u] is unspecified) and evaluates them without
// branches between them, so the U dependent chains can be interleaved.  Results must be combined
// in u order to sum like the plain loop.
template <int TL, int U, typename F>
__device__ inline void for_row_batched(const uint32_t *__restrict__ nbr, int64_t st, int64_t i, int nn, int lane,
                                       F &&f, int k_begin = 0) {
  uint32_t cur[U], nxt[U];
  if constexpr ((U * TL) % kRowBlock == 0) {
    // A batch advances every visit u by whole row blocks, so each visit keeps its position in the
    // block and its byte offset grows by a fixed amount: 32-bit offsets from the list base (the list
    // is below 4 GiB, checked by the host) replace the 64-bit index arithmetic of row_index.  Past
    // the end of the row a visit reads the same position of the row's last block (allocated:
    // n_nbr <= max_nbr), so the loads carry no branch and stay in flight during the evaluation.
    const char *base = reinterpret_cast<const char *>(nbr);
    const uint32_t s32 = (uint32_t)st, i32 = (uint32_t)i;
    const uint32_t inc = (uint32_t)(U * TL / kRowBlock) * s32 * (uint32_t)(kRowBlock * 4);
    const uint32_t last = (uint32_t)(nn > 0 ? (nn - 1) / kRowBlock : 0);
    uint32_t off[U], lim[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t kk = (uint32_t)(k_begin + lane + u * TL), w = (kk % kRowBlock) * 4u;
      off[u] = ((kk / kRowBlock) * s32 + i32) * (uint32_t)(kRowBlock * 4) + w;
      lim[u] = (last * s32 + i32) * (uint32_t)(kRowBlock * 4) + w;
      cur[u] = *reinterpret_cast<const uint32_t *>(base + (off[u] < lim[u] ? off[u] : lim[u]));
    }
    for (int k = k_begin + lane; k < nn; k += U * TL) {
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        off[u] += inc;
        nxt[u] = *reinterpret_cast<const uint32_t *>(base + (off[u] < lim[u] ? off[u] : lim[u]));
        ok[u] = k + u * TL < nn;
      }
      f(cur, ok);
#pragma unroll
      for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
  } else {
    // unconditional loads as in for_row (entries past the end are masked by ok)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int kk = k_begin + lane + u * TL;
      cur[u] = nbr[row_index(kk < nn ? kk : (kk & (kRowBlock - 1)), i, st)];
    }
    for (int k = k_begin + lane; k < nn; k += U * TL) {
      bool ok[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int kk = k + (U + u) * TL;
        nxt[u] = nbr[row_index(kk < nn ? kk : (kk & (kRowBlock - 1)), i, st)];
        ok[u] = k + u * TL < nn;
      }
      f(cur, ok);
#pragma unroll
      for (int u = 0; u < U; ++u) cur[u] = nxt[u];
    }
  }
}

// Copy the species-pair table into LDS.  Every kernel that takes a PairTable takes it as its FIRST
// argument, so the table's kernarg copy starts at the kernarg segment base; reading it through that
// pointer allows a run-time index (one lane per entry, all loads issued together), whereas a
// by-value parameter indexed at run time gets a private per-lane copy and a static-index loop
// issues one dependent kernarg load per entry.  Must be reached by every thread of the workgroup.
__device__ inline void table_to_lds(PairCoef *dst) {
  const PairTable *t = (const PairTable *)__builtin_amdgcn_kernarg_segment_ptr();
  if (threadIdx.x < TS_MAX_SPECIES * TS_MAX_SPECIES) dst[threadIdx.x] = t->c[threadIdx.x];
  __syncthreads();
}

// Pair function: returns g = phi'(r)/r and (optionally) phi(r) - shift.  d is the pair vector in
// the pair precision, r2 its squared norm (float64) for masks and the soft-sphere overlap.
template <int KIND, typename T>
__device__ inline T pair_g(const PairCoef &pc, T r2t, double r2, T *phi, bool want_phi);

template <>
__device__ inline float pair_g<TS_LJ, float>(const PairCoef &pc, float r2t, double, float *phi, bool want_phi) {
  const float ir2 = __builtin_amdgcn_rcpf(r2t);  // hardware reciprocal, 1 ulp
  const float ir6 = ir2 * ir2 * ir2;
  const float a = (float)pc.a, b = (float)pc.b;
  if (want_phi) *phi = ir6 * (a * ir6 - b) - (float)pc.shift;
  return ir2 * ir6 * (6.0f * b - 12.0f * a * ir6);
}
template <>
__device__ inline double pair_g<TS_LJ, double>(const PairCoef &pc, double r2t, double, double *phi, bool want_phi) {
  const double ir2 = 1.0 / r2t;
  const double ir6 = ir2 * ir2 * ir2;
  if (want_phi) *phi = ir6 * (pc.a * ir6 - pc.b) - pc.shift;
  return ir2 * ir6 * (6.0 * pc.b - 12.0 * pc.a * ir6);
}
template <>
__device__ inline float pair_g<TS_MORSE, float>(const PairCoef &pc, float r2t, double, float *phi, bool want_phi) {
  const float r = sqrtf(r2t);
  const float x = expf(-(float)pc.b * (r - (float)pc.c));
  const float D = (float)pc.a;
  if (want_phi) *phi = D * (x * x - 2.0f * x) - (float)pc.shift;
  return 2.0f * (float)pc.b * D * (x - x * x) / r;
}
template <>
__device__ inline double pair_g<TS_MORSE, double>(const PairCoef &pc, double r2t, double, double *phi,
                                                  bool want_phi) {
  const double r = sqrt(r2t);
  const double x = exp(-pc.b * (r - pc.c));
  if (want_phi) *phi = pc.a * (x * x - 2.0 * x) - pc.shift;
  return 2.0 * pc.b * pc.a * (x - x * x) / r;
}
template <>
__device__ inline float pair_g<TS_SOFT_SPHERE, float>(const PairCoef &pc, float r2t, double r2, float *phi,
                                                      bool want_phi) {
  // overlap 1 - r/sigma in float64: it cancels catastrophically near contact
  const double r64 = sqrt(r2);
  const float u = (float)(1.0 - r64 * pc.c);
  const float eps = (float)pc.a;
  if (want_phi) *phi = 0.5f * eps * u * u;
  return -eps * (float)pc.c * u / (float)r64;
}
template <>
__device__ inline double pair_g<TS_SOFT_SPHERE, double>(const PairCoef &pc, double, double r2, double *phi,
                                                        bool want_phi) {
  const double r = sqrt(r2);
  const double u = 1.0 - r * pc.c;
  if (want_phi) *phi = 0.5 * pc.a * u * u;
  return -pc.a * pc.c * u / r;
}

// Shifted-force kinds: g_sf = g - phi'(r_c) / r and phi_sf = phi - phi(r_c) - (r - r_c) phi'(r_c)
// (the base form already subtracts shift = phi(r_c)).
template <int KIND, typename T>
__device__ inline T pair_g_sf(const PairCoef &pc, T r2t, double r2, T *phi, bool want_phi) {
  constexpr int B = BaseKind<KIND>::value;
  const T g = pair_g<B, T>(pc, r2t, r2, phi, want_phi);
  T ir;
  if constexpr (std::is_same<T, float>::value) ir = __builtin_amdgcn_rsqf(r2t);
  else ir = 1.0 / sqrt(r2t);
  if (want_phi) *phi -= (r2t * ir - (T)pc.rc) * (T)pc.fs;
  return g - (T)pc.fs * ir;
}
template <>
__device__ inline float pair_g<TS_LJ_SF, float>(const PairCoef &pc, float r2t, double r2, float *phi, bool want_phi) {
  return pair_g_sf<TS_LJ_SF, float>(pc, r2t, r2, phi, want_phi);
}
template <>
__device__ inline double pair_g<TS_LJ_SF, double>(const PairCoef &pc, double r2t, double r2, double *phi,
                                                  bool want_phi) {
  return pair_g_sf<TS_LJ_SF, double>(pc, r2t, r2, phi, want_phi);
}
template <>
__device__ inline float pair_g<TS_MORSE_SF, float>(const PairCoef &pc, float r2t, double r2, float *phi,
                                                   bool want_phi) {
  return pair_g_sf<TS_MORSE_SF, float>(pc, r2t, r2, phi, want_phi);
}
template <>
__device__ inline double pair_g<TS_MORSE_SF, double>(const PairCoef &pc, double r2t, double r2, double *phi,
                                                     bool want_phi) {
  return pair_g_sf<TS_MORSE_SF, double>(pc, r2t, r2, phi, want_phi);
}

// One pair's contribution to atom i: g = phi'(r)/r comes from the pair function (pair precision);
// it multiplies the float64 pair vector d = r_j - r_i + S h in float64 and the force sums in
// float64 (F_i += g d).  The virial variant also accumulates the six distinct entries of
// sum g d (x) d (xx yy zz xy xz yz).  Every force kernel uses these, so they agree bitwise.
__device__ inline void acc_force(double g, double dx, double dy, double dz, double &fx, double &fy, double &fz) {
  fx = fma(g, dx, fx);
  fy = fma(g, dy, fy);
  fz = fma(g, dz, fz);
}
__device__ inline void acc_virial(double g, double dx, double dy, double dz, double (&w)[6]) {
  const double gx = g * dx, gy = g * dy, gz = g * dz;
  w[0] = fma(gx, dx, w[0]);
  w[1] = fma(gy, dy, w[1]);
  w[2] = fma(gz, dz, w[2]);
  w[3] = fma(gx, dy, w[3]);
  w[4] = fma(gx, dz, w[4]);
  w[5] = fma(gy, dz, w[5]);
}

// Second-derivative data for the adjoint: returns g = phi'/r and h = phi''(r); all in T.
template <int KIND, typename T>
__device__ inline void pair_g_h(const PairCoef &pc, T r2t, double r2, T *g, T *h);

template <>
__device__ inline void pair_g_h<TS_LJ, float>(const PairCoef &pc, float r2t, double, float *g, float *h) {
  const float ir2 = 1.0f / r2t;
  const float ir6 = ir2 * ir2 * ir2;
  const float a = (float)pc.a, b = (float)pc.b;
  *g = ir2 * ir6 * (6.0f * b - 12.0f * a * ir6);
  *h = ir2 * ir6 * (156.0f * a * ir6 - 42.0f * b);
}
template <>
__device__ inline void pair_g_h<TS_LJ, double>(const PairCoef &pc, double r2t, double, double *g, double *h) {
  const double ir2 = 1.0 / r2t;
  const double ir6 = ir2 * ir2 * ir2;
  *g = ir2 * ir6 * (6.0 * pc.b - 12.0 * pc.a * ir6);
  *h = ir2 * ir6 * (156.0 * pc.a * ir6 - 42.0 * pc.b);
}
template <>
__device__ inline void pair_g_h<TS_MORSE, float>(const PairCoef &pc, float r2t, double, float *g, float *h) {
  const float r = sqrtf(r2t);
  const float al = (float)pc.b, D = (float)pc.a;
  const float x = expf(-al * (r - (float)pc.c));
  *g = 2.0f * al * D * (x - x * x) / r;
  *h = 2.0f * al * al * D * (2.0f * x * x - x);
}
template <>
__device__ inline void pair_g_h<TS_MORSE, double>(const PairCoef &pc, double r2t, double, double *g, double *h) {
  const double r = sqrt(r2t);
  const double x = exp(-pc.b * (r - pc.c));
  *g = 2.0 * pc.b * pc.a * (x - x * x) / r;
  *h = 2.0 * pc.b * pc.b * pc.a * (2.0 * x * x - x);
}
template <>
__device__ inline void pair_g_h<TS_SOFT_SPHERE, float>(const PairCoef &pc, float, double r2, float *g, float *h) {
  const double r64 = sqrt(r2);
  const float u = (float)(1.0 - r64 * pc.c);
  *g = -(float)pc.a * (float)pc.c * u / (float)r64;
  *h = (float)(pc.a * pc.c * pc.c);
}
template <>
__device__ inline void pair_g_h<TS_SOFT_SPHERE, double>(const PairCoef &pc, double, double r2, double *g,
                                                        double *h) {
  const double r = sqrt(r2);
  const double u = 1.0 - r * pc.c;
  *g = -pc.a * pc.c * u / r;
  *h = pc.a * pc.c * pc.c;
}
// Shifted-force kinds: phi_sf'' = phi'' and g_sf = g - phi'(r_c) / r.
template <int KIND, typename T>
__device__ inline void pair_g_h_sf(const PairCoef &pc, T r2t, double r2, T *g, T *h) {
  pair_g_h<BaseKind<KIND>::value, T>(pc, r2t, r2, g, h);
  *g -= (T)pc.fs / sqrt(r2t);
}
template <>
__device__ inline void pair_g_h<TS_LJ_SF, float>(const PairCoef &pc, float r2t, double r2, float *g, float *h) {
  pair_g_h_sf<TS_LJ_SF, float>(pc, r2t, r2, g, h);
}
template <>
__device__ inline void pair_g_h<TS_LJ_SF, double>(const PairCoef &pc, double r2t, double r2, double *g, double *h) {
  pair_g_h_sf<TS_LJ_SF, double>(pc, r2t, r2, g, h);
}
template <>
__device__ inline void pair_g_h<TS_MORSE_SF, float>(const PairCoef &pc, float r2t, double r2, float *g, float *h) {
  pair_g_h_sf<TS_MORSE_SF, float>(pc, r2t, r2, g, h);
}
template <>
__device__ inline void pair_g_h<TS_MORSE_SF, double>(const PairCoef &pc, double r2t, double r2, double *g,
                                                      double *h) {
  pair_g_h_sf<TS_MORSE_SF, double>(pc, r2t, r2, g, h);
}

// Derivatives of g = phi'/r with respect to the raw parameter triple (float64).  One division per
// pair (1/r^2 or 1/r); quotients of the parameters alone are loop invariants for a one-species
// table and are hoisted by the compiler.
template <int KIND>
__device__ inline void pair_dg_dparams(const PairCoef &pc, double r2, double out[3]);

template <>
__device__ inline void pair_dg_dparams<TS_LJ>(const PairCoef &pc, double r2, double out[3]) {
  // g = 24 eps / r^2 (s^6 - 2 s^12), s = sigma / r
  const double eps = pc.raw[0], sig = pc.raw[1];
  const double ir2 = 1.0 / r2;
  const double s2 = sig * sig * ir2;
  const double sr6 = s2 * s2 * s2;
  const double sr12 = sr6 * sr6;
  out[0] = 24.0 * ir2 * (sr6 - 2.0 * sr12);                    // dg/deps = g / eps
  out[1] = (24.0 * eps / sig) * ir2 * (6.0 * sr6 - 24.0 * sr12);  // dg/dsigma
  out[2] = 0.0;
}
template <>
__device__ inline void pair_dg_dparams<TS_MORSE>(const PairCoef &pc, double r2, double out[3]) {
  // g = 2 alpha D (x - x^2) / r, x = exp(-alpha (r - r0))
  const double D = pc.raw[0], al = pc.raw[1], r0 = pc.raw[2];
  const double r = sqrt(r2);
  const double ir = 1.0 / r;
  const double x = exp(-al * (r - r0));
  const double q = x - x * x, p = 1.0 - 2.0 * x;
  out[0] = 2.0 * al * q * ir;
  out[1] = (2.0 * D * q - 2.0 * al * D * p * (r - r0) * x) * ir;
  out[2] = 2.0 * al * al * D * p * x * ir;
}
template <>
__device__ inline void pair_dg_dparams<TS_SOFT_SPHERE>(const PairCoef &pc, double r2, double out[3]) {
  // g = -(eps / sigma) (1 - r / sigma) / r
  const double eps = pc.raw[0], sig = pc.raw[1];
  const double isig = 1.0 / sig;
  const double r = sqrt(r2);
  const double ir = 1.0 / r;
  const double u = 1.0 - r * isig;
  out[0] = -u * isig * ir;
  out[1] = eps * isig * isig * (ir - 2.0 * isig);
  out[2] = 0.0;
}
// Shifted-force kinds: d g_sf / d theta = d g / d theta - (d phi'(r_c) / d theta) / r.
template <>
__device__ inline void pair_dg_dparams<TS_LJ_SF>(const PairCoef &pc, double r2, double out[3]) {
  pair_dg_dparams<TS_LJ>(pc, r2, out);
  const double ir = 1.0 / sqrt(r2);
  out[0] -= pc.dfs[0] * ir;
  out[1] -= pc.dfs[1] * ir;
}
template <>
__device__ inline void pair_dg_dparams<TS_MORSE_SF>(const PairCoef &pc, double r2, double out[3]) {
  pair_dg_dparams<TS_MORSE>(pc, r2, out);
  const double ir = 1.0 / sqrt(r2);
  out[0] -= pc.dfs[0] * ir;
  out[1] -= pc.dfs[1] * ir;
  out[2] -= pc.dfs[2] * ir;
}

// ----------------------------------------------------------------------------- reductions

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Raise status word k to at least v.  Status words only grow, so the atomic is skipped when a
// coherent read already shows a value >= v: atomics on one address serialise in L2, and issuing
// one per atom costs microseconds per thousand atoms.
__device__ inline void status_raise(int64_t *status, int k, int64_t v) {
  if (v > __hip_atomic_load(&status[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    atomicMax((unsigned long long *)&status[k], (unsigned long long)v);
}

// Workgroup-level status update after a row build: the largest row length and the overflow /
// image-shift / non-finite flags of all threads go through LDS, then one thread raises the global
// words.  Must be reached by every thread of the workgroup.
__device__ inline void block_status(int64_t *status, int cnt, int max_nbr, bool shift_bad, bool nonfinite) {
  __shared__ int s_max, s_flags;
  if (threadIdx.x == 0) {
    s_max = 0;
    s_flags = 0;
  }
  __syncthreads();
  if (cnt > 0) atomicMax(&s_max, cnt);
  const int fl = (shift_bad ? 1 : 0) | (nonfinite ? 2 : 0);
  if (fl) atomicOr(&s_flags, fl);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_max > 0) status_raise(status, TS_STATUS_MAX_NBR, s_max);
    if (s_max > max_nbr) status_raise(status, TS_STATUS_OVERFLOW, 1);
    if (s_flags & 1) status_raise(status, TS_STATUS_SHIFT, 1);
    if (s_flags & 2) status_raise(status, TS_STATUS_NONFINITE, 1);
  }
}

// Add the NV per-lane values v[k] into out[s * out_stride + k].  Must be reached by every lane of
// the wavefront (convergent control flow).  One atomic per value and wavefront when all valid lanes
// share a system (the common case: systems are contiguous), one per lane otherwise.
template <int NV>
__device__ inline void add_by_system(double *out, int out_stride, int s, bool valid, const double (&v)[NV]) {
  const uint64_t act = __ballot(valid);
  if (act == 0) return;
  const int first = __ffsll((unsigned long long)act) - 1;
  const int s_first = __shfl(s, first, kWave);
  if (__all(!valid || s == s_first)) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const double t = wave_sum(valid ? v[k] : 0.0);
      if ((int)__lane_id() == first) atomicAdd(&out[(int64_t)s_first * out_stride + k], t);
    }
  } else if (valid) {
#pragma unroll
    for (int k = 0; k < NV; ++k) atomicAdd(&out[(int64_t)s * out_stride + k], v[k]);
  }
}

// Fill kernel (used instead of hipMemsetAsync so that calls remain safe inside captured graphs).
template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename T>
inline int fill_async(T *p, int64_t n, T v, hipStream_t st) {
  if (n <= 0 || p == nullptr) return TS_OK;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, p, n, v);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

}  // namespace ts
