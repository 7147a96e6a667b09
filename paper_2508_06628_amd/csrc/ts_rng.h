// Counter-based normal numbers for the Langevin O step: Philox4x32-10 (Salmon, Moraes, Dror and
// Shaw, SC 2011) keyed by the run's 64-bit seed, counter (atom, step low word, step high word, 0),
// and the Box-Muller transform of its four outputs.  Every atom and step has its own draw and no
// generator state lives in memory.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace ts {

// Ten rounds of Philox4x32 on the counter c with the key (k0, k1).
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;  // round multipliers
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;  // key increments
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(kM0, c[0]), lo0 = kM0 * c[0];
    const uint32_t hi1 = __umulhi(kM1, c[2]), lo1 = kM1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += kW0;
    k1 += kW1;
  }
}

// Standard normals of atom i at step t: Box-Muller on the four uniforms (x + 1/2) 2^-32, giving
// (sqrt(-2 ln u0) cos 2 pi u1, sqrt(-2 ln u0) sin 2 pi u1, sqrt(-2 ln u2) cos 2 pi u3).
__device__ inline void atom_normals(uint64_t i, uint64_t t, uint32_t key0, uint32_t key1, double z[3]) {
  uint32_t c[4] = {(uint32_t)i, (uint32_t)t, (uint32_t)(t >> 32), 0u};
  philox4x32_10(c, key0, key1);
  double u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = ((double)c[k] + 0.5) * 0x1p-32;
  // cos(2 pi u) = cospi(2u): 2u = (2x + 1) 2^-32 is exact and the reduction of cospi is exact
  const double r0 = sqrt(-2.0 * log(u[0])), r2 = sqrt(-2.0 * log(u[2]));
  z[0] = r0 * cospi(2.0 * u[1]);
  z[1] = r0 * sinpi(2.0 * u[1]);
  z[2] = r2 * cospi(2.0 * u[3]);
}

// Parameters of the O step v = c1 v + c2 sqrt(kT_s a / m) xi, with c1 = exp(-gamma dt) and
// c2 = sqrt(1 - c1^2); the normals of step k of a call use the counter *rng_step + k, and the last
// launch of the call advances *rng_step by the call's step count.
struct LangParams {
  const double *kT;    // [n_systems] (energy units)
  double c1, c2;
  uint32_t key0, key1;  // seed low and high words
  uint64_t *rng_step;
};

}  // namespace ts
