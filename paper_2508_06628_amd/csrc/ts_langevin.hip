// Langevin (NVT) dynamics over the whole batch: BAOAB splitting with one force evaluation per
// step; the normals come from Philox4x32-10, a counter-based generator, so that every atom and
// step has its own reproducible draw without generator state in memory.  Batches whose systems fit
// in LDS run the fused step kernel (the O step in its drift); others run the per-atom kernels below
// around the general force kernel.
#include <string>

#include "ts_forces.h"
#include "ts_graph.h"
#include "ts_neighbor.h"
#include "ts_rng.h"
#include "ts_step.h"

namespace ts {

// B A O A of step k of the call: v += dt/2 a F/m; r += dt/2 v; v = c1 v + c2 sqrt(a kT_s / m) xi;
// r += dt/2 v.  From the second step of a call on, the closing B of the previous step (the same
// force) is applied first, as a separate half kick.
template <typename T>
__global__ void k_lang_baoa(int64_t n, int64_t st, const int32_t *__restrict__ sys_idx, double *__restrict__ pos,
                            double *__restrict__ vel, const T *__restrict__ F, const double *__restrict__ mass,
                            const double *__restrict__ kT, double half_dt, double accel, double c1, double c2,
                            uint32_t key0, uint32_t key1, const uint64_t *__restrict__ rng_step, int k) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = mass ? accel / mass[i] : accel;
  const double sd = c2 * sqrt(kT[sys_idx[i]] * sc);
  double z[3];
  atom_normals((uint64_t)i, *rng_step + (uint64_t)k, key0, key1, z);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double kick = half_dt * (double)F[c * st + i];
    double v = vel[c * st + i];
    if (k > 0) v = fma(kick, sc, v);
    v = fma(kick, sc, v);
    double r = fma(half_dt, v, pos[c * st + i]);
    v = fma(c1, v, sd * z[c]);
    r = fma(half_dt, v, r);
    vel[c * st + i] = v;
    pos[c * st + i] = r;
  }
}

// the closing B (v += dt/2 a F/m) and the counter advance by the call's n_steps
template <typename T>
__global__ void k_lang_b(int64_t n, int64_t st, double *__restrict__ vel, const T *__restrict__ F,
                         const double *__restrict__ mass, double half_dt, double accel, uint64_t *__restrict__ rng_step,
                         int n_steps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) *rng_step += (uint64_t)n_steps;  // read by earlier launches only
  if (i >= n) return;
  const double sc = mass ? accel / mass[i] : accel;
#pragma unroll
  for (int c = 0; c < 3; ++c) vel[c * st + i] = fma(half_dt * (double)F[c * st + i], sc, vel[c * st + i]);
}

template <typename T>
static int langevin_sequence(const ts_batch *b, ts_neighbor_list *nl, const PairTable &tab, int prec, double dt,
                             double accel, double gamma, const double *kT, uint64_t seed, uint64_t *rng_step,
                             int n_steps, void *force, int64_t max_atoms, hipStream_t st) {
  const int64_t n = b->n_atoms, s_ = stride_of(b);
  const dim3 g((unsigned)ceil_div(n > 0 ? n : 1, 256));
  const double c1 = std::exp(-gamma * dt), c2 = std::sqrt(1.0 - c1 * c1);
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  const T *F = static_cast<const T *>(force);
  if (n_steps >= 1 && n > 0 && max_atoms <= kLdsMaxAtoms && !nl->half && fused_enabled()) {
    const LangParams lp{kT, c1, c2, key0, key1, rng_step};
    return nve_fused_sequence(b, nl, tab, prec, dt, accel, n_steps, force, nullptr, nullptr, nullptr, max_atoms, st,
                              nullptr, &lp);
  }
  for (int k = 0; k < n_steps; ++k) {
    if (n > 0) {
      hipLaunchKernelGGL(k_lang_baoa<T>, g, dim3(256), 0, st, n, s_, b->system_idx, b->pos, b->vel, F, b->mass, kT,
                         0.5 * dt, accel, c1, c2, key0, key1, rng_step, k);
      TS_LAUNCH_CHECK();
    }
    int rc = nl_update(b, nl, 0, max_atoms, st);
    if (rc != TS_OK) return rc;
    rc = launch_forces(make_force_args(b, nl, force, nullptr, nullptr, nullptr), b->n_systems, tab, prec, false, st);
    if (rc != TS_OK) return rc;
  }
  if (n_steps > 0) {
    hipLaunchKernelGGL(k_lang_b<T>, g, dim3(256), 0, st, n, s_, b->vel, F, b->mass, 0.5 * dt, accel, rng_step,
                       n_steps);
    TS_LAUNCH_CHECK();
  }
  return TS_OK;
}

}  // namespace ts

extern "C" int ts_langevin_step(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp, double dt,
                                double accel, double gamma, const double *kT, uint64_t seed, uint64_t *rng_step,
                                int32_t n_steps, void *force, int32_t use_graph, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, true);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(force != nullptr && kT != nullptr && rng_step != nullptr);
  TS_CHECK_ARG(std::isfinite(dt) && dt > 0.0 && std::isfinite(accel) && accel > 0.0 && n_steps >= 0);
  TS_CHECK_ARG(std::isfinite(gamma) && gamma >= 0.0 && batch->n_atoms < ((int64_t)1 << 32));
  if (n_steps == 0) return TS_OK;  // nothing to advance, the counter included
  std::string key("langevin");
  ts::key_add(key, *batch);
  ts::key_add(key, *nl);
  ts::key_add(key, *pp);
  ts::key_add(key, dt);
  ts::key_add(key, accel);
  ts::key_add(key, gamma);
  ts::key_add(key, kT);
  ts::key_add(key, seed);
  ts::key_add(key, rng_step);
  ts::key_add(key, n_steps);
  ts::key_add(key, max_atoms);
  ts::key_add(key, force);
  ts::key_add(key, ts::fused_enabled());
  ts::key_add(key, ts::defer_pre_factor());
  const ts::PairTable tab = ts::make_table(pp);
  return ts::run_graph_cached(use_graph != 0, key, ts::as_stream(stream), [&](hipStream_t s) {
    if (pp->prec == TS_PAIR_F32)
      return ts::langevin_sequence<float>(batch, nl, tab, pp->prec, dt, accel, gamma, kT, seed, rng_step, n_steps,
                                          force, max_atoms, s);
    return ts::langevin_sequence<double>(batch, nl, tab, pp->prec, dt, accel, gamma, kT, seed, rng_step, n_steps,
                                         force, max_atoms, s);
  });
}
