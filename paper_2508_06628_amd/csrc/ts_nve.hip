// Velocity-Verlet NVE over the whole batch (the molecular-dynamics integrators of the paper's
// Abstract; every system advances in the same launches, Section 3), with the per-step neighbor
// validity test and rebuild on the device and an optional hipGraph of the whole step loop.
#include <cmath>
#include <cstdlib>
#include <string>

#include "ts_forces.h"
#include "ts_graph.h"
#include "ts_neighbor.h"
#include "ts_step.h"

namespace ts {

// TS_NVE_UNFUSED=1 selects the multi-kernel step (separate list update, force and kick launches)
// instead of the fused one; both compute the same trajectory up to rounding.
bool fused_enabled() {
  const char *e = std::getenv("TS_NVE_UNFUSED");
  return !(e && e[0] == '1');
}

double defer_pre_factor() {
  const char *e = std::getenv("TS_DEFER_PREFACTOR");
  if (!e || !e[0]) return 2.0;
  const double v = std::atof(e);
  return std::isfinite(v) && v >= 0.0 ? v : 2.0;
}

// v += (dt/2) a F / m ; r += dt v
template <typename T>
__global__ void k_vv_kick_drift(int64_t n, int64_t st, double *__restrict__ pos, double *__restrict__ vel,
                                const T *__restrict__ F, const double *__restrict__ mass, double half_dt,
                                double accel, double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = mass ? accel / mass[i] : accel;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double v = fma(half_dt * (double)F[c * st + i], sc, vel[c * st + i]);
    vel[c * st + i] = v;
    pos[c * st + i] = fma(dt, v, pos[c * st + i]);
  }
}

// v += (dt/2) a F / m
template <typename T>
__global__ void k_vv_kick(int64_t n, int64_t st, double *__restrict__ vel, const T *__restrict__ F,
                          const double *__restrict__ mass, double half_dt, double accel) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = mass ? accel / mass[i] : accel;
#pragma unroll
  for (int c = 0; c < 3; ++c) vel[c * st + i] = fma(half_dt * (double)F[c * st + i], sc, vel[c * st + i]);
}

// ekin[s] += 1/2 m |v|^2 / accel
__global__ void __launch_bounds__(256) k_kinetic(int64_t n, int64_t st, const int32_t *__restrict__ sys_idx,
                                                 const double *__restrict__ vel, const double *__restrict__ mass,
                                                 double half_inv_accel, double *__restrict__ ekin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < n;
  const int64_t ii = valid ? i : 0;
  const int s = valid ? sys_idx[ii] : 0;
  double k = 0.0;
  if (valid) {
    const double vx = vel[ii], vy = vel[st + ii], vz = vel[2 * st + ii];
    const double m = mass ? mass[ii] : 1.0;
    k = half_inv_accel * (m * (vx * vx + vy * vy + vz * vz));
  }
  const double kv[1] = {k};
  add_by_system<1>(ekin, 1, s, valid, kv);
}

int launch_kinetic(const ts_batch *b, double accel, double *ekin, hipStream_t st) {
  int rc = fill_async<double>(ekin, b->n_systems, 0.0, st);
  if (rc != TS_OK) return rc;
  if (b->n_atoms == 0) return TS_OK;
  hipLaunchKernelGGL(k_kinetic, dim3((unsigned)ceil_div(b->n_atoms, 256)), dim3(256), 0, st, b->n_atoms, stride_of(b),
                     b->system_idx, b->vel, b->mass, 0.5 / accel, ekin);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

template <typename T>
static int nve_sequence_t(const ts_batch *b, ts_neighbor_list *nl, const PairTable &tab, int prec, double dt,
                          double accel, int n_steps, void *force, double *epot, double *ekin, double *virial,
                          int64_t max_atoms, hipStream_t st) {
  const int64_t n = b->n_atoms, s_ = stride_of(b);
  const dim3 g((unsigned)ceil_div(n > 0 ? n : 1, 256));
  const bool want_ev = epot != nullptr || virial != nullptr;
  T *F = static_cast<T *>(force);
  int rc;
  if (n_steps == 0 && want_ev) {
    rc = nl_update(b, nl, 0, max_atoms, st);
    if (rc != TS_OK) return rc;
    rc = launch_forces(make_force_args(b, nl, force, epot, virial, nullptr), b->n_systems, tab, prec, true, st);
    if (rc != TS_OK) return rc;
  }
  for (int step = 0; step < n_steps; ++step) {
    if (n > 0) {
      hipLaunchKernelGGL(k_vv_kick_drift<T>, g, dim3(256), 0, st, n, s_, b->pos, b->vel, F, b->mass, 0.5 * dt, accel,
                         dt);
      TS_LAUNCH_CHECK();
    }
    rc = nl_update(b, nl, 0, max_atoms, st);
    if (rc != TS_OK) return rc;
    const bool last = step == n_steps - 1;
    rc = launch_forces(make_force_args(b, nl, force, last ? epot : nullptr, last ? virial : nullptr, nullptr),
                       b->n_systems, tab, prec, last && want_ev, st);
    if (rc != TS_OK) return rc;
    if (n > 0) {
      hipLaunchKernelGGL(k_vv_kick<T>, g, dim3(256), 0, st, n, s_, b->vel, F, b->mass, 0.5 * dt, accel);
      TS_LAUNCH_CHECK();
    }
  }
  if (ekin) {
    rc = launch_kinetic(b, accel, ekin, st);
    if (rc != TS_OK) return rc;
  }
  return TS_OK;
}

// One launch per step (see ts_step.hip): systems of at most kLdsMaxAtoms atoms, full list.
// With traj != null every position r_0..r_N is written to traj ([N+1][3][n_atoms]), which then
// serves as the ping-pong position storage of the loop.
int nve_fused_sequence(const ts_batch *b, ts_neighbor_list *nl, const PairTable &tab, int prec, double dt,
                       double accel, int n_steps, void *force, double *epot, double *ekin, double *virial,
                       int64_t max_atoms, hipStream_t st, double *traj, const LangParams *lang) {
  const int64_t n = b->n_atoms, S = b->n_systems;
  NlWork w = nl_work(nl->workspace, n, S);
  const int tl = lanes_for(nl, n);
  int rc = fill_async<int32_t>(w.flags3, 6 * S + 8, 0, st);
  if (rc != TS_OK) return rc;
  if (epot) {
    rc = fill_async<double>(epot, S, 0.0, st);
    if (rc != TS_OK) return rc;
  }
  if (virial) {
    rc = fill_async<double>(virial, 9 * S, 0.0, st);
    if (rc != TS_OK) return rc;
  }
  double *buf[2] = {b->pos, w.pos_alt};
  const int64_t sts[2] = {stride_of(b), n};
  StepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.offs = b->sys_offsets;
  a.vel = b->vel;
  a.st_vel = stride_of(b);
  a.mass = b->mass;
  a.species = b->species;
  a.cell = b->cell;
  a.force = force;
  a.nbr = reinterpret_cast<uint32_t *>(nl->nbr);
  a.n_nbr = nl->n_nbr;
  a.max_nbr = nl->max_nbr;
  a.half = nl->half;
  a.ref_pos = nl->ref_pos;
  a.ref_cell = nl->ref_cell;
  a.status = nl->status;
  a.r_list = nl->cutoff + nl->skin;
  a.skin = nl->skin;
  a.half_dt = 0.5 * dt;
  a.dt = dt;
  a.accel = accel;
  a.n_sys = (int)S;
  if (lang) {
    a.lang = *lang;
    a.lang_adv = n_steps;
  }
  // the cells do not change during the loop: their rebuild geometry is computed once
  static_assert(sizeof(RowGeom) == 14 * sizeof(double), "row geometry record");
  rc = launch_row_geometry(S, b->cell, a.r_list, reinterpret_cast<RowGeom *>(w.row_geom), st);
  if (rc != TS_OK) return rc;
  a.row_geom = reinterpret_cast<const RowGeom *>(w.row_geom);
  // deferred rebuild when the list has its second row buffer: every system starts in buffer 0
  const bool defer = nl->nbr_alt != nullptr;
  if (defer) {
    rc = fill_async<int32_t>(w.sel2, 2 * S, 0, st);
    if (rc != TS_OK) return rc;
    rc = fill_async<int32_t>(w.pflags3, 6 * S + 8, 0, st);
    if (rc != TS_OK) return rc;
    a.nbr_alt = reinterpret_cast<uint32_t *>(nl->nbr_alt);
    a.n_nbr_alt = nl->n_nbr_alt;
    a.ref_pos_alt = nl->ref_pos_alt;
    a.pre_factor = defer_pre_factor();
  }
  for (int step = 0; step <= n_steps; ++step) {
    const int mid = defer ? (lang ? kStepLangMidDefer : kStepMidDefer) : (lang ? kStepLangMid : kStepMid);
    const int mode = step == 0 ? (lang ? kStepLangFirst : kStepFirst) : (step == n_steps ? kStepLast : mid);
    a.lang_k = step;
    a.pos_in = buf[step % 2];
    a.st_in = sts[step % 2];
    a.pos_out = buf[(step + 1) % 2];
    a.st_out = sts[(step + 1) % 2];
    a.flag_cur = w.flags3 + S * (step % 3);
    a.flag_next = w.flags3 + S * ((step + 1) % 3);
    a.flag_clear = w.flags3 + S * ((step + 2) % 3);
    a.list_cur = w.flags3 + 3 * S + S * (step % 3);
    a.list_next = w.flags3 + 3 * S + S * ((step + 1) % 3);
    a.count_cur = w.flags3 + 6 * S + step % 3;
    a.count_next = w.flags3 + 6 * S + (step + 1) % 3;
    a.count_clear = w.flags3 + 6 * S + (step + 2) % 3;
    a.pos_final = (mode == kStepLast && step % 2 == 1) ? b->pos : nullptr;
    a.n_atoms = n;
    a.pos_copy = nullptr;
    if (traj) {
      a.pos_in = step == 0 ? b->pos : traj + 3 * n * step;
      a.st_in = step == 0 ? stride_of(b) : n;
      a.pos_out = traj + 3 * n * (step + 1);
      a.st_out = n;
      a.pos_copy = step == 0 ? traj : nullptr;
      a.pos_final = mode == kStepLast ? b->pos : nullptr;
    }
    a.epot = mode == kStepLast ? epot : nullptr;
    a.virial = mode == kStepLast ? virial : nullptr;
    if (defer) {
      a.sel_cur = w.sel2 + S * (step % 2);
      a.sel_next = w.sel2 + S * ((step + 1) % 2);
      a.pflag_cur = w.pflags3 + S * (step % 3);
      a.pflag_next = w.pflags3 + S * ((step + 1) % 3);
      a.pflag_clear = w.pflags3 + S * ((step + 2) % 3);
      a.plist_cur = w.pflags3 + 3 * S + S * (step % 3);
      a.plist_next = w.pflags3 + 3 * S + S * ((step + 1) % 3);
      a.pcount_cur = w.pflags3 + 6 * S + step % 3;
      a.pcount_next = w.pflags3 + 6 * S + (step + 1) % 3;
      a.pcount_clear = w.pflags3 + 6 * S + (step + 2) % 3;
      a.n_defer_wgs = (mode == kStepMidDefer || mode == kStepLangMidDefer) ? kDeferWgs : 0;
    }
    if (step != 0) {
      rc = launch_rebuild(a, S, max_atoms, st);
      if (rc != TS_OK) return rc;
    }
    rc = launch_step(mode, tl, nl->group_atoms, a, tab, prec, S, max_atoms, b->h_sys_offsets, st);
    if (rc != TS_OK) return rc;
  }
  if (defer) {
    // rows of systems rebuilt into the second buffer go back to the list's own buffer
    rc = launch_rows_restore(a, w.sel2 + S * (n_steps % 2), S, st);
    if (rc != TS_OK) return rc;
  }
  if (ekin) {
    rc = launch_kinetic(b, accel, ekin, st);
    if (rc != TS_OK) return rc;
  }
  return TS_OK;
}

static int nve_sequence(const ts_batch *b, ts_neighbor_list *nl, const ts_pair_params *pp, double dt, double accel,
                        int n_steps, void *force, double *epot, double *ekin, double *virial, int64_t max_atoms,
                        hipStream_t st) {
  const PairTable tab = make_table(pp);
  if (n_steps >= 1 && b->n_atoms > 0 && max_atoms <= kLdsMaxAtoms && !nl->half && fused_enabled())
    return nve_fused_sequence(b, nl, tab, pp->prec, dt, accel, n_steps, force, epot, ekin, virial, max_atoms, st);
  if (pp->prec == TS_PAIR_F32)
    return nve_sequence_t<float>(b, nl, tab, pp->prec, dt, accel, n_steps, force, epot, ekin, virial, max_atoms, st);
  return nve_sequence_t<double>(b, nl, tab, pp->prec, dt, accel, n_steps, force, epot, ekin, virial, max_atoms, st);
}

}  // namespace ts

extern "C" int ts_kinetic_energy(const ts_batch *batch, double accel, double *ekin, ts_stream_t stream) {
  int rc = ts::validate_batch(batch, true, nullptr);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(ekin != nullptr && std::isfinite(accel) && accel > 0.0);
  return ts::launch_kinetic(batch, accel, ekin, ts::as_stream(stream));
}

extern "C" int ts_nve_step(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp, double dt,
                           double accel, int32_t n_steps, void *force, double *epot, double *ekin, double *virial,
                           int32_t use_graph, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, true);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(force != nullptr);
  TS_CHECK_ARG(std::isfinite(dt) && dt > 0.0 && std::isfinite(accel) && accel > 0.0 && n_steps >= 0);
  std::string key("nve");
  ts::key_add(key, *batch);
  ts::key_add(key, *nl);
  ts::key_add(key, *pp);
  ts::key_add(key, dt);
  ts::key_add(key, accel);
  ts::key_add(key, n_steps);
  ts::key_add(key, max_atoms);
  ts::key_add(key, force);
  ts::key_add(key, epot);
  ts::key_add(key, ekin);
  ts::key_add(key, virial);
  const bool fused = ts::fused_enabled();
  ts::key_add(key, fused);
  ts::key_add(key, ts::defer_pre_factor());
  return ts::run_graph_cached(use_graph != 0, key, ts::as_stream(stream), [&](hipStream_t s) {
    return ts::nve_sequence(batch, nl, pp, dt, accel, n_steps, force, epot, ekin, virial, max_atoms, s);
  });
}

extern "C" int ts_nve_record(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp, double dt,
                             double accel, int32_t n_steps, void *force, double *traj, int32_t use_graph,
                             ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, true);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(force != nullptr && traj != nullptr);
  TS_CHECK_ARG(std::isfinite(dt) && dt > 0.0 && std::isfinite(accel) && accel > 0.0 && n_steps >= 1);
  if (max_atoms > ts::kLdsMaxAtoms || nl->half || batch->n_atoms == 0) return TS_E_UNSUPPORTED;
  std::string key("record");
  ts::key_add(key, *batch);
  ts::key_add(key, *nl);
  ts::key_add(key, *pp);
  ts::key_add(key, dt);
  ts::key_add(key, accel);
  ts::key_add(key, n_steps);
  ts::key_add(key, max_atoms);
  ts::key_add(key, force);
  ts::key_add(key, traj);
  ts::key_add(key, ts::defer_pre_factor());
  const ts::PairTable tab = ts::make_table(pp);
  return ts::run_graph_cached(use_graph != 0, key, ts::as_stream(stream), [&](hipStream_t s) {
    return ts::nve_fused_sequence(batch, nl, tab, pp->prec, dt, accel, n_steps, force, nullptr, nullptr, nullptr,
                                  max_atoms, s, traj);
  });
}
