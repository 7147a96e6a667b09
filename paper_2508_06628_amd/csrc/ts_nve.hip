// Velocity-Verlet NVE over the whole batch (the molecular-dynamics integrators of the paper's
// Abstract; every system advances in the same launches, Section 3), with the per-step neighbor
// validity test and rebuild on the device and an optional hipGraph of the whole step loop.
#include <map>
#include <mutex>
#include <vector>

#include <cstdlib>

#include "ts_forces.h"
#include "ts_neighbor.h"
#include "ts_step.h"

namespace ts {

// TS_NVE_UNFUSED=1 selects the multi-kernel step (separate list update, force and kick launches)
// instead of the fused one; both compute the same trajectory.
static bool fused_enabled() {
  const char *e = std::getenv("TS_NVE_UNFUSED");
  return !(e && e[0] == '1');
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
static int nve_fused_sequence(const ts_batch *b, ts_neighbor_list *nl, const PairTable &tab, int prec, double dt,
                              double accel, int n_steps, void *force, double *epot, double *ekin, double *virial,
                              int64_t max_atoms, hipStream_t st) {
  const int64_t n = b->n_atoms, S = b->n_systems;
  NlWork w = nl_work(nl->workspace, n, S);
  const int tl = nl->lanes_per_atom > 0 ? nl->lanes_per_atom : 4;
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
  for (int step = 0; step <= n_steps; ++step) {
    const int mode = step == 0 ? kStepFirst : (step == n_steps ? kStepLast : kStepMid);
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
    a.epot = mode == kStepLast ? epot : nullptr;
    a.virial = mode == kStepLast ? virial : nullptr;
    if (mode != kStepFirst) {
      rc = launch_rebuild(a, S, max_atoms, st);
      if (rc != TS_OK) return rc;
    }
    rc = launch_step(mode, tl, a, tab, prec, S, max_atoms, st);
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

// ----------------------------------------------------------------------------- graph cache

namespace {

struct NveKey {
  ts_batch b;
  ts_neighbor_list nl;
  ts_pair_params pp;
  double dt, accel;
  int64_t n_steps, max_atoms;
  void *force;
  double *epot, *ekin, *virial;
  int device;
};

struct KeyLess {
  bool operator()(const NveKey &x, const NveKey &y) const { return std::memcmp(&x, &y, sizeof(NveKey)) < 0; }
};

struct GraphEntry {
  hipGraph_t graph;
  hipGraphExec_t exec;
  uint64_t stamp;
};

std::mutex g_mu;
std::map<NveKey, GraphEntry, KeyLess> g_cache;
uint64_t g_clock = 0;
std::map<int, hipStream_t> g_capture_stream;
constexpr size_t kMaxGraphs = 16;

void destroy_entry(GraphEntry &e) {
  (void)hipGraphExecDestroy(e.exec);
  (void)hipGraphDestroy(e.graph);
}

}  // namespace

int capture_stream(int device, hipStream_t *out) {
  auto it = g_capture_stream.find(device);
  if (it != g_capture_stream.end()) {
    *out = it->second;
    return TS_OK;
  }
  hipStream_t s;
  TS_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  g_capture_stream[device] = s;
  *out = s;
  return TS_OK;
}

void release_graphs() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_cache.empty()) (void)hipDeviceSynchronize();
  for (auto &kv : g_cache) destroy_entry(kv.second);
  g_cache.clear();
}

}  // namespace ts

extern "C" void ts_release_graphs(void) { ts::release_graphs(); }

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
  hipStream_t st = ts::as_stream(stream);
  if (!use_graph) return ts::nve_sequence(batch, nl, pp, dt, accel, n_steps, force, epot, ekin, virial, max_atoms, st);

  ts::NveKey key;
  std::memset(&key, 0, sizeof(key));
  key.b = *batch;
  key.nl = *nl;
  key.pp = *pp;
  key.dt = dt;
  key.accel = accel;
  key.n_steps = n_steps;
  key.max_atoms = max_atoms;
  key.force = force;
  key.epot = epot;
  key.ekin = ekin;
  key.virial = virial;
  TS_HIP(hipGetDevice(&key.device));

  std::lock_guard<std::mutex> lk(ts::g_mu);
  auto it = ts::g_cache.find(key);
  if (it == ts::g_cache.end()) {
    hipStream_t cap;
    rc = ts::capture_stream(key.device, &cap);
    if (rc != TS_OK) return rc;
    TS_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    rc = ts::nve_sequence(batch, nl, pp, dt, accel, n_steps, force, epot, ekin, virial, max_atoms, cap);
    hipGraph_t graph = nullptr;
    hipError_t ce = hipStreamEndCapture(cap, &graph);
    if (rc != TS_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    if (ce != hipSuccess || graph == nullptr) return TS_E_HIP;
    hipGraphExec_t exec;
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return TS_E_HIP;
    }
    if (ts::g_cache.size() >= ts::kMaxGraphs) {
      auto old = ts::g_cache.begin();
      for (auto jt = ts::g_cache.begin(); jt != ts::g_cache.end(); ++jt)
        if (jt->second.stamp < old->second.stamp) old = jt;
      (void)hipDeviceSynchronize();
      ts::destroy_entry(old->second);
      ts::g_cache.erase(old);
    }
    it = ts::g_cache.emplace(key, ts::GraphEntry{graph, exec, 0}).first;
  }
  it->second.stamp = ++ts::g_clock;
  TS_HIP(hipGraphLaunch(it->second.exec, st));
  return TS_OK;
}
