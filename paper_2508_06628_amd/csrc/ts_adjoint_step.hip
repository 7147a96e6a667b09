// Reverse (adjoint) velocity-Verlet over a recorded trajectory segment: one launch per step for
// systems that fit in LDS (differentiable simulation, paper Section 2).
//
// For each position r_n of the segment, from the last to the first, the adjoint state (lr, lv)
// is advanced by   lv <- lv + dt_drift lr,   lr <- lr + w J(r_n) u(lv),   u = accel lv / m,
// and the parameter gradient by w sum_i u_i . dF_i/dtheta (the composition of the reverse half
// kicks and drift, consecutive half kicks at the same positions merged).  A workgroup stages its
// system's r_n and drifted u in LDS (the drift is applied on the fly from the previous adjoint
// state, which is read from one buffer while the new state goes to the other), evaluates the
// Hessian-vector product of its atoms with TL lanes per atom, and tests the neighbor-list
// validity of the next position to process, so the rows are rebuilt (k_rebuild_rows, the same
// flagged-system list as the forward loop) before the next reverse step needs them.
#include <string>

#include "ts_adjoint.h"
#include "ts_forces.h"
#include "ts_graph.h"
#include "ts_neighbor.h"
#include "ts_step.h"

namespace ts {

struct AdjStepArgs {
  const int64_t *offs;
  const double *pos;       // r_n, compact stride n
  const double *pos_next;  // the next position to process (r_{n-1}), or null
  int64_t n;               // compact stride of the trajectory
  const double *mass;
  const int32_t *species;
  const double *cell;
  const uint32_t *nbr;
  const int32_t *n_nbr;
  int64_t st;  // batch stride: list rows, reference positions
  const double *ref_pos;
  const double *lr_in, *lv_in;
  double *lr_out, *lv_out;
  int64_t st_in, st_out;
  double *adj_params;  // non-null: accumulate the parameter gradient
  double *slots;       // [S][kAdjSlot] per-system partial sums of the parameter gradient
  double dt_drift, w, accel;
  int32_t *flag_next, *flag_clear, *list_next, *count_next, *count_clear;
  double r_list, skin;
  int n_sys;
};

// Validity of the list for positions `pos` (compact stride n): flag systems for a rebuild.
__global__ void k_list_check(StepArgs a, const double *pos, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // system of atom i: binary search of the offsets
  int lo = 0, hi = (int)a.n_atoms;  // n_atoms holds the number of systems here
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (a.offs[mid] <= i) lo = mid;
    else hi = mid;
  }
  const int s = lo;
  const double r[3] = {pos[i], pos[n + i], pos[2 * n + i]};
  if (list_invalid(r, a.ref_pos, a.st_vel, i, a.cell + 9 * (int64_t)s, a.ref_cell + 9 * (int64_t)s, a.skin,
                   a.r_list) &&
      __hip_atomic_load(&a.flag_next[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
      atomicExch(&a.flag_next[s], 1) == 0) {
    const int q = atomicAdd(a.count_next, 1);
    if (q < (int)a.n_atoms) a.list_next[q] = s;  // a.n_atoms: number of systems (see above)
  }
}

template <int KIND, typename T, int TL, bool SINGLE>
__global__ void __launch_bounds__(256) k_adj_step(PairTable tab, AdjStepArgs a) {
  extern __shared__ double lds[];
  __shared__ PairCoef ltab[TS_MAX_SPECIES * TS_MAX_SPECIES];
  __shared__ double acc[TS_MAX_SPECIES * TS_MAX_SPECIES * 3];
  constexpr int APB = 256 / TL;
  const int s = blockIdx.y;
  const int64_t a0 = a.offs[s];
  const int ns = (int)(a.offs[s + 1] - a0);
  const int first = blockIdx.x * APB;
  // flags and list count of the position after next are cleared ahead of every early exit (an
  // empty system still clears its flag, and system 0 the count, whatever its size)
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.flag_clear[s] = 0;
    if (s == 0) *a.count_clear = 0;
  }
  if (first >= ns) return;
  const int tid = threadIdx.x, grp = tid / TL, lane = tid % TL;
  const int li = first + grp;
  const bool own = li < ns;
  const int64_t i = a0 + li;
  if (!SINGLE) {
    table_to_lds(ltab);
    for (int k = tid; k < TS_MAX_SPECIES * TS_MAX_SPECIES * 3; k += 256) acc[k] = 0.0;
  }
  const PairCoef pc0 = tab.c[0];  // one species: loop-invariant coefficients in registers
  // stage r_n and the drifted u of the whole system
  double *lx = lds, *ly = lds + ns, *lz = lds + 2 * ns;
  double *ux = lds + 3 * ns, *uy = lds + 4 * ns, *uz = lds + 5 * ns;
  for (int k = tid; k < ns; k += 256) {
    const int64_t g = a0 + k;
    lx[k] = a.pos[g];
    ly[k] = a.pos[a.n + g];
    lz[k] = a.pos[2 * a.n + g];
    const double sc = a.mass ? a.accel / a.mass[g] : a.accel;
    ux[k] = sc * fma(a.dt_drift, a.lr_in[g], a.lv_in[g]);
    uy[k] = sc * fma(a.dt_drift, a.lr_in[a.st_in + g], a.lv_in[a.st_in + g]);
    uz[k] = sc * fma(a.dt_drift, a.lr_in[2 * a.st_in + g], a.lv_in[2 * a.st_in + g]);
  }
  __syncthreads();
  const double *__restrict__ h = a.cell + 9 * (int64_t)s;
  const double h00 = h[0], h01 = h[1], h02 = h[2], h10 = h[3], h11 = h[4], h12 = h[5], h20 = h[6], h21 = h[7],
               h22 = h[8];
  const bool diag = h01 == 0.0 && h02 == 0.0 && h10 == 0.0 && h12 == 0.0 && h20 == 0.0 && h21 == 0.0 && h00 > 0.0 &&
                    h11 > 0.0 && h22 > 0.0;
  double jx = 0.0, jy = 0.0, jz = 0.0, t0 = 0.0, t1 = 0.0, t2 = 0.0;
  if (own) {
    const double rx = lx[li], ry = ly[li], rz = lz[li];
    const double uix = ux[li], uiy = uy[li], uiz = uz[li];
    const int si = SINGLE ? 0 : a.species[i];
    const int nn = a.n_nbr[i];
    const double cut2 = tab.cut2;
    const bool want_params = a.adj_params != nullptr;
    for_row<TL>(a.nbr, a.st, i, nn, lane, [&](uint32_t ent) {
      const int j = entry_j(ent);
      const double S0 = (double)entry_s0(ent), S1 = (double)entry_s1(ent), S2 = (double)entry_s2(ent);
      double dx, dy, dz;
      if (diag) {
        dx = (lx[j] - rx) + S0 * h00;
        dy = (ly[j] - ry) + S1 * h11;
        dz = (lz[j] - rz) + S2 * h22;
      } else {
        dx = shift_comp(lx[j] - rx, S0, S1, S2, h00, h10, h20);
        dy = shift_comp(ly[j] - ry, S0, S1, S2, h01, h11, h21);
        dz = shift_comp(lz[j] - rz, S0, S1, S2, h02, h12, h22);
      }
      const double r2 = norm2(dx, dy, dz);
      if (!(r2 < cut2)) return;
      const int sj = SINGLE ? 0 : a.species[a0 + j];
      const PairCoef &pc = SINGLE ? pc0 : ltab[si * TS_MAX_SPECIES + sj];
      if (KIND == TS_SOFT_SPHERE && !(r2 < pc.sig2)) return;
      T g, hh;
      pair_g_h<KIND, T>(pc, (T)r2, r2, &g, &hh);
      const T tx = (T)dx, tyy = (T)dy, tz = (T)dz;
      const T dux = (T)(ux[j] - uix), duy = (T)(uy[j] - uiy), duz = (T)(uz[j] - uiz);
      const T proj = tx * dux + tyy * duy + tz * duz;
      const T coef = (hh - g) * proj / (T)r2;
      jx += (double)(coef * tx + g * dux);
      jy += (double)(coef * tyy + g * duy);
      jz += (double)(coef * tz + g * duz);
      if (want_params) {
        double dg[3];
        pair_dg_dparams<KIND>(pc, r2, dg);
        const double ud = uix * dx + uiy * dy + uiz * dz;
        if (SINGLE) {
          t0 += dg[0] * ud;
          t1 += dg[1] * ud;
          t2 += dg[2] * ud;
        } else {
          double *q = acc + 3 * (si * TS_MAX_SPECIES + sj);
          atomicAdd(&q[0], a.w * dg[0] * ud);
          atomicAdd(&q[1], a.w * dg[1] * ud);
          atomicAdd(&q[2], a.w * dg[2] * ud);
        }
      }
    });
  }
#pragma unroll
  for (int o = 1; o < TL; o <<= 1) {
    jx += __shfl_xor(jx, o, TL);
    jy += __shfl_xor(jy, o, TL);
    jz += __shfl_xor(jz, o, TL);
  }
  if (own && lane == 0) {
    a.lv_out[i] = fma(a.dt_drift, a.lr_in[i], a.lv_in[i]);
    a.lv_out[a.st_out + i] = fma(a.dt_drift, a.lr_in[a.st_in + i], a.lv_in[a.st_in + i]);
    a.lv_out[2 * a.st_out + i] = fma(a.dt_drift, a.lr_in[2 * a.st_in + i], a.lv_in[2 * a.st_in + i]);
    a.lr_out[i] = fma(a.w, jx, a.lr_in[i]);
    a.lr_out[a.st_out + i] = fma(a.w, jy, a.lr_in[a.st_in + i]);
    a.lr_out[2 * a.st_out + i] = fma(a.w, jz, a.lr_in[2 * a.st_in + i]);
    if (a.pos_next) {
      // the cell does not change along an NVE trajectory: displacement part of the bound only
      const double dx = a.pos_next[i] - a.ref_pos[i], dy = a.pos_next[a.n + i] - a.ref_pos[a.st + i],
                   dz = a.pos_next[2 * a.n + i] - a.ref_pos[2 * a.st + i];
      // (a plain read first: the exchange of every atom over the bound would serialise on one word)
      if (bound_exceeded(sqrt(norm2(dx, dy, dz)), 0.0, a.skin, a.r_list) &&
          __hip_atomic_load(&a.flag_next[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
          atomicExch(&a.flag_next[s], 1) == 0) {
        const int q = atomicAdd(a.count_next, 1);
        if (q < a.n_sys) a.list_next[q] = s;
      }
    }
  }
  if (a.adj_params) {
    // workgroup sums go to the system's slot (atomics shared by the workgroups of one system only:
    // one word for the whole launch would serialise every wavefront of the batch); the slots are
    // summed into adj_params once per segment
    double *slot = a.slots + (int64_t)kAdjSlot * s;
    if (SINGLE) {
      __shared__ double wsum[256 / kWave][3];
      const double v0 = wave_sum(a.w * t0), v1 = wave_sum(a.w * t1), v2 = wave_sum(a.w * t2);
      if ((tid % kWave) == 0) {
        wsum[tid / kWave][0] = v0;
        wsum[tid / kWave][1] = v1;
        wsum[tid / kWave][2] = v2;
      }
      __syncthreads();
      if (tid < 3) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 256 / kWave; ++q) v += wsum[q][tid];
        atomicAdd(&slot[tid], v);
      }
    } else {
      __syncthreads();
      for (int k = tid; k < kAdjSlot; k += 256)
        if (acc[k] != 0.0) atomicAdd(&slot[k], acc[k]);
    }
  }
}

__global__ void k_copy3(int64_t n, const double *src, int64_t st_src, double *dst, int64_t st_dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int c = 0; c < 3; ++c) dst[c * st_dst + i] = src[c * st_src + i];
}

template <int KIND, typename T, int TL>
static void launch_adj_k(bool single, dim3 g, size_t shm, const AdjStepArgs &a, const PairTable &t, hipStream_t st) {
  if (single)
    hipLaunchKernelGGL((k_adj_step<KIND, T, TL, true>), g, dim3(256), shm, st, t, a);
  else
    hipLaunchKernelGGL((k_adj_step<KIND, T, TL, false>), g, dim3(256), shm, st, t, a);
}

template <int KIND, typename T>
static void launch_adj_kt(int tl, bool single, int64_t n_sys, int64_t max_atoms, const AdjStepArgs &a,
                          const PairTable &t, hipStream_t st) {
  const dim3 g((unsigned)ceil_div(max_atoms, 256 / tl), (unsigned)n_sys);
  const size_t shm = (size_t)6 * sizeof(double) * (size_t)max_atoms;
  switch (tl) {
    case 1: launch_adj_k<KIND, T, 1>(single, g, shm, a, t, st); break;
    case 2: launch_adj_k<KIND, T, 2>(single, g, shm, a, t, st); break;
    case 4: launch_adj_k<KIND, T, 4>(single, g, shm, a, t, st); break;
    default: launch_adj_k<KIND, T, 8>(single, g, shm, a, t, st); break;
  }
}

static int adjoint_segment(const ts_batch *b, ts_neighbor_list *nl, const ts_pair_params *pp, const double *traj,
                           int n_steps, double dt, double accel, bool top, bool bottom, double *adj_pos,
                           double *adj_vel, double *adj_params, int64_t max_atoms, hipStream_t st) {
  const int64_t n = b->n_atoms, S = b->n_systems, sb = stride_of(b);
  NlWork w = nl_work(nl->workspace, n, S);
  const PairTable tab = make_table(pp);
  const int tl = lanes_for(nl, n);
  const bool single = tab.n_species == 1 || b->species == nullptr;
  int rc = fill_async<int32_t>(w.flags3, 6 * S + 8, 0, st);
  if (rc != TS_OK) return rc;
  // list arguments shared with the rebuild kernel
  StepArgs r;
  std::memset(&r, 0, sizeof(r));
  r.offs = b->sys_offsets;
  r.st_vel = sb;
  r.cell = b->cell;
  r.nbr = reinterpret_cast<uint32_t *>(nl->nbr);
  r.n_nbr = nl->n_nbr;
  r.max_nbr = nl->max_nbr;
  r.half = nl->half;
  r.ref_pos = nl->ref_pos;
  r.ref_cell = nl->ref_cell;
  r.status = nl->status;
  r.r_list = nl->cutoff + nl->skin;
  r.skin = nl->skin;
  r.st_in = n;
  // validity of the first position to process
  r.flag_next = w.flags3;
  r.list_next = w.flags3 + 3 * S;
  r.count_next = w.flags3 + 6 * S;
  r.n_atoms = S;
  hipLaunchKernelGGL(k_list_check, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, r, traj + 3 * n * n_steps, n);
  TS_LAUNCH_CHECK();
  double *bufr[2] = {adj_pos, w.adj_alt};
  double *bufv[2] = {adj_vel, w.adj_alt + 3 * n};
  const int64_t sts[2] = {sb, n};
  const int P = n_steps + (bottom ? 1 : 0);
  AdjStepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.offs = b->sys_offsets;
  a.n = n;
  a.mass = b->mass;
  a.species = b->species;
  a.cell = b->cell;
  a.nbr = reinterpret_cast<const uint32_t *>(nl->nbr);
  a.n_nbr = nl->n_nbr;
  a.st = sb;
  a.ref_pos = nl->ref_pos;
  a.adj_params = adj_params;
  a.slots = w.adj_slots;
  a.accel = accel;
  if (adj_params) {
    rc = fill_async<double>(w.adj_slots, (int64_t)kAdjSlot * S, 0.0, st);
    if (rc != TS_OK) return rc;
  }
  a.r_list = r.r_list;
  a.skin = r.skin;
  a.n_sys = (int)S;
  for (int p = 0; p < P; ++p) {
    const int m = n_steps - p;
    const bool first_kick = top && p == 0;
    const bool last_kick = bottom && m == 0;
    a.dt_drift = first_kick ? 0.0 : dt;
    a.w = (first_kick || last_kick) ? 0.5 * dt : dt;
    a.pos = traj + 3 * n * m;
    a.pos_next = p + 1 < P ? traj + 3 * n * (m - 1) : nullptr;
    a.lr_in = bufr[p % 2];
    a.lv_in = bufv[p % 2];
    a.st_in = sts[p % 2];
    a.lr_out = bufr[(p + 1) % 2];
    a.lv_out = bufv[(p + 1) % 2];
    a.st_out = sts[(p + 1) % 2];
    a.flag_next = w.flags3 + S * ((p + 1) % 3);
    a.flag_clear = w.flags3 + S * ((p + 2) % 3);
    a.list_next = w.flags3 + 3 * S + S * ((p + 1) % 3);
    a.count_next = w.flags3 + 6 * S + (p + 1) % 3;
    a.count_clear = w.flags3 + 6 * S + (p + 2) % 3;
    // rebuild the rows of the systems flagged for this position
    r.pos_in = a.pos;
    r.list_cur = w.flags3 + 3 * S + S * (p % 3);
    r.count_cur = w.flags3 + 6 * S + p % 3;
    rc = launch_rebuild(r, S, max_atoms, st);
    if (rc != TS_OK) return rc;
    with_kind(tab.kind, [&](auto k) {
      constexpr int KIND = decltype(k)::value;
      if (pp->prec == TS_PAIR_F32) launch_adj_kt<KIND, float>(tl, single, S, max_atoms, a, tab, st);
      else launch_adj_kt<KIND, double>(tl, single, S, max_atoms, a, tab, st);
    });
    TS_LAUNCH_CHECK();
  }
  if (adj_params) {
    rc = launch_sum_slots(S, w.adj_slots, adj_params, st);
    if (rc != TS_OK) return rc;
  }
  if (P % 2 == 1) {
    // the final state is in the second buffers: copy it to the caller's
    hipLaunchKernelGGL(k_copy3, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, bufr[1], n, adj_pos, sb);
    hipLaunchKernelGGL(k_copy3, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, n, bufv[1], n, adj_vel, sb);
    TS_LAUNCH_CHECK();
  }
  return TS_OK;
}

}  // namespace ts

extern "C" int ts_adjoint_segment(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp,
                                  const double *traj, int32_t n_steps, double dt, double accel, int32_t top,
                                  int32_t bottom, double *adj_pos, double *adj_vel, double *adj_params,
                                  int32_t use_graph, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, false);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(traj && adj_pos && adj_vel && n_steps >= 1);
  TS_CHECK_ARG(std::isfinite(dt) && dt > 0.0 && std::isfinite(accel) && accel > 0.0);
  if (max_atoms > ts::kLdsMaxAtoms || batch->n_atoms == 0) return TS_E_UNSUPPORTED;
  std::string key("adjoint");
  ts::key_add(key, *batch);
  ts::key_add(key, *nl);
  ts::key_add(key, *pp);
  ts::key_add(key, traj);
  ts::key_add(key, n_steps);
  ts::key_add(key, dt);
  ts::key_add(key, accel);
  ts::key_add(key, top);
  ts::key_add(key, bottom);
  ts::key_add(key, adj_pos);
  ts::key_add(key, adj_vel);
  ts::key_add(key, adj_params);
  ts::key_add(key, max_atoms);
  return ts::run_graph_cached(use_graph != 0, key, ts::as_stream(stream), [&](hipStream_t s) {
    return ts::adjoint_segment(batch, nl, pp, traj, n_steps, dt, accel, top != 0, bottom != 0, adj_pos, adj_vel,
                               adj_params, max_atoms, s);
  });
}
