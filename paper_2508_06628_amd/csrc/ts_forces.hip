// Pair energy / force / virial over a padded full neighbor list (Lennard-Jones, Morse,
// soft-sphere: the classical potentials of the paper's Abstract; output schema of energies,
// forces and stress, Section 2).
//
// One lane per atom.  The pair vector d = r_j - r_i + S cell and the interaction mask are float64;
// the pair function runs in the pair precision T; forces, energies and virials accumulate in
// float64.  Per-system energy and virial are reduced across the wavefront and added with one
// float64 atomic per wavefront (lanes of a wavefront almost always share a system).
#include "ts_forces.h"
#include "ts_neighbor.h"
#include "ts_step.h"

namespace ts {

constexpr int kFwdUnroll = 4;  // row entries a thread evaluates together in k_pair_forces

// pos4[i] = (x_i, y_i, z_i, 0): one 32-byte block per atom, so that a neighbor gather touches one
// cache line instead of one line in each of the three coordinate arrays
__global__ void k_pack_pos4(int64_t n, int64_t st, const double *__restrict__ pos, double4 *__restrict__ pos4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  pos4[i] = make_double4(pos[i], pos[st + i], pos[2 * st + i], 0.0);
}

template <int KIND, typename T, bool EV, bool SINGLE>
__global__ void __launch_bounds__(256) k_pair_forces(PairTable tab, ForceArgs a) {
  __shared__ PairCoef ltab[TS_MAX_SPECIES * TS_MAX_SPECIES];
  if (!SINGLE) table_to_lds(ltab);
  // consecutive atoms (those of one system, whose positions the rows gather) on one XCD's L2
  const int64_t i = xcd_order(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  bool valid = i < a.n;
  const int64_t ii = valid ? i : 0;
  const int s = valid ? a.sys_idx[ii] : 0;
  if (valid && a.skip && a.skip[s]) valid = false;
  double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
  double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // xx yy zz xy xz yz
  if (valid) {
    const int64_t st = a.stride;
    const int64_t a0 = a.offs[s];
    const double *h = a.cell + 9 * (int64_t)s;
    const double h00 = h[0], h01 = h[1], h02 = h[2], h10 = h[3], h11 = h[4], h12 = h[5], h20 = h[6], h21 = h[7],
                 h22 = h[8];
    const double rx = a.pos[ii], ry = a.pos[st + ii], rz = a.pos[2 * st + ii];
    const bool multi = !SINGLE && a.species != nullptr;  // uniform
    const int si = multi ? a.species[ii] : 0;
    const int nn = a.n_nbr[ii];
    const double cut2 = tab.cut2;
    const PairCoef pc0 = tab.c[0];
    // kFwdUnroll entries at a time: their neighbor loads are issued together and the pairs are
    // evaluated without branches (entries past the row end or beyond the cutoff add exact zeros,
    // so the sums round as in a plain loop over the in-range pairs)
    for_row_batched<1, kFwdUnroll>(a.nbr, st, ii, nn, 0, [&](const uint32_t *ent, const bool *ok) {
      double xj[kFwdUnroll], yj[kFwdUnroll], zj[kFwdUnroll];
      int sj[kFwdUnroll];
#pragma unroll
      for (int u = 0; u < kFwdUnroll; ++u) {
        const int64_t j = ok[u] ? a0 + entry_j(ent[u]) : ii;  // masked visits read atom i itself
        const double4 pj = reinterpret_cast<const double4 *>(a.pos4)[j];
        xj[u] = pj.x;
        yj[u] = pj.y;
        zj[u] = pj.z;
        sj[u] = multi ? a.species[j] : 0;
      }
#pragma unroll
      for (int u = 0; u < kFwdUnroll; ++u) {
        const double S0 = (double)entry_s0(ent[u]), S1 = (double)entry_s1(ent[u]), S2 = (double)entry_s2(ent[u]);
        const double dx = shift_comp(xj[u] - rx, S0, S1, S2, h00, h10, h20);
        const double dy = shift_comp(yj[u] - ry, S0, S1, S2, h01, h11, h21);
        const double dz = shift_comp(zj[u] - rz, S0, S1, S2, h02, h12, h22);
        const double r2 = norm2(dx, dy, dz);
        const PairCoef &pc = multi ? ltab[si * TS_MAX_SPECIES + sj[u]] : pc0;
        bool in = ok[u] && r2 < cut2;
        if (KIND == TS_SOFT_SPHERE) in = in && r2 < pc.sig2;
        T phi = (T)0;
        const T gt = pair_g<KIND, T>(pc, (T)r2, r2, &phi, EV);
        const double g = in ? (double)gt : 0.0;
        acc_force(g, dx, dy, dz, fx, fy, fz);
        if (EV) {
          e += in ? (double)phi : 0.0;
          acc_virial(g, dx, dy, dz, w);
        }
      }
    });
    T *F = static_cast<T *>(a.force);
    F[ii] = (T)fx;
    F[st + ii] = (T)fy;
    F[2 * st + ii] = (T)fz;
  }
  if (EV) {
    if (a.energy) {
      const double ev[1] = {0.5 * e};
      add_by_system<1>(a.energy, 1, s, valid, ev);
    }
    if (a.virial) {
      const double wv[9] = {-0.5 * w[0], -0.5 * w[3], -0.5 * w[4], -0.5 * w[3], -0.5 * w[1],
                            -0.5 * w[5], -0.5 * w[4], -0.5 * w[5], -0.5 * w[2]};
      add_by_system<9>(a.virial, 9, s, valid, wv);
    }
  }
}

__global__ void k_zero_ev(int64_t n_sys, double *energy, double *virial, const int32_t *skip) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  if (skip && skip[s]) return;
  if (energy) energy[s] = 0.0;
  if (virial)
    for (int k = 0; k < 9; ++k) virial[9 * s + k] = 0.0;
}

template <int KIND, typename T>
static void launch_kt(const ForceArgs &a, const PairTable &t, bool ev, bool single, dim3 g, hipStream_t st) {
  if (ev) {
    if (single)
      hipLaunchKernelGGL((k_pair_forces<KIND, T, true, true>), g, dim3(256), 0, st, t, a);
    else
      hipLaunchKernelGGL((k_pair_forces<KIND, T, true, false>), g, dim3(256), 0, st, t, a);
  } else {
    if (single)
      hipLaunchKernelGGL((k_pair_forces<KIND, T, false, true>), g, dim3(256), 0, st, t, a);
    else
      hipLaunchKernelGGL((k_pair_forces<KIND, T, false, false>), g, dim3(256), 0, st, t, a);
  }
}

int launch_forces(const ForceArgs &a, int64_t n_sys, const PairTable &t, int prec, bool ev, hipStream_t st) {
  if (ev && (a.energy || a.virial)) {
    hipLaunchKernelGGL(k_zero_ev, dim3((unsigned)ceil_div(n_sys, 64)), dim3(64), 0, st, n_sys, a.energy, a.virial,
                       a.skip);
    TS_LAUNCH_CHECK();
  }
  if (a.n == 0) return TS_OK;
  hipLaunchKernelGGL(k_pack_pos4, dim3((unsigned)ceil_div(a.n, 256)), dim3(256), 0, st, a.n, a.stride, a.pos,
                     reinterpret_cast<double4 *>(a.pos4));
  TS_LAUNCH_CHECK();
  const dim3 g((unsigned)(ceil_div(ceil_div(a.n, 256), kXcds) * kXcds));  // a multiple of kXcds for xcd_order
  const bool single = t.n_species == 1 || a.species == nullptr;
  const bool do_ev = ev && (a.energy || a.virial);
  with_kind(t.kind, [&](auto k) {
    constexpr int KIND = decltype(k)::value;
    if (prec == TS_PAIR_F32) launch_kt<KIND, float>(a, t, do_ev, single, g, st);
    else launch_kt<KIND, double>(a, t, do_ev, single, g, st);
  });
  TS_LAUNCH_CHECK();
  return TS_OK;
}

ForceArgs make_force_args(const ts_batch *b, const ts_neighbor_list *nl, void *force, double *energy, double *virial,
                          const int32_t *skip) {
  ForceArgs a;
  a.n = b->n_atoms;
  a.stride = stride_of(b);
  a.sys_idx = b->system_idx;
  a.offs = b->sys_offsets;
  a.pos = b->pos;
  a.cell = b->cell;
  a.species = b->species;
  a.nbr = reinterpret_cast<const uint32_t *>(nl->nbr);
  a.n_nbr = nl->n_nbr;
  a.force = force;
  a.energy = energy;
  a.virial = virial;
  a.skip = skip;
  a.pos4 = nl_work(nl->workspace, b->n_atoms, b->n_systems).pos4;
  return a;
}

int validate_pair_call(const ts_batch *b, const ts_neighbor_list *nl, const ts_pair_params *pp, int64_t *max_atoms,
                       bool need_vel, bool need_workspace) {
  int rc = validate_batch(b, need_vel, max_atoms);
  if (rc != TS_OK) return rc;
  rc = validate_params(pp);
  if (rc != TS_OK) return rc;
  rc = validate_list(b, nl, need_workspace);
  if (rc != TS_OK) return rc;
  if (nl->half) return TS_E_UNSUPPORTED;
  // the list must cover the interaction range
  TS_CHECK_ARG(nl->cutoff + nl->skin >= pp->cutoff);
  return TS_OK;
}

// Forces (energy and virial when asked) of every system whose skip entry is zero (skip may be
// null): systems that fit in LDS take the workgroup-per-system kernel of the step loop, larger
// ones the row-per-atom kernel.  Skipped systems keep their forces, energy and virial.
int launch_forces_batch(const ts_batch *b, const ts_neighbor_list *nl, const PairTable &t, int prec, void *force,
                        double *energy, double *virial, const int32_t *skip, int64_t max_atoms, hipStream_t st) {
  if (max_atoms > kLdsMaxAtoms || b->n_atoms == 0)
    return launch_forces(make_force_args(b, nl, force, energy, virial, skip), b->n_systems, t, prec,
                         energy != nullptr || virial != nullptr, st);
  if (energy || virial) {
    hipLaunchKernelGGL(k_zero_ev, dim3((unsigned)ceil_div(b->n_systems, 64)), dim3(64), 0, st, b->n_systems, energy,
                       virial, skip);
    TS_LAUNCH_CHECK();
  }
  StepArgs s;
  std::memset(&s, 0, sizeof(s));
  s.offs = b->sys_offsets;
  s.pos_in = b->pos;
  s.st_in = stride_of(b);
  s.st_vel = stride_of(b);
  s.species = b->species;
  s.cell = b->cell;
  s.force = force;
  s.nbr = reinterpret_cast<uint32_t *>(nl->nbr);
  s.n_nbr = nl->n_nbr;
  s.max_nbr = nl->max_nbr;
  s.epot = energy;
  s.virial = virial;
  s.skip = skip;
  const int mode = (energy || virial) ? kStepForceEV : kStepForce;
  return launch_step(mode, lanes_for(nl, b->n_atoms), nl->group_atoms, s, t, prec, b->n_systems, max_atoms,
                     b->h_sys_offsets, st);
}

}  // namespace ts

extern "C" int ts_pair_forces(const ts_batch *batch, const ts_neighbor_list *nl, const ts_pair_params *pp, void *force,
                              double *energy, double *virial, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, false);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(force != nullptr);
  return ts::launch_forces_batch(batch, nl, ts::make_table(pp), pp->prec, force, energy, virial, nullptr, max_atoms,
                                 ts::as_stream(stream));
}
