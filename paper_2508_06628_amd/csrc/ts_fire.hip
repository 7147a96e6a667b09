// FIRE relaxation of positions, or positions and cell, for every system of a batch (the
// structural relaxation optimizers of the paper's Abstract; relaxation is the variable-length
// workload of Section 3).  Each iteration is: neighbor validity test/rebuild, pair forces of the
// unconverged systems, and the FIRE update in three launches (chunked reductions of the FIRE
// scalars max |F|, g.v, |v|^2, |g|^2; one wavefront per system combining them in a fixed order and
// taking the decision; the chunked update of the atoms), so that systems of any size spread over
// the whole GPU.  The persistent path for systems that fit in LDS is in ts_fire_persistent.hip.
#include "ts_fire.h"
#include "ts_step.h"

namespace ts {



__device__ inline void inv3d(const double *h, double *inv) {
  const double det = h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                     h[2] * (h[3] * h[7] - h[4] * h[6]);
  const double id = 1.0 / det;
  inv[0] = (h[4] * h[8] - h[5] * h[7]) * id;
  inv[1] = (h[2] * h[7] - h[1] * h[8]) * id;
  inv[2] = (h[1] * h[5] - h[2] * h[4]) * id;
  inv[3] = (h[5] * h[6] - h[3] * h[8]) * id;
  inv[4] = (h[0] * h[8] - h[2] * h[6]) * id;
  inv[5] = (h[2] * h[3] - h[0] * h[5]) * id;
  inv[6] = (h[3] * h[7] - h[4] * h[6]) * id;
  inv[7] = (h[1] * h[6] - h[0] * h[7]) * id;
  inv[8] = (h[0] * h[4] - h[1] * h[3]) * id;
}

// Block (256 threads) reductions with a fixed combination order.
__device__ inline double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  return (sh[0] + sh[1]) + (sh[2] + sh[3]);
}
__device__ inline double block_max(double v, double *sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  return fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// The FIRE iteration of the non-persistent path, for systems of any size, in three launches:
//   k_fire_reduce: each workgroup reduces max |F|^2, g.v, |v|^2, |g|^2 over a chunk of kFireChunk
//     atoms of one system (g = F D^T with the cell's deformation gradient D when the cell relaxes)
//     and writes the four partial values to its slot;
//   k_fire_decide: one wavefront per system combines the slots of its system in a fixed order,
//     adds the cell terms, takes the FIRE decision, updates the per-system state and the cell and
//     writes the mixing coefficients;
//   k_fire_apply: each workgroup updates the velocities and positions of its chunk.
// The slot of chunk c of system s is s + floor((a0_s + kFireChunk c) / kFireChunk): unique, and at
// most S + N / kFireChunk + 1 slots of 4 doubles.
constexpr int kFireChunk = 256;

__device__ inline int64_t fire_slot(int s, int64_t a0, int c) { return s + (a0 + (int64_t)kFireChunk * c) / kFireChunk; }

template <typename T, bool CELL>
__global__ void __launch_bounds__(kFireChunk) k_fire_reduce(FireArgs a, double *part) {
  const int s = blockIdx.y, c = blockIdx.x;
  if (a.converged[s]) return;
  const int64_t a0 = a.offs[s], a1 = a.offs[s + 1];
  if (a0 + (int64_t)kFireChunk * c >= a1) return;  // uniform over the workgroup
  const int64_t i = a0 + (int64_t)kFireChunk * c + threadIdx.x;
  const int64_t st = a.stride;
  const T *F = static_cast<const T *>(a.force);
  __shared__ double sh[4];
  double fmax2 = 0.0, P = 0.0, vv = 0.0, gg = 0.0;
  if (i < a1) {
    const double f0 = (double)F[i], f1 = (double)F[st + i], f2 = (double)F[2 * st + i];
    fmax2 = f0 * f0 + f1 * f1 + f2 * f2;
    double g0 = f0, g1 = f1, g2 = f2;
    if (CELL) {
      const double *D = a.deform + 9 * (int64_t)s;
      g0 = f0 * D[0] + f1 * D[1] + f2 * D[2];
      g1 = f0 * D[3] + f1 * D[4] + f2 * D[5];
      g2 = f0 * D[6] + f1 * D[7] + f2 * D[8];
    }
    const double v0 = a.vel[i], v1 = a.vel[st + i], v2 = a.vel[2 * st + i];
    P = g0 * v0 + g1 * v1 + g2 * v2;
    vv = v0 * v0 + v1 * v1 + v2 * v2;
    gg = g0 * g0 + g1 * g1 + g2 * g2;
  }
  fmax2 = block_max(fmax2, sh);
  P = block_sum(P, sh);
  vv = block_sum(vv, sh);
  gg = block_sum(gg, sh);
  if (threadIdx.x == 0) {
    double *q = part + 4 * fire_slot(s, a0, c);
    q[0] = fmax2;
    q[1] = P;
    q[2] = vv;
    q[3] = gg;
  }
}

// Per-system coefficients written by k_fire_decide: cv, cg, dt, skip, D_old (9), D_new (9).
constexpr int kFireCoef = 22;

template <bool CELL>
__global__ void __launch_bounds__(kWave) k_fire_decide(FireArgs a, const double *part, double *coef, int final_check) {
  const int s = blockIdx.x;
  double *co = coef + (int64_t)kFireCoef * s;
  if (a.converged[s]) {
    if (threadIdx.x == 0) co[3] = 1.0;
    return;
  }
  const int64_t a0 = a.offs[s], a1 = a.offs[s + 1];
  const int64_t na = a1 - a0;
  const int nc = (int)((na + kFireChunk - 1) / kFireChunk);
  // fixed order: lane l takes chunks l, l + 64, ... in turn, then a fixed butterfly across lanes
  double fmax2 = 0.0, P = 0.0, vv = 0.0, gg = 0.0;
  for (int c = threadIdx.x; c < nc; c += kWave) {
    const double *q = part + 4 * fire_slot(s, a0, c);
    fmax2 = fmax(fmax2, q[0]);
    P += q[1];
    vv += q[2];
    gg += q[3];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) fmax2 = fmax(fmax2, __shfl_xor(fmax2, o, kWave));
  P = wave_sum(P);
  vv = wave_sum(vv);
  gg = wave_sum(gg);
  if (threadIdx.x != 0) return;
  const ts_fire_config &c = a.cfg;
  bool conv = sqrt(fmax2) < c.fmax;
  double D[9], Di[9], G[9], V[9];
  if (CELL) {
    for (int k = 0; k < 9; ++k) D[k] = a.deform[9 * s + k];
    inv3d(D, Di);
    const double *W = a.virial + 9 * s;
    double gmax = 0.0;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        // G = D^-T W / N
        const double v =
            (Di[0 * 3 + p] * W[0 * 3 + q] + Di[1 * 3 + p] * W[1 * 3 + q] + Di[2 * 3 + p] * W[2 * 3 + q]) / (double)na;
        G[3 * p + q] = v;
        gmax = fmax(gmax, fabs(v));
      }
    conv = conv && gmax < c.fmax;
    for (int k = 0; k < 9; ++k) V[k] = a.deform_vel[9 * s + k];
  }
  double skip = 0.0;
  if (conv) {
    a.converged[s] = 1;
    skip = 1.0;
  } else if (final_check || a.n_iter[s] >= c.max_iter ||
             (a.iter_start && a.budget >= 0 && a.n_iter[s] - a.iter_start[s] >= a.budget)) {
    skip = 1.0;
  } else {
    double dt = a.dt[s], al = a.alpha[s];
    int np = a.n_pos[s];
    double cv = 1.0, cg = 0.0;
    if (a.n_iter[s] > 0) {
      double Pt = P, vvt = vv, ggt = gg;
      if (CELL)
        for (int k = 0; k < 9; ++k) {
          Pt += G[k] * V[k];
          vvt += V[k] * V[k];
          ggt += G[k] * G[k];
        }
      if (Pt > 0.0) {
        if (ggt > 0.0) {
          cv = 1.0 - al;
          cg = al * sqrt(vvt) / sqrt(ggt);
        }
        np += 1;
        if (np > c.n_min) {
          dt = fmin(dt * c.f_inc, c.dt_max);
          al = al * c.f_alpha;
        }
      } else {
        cv = 0.0;
        cg = 0.0;
        dt = dt * c.f_dec;
        al = c.alpha_start;
        np = 0;
      }
    }
    a.dt[s] = dt;
    a.alpha[s] = al;
    a.n_pos[s] = np;
    a.n_iter[s] += 1;
    co[0] = cv;
    co[1] = cg;
    co[2] = dt;
    if (CELL) {
      double Dn[9];
      for (int k = 0; k < 9; ++k) {
        V[k] = cv * V[k] + cg * G[k];
        V[k] = V[k] + dt * G[k] / c.cell_mass;
        Dn[k] = D[k] + (dt / (double)na) * V[k];
        a.deform_vel[9 * s + k] = V[k];
        a.deform[9 * s + k] = Dn[k];
        co[13 + k] = Dn[k];
      }
      for (int p = 0; p < 3; ++p)
        for (int q = 0; q < 3; ++q)
          a.cell[9 * s + 3 * p + q] = a.ref_cell[9 * s + 3 * p + 0] * Dn[0 * 3 + q] +
                                      a.ref_cell[9 * s + 3 * p + 1] * Dn[1 * 3 + q] +
                                      a.ref_cell[9 * s + 3 * p + 2] * Dn[2 * 3 + q];
      // the apply kernel needs the old D (g = F D^T, and D^-1 for q = r D^-1 + dt v)
      for (int k = 0; k < 9; ++k) co[4 + k] = D[k];
    }
  }
  co[3] = skip;
}

template <typename T, bool CELL>
__global__ void __launch_bounds__(kFireChunk) k_fire_apply(FireArgs a, const double *coef) {
  const int s = blockIdx.y, c = blockIdx.x;
  const double *co = coef + (int64_t)kFireCoef * s;
  if (co[3] != 0.0) return;
  const int64_t a0 = a.offs[s], a1 = a.offs[s + 1];
  const int64_t i = a0 + (int64_t)kFireChunk * c + threadIdx.x;
  if (i >= a1) return;
  const int64_t st = a.stride;
  const T *F = static_cast<const T *>(a.force);
  const double cv = co[0], cg = co[1], dt = co[2];
  double D[9], Di[9], Dn[9];
  if (CELL) {
    for (int k = 0; k < 9; ++k) {
      D[k] = co[4 + k];
      Dn[k] = co[13 + k];
    }
    inv3d(D, Di);
  }
  const double f0 = (double)F[i], f1 = (double)F[st + i], f2 = (double)F[2 * st + i];
  double g[3] = {f0, f1, f2};
  if (CELL) {
    g[0] = f0 * D[0] + f1 * D[1] + f2 * D[2];
    g[1] = f0 * D[3] + f1 * D[4] + f2 * D[5];
    g[2] = f0 * D[6] + f1 * D[7] + f2 * D[8];
  }
  const double m = a.mass ? a.mass[i] : 1.0;
  double v[3], r[3];
  for (int k = 0; k < 3; ++k) {
    v[k] = cv * a.vel[k * st + i] + cg * g[k];
    v[k] = v[k] + dt * g[k] / m;
    a.vel[k * st + i] = v[k];
    r[k] = a.pos[k * st + i];
  }
  if (CELL) {
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = (r[0] * Di[k] + r[1] * Di[3 + k] + r[2] * Di[6 + k]) + dt * v[k];
    for (int k = 0; k < 3; ++k) a.pos[k * st + i] = q[0] * Dn[k] + q[1] * Dn[3 + k] + q[2] * Dn[6 + k];
  } else {
    for (int k = 0; k < 3; ++k) a.pos[k * st + i] = r[k] + dt * v[k];
  }
}

template <typename T>
static int launch_fire_update(const FireArgs &fa, bool cell, int final_check, int64_t n_sys, int64_t max_atoms,
                              double *part, double *coef, hipStream_t st) {
  const dim3 g((unsigned)ceil_div(max_atoms, kFireChunk), (unsigned)n_sys);
  if (cell) {
    hipLaunchKernelGGL((k_fire_reduce<T, true>), g, dim3(kFireChunk), 0, st, fa, part);
    hipLaunchKernelGGL((k_fire_decide<true>), dim3((unsigned)n_sys), dim3(kWave), 0, st, fa, part, coef, final_check);
    hipLaunchKernelGGL((k_fire_apply<T, true>), g, dim3(kFireChunk), 0, st, fa, coef);
  } else {
    hipLaunchKernelGGL((k_fire_reduce<T, false>), g, dim3(kFireChunk), 0, st, fa, part);
    hipLaunchKernelGGL((k_fire_decide<false>), dim3((unsigned)n_sys), dim3(kWave), 0, st, fa, part, coef, final_check);
    hipLaunchKernelGGL((k_fire_apply<T, false>), g, dim3(kFireChunk), 0, st, fa, coef);
  }
  TS_LAUNCH_CHECK();
  return TS_OK;
}

FireArgs make_fire_args(const ts_batch *b, const ts_fire_state *fs, const ts_fire_config *cfg, void *force,
                        double *virial) {
  FireArgs fa;
  fa.stride = stride_of(b);
  fa.offs = b->sys_offsets;
  fa.pos = b->pos;
  fa.vel = b->vel;
  fa.mass = b->mass;
  fa.cell = b->cell;
  fa.force = force;
  fa.virial = virial;
  fa.dt = fs->dt;
  fa.alpha = fs->alpha;
  fa.n_pos = fs->n_pos;
  fa.converged = fs->converged;
  fa.n_iter = fs->n_iter;
  fa.deform = fs->deform;
  fa.deform_vel = fs->deform_vel;
  fa.ref_cell = fs->ref_cell;
  fa.cfg = *cfg;
  fa.iter_start = nullptr;
  fa.budget = -1;
  return fa;
}

// n_iter FIRE iterations of every open system with the per-iteration kernels, then a convergence
// check of the final positions.
static int fire_iterations(const ts_batch *batch, const ts_fire_state *fs, const ts_fire_config *cfg,
                           ts_neighbor_list *nl, const ts_pair_params *pp, const FireArgs &fa, int64_t n_iter,
                           void *force, double *energy, double *virial, int64_t max_atoms, hipStream_t st) {
  const bool cell = cfg->relax_cell != 0;
  const PairTable tab = make_table(pp);
  const int64_t S = batch->n_systems;
  // per-chunk partial sums in the list workspace's second adjoint buffer (6 N doubles, free during
  // a relaxation) and the per-system coefficients in the state's scratch after the virial slots
  const NlWork w = nl_work(nl->workspace, batch->n_atoms, S);
  double *part = w.adj_alt;
  double *coef = fs->scratch + 9 * S;
  // energy and virial are evaluated at every iteration: a system that converges (and is frozen)
  // before the last one keeps the values of its final configuration
  const bool ev = cell || energy || virial;
  for (int64_t it = 0; it <= n_iter; ++it) {
    const bool last = it == n_iter;
    int rc = nl_update(batch, nl, 0, max_atoms, st);
    if (rc != TS_OK) return rc;
    rc = launch_forces_batch(batch, nl, tab, pp->prec, force, energy, ev ? fa.virial : nullptr, fs->converged,
                             max_atoms, st);
    if (rc != TS_OK) return rc;
    rc = pp->prec == TS_PAIR_F32 ? launch_fire_update<float>(fa, cell, last ? 1 : 0, S, max_atoms, part, coef, st)
                                 : launch_fire_update<double>(fa, cell, last ? 1 : 0, S, max_atoms, part, coef, st);
    if (rc != TS_OK) return rc;
  }
  return TS_OK;
}

}  // namespace ts

extern "C" int ts_fire_step(const ts_batch *batch, ts_fire_state *fs, const ts_fire_config *cfg, ts_neighbor_list *nl,
                            const ts_pair_params *pp, int64_t n_iter, void *force, double *energy, double *virial,
                            int32_t persistent, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, true);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(fs && cfg && force && (n_iter >= 1 || n_iter == -1));
  TS_CHECK_ARG(fs->dt && fs->alpha && fs->n_pos && fs->converged && fs->n_iter && fs->scratch);
  TS_CHECK_ARG(cfg->fmax > 0.0 && cfg->dt_start > 0.0 && cfg->dt_max > 0.0 && cfg->f_dec > 0.0 && cfg->f_inc > 0.0);
  const bool cell = cfg->relax_cell != 0;
  if (cell) {
    TS_CHECK_ARG(fs->deform && fs->deform_vel && fs->ref_cell && cfg->cell_mass > 0.0);
    for (int64_t s = 0; s < batch->n_systems; ++s)
      TS_CHECK_ARG(batch->h_sys_offsets[s + 1] > batch->h_sys_offsets[s]);
  }
  hipStream_t st = ts::as_stream(stream);
  const int64_t S = batch->n_systems;
  double *vir = virial ? virial : fs->scratch;  // scratch holds [S][9] when the caller wants no virial
  ts::FireArgs fa = ts::make_fire_args(batch, fs, cfg, force, vir);
  // iterations of the per-iteration kernels enqueued by one call when the budget is open or larger
  const int64_t tail = (n_iter < 0 || n_iter > TS_FIRE_TAIL_ITERS) ? TS_FIRE_TAIL_ITERS : n_iter;
  if (persistent && max_atoms <= ts::kLdsMaxAtoms) {
    // n_iter at the start of the call, for the per-call budget of the tail (scratch slots 31 S..32 S)
    int64_t *iter_start = reinterpret_cast<int64_t *>(fs->scratch + 31 * S);
    TS_HIP(hipMemcpyAsync(iter_start, fs->n_iter, sizeof(int64_t) * S, hipMemcpyDeviceToDevice, st));
    bool handed_off = false;
    rc = ts::fire_persistent(batch, fs, cfg, nl, pp, n_iter, force, energy, virial, max_atoms, true, &handed_off, st);
    if (rc != TS_OK || !handed_off) return rc;
    // the tail: systems still iterating when the persistent launch stopped (it stops once most of
    // its workgroups are idle) continue with the per-iteration kernels, which spread every system
    // over many workgroups.  A fixed number of iterations is enqueued (the host reads nothing);
    // each one leaves converged systems, systems at max_iter and systems whose budget for this
    // call is spent untouched.
    fa.iter_start = iter_start;
    fa.budget = n_iter;
    return ts::fire_iterations(batch, fs, cfg, nl, pp, fa, tail, force, energy, virial, max_atoms, st);
  }
  rc = ts::fire_iterations(batch, fs, cfg, nl, pp, fa, tail, force, energy, virial, max_atoms, st);
  if (rc != TS_OK) return rc;
  return TS_OK;
}
