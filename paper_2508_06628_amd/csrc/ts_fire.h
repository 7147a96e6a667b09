// FIRE launch interface shared by the per-iteration and the persistent paths.
#pragma once

#include "ts_forces.h"
#include "ts_neighbor.h"

namespace ts {

struct FireArgs {
  int64_t stride;
  const int64_t *offs;
  double *pos, *vel;
  const double *mass;
  double *cell;
  void *force;
  double *virial;  // [S][9] (relax_cell)
  double *dt, *alpha;
  int32_t *n_pos, *converged;
  int64_t *n_iter;
  double *deform, *deform_vel, *ref_cell;
  ts_fire_config cfg;
  const int64_t *iter_start;  // n_iter at the start of the call, or null (no per-call budget)
  int64_t budget;             // iterations per system in this call when iter_start is set (< 0: none)
};

FireArgs make_fire_args(const ts_batch *b, const ts_fire_state *fs, const ts_fire_config *cfg, void *force,
                        double *virial);

// One persistent launch over a work queue of systems (systems of at most kLdsMaxAtoms atoms).  With
// hand_off, workgroups still iterating stop (state written back, not converged) once most of the
// launch's workgroups have gone idle; *handed_off tells whether that can happen for this batch,
// in which case the caller continues the remaining systems with the per-iteration path.
int fire_persistent(const ts_batch *b, const ts_fire_state *fs, const ts_fire_config *cfg, ts_neighbor_list *nl,
                    const ts_pair_params *pp, int64_t n_iter, void *force, double *energy, double *virial,
                    int64_t max_atoms, bool hand_off, bool *handed_off, hipStream_t st);

}  // namespace ts
