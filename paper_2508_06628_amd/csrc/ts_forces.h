// Pair-force launch interface shared by the step loops.
#pragma once

#include "ts_internal.h"

namespace ts {

struct ForceArgs {
  int64_t n, stride;
  const int32_t *sys_idx;
  const int64_t *offs;
  const double *pos;
  const double *cell;
  const int32_t *species;
  const uint32_t *nbr;
  const int32_t *n_nbr;
  void *force;
  double *energy;
  double *virial;
  const int32_t *skip;  // per-system flag: leave the system untouched (converged FIRE systems)
  double *pos4;         // workspace [N][4]: positions packed per atom for the neighbor gathers
};

ForceArgs make_force_args(const ts_batch *b, const ts_neighbor_list *nl, void *force, double *energy, double *virial,
                          const int32_t *skip);

// Zero energy/virial of the non-skipped systems (when requested) and launch the force kernel.
int launch_forces(const ForceArgs &a, int64_t n_sys, const PairTable &t, int prec, bool ev, hipStream_t st);

// Forces (and energy / virial when asked) of the systems whose skip entry is zero (skip may be
// null): the step loop's workgroup-per-system kernel when max_atoms fits in LDS, else launch_forces.
int launch_forces_batch(const ts_batch *b, const ts_neighbor_list *nl, const PairTable &t, int prec, void *force,
                        double *energy, double *virial, const int32_t *skip, int64_t max_atoms, hipStream_t st);

int validate_pair_call(const ts_batch *b, const ts_neighbor_list *nl, const ts_pair_params *pp, int64_t *max_atoms,
                       bool need_vel, bool need_workspace = true);

}  // namespace ts
