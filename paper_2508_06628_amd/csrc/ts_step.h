// Fused velocity-Verlet step kernels (one launch per step for systems that fit in LDS).
#pragma once

#include "ts_internal.h"
#include "ts_rng.h"

namespace ts {

constexpr int kStepFirst = 0;  // first half kick and drift (forces given)
constexpr int kStepMid = 1;    // forces, two half kicks, drift, validity test
constexpr int kStepLast = 2;   // forces (+ energy, virial), last half kick
constexpr int kStepForce = 3;  // forces only (ts_pair_forces)
constexpr int kStepForceEV = 4;  // forces, energy and virial (ts_pair_forces)
constexpr int kStepLangFirst = 5;  // Langevin: first half kick, half drift, O step, half drift
constexpr int kStepLangMid = 6;    // Langevin: forces, two half kicks, half drift, O step, half drift, validity
constexpr int kStepMidDefer = 7;      // kStepMid with the deferred rebuild (second row buffer)
constexpr int kStepLangMidDefer = 8;  // kStepLangMid with the deferred rebuild
constexpr int kStepThreads = 256;  // workgroup size of the step kernel
constexpr int kStepUnroll = 4;      // row entries a lane evaluates together in the step kernel
constexpr int kLdsMaxAtoms = 2048;  // largest system staged in LDS (3 x 8 B x atoms = 48 KiB)
constexpr int kDeferWgs = 256;      // rebuild workgroups of a step launch with the deferred rebuild
constexpr int kDeferRowsPerWave = 4;  // rows a wavefront of those builds per staging of its system
constexpr int kDeferSurvCap = 3 * 64;  // survivor queue of a rebuild wavefront (ints)

// Geometry of a cell for the row rebuild: inverse, determinant and reach per lattice direction.
struct RowGeom {
  double inv[9];
  double reach[3];
  double det;
  double bound;  // r_list + delta, the distance bound of the float32 prefilters of a rebuild
};

// Cell inverse (row convention: fractional = r inv), determinant, reach_k = r_list / w_k, with
// w_k = V / |a_{k+1} x a_{k+2}| the perpendicular width, and the prefilter bound of the cell h
// (rows are lattice vectors).
__device__ inline void row_geometry(const double *h, double r_list, RowGeom *g) {
  const double h00 = h[0], h01 = h[1], h02 = h[2], h10 = h[3], h11 = h[4], h12 = h[5], h20 = h[6], h21 = h[7],
               h22 = h[8];
  const double det = h00 * (h11 * h22 - h12 * h21) - h01 * (h10 * h22 - h12 * h20) + h02 * (h10 * h21 - h11 * h20);
  const double id = 1.0 / det;
  g->inv[0] = (h11 * h22 - h12 * h21) * id;
  g->inv[1] = (h02 * h21 - h01 * h22) * id;
  g->inv[2] = (h01 * h12 - h02 * h11) * id;
  g->inv[3] = (h12 * h20 - h10 * h22) * id;
  g->inv[4] = (h00 * h22 - h02 * h20) * id;
  g->inv[5] = (h02 * h10 - h00 * h12) * id;
  g->inv[6] = (h10 * h21 - h11 * h20) * id;
  g->inv[7] = (h01 * h20 - h00 * h21) * id;
  g->inv[8] = (h00 * h11 - h01 * h10) * id;
  g->det = det;
  const double vol = fabs(det);
  const double c0x = h11 * h22 - h12 * h21, c0y = h12 * h20 - h10 * h22, c0z = h10 * h21 - h11 * h20;
  const double c1x = h21 * h02 - h22 * h01, c1y = h22 * h00 - h20 * h02, c1z = h20 * h01 - h21 * h00;
  const double c2x = h01 * h12 - h02 * h11, c2y = h02 * h10 - h00 * h12, c2z = h00 * h11 - h01 * h10;
  g->reach[0] = r_list / (vol / sqrt(c0x * c0x + c0y * c0y + c0z * c0z));
  g->reach[1] = r_list / (vol / sqrt(c1x * c1x + c1y * c1y + c1z * c1z));
  g->reach[2] = r_list / (vol / sqrt(c2x * c2x + c2y * c2y + c2z * c2z));
  // delta bounds the float32 rounding of wrapped fractional coordinates and of the distances built
  // from them (a few 1e-5 A at most) with a wide margin
  const double rowsum = sqrt(h00 * h00 + h01 * h01 + h02 * h02) + sqrt(h10 * h10 + h11 * h11 + h12 * h12) +
                        sqrt(h20 * h20 + h21 * h21 + h22 * h22);
  g->bound = r_list + 1e-4 + 4e-6 * rowsum;
}

struct StepArgs {
  const int64_t *offs;
  const double *pos_in;  // r_n
  int64_t st_in;
  double *pos_out;  // r_{n+1}
  int64_t st_out;
  double *pos_final;  // last step: where r_N is copied (the caller's buffer), or null
  double *pos_copy;   // first step: where r_0 is copied (compact stride n_atoms), or null
  int64_t n_atoms;
  double *vel;        // velocities, forces, list rows and reference positions use st_vel
  int64_t st_vel;
  const double *mass;
  const int32_t *species;
  const double *cell;
  void *force;
  uint32_t *nbr;
  int32_t *n_nbr;
  int max_nbr;
  int half;
  double *ref_pos;
  double *ref_cell;
  int32_t *flag_cur, *flag_next, *flag_clear;  // per-system rebuild flags of steps n, n+1, n+2
  int32_t *list_cur, *list_next;               // flagged systems of steps n, n+1
  int32_t *count_cur, *count_next, *count_clear;
  int64_t *status;
  double r_list, skin;
  double half_dt, dt, accel;
  double *epot, *virial;
  int chunks;      // workgroups per system; chunk c owns atoms [c span, (c + 1) span) of its system
  int rounds;      // groups of kStepThreads/TL atoms a workgroup evaluates one after another
  int span;        // atoms per chunk: ceil(largest system / chunks) <= rounds * kStepThreads/TL
  int64_t n_work;  // n_systems * chunks (the grid is n_work rounded up to a multiple of kXcds)
  int n_sys;       // systems in the batch (rebuild launch)
  // Deferred rebuild (the list has its second row buffer): a system whose rows will soon fail the
  // validity bound is "pre-flagged" and rebuilt from r_n by extra workgroups of launch n (the first
  // n_defer_wgs of the grid) into the buffer it does not use in launch n; from launch n + 1 on it
  // reads that buffer.  sel_cur[s] / sel_next[s]: the buffer of system s in this / the next launch.
  uint32_t *nbr_alt;
  int32_t *n_nbr_alt;
  double *ref_pos_alt;
  const int32_t *sel_cur;
  int32_t *sel_next;
  int32_t *pflag_cur, *pflag_next, *pflag_clear;  // pre-flags of launches n-1 (rebuilt now), n, n+1
  int32_t *plist_cur, *plist_next;
  int32_t *pcount_cur, *pcount_next, *pcount_clear;
  int n_defer_wgs;       // rebuild workgroups at the start of the grid (0: none in this launch)
  int defer_chunks1;     // their chunks per system at one row per wavefront (largest system / 4 waves)
  double pre_factor;     // pre-flag when 2 (|r_{n+1} - ref| + pre_factor |r_{n+1} - r_n|) > skin
  const RowGeom *row_geom;  // per-system cell geometry of the rebuilds, or null (computed inline)
  const int32_t *skip;      // forces-only modes: systems whose forces, energy and virial stay as they are
  // Langevin modes: O step of this launch (step index lang_k of the call) and, with a non-null
  // rng_step, the counter advance by lang_adv done by the call's last launch
  LangParams lang;
  int lang_k;
  int lang_adv;
};

// Target number of non-empty workgroups of a step launch when the caller leaves the grouping open.
constexpr int64_t kStepTargetWgs = 4096;

// List validity bound of one atom: 2 |r - ref M| + r_list ||M - I||_F > skin, with
// M = ref_cell^-1 cell, and M = I exactly when the cell is bitwise unchanged.
__device__ inline bool bound_exceeded(double dm, double strain, double skin, double r_list) {
  const double lhs = 2.0 * dm + r_list * strain;
  return !(lhs <= skin);
}

__device__ inline bool list_invalid(const double r[3], const double *ref_pos, int64_t st, int64_t i, const double *h,
                                    const double *h0, double skin, double r_list) {
  bool same = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) same &= (h[k] == h0[k]);
  double r0[3], dlt[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r0[c] = ref_pos[c * st + i];
  double strain = 0.0;
  if (same) {
#pragma unroll
    for (int c = 0; c < 3; ++c) dlt[c] = r[c] - r0[c];
  } else {
    const double det = h0[0] * (h0[4] * h0[8] - h0[5] * h0[7]) - h0[1] * (h0[3] * h0[8] - h0[5] * h0[6]) +
                       h0[2] * (h0[3] * h0[7] - h0[4] * h0[6]);
    const double id = 1.0 / det;
    double hi[9], M[9];
    hi[0] = (h0[4] * h0[8] - h0[5] * h0[7]) * id;
    hi[1] = (h0[2] * h0[7] - h0[1] * h0[8]) * id;
    hi[2] = (h0[1] * h0[5] - h0[2] * h0[4]) * id;
    hi[3] = (h0[5] * h0[6] - h0[3] * h0[8]) * id;
    hi[4] = (h0[0] * h0[8] - h0[2] * h0[6]) * id;
    hi[5] = (h0[2] * h0[3] - h0[0] * h0[5]) * id;
    hi[6] = (h0[3] * h0[7] - h0[4] * h0[6]) * id;
    hi[7] = (h0[1] * h0[6] - h0[0] * h0[7]) * id;
    hi[8] = (h0[0] * h0[4] - h0[1] * h0[3]) * id;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) M[3 * p + q] = hi[3 * p] * h[q] + hi[3 * p + 1] * h[3 + q] + hi[3 * p + 2] * h[6 + q];
    double acc = 0.0;
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        const double e = M[3 * p + q] - (p == q ? 1.0 : 0.0);
        acc += e * e;
      }
    strain = sqrt(acc);
    for (int c = 0; c < 3; ++c) dlt[c] = r[c] - (r0[0] * M[c] + r0[1] * M[3 + c] + r0[2] * M[6 + c]);
  }
  return bound_exceeded(sqrt(norm2(dlt[0], dlt[1], dlt[2])), strain, skin, r_list);
}

// Candidate images of one (i, j) pair along one lattice direction: integers S with
// |f + S| < reach (+ a rounding margin), f the fractional difference.  The range is clipped to
// |S| <= TS_MAX_IMAGE_SHIFT + 1, so the candidate loops stay short whatever the input (an image
// at +-16 that is in range is reported by the caller's shift test); a range lying wholly beyond
// the clip sets *clipped; a non-finite f gives no candidate.
__device__ inline void image_range(double f, double reach, int *lo, int *hi, bool *clipped) {
  double l = ceil(-f - reach - 1e-9), h = floor(-f + reach + 1e-9);
  const double lim = TS_MAX_IMAGE_SHIFT + 1;
  if (!(l <= h)) {  // empty, or NaN
    *lo = 0;
    *hi = -1;
    return;
  }
  if (l > lim || h < -lim) {
    *clipped = true;
    *lo = 0;
    *hi = -1;
    return;
  }
  *lo = (int)fmax(l, -lim);
  *hi = (int)fmin(h, lim);
}

int launch_rebuild(const StepArgs &a, int64_t n_sys, int64_t max_atoms, hipStream_t st);

// Per-system RowGeom of the cells (cell inverse, determinant, reach at r_list) into out[S].
int launch_row_geometry(int64_t n_sys, const double *cell, double r_list, RowGeom *out, hipStream_t st);

// Copy back to the list's own buffer the rows of the systems with sel[s] = 1 (deferred rebuild).
int launch_rows_restore(const StepArgs &a, const int32_t *sel, int64_t n_sys, hipStream_t st);

// Pre-flag factor of the deferred rebuild: 2.0, or TS_DEFER_PREFACTOR from the environment.
double defer_pre_factor();

// Lanes per atom of the pair kernels: the list's choice, else 8 for batches too small to fill the
// chip with 4 (fewer than 2048 wavefronts, i.e. under 32768 atoms), 4 otherwise.
inline int lanes_for(const ts_neighbor_list *nl, int64_t n_atoms) {
  if (nl->lanes_per_atom > 0) return nl->lanes_per_atom;
  return n_atoms * 4 / kWave < 2048 ? 8 : 4;
}

// Fills a.chunks / a.rounds / a.n_work for lanes-per-atom tl and the caller's group size (0: from
// the batch shape; h_offs are the host system offsets) and launches the step kernel.
int launch_step(int mode, int tl, int group_atoms, StepArgs a, const PairTable &t, int prec, int64_t n_sys,
                int64_t max_atoms, const int64_t *h_offs, hipStream_t st);

// TS_NVE_UNFUSED=1 in the environment selects the multi-kernel step loops instead of the fused one.
bool fused_enabled();

// Fused step loop (k_rebuild_rows + k_step per step) over a batch whose systems fit in LDS, full
// list.  With traj != null every position r_0..r_N is written to traj ([N+1][3][n_atoms]); with
// lang != null the steps are BAOAB Langevin steps instead of velocity-Verlet ones.
int nve_fused_sequence(const ts_batch *b, ts_neighbor_list *nl, const PairTable &tab, int prec, double dt,
                       double accel, int n_steps, void *force, double *epot, double *ekin, double *virial,
                       int64_t max_atoms, hipStream_t st, double *traj = nullptr, const LangParams *lang = nullptr);

}  // namespace ts
