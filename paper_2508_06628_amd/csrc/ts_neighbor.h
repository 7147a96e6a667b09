// Neighbor-list workspace layout and the update routine used by the step loops.
#pragma once

#include "ts_internal.h"

namespace ts {

// Bin geometry of one system at its last build.
struct NlGeom {
  double inv[9];    // cell^-1 (row convention: s = r inv)
  double reach[3];  // r_list / w_k  (w_k perpendicular width)
  int n[3];         // bins along each direction
  int m[3];         // stencil half-width in bins
  int active;       // rebuilt by the current update
  int pad;
};

// Views into the caller's workspace.  Bins of system s start at 2 sys_offsets[s] + s (at most
// 2 N_s + 1 bins per system).
struct NlWork {
  NlGeom *geom;
  int32_t *flags;     // [S] rebuild requests
  int32_t *atom_bin;  // [N] local bin of each atom
  int32_t *atom_img;  // [N] packed integer image offset floor(s) of each atom
  int32_t *count;     // [2N+S] atoms per bin
  int32_t *start;     // [2N+S] first slot of each bin in perm (global atom index space)
  int32_t *fill;      // [2N+S] scatter cursors
  int32_t *perm;      // [N] atoms sorted by (system, bin, index)
  double *pos_alt;    // [3][N] second position buffer of the fused step loop
  double *adj_alt;    // [6][N] second adjoint buffers (positions, velocities) of the reverse loop
  int32_t *flags3;    // fused step loop: rebuild flags [3][S], flagged lists [3][S], counts [3]
  double *pos4;       // [N][4] positions packed per atom (x, y, z, unused) for neighbor gathers
  double *adj_slots;  // [adj_slot_count(S)][kAdjSlot] parameter-gradient partial sums (reverse loop, VJP)
  int32_t *sel2;      // deferred rebuild: row buffer of each system [2][S] (launch parity)
  int32_t *pflags3;   // deferred rebuild: pre-flags [3][S], pre-flagged lists [3][S], counts [3]
  double *row_geom;   // fused step loops: per-system cell geometry of the rebuilds [S][14]
  size_t bytes;
};

constexpr int kAdjSlot = TS_MAX_SPECIES * TS_MAX_SPECIES * 3;
// Partial-sum slots of the parameter gradient: one per system, at least 256 (so that workgroups
// spread over many words even for a single large system).
inline int64_t adj_slot_count(int64_t n_sys) { return n_sys > 256 ? n_sys : 256; }

NlWork nl_work(void *ws, int64_t n_atoms, int64_t n_sys);

// Enqueue the device-side validity test (force = 0) and the rebuild of the flagged systems.
int nl_update(const ts_batch *b, ts_neighbor_list *nl, int force, int64_t max_atoms, hipStream_t st);

}  // namespace ts
