/*
 * ts_api.h -- C ABI of the MI355X (gfx950) batched pair-potential simulation library.
 *
 * The library advances many periodic systems of uneven size together, as the paper's batched
 * state does (TorchSim, arXiv 2508.06628, Section 3: atom-wise attributes concatenated,
 * system-wise attributes stacked).  It implements the classical pair-potential hot path:
 * cell-list neighbor build under triclinic periodic boundaries, Lennard-Jones / Morse /
 * soft-sphere energy, forces and virial (the model output schema of energies, forces and
 * stress, Section 2), velocity-Verlet NVE and FIRE relaxation (the integrators and relaxation
 * optimizers of the Abstract), and the adjoint of the pair step and the integrator used to
 * differentiate a trajectory observable (differentiable simulation, Section 2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every array pointer inside the structs below is a DEVICE pointer (memory from hipMalloc,
 *   e.g. a torch tensor's data_ptr) owned by the caller, unless the field says "host".
 *   The library never frees caller memory and never allocates inside a ts_* call, except
 *   for the hipGraph objects ts_nve_step keeps in its replay cache (see there).
 * - Positions, velocities, forces and adjoints are structure-of-arrays: component c of atom i
 *   is at p[c * stride + i], 0 <= i < n_atoms (stride >= n_atoms; 0 means n_atoms).
 * - cell is [S][3][3] row-major with row a = lattice vector a; Cartesian = fractional @ cell.
 *   The pair vector of the periodic image S in Z^3 is d = r_j - r_i + S @ cell.  Positions are
 *   never wrapped: whole lattice vectors by which a position sits outside its cell go into S.
 * - Atoms of system s are the contiguous range [sys_offsets[s], sys_offsets[s+1]).
 * - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default stream).  The
 *   return value reports only synchronous argument errors, checked before any launch.
 *   Conditions found while kernels run (neighbor-list overflow, non-finite positions,
 *   image-shift overflow) are written to the caller-owned device status words of the neighbor
 *   list, which the caller reads at a synchronisation point.  No exception crosses the ABI.
 * - Calls on one stream are ordered; calls that share output buffers on different streams race.
 */
#ifndef TS_API_H
#define TS_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef void *ts_stream_t; /* hipStream_t */

typedef enum {
  TS_OK = 0,
  TS_NOT_CONVERGED = 1,
  TS_E_INVALID = -1,     /* bad argument (null pointer, inconsistent sizes, singular cell ...) */
  TS_E_UNSUPPORTED = -2, /* valid but outside what this build implements */
  TS_E_CAPACITY = -3,    /* a size exceeds a documented limit of the library */
  TS_E_HIP = -4          /* the HIP runtime reported an error (launch, graph, device query) */
} ts_status;

typedef enum { TS_LJ = 0, TS_MORSE = 1, TS_SOFT_SPHERE = 2, TS_LJ_SF = 3, TS_MORSE_SF = 4 } ts_potential;
typedef enum { TS_PAIR_F32 = 0, TS_PAIR_F64 = 1 } ts_pair_prec;

#define TS_MAX_SPECIES 4
#define TS_MAX_SYSTEM_ATOMS 131072 /* atoms per system: 17-bit local index in a list entry */
#define TS_MAX_IMAGE_SHIFT 15      /* |S_k| per pair: 5-bit field in a list entry */

/* Neighbor-list status words (device int64[TS_STATUS_WORDS]); cumulative until the caller clears
   them (e.g. with a fill kernel or torch.zero_()). */
#define TS_STATUS_MAX_NBR 0   /* largest per-atom neighbor count found by any build (atomic max) */
#define TS_STATUS_OVERFLOW 1  /* 1 if some atom had more neighbors than max_nbr (list truncated) */
#define TS_STATUS_REBUILDS 2  /* number of system rebuilds performed */
#define TS_STATUS_NONFINITE 3 /* 1 if a build met a non-finite position or a singular cell */
#define TS_STATUS_SHIFT 4     /* 1 if an image shift fell outside [-15, 15] (entry dropped) */
#define TS_STATUS_WORDS 8

/* Batched state (paper Section 3: concatenated atom-wise, stacked system-wise attributes). */
typedef struct {
  int64_t n_atoms;              /* N: total atoms of all systems */
  int64_t n_systems;            /* S */
  int64_t stride;               /* leading dimension of the SoA arrays (0 = n_atoms) */
  const int64_t *sys_offsets;   /* device [S+1], nondecreasing, sys_offsets[0] = 0, [S] = N */
  const int64_t *h_sys_offsets; /* HOST copy of sys_offsets (launch planning and validation) */
  const int32_t *system_idx;    /* device [N]: system of each atom, consistent with sys_offsets */
  double *pos;                  /* device SoA [3][stride] float64 */
  double *vel;                  /* device SoA [3][stride] float64 (may be NULL for ts_pair_forces) */
  const double *mass;           /* device [N] float64; NULL = unit masses */
  const int32_t *species;       /* device [N] int32 in [0, n_species); NULL = all species 0 */
  double *cell;                 /* device [S][3][3] float64 */
} ts_batch;

/* Pair potential (paper Abstract: Lennard-Jones, Morse, soft-sphere).  Host struct, passed by
   pointer and copied at launch.  params[si][sj] holds
     TS_LJ:          (epsilon, sigma, unused)   phi = 4 eps ((sigma/r)^12 - (sigma/r)^6)
     TS_MORSE:       (D, alpha, r0)             phi = D (exp(-2 alpha (r - r0)) - 2 exp(-alpha (r - r0)))
     TS_SOFT_SPHERE: (epsilon, sigma_ij, unused) phi = eps/2 (1 - r/sigma_ij)^2 for r < sigma_ij
     TS_LJ_SF, TS_MORSE_SF: the LJ / Morse parameters, shifted-force truncation
                     phi_sf(r) = phi(r) - phi(r_c) - (r - r_c) phi'(r_c): energy and force both go
                     to zero continuously at the cutoff (smooth trajectory gradients)
   A pair interacts when r^2 < cutoff^2 (decided in float64), and for the soft sphere also
   r^2 < sigma_ij^2.  shift_energy = 1 subtracts phi(cutoff) inside the cutoff (LJ, Morse; the
   shifted-force kinds ignore it: they vanish at the cutoff by construction).
   prec = TS_PAIR_F32: the pair vector and the cutoff test are float64, the pair function is
   evaluated in float32 (soft sphere: overlap 1 - r/sigma_ij in float64), and forces, energies,
   virials are accumulated in float64; forces are stored as float32.  TS_PAIR_F64: all float64. */
typedef struct {
  int32_t kind;         /* ts_potential */
  int32_t prec;         /* ts_pair_prec */
  int32_t n_species;    /* 1..TS_MAX_SPECIES */
  int32_t shift_energy; /* 0 or 1 */
  double cutoff;        /* r_c > 0 */
  double params[TS_MAX_SPECIES][TS_MAX_SPECIES][3];
} ts_pair_params;

/* Neighbor list: padded per-atom rows in blocks of 8 entries.  Entry k of atom i is
   nbr[((k / 8) * stride + i) * 8 + k % 8] for k < n_nbr[i] <= max_nbr (so the 8 entries of a block
   of one atom are contiguous), packed as  j_local << 15 | (S0+16) << 10 | (S1+16) << 5 | (S2+16)
   with j_local = j - sys_offsets[system of i] (so each system may hold up to 2^17 atoms).
   Rows are sorted by the unsigned entry value, i.e. by (j_local, S0, S1, S2): every builder
   produces the same row for the same pair set. 
   A list built at (ref_pos, ref_cell) with list radius r_list = cutoff + skin holds every (j, S)
   with |d| < r_list (float64 test), j != i or S != 0, and stays valid while
   2 max_i |r_i - ref_i M| + r_list ||M - I||_F <= skin, M = ref_cell^-1 cell (M = I when the
   cell is bitwise unchanged); a system is rebuilt as soon as that bound is exceeded. */
typedef struct {
  double cutoff;       /* r_c of the consumer (pair potential cutoff, or the RDF range) */
  double skin;         /* >= 0 */
  int32_t half;        /* 0 = full list (each pair from both sides).  1 = half list (i<j, or
                          i==j with S lexicographically positive); the force, NVE, FIRE and
                          adjoint entry points require half = 0 */
  int32_t max_nbr;     /* per-atom capacity (rows of nbr) */
  int32_t bin_factor;  /* cell-list bins per list radius along each direction (1..4) */
  int32_t lanes_per_atom; /* lanes of a wavefront sharing one atom's row in the fused step
                             kernels: 1, 2, 4 or 8 (0 = 8 for batches under 32768 atoms, else 4) */
  int32_t group_atoms;  /* atoms one 256-lane workgroup of the fused step kernels owns (its system's
                           positions are staged in LDS once for all of them): rounded down to a
                           multiple of 256 / lanes_per_atom; 0 = chosen from the batch shape */
  int32_t reserved;     /* must be 0 */
  int32_t *nbr;        /* device [ceil(max_nbr / 8)][stride][8], at most 4 GiB (TS_E_CAPACITY) */
  int32_t *n_nbr;      /* device [N] */
  double *ref_pos;     /* device SoA [3][stride]: positions at the last build of each system */
  double *ref_cell;    /* device [S][9]: cell at the last build */
  int64_t *status;     /* device int64[TS_STATUS_WORDS] */
  void *workspace;     /* device, ts_neighbor_workspace_bytes(N, S) bytes, caller-owned */
  size_t workspace_bytes;
  /* Optional second row buffer (all three NULL, or all three set), used by the fused step loops
     (ts_nve_step, ts_langevin_step and ts_nve_record on systems of at most 2048 atoms) to rebuild
     lists one step ahead: a system whose rows are predicted to fail the validity bound at the next
     step (2 (|r_{n+1} - ref| + 2 |r_{n+1} - r_n|) > skin, the factor 2 overridable by the
     environment variable TS_DEFER_PREFACTOR) is rebuilt from r_n by extra workgroups of the next
     step launch into the buffer it does not read there, and reads that buffer from the launch
     after; a system whose rows do fail the bound is still rebuilt before the step that needs
     them, as without the second buffer.  Forces and trajectories are identical with and without
     it (pairs beyond the cutoff contribute exact zeros; rows are canonical).  On return every
     system's rows, lengths and reference positions are back in nbr, n_nbr and ref_pos. */
  int32_t *nbr_alt;     /* device, same shape as nbr */
  int32_t *n_nbr_alt;   /* device [N] */
  double *ref_pos_alt;  /* device SoA [3][stride] */
} ts_neighbor_list;

/* Bytes of device workspace a neighbor list needs for N atoms in S systems. */
size_t ts_neighbor_workspace_bytes(int64_t n_atoms, int64_t n_systems);

/* Build (force = 1) or update (force = 0) the neighbor list of every system.  With force = 0 a
   system is rebuilt only when the validity bound above is exceeded for it; the test and the
   rebuild both run on the device (no host synchronisation).  Binning: fractional coordinates
   s = r cell^-1 (float64) wrapped to [0, 1); n_k = max(1, floor(bin_factor w_k / r_list)) bins
   along direction k (w_k the perpendicular width), reduced until a system has at most 2 N_s + 1
   bins; every bin within reach (stencil ceil(r_list n_k / w_k), several images of one bin when
   the cell is narrower than 2 r_list) is searched.  Rows are in the canonical sorted order, so a
   list is a deterministic function of positions and cells.
   Errors: TS_E_INVALID (null pointers, sizes, cutoff <= 0, skin < 0, max_nbr < 1,
   workspace too small), TS_E_CAPACITY (a system above TS_MAX_SYSTEM_ATOMS). */
int ts_neighbor_build(const ts_batch *batch, ts_neighbor_list *nl, int32_t force, ts_stream_t stream);

/* The list exported as the graph a learned potential consumes (the graph construction whose cost
   dominates the differences between models, Section 4): every (i, j, S) of the list with
   |d| < r_graph, d = r_j - r_i + S cell (float64 test), as one edge, in the order (system,
   i, j, S0, S1, S2).  A full list gives both directions of every pair, a half list each pair once.
   Outputs (device, overwritten; E = edge_offsets[S] after the call):
     row_ptr      int64 [N + 1]  edges of atom i are row_ptr[i] .. row_ptr[i + 1] - 1
     edge_offsets int64 [S + 1]  edges of system s are edge_offsets[s] .. edge_offsets[s + 1] - 1
     edge_index   int64 [2][capacity]  row 0 = i (center), row 1 = j (global atom indices)
     edge_shift   int32 [capacity][3]  integer image S, or NULL to skip
     edge_vec     float64 [capacity][3]  d, or NULL to skip
   Edges at positions >= capacity are not written; the counts and offsets are complete, so a caller
   compares edge_offsets[S] with capacity after the call.  The list must be valid for the batch's
   positions (build or update it first) and r_graph <= cutoff + skin.  Asynchronous on `stream`.
   Errors: TS_E_INVALID (null pointers, r_graph outside (0, cutoff + skin], capacity < 0). */
int ts_graph_export(const ts_batch *batch, const ts_neighbor_list *nl, double r_graph, int64_t *row_ptr,
                    int64_t *edge_offsets, int64_t *edge_index, int32_t *edge_shift, double *edge_vec,
                    int64_t capacity, ts_stream_t stream);

/* Pair table of a Lennard-Jones mixture from per-species parameters by the Lorentz-Berthelot
   rules (the paper's classical potentials, Abstract, applied to several species):
     epsilon_ab = sqrt(epsilon_a epsilon_b),   sigma_ab = (sigma_a + sigma_b) / 2.
   Host call (no device work): eps and sigma are HOST arrays of n_species values; writes
   pp->params[a][b] = (epsilon_ab, sigma_ab, 0) for a, b < n_species, zeroes the other entries and
   sets pp->n_species; the caller sets kind = TS_LJ, prec, cutoff and shift_energy.
   Errors: TS_E_INVALID (null pointers, n_species outside 1..TS_MAX_SPECIES, an epsilon negative or
   not finite, a sigma not positive or not finite). */
int ts_lorentz_berthelot(int32_t n_species, const double *eps, const double *sigma, ts_pair_params *pp);

/* Energy per system, force per atom and virial per system from the pair potential:
     E_s = 1/2 sum_{(i,j,S)} [phi(r) - shift],  F_i = sum_{(j,S)} (phi'(r)/r) d,
     W_s = -1/2 sum_{(i,j,S)} (phi'(r)/r) d (x) d  (stress = -W/V).
   force: SoA [3][stride], float32 when prec = TS_PAIR_F32, float64 when TS_PAIR_F64 (overwritten).
   energy [S] and virial [S][9] (float64) are overwritten; either may be NULL to skip it.
   The list must be valid for the batch's positions (build it first).
   Errors: TS_E_INVALID, TS_E_UNSUPPORTED (half list, unknown kind/prec). */
int ts_pair_forces(const ts_batch *batch, const ts_neighbor_list *nl, const ts_pair_params *pp, void *force,
                   double *energy, double *virial, ts_stream_t stream);

/* n_steps of velocity-Verlet NVE on every system (kick-drift-kick, one force evaluation per step):
     v += dt/2 a F/m;  r += dt v;  [list update];  F = F(r);  v += dt/2 a F/m
   with a = accel (force/mass -> length/time^2; 0.009648533215665327 for eV, A, amu, fs).
   force: in: F(r_0) valid (f32 or f64 as pp->prec); out: F(r_n).  The neighbor list is updated
   on the device each step by the validity bound.  On return (when the stream completes)
   epot [S], ekin [S] = 1/2 sum m v^2 / accel and virial [S][9] hold the final state's values
   (each may be NULL).  use_graph = 1 captures the whole step loop in one hipGraph that is cached
   (keyed by every argument) and replayed on later identical calls; the cache holds at most 16
   graphs per process and is released by ts_release_graphs().  use_graph = 0 launches eagerly.
   Errors: TS_E_INVALID (dt or accel not finite/positive, n_steps < 0, vel NULL ...),
   TS_E_UNSUPPORTED, TS_E_HIP (graph capture failed). */
int ts_nve_step(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp, double dt, double accel,
                int32_t n_steps, void *force, double *epot, double *ekin, double *virial, int32_t use_graph,
                ts_stream_t stream);

/* ts_nve_step that also records the trajectory: traj is device float64 [n_steps+1][3][n_atoms]
   (compact structure-of-arrays, stride n_atoms) and receives r_0 .. r_{n_steps}; the batch ends at
   r_{n_steps} as with ts_nve_step.  This is the forward recomputation of a checkpointed segment
   for ts_adjoint_segment.  Systems of at most 2048 atoms (TS_E_UNSUPPORTED otherwise).
   Graph caching as ts_nve_step. */
int ts_nve_record(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp, double dt, double accel,
                  int32_t n_steps, void *force, double *traj, int32_t use_graph, ts_stream_t stream);

/* n_steps of Langevin (NVT) dynamics, the integrator of the paper's batched MD benchmark
   (Section 4), as the BAOAB splitting (Leimkuhler and Matthews 2013; the paper names no scheme):
     v += dt/2 a F/m;  r += dt/2 v;  v = c1 v + sqrt((1 - c1^2) a kT_s / m) xi;  r += dt/2 v;
     [list update];  F = F(r);  v += dt/2 a F/m,        c1 = exp(-gamma dt),
   a = accel as in ts_nve_step, gamma >= 0 the friction (1/time), kT device [S] the per-system
   temperature in energy units.  The normals xi of atom i at step t come from the counter-based
   generator Philox4x32-10 (Salmon et al., SC 2011) with key (seed low word, seed high word) and
   counter (i, t low word, t high word, 0): uniforms (x_k + 1/2) 2^-32, Box-Muller pairs
   (u0, u1) -> x, y and (u2, u3) -> z (cosine branch).  rng_step: device uint64 counter t of the
   first step, advanced by n_steps by the call (so a cached graph replays new numbers).
   force: in F(r_0), out F(r_n), as ts_nve_step.  gamma = 0 gives velocity Verlet (with the drift
   in two halves).  Graph caching as ts_nve_step (the key holds seed and gamma, not the counter).
   Errors: TS_E_INVALID (dt, accel not finite/positive, gamma negative or not finite, kT or
   rng_step NULL, n_steps < 0, vel NULL, more than 2^32 atoms), TS_E_UNSUPPORTED, TS_E_HIP. */
int ts_langevin_step(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp, double dt, double accel,
                     double gamma, const double *kT, uint64_t seed, uint64_t *rng_step, int32_t n_steps, void *force,
                     int32_t use_graph, ts_stream_t stream);

/* FIRE relaxation (Bitzek et al., PRL 97, 170201 (2006); the paper's structural relaxation
   optimizers, Abstract).  Per system and iteration: forces; stop if converged
   (max_i |F_i| < fmax, and with relax_cell also max |G_ab| < fmax); from the second iteration on
   P = g.v: P > 0 -> v = (1-alpha) v + alpha |v| g/|g|, n_pos++, and after n_min such steps
   dt = min(f_inc dt, dt_max), alpha *= f_alpha; P <= 0 -> v = 0, dt *= f_dec, alpha = alpha_start,
   n_pos = 0; then v += dt g/m and x += dt v (time unit: acceleration = F/m).
   relax_cell = 1 adds the cell: r_i = q_i D, cell = ref_cell D (D_0 = I); atom coordinates q_i
   with g_i = F_i D^T; cell coordinate Y = N_s D with force G = D^-T W / N_s and mass cell_mass;
   zero external pressure.  Velocities of q live in batch->vel. */
typedef struct {
  double dt_start, dt_max, alpha_start, f_inc, f_dec, f_alpha, fmax, cell_mass;
  int32_t n_min, relax_cell;
  int64_t max_iter; /* per system; a system that reaches it stops with converged = 0 */
} ts_fire_config;

typedef struct {
  double *dt;         /* device [S] */
  double *alpha;      /* device [S] */
  int32_t *n_pos;     /* device [S] */
  int32_t *converged; /* device [S] */
  int64_t *n_iter;    /* device [S]: updates performed so far */
  double *deform;     /* device [S][9]: D (relax_cell only; may be NULL otherwise) */
  double *deform_vel; /* device [S][9]: velocity of Y (relax_cell only) */
  double *ref_cell;   /* device [S][9]: cell at D = I (relax_cell only) */
  double *scratch;    /* device [S][32] float64 working space */
} ts_fire_state;

/* Advance every unconverged system by up to n_iter FIRE iterations (n_iter >= 1, or -1 for no
   per-call budget), then evaluate forces and the convergence test at the final configuration: on
   completion force/energy/virial (each may be NULL; force is required) describe each system's
   final positions and converged[] is current.  Like every call, ts_fire_step only enqueues work:
   it never waits for the device and reads nothing back, so the host learns where each system
   stands from converged[] and n_iter[] after synchronising.
   persistent = 0: each iteration is a few launches over the whole batch; the call enqueues
   min(n_iter, TS_FIRE_TAIL_ITERS) iterations (TS_FIRE_TAIL_ITERS when n_iter = -1).
   persistent = 1: one persistent launch; workgroups take systems from a device work queue
   (largest first), keep a system's positions in LDS and iterate it until it converges, reaches
   max_iter or spends the call's budget, before taking the next, so a converged system frees its
   workgroup at once (the in-flight batching of the paper's Section 3, on the device).  With more
   systems than a quarter of the compute units, the launch stops once only that many workgroups
   are still iterating, and the systems still open continue with the per-iteration kernels for
   min(n_iter, TS_FIRE_TAIL_ITERS) more iterations (TS_FIRE_TAIL_ITERS when n_iter = -1).  So a
   call with n_iter = -1, or with n_iter > TS_FIRE_TAIL_ITERS, may return with systems still open
   (converged = 0, n_iter below max_iter): call again until converged[] or max_iter says stop.
   Systems above 2048 atoms use the per-iteration path.
   The caller initialises the state (vel = 0, dt = dt_start, alpha = alpha_start, n_pos = 0,
   converged = 0, n_iter = 0, deform = I, deform_vel = 0, ref_cell = cell).
   Errors: TS_E_INVALID, TS_E_UNSUPPORTED. */
#define TS_FIRE_TAIL_ITERS 256
int ts_fire_step(const ts_batch *batch, ts_fire_state *fs, const ts_fire_config *cfg, ts_neighbor_list *nl,
                 const ts_pair_params *pp, int64_t n_iter, void *force, double *energy, double *virial,
                 int32_t persistent, ts_stream_t stream);

/* Adjoint of velocity-Verlet sub-steps (differentiable simulation, paper Section 2).  With
   lr = adj_pos = dL/dr and lv = adj_vel = dL/dv (SoA float64), u = accel lv / m and J = dF/dr
   evaluated at batch->pos:
     lv += dt_drift lr;   lr += w_kick J u;   adj_params[si][sj][k] += w_kick sum_i u_i . dF_i/dtheta
   where theta = params[si][sj][k] of the pair potential, accumulated per ordered species pair of
   the full list (for a symmetric parameter the gradient is [a][b][k] + [b][a][k] when a != b).
   Per pair: (J u)_i += phi'' (d^.du) d^ + (phi'/r)(du - (d^.du) d^), du = u_j - u_i.
   One reverse velocity-Verlet step from (lr, lv) at step n+1 to step n is
     (dt_drift = 0, w_kick = dt/2) at r_{n+1}, then (dt_drift = dt, w_kick = dt/2) at r_n;
   consecutive half kicks at the same positions merge into one call with w_kick = dt.
   adj_params is device float64 [TS_MAX_SPECIES][TS_MAX_SPECIES][3] (may be NULL).
   Pair arithmetic follows pp->prec; every accumulator is float64. */
int ts_pair_adjoint(const ts_batch *batch, const ts_neighbor_list *nl, const ts_pair_params *pp, double dt_drift,
                    double w_kick, double accel, double *adj_pos, double *adj_vel, double *adj_params,
                    ts_stream_t stream);

/* ts_pair_adjoint for callers that cannot allocate device memory (code under hipGraph capture,
   tight serving loops, harnesses that forbid hipMalloc): the same operation, arguments and results,
   but the parameter-gradient partial sums live in a library-held device array instead of the list's
   workspace, so nl->workspace may be NULL (nl->workspace_bytes is then ignored) and the call makes no
   allocation of any kind.  Limit: with adj_params != NULL at most 4096 systems (TS_E_CAPACITY
   beyond; without adj_params any batch size).  The array is 1.5 MiB per GPU, held from the first
   call on that GPU until the process ends; its address is looked up once per device.  Every call
   on one GPU shares that GPU's array (each call clears what it uses): calls that overlap in time
   on one GPU (different streams, or host threads) race and must be serialised by the caller. */
int ts_pair_adjoint_noalloc(const ts_batch *batch, const ts_neighbor_list *nl, const ts_pair_params *pp,
                            double dt_drift, double w_kick, double accel, double *adj_pos, double *adj_vel,
                            double *adj_params, ts_stream_t stream);

/* Reverse velocity-Verlet over one recorded segment r_{n0} .. r_{n0+n_steps} (traj as written by
   ts_nve_record; the batch supplies masses, species and cells).  Positions are processed from
   r_{n0+n_steps} down to r_{n0+1}, and also r_{n0} when bottom = 1 (n0 = 0); at each the adjoint
   state advances as in ts_pair_adjoint with (dt_drift, w_kick) = (dt, dt), except (0, dt/2) at the
   trajectory's last position when top = 1 and (dt, dt/2) at r_0 when bottom = 1.  Chaining the
   segments from the last to the first (top = 1 on the last one, bottom = 1 on the first) is the
   full reverse pass.  One launch per step (plus a rebuild launch that exits at once when no list
   needs one); graph caching as ts_nve_step.  Systems of at most 2048 atoms. */
int ts_adjoint_segment(const ts_batch *batch, ts_neighbor_list *nl, const ts_pair_params *pp, const double *traj,
                       int32_t n_steps, double dt, double accel, int32_t top, int32_t bottom, double *adj_pos,
                       double *adj_vel, double *adj_params, int32_t use_graph, ts_stream_t stream);

/* Gaussian-smeared radial distribution function per system over the full pair set within r_max
   (the list's radius must be >= r_max):
     g_s(r_b) = sum_{(i,j,S), |d| < r_max} N(r_b - |d|; sigma) / (4 pi r_b^2 rho_s N_s),
   r_b = (b + 1/2) r_end / n_bins, rho_s = N_s / V_s, N the normal density of std sigma.
   g: device float64 [S][n_bins], overwritten. */
int ts_rdf_smeared(const ts_batch *batch, const ts_neighbor_list *nl, int32_t n_bins, double r_end, double sigma,
                   double r_max, double *g, ts_stream_t stream);

/* Mean-squared RDF loss L = 1/(S n_bins) sum (g - g_target)^2 and dL/dg.  loss: device float64[1];
   dl_dg: device [S][n_bins] (either may be NULL). */
int ts_rdf_loss(const double *g, const double *g_target, int64_t n_systems, int32_t n_bins, double *loss,
                double *dl_dg, ts_stream_t stream);

/* Accumulate grad_pos += d(sum_{s,b} dl_dg[s][b] g_s(r_b)) / d pos (SoA float64 [3][stride]). */
int ts_rdf_vjp(const ts_batch *batch, const ts_neighbor_list *nl, int32_t n_bins, double r_end, double sigma,
               double r_max, const double *dl_dg, double *grad_pos, ts_stream_t stream);

/* ekin[s] = 1/2 sum_{i in s} m_i |v_i|^2 / accel (float64, overwritten). */
int ts_kinetic_energy(const ts_batch *batch, double accel, double *ekin, ts_stream_t stream);

/* Release every cached hipGraph (see ts_nve_step). */
void ts_release_graphs(void);

/* Static description of a status code. */
const char *ts_strerror(int status);

/* Library version string. */
const char *ts_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TS_API_H */
