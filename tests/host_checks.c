/* Host-side argument validation of every C-ABI entry point, run against the host-only build of the
 * library instrumented with AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_host_sanitized.py).
 * Every call below is rejected (or has nothing to do) before any device work, so no GPU is needed:
 * device pointers are fake addresses that are never dereferenced; host arrays are real.
 * Exit status 0 when every return code is the expected one. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ts_api.h"

static int failures = 0;
#define EXPECT(call, want)                                                                   \
  do {                                                                                       \
    int got_ = (call);                                                                       \
    if (got_ != (want)) {                                                                    \
      fprintf(stderr, "line %d: %s returned %d, expected %d\n", __LINE__, #call, got_, want); \
      ++failures;                                                                            \
    }                                                                                        \
  } while (0)

#define FAKE(T) ((T)(void *)0x1000)

static ts_batch make_batch(const int64_t *h_offs, int64_t n_sys) {
  ts_batch b;
  memset(&b, 0, sizeof(b));
  b.n_systems = n_sys;
  b.n_atoms = h_offs[n_sys];
  b.h_sys_offsets = h_offs;
  b.sys_offsets = FAKE(const int64_t *);
  b.system_idx = FAKE(const int32_t *);
  b.pos = FAKE(double *);
  b.vel = FAKE(double *);
  b.cell = FAKE(double *);
  return b;
}

static ts_pair_params make_pp(void) {
  ts_pair_params pp;
  memset(&pp, 0, sizeof(pp));
  pp.kind = TS_LJ;
  pp.prec = TS_PAIR_F32;
  pp.n_species = 1;
  pp.cutoff = 2.5;
  pp.params[0][0][0] = 1.0;
  pp.params[0][0][1] = 1.0;
  return pp;
}

static ts_neighbor_list make_nl(int64_t n_atoms, int64_t n_sys) {
  ts_neighbor_list nl;
  memset(&nl, 0, sizeof(nl));
  nl.cutoff = 2.5;
  nl.skin = 0.3;
  nl.max_nbr = 64;
  nl.bin_factor = 1;
  nl.nbr = FAKE(int32_t *);
  nl.n_nbr = FAKE(int32_t *);
  nl.ref_pos = FAKE(double *);
  nl.ref_cell = FAKE(double *);
  nl.status = FAKE(int64_t *);
  nl.workspace = FAKE(void *);
  nl.workspace_bytes = ts_neighbor_workspace_bytes(n_atoms, n_sys);
  return nl;
}

int main(void) {
  const int64_t offs[3] = {0, 10, 25};
  ts_batch b = make_batch(offs, 2);
  ts_pair_params pp = make_pp();
  ts_neighbor_list nl = make_nl(25, 2);
  void *F = FAKE(void *);

  /* library strings and sizes */
  if (strncmp(ts_version(), "ts-mi355x", 9) != 0) ++failures;
  for (int c = -5; c <= 2; ++c)
    if (ts_strerror(c) == NULL) ++failures;
  if (ts_neighbor_workspace_bytes(25, 2) == 0 || ts_neighbor_workspace_bytes(0, 1) == 0) ++failures;

  /* batch and parameter checks */
  const int64_t bad_last[3] = {0, 10, 24};
  ts_batch bb = make_batch(bad_last, 2);
  bb.n_atoms = 25;
  EXPECT(ts_pair_forces(&bb, &nl, &pp, F, NULL, NULL, NULL), TS_E_INVALID);
  const int64_t nonmono[4] = {0, 12, 10, 25};
  ts_batch bn = make_batch(nonmono, 3);
  ts_neighbor_list nl3 = make_nl(25, 3);
  EXPECT(ts_neighbor_build(&bn, &nl3, 1, NULL), TS_E_INVALID);
  ts_pair_params p2 = pp;
  p2.kind = 9;
  EXPECT(ts_pair_forces(&b, &nl, &p2, F, NULL, NULL, NULL), TS_E_UNSUPPORTED);
  p2 = pp;
  p2.prec = 7;
  EXPECT(ts_pair_forces(&b, &nl, &p2, F, NULL, NULL, NULL), TS_E_UNSUPPORTED);
  p2 = pp;
  p2.n_species = TS_MAX_SPECIES + 1;
  EXPECT(ts_pair_forces(&b, &nl, &p2, F, NULL, NULL, NULL), TS_E_INVALID);
  p2 = pp;
  p2.cutoff = NAN;
  EXPECT(ts_pair_forces(&b, &nl, &p2, F, NULL, NULL, NULL), TS_E_INVALID);
  p2 = pp;
  p2.params[0][0][1] = -1.0;
  EXPECT(ts_pair_forces(&b, &nl, &p2, F, NULL, NULL, NULL), TS_E_INVALID);
  EXPECT(ts_pair_forces(&b, &nl, &pp, NULL, NULL, NULL, NULL), TS_E_INVALID);
  EXPECT(ts_pair_forces(NULL, &nl, &pp, F, NULL, NULL, NULL), TS_E_INVALID);
  EXPECT(ts_pair_forces(&b, NULL, &pp, F, NULL, NULL, NULL), TS_E_INVALID);
  EXPECT(ts_pair_forces(&b, &nl, NULL, F, NULL, NULL, NULL), TS_E_INVALID);

  /* list checks */
  ts_neighbor_list n2 = nl;
  n2.workspace_bytes = 16;
  EXPECT(ts_neighbor_build(&b, &n2, 1, NULL), TS_E_INVALID);
  n2 = nl;
  n2.max_nbr = 0;
  EXPECT(ts_neighbor_build(&b, &n2, 1, NULL), TS_E_INVALID);
  n2 = nl;
  n2.skin = -0.5;
  EXPECT(ts_neighbor_build(&b, &n2, 1, NULL), TS_E_INVALID);
  n2 = nl;
  n2.bin_factor = 5;
  EXPECT(ts_neighbor_build(&b, &n2, 1, NULL), TS_E_INVALID);
  n2 = nl;
  n2.lanes_per_atom = 3;
  EXPECT(ts_pair_forces(&b, &n2, &pp, F, NULL, NULL, NULL), TS_E_INVALID);
  n2 = nl;
  n2.half = 1;
  EXPECT(ts_pair_forces(&b, &n2, &pp, F, NULL, NULL, NULL), TS_E_UNSUPPORTED);
  n2 = nl;
  n2.cutoff = 2.0;
  n2.skin = 0.1;
  EXPECT(ts_pair_forces(&b, &n2, &pp, F, NULL, NULL, NULL), TS_E_INVALID);
  n2 = nl;
  n2.max_nbr = 1 << 30; /* list beyond 4 GiB */
  EXPECT(ts_pair_forces(&b, &n2, &pp, F, NULL, NULL, NULL), TS_E_CAPACITY);
  const int64_t big[2] = {0, TS_MAX_SYSTEM_ATOMS + 1};
  ts_batch bbig = make_batch(big, 1);
  ts_neighbor_list nbig = make_nl(TS_MAX_SYSTEM_ATOMS + 1, 1);
  EXPECT(ts_neighbor_build(&bbig, &nbig, 1, NULL), TS_E_CAPACITY);

  /* integrators */
  EXPECT(ts_nve_step(&b, &nl, &pp, -1.0, 1.0, 10, F, NULL, NULL, NULL, 0, NULL), TS_E_INVALID);
  EXPECT(ts_nve_step(&b, &nl, &pp, 1.0, 0.0, 10, F, NULL, NULL, NULL, 0, NULL), TS_E_INVALID);
  ts_batch bv = b;
  bv.vel = NULL;
  EXPECT(ts_nve_step(&bv, &nl, &pp, 1.0, 1.0, 10, F, NULL, NULL, NULL, 0, NULL), TS_E_INVALID);
  double *kT = FAKE(double *);
  uint64_t *ctr = FAKE(uint64_t *);
  EXPECT(ts_langevin_step(&b, &nl, &pp, 1.0, 1.0, -0.1, kT, 1, ctr, 5, F, 0, NULL), TS_E_INVALID);
  EXPECT(ts_langevin_step(&b, &nl, &pp, 1.0, 1.0, NAN, kT, 1, ctr, 5, F, 0, NULL), TS_E_INVALID);
  EXPECT(ts_langevin_step(&b, &nl, &pp, 1.0, 1.0, 0.1, NULL, 1, ctr, 5, F, 0, NULL), TS_E_INVALID);
  EXPECT(ts_langevin_step(&b, &nl, &pp, 1.0, 1.0, 0.1, kT, 1, NULL, 5, F, 0, NULL), TS_E_INVALID);
  EXPECT(ts_langevin_step(&b, &nl, &pp, 1.0, 1.0, 0.1, kT, 1, ctr, -1, F, 0, NULL), TS_E_INVALID);
  ts_fire_config cfg;
  memset(&cfg, 0, sizeof(cfg));
  cfg.dt_start = 0.1;
  cfg.dt_max = 1.0;
  cfg.alpha_start = 0.1;
  cfg.f_inc = 1.1;
  cfg.f_dec = 0.5;
  cfg.f_alpha = 0.99;
  cfg.fmax = 0.01;
  cfg.cell_mass = 1.0;
  cfg.n_min = 5;
  cfg.max_iter = 1000;
  ts_fire_state fs;
  memset(&fs, 0, sizeof(fs));
  EXPECT(ts_fire_step(&b, &fs, &cfg, &nl, &pp, 10, F, NULL, NULL, 1, NULL), TS_E_INVALID); /* null state */
  fs.dt = fs.alpha = fs.scratch = FAKE(double *);
  fs.n_pos = fs.converged = FAKE(int32_t *);
  fs.n_iter = FAKE(int64_t *);
  EXPECT(ts_fire_step(&b, &fs, &cfg, &nl, &pp, 0, F, NULL, NULL, 1, NULL), TS_E_INVALID); /* n_iter */
  ts_fire_config c2 = cfg;
  c2.fmax = 0.0;
  EXPECT(ts_fire_step(&b, &fs, &c2, &nl, &pp, 10, F, NULL, NULL, 1, NULL), TS_E_INVALID);

  /* adjoint, RDF, export */
  double *lr = FAKE(double *), *lv = FAKE(double *), *tb = FAKE(double *);
  EXPECT(ts_pair_adjoint(&b, &nl, &pp, 0.0, 0.0, 0.0, lr, lv, tb, NULL), TS_E_INVALID);
  EXPECT(ts_pair_adjoint(&b, &nl, &pp, 0.0, 0.0, 1.0, NULL, lv, tb, NULL), TS_E_INVALID);
  ts_neighbor_list nows = nl;
  nows.workspace = NULL;
  nows.workspace_bytes = 0;
  EXPECT(ts_pair_adjoint(&b, &nows, &pp, 0.0, 0.0, 1.0, lr, lv, tb, NULL), TS_E_INVALID);
  EXPECT(ts_pair_adjoint_noalloc(&b, &nows, &pp, 0.0, 0.0, 1.0, lr, lv, tb, NULL), TS_OK);
  int64_t *many = (int64_t *)malloc(sizeof(int64_t) * 4098);
  for (int s = 0; s < 4098; ++s) many[s] = s;
  ts_batch bm = make_batch(many, 4097);
  ts_neighbor_list nm = make_nl(4097, 4097);
  nm.workspace = NULL;
  EXPECT(ts_pair_adjoint_noalloc(&bm, &nm, &pp, 0.0, 0.0, 1.0, lr, lv, tb, NULL), TS_E_CAPACITY);
  EXPECT(ts_pair_adjoint_noalloc(&bm, &nm, &pp, 0.0, 0.0, 1.0, lr, lv, NULL, NULL), TS_OK);
  free(many);
  double *g = FAKE(double *);
  EXPECT(ts_rdf_smeared(&b, &nl, 0, 10.0, 0.05, 2.8, g, NULL), TS_E_INVALID);
  EXPECT(ts_rdf_smeared(&b, &nl, 100, 10.0, -0.05, 2.8, g, NULL), TS_E_INVALID);
  EXPECT(ts_rdf_loss(NULL, g, 2, 100, g, g, NULL), TS_E_INVALID);
  EXPECT(ts_rdf_loss(g, g, 0, 100, g, g, NULL), TS_E_INVALID);
  int64_t *rp = FAKE(int64_t *), *eo = FAKE(int64_t *), *ei = FAKE(int64_t *);
  const double r_list = nl.cutoff + nl.skin;
  EXPECT(ts_graph_export(&b, &nl, r_list * 1.01, rp, eo, ei, NULL, NULL, 10, NULL), TS_E_INVALID);
  EXPECT(ts_graph_export(&b, &nl, 0.0, rp, eo, ei, NULL, NULL, 10, NULL), TS_E_INVALID);
  EXPECT(ts_graph_export(&b, &nl, 1.0, rp, eo, ei, NULL, NULL, -1, NULL), TS_E_INVALID);
  EXPECT(ts_kinetic_energy(NULL, 1.0, g, NULL), TS_E_INVALID);

  /* the Lorentz-Berthelot table: host arithmetic only */
  const double eps[3] = {1.0, 0.6, 1.4}, sig[3] = {1.0, 1.15, 0.9};
  ts_pair_params lb;
  memset(&lb, 0, sizeof(lb));
  EXPECT(ts_lorentz_berthelot(3, eps, sig, &lb), TS_OK);
  if (lb.n_species != 3 || fabs(lb.params[0][1][0] - sqrt(0.6)) > 1e-15 ||
      fabs(lb.params[1][2][1] - 0.5 * (1.15 + 0.9)) > 1e-15 || lb.params[3][3][0] != 0.0)
    ++failures;
  EXPECT(ts_lorentz_berthelot(0, eps, sig, &lb), TS_E_INVALID);
  EXPECT(ts_lorentz_berthelot(TS_MAX_SPECIES + 1, eps, sig, &lb), TS_E_INVALID);
  const double neg[1] = {-1.0};
  EXPECT(ts_lorentz_berthelot(1, neg, sig, &lb), TS_E_INVALID);

  if (failures) {
    fprintf(stderr, "%d host check(s) failed\n", failures);
    return 1;
  }
  printf("host checks ok\n");
  return 0;
}
