// Host-side validation, parameter tables and status strings.
#include <atomic>
#include <cmath>
#include <limits>

#include "ts_internal.h"

namespace ts {

int device_cus() {
  static std::atomic<int> cache[64];  // 0: not queried yet
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v > 0) return v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
  cache[dev].store(v, std::memory_order_relaxed);
  return v;
}

int validate_batch(const ts_batch *b, bool need_vel, int64_t *max_atoms) {
  TS_CHECK_ARG(b != nullptr);
  TS_CHECK_ARG(b->n_atoms >= 0 && b->n_systems >= 1);
  TS_CHECK_ARG(b->stride == 0 || b->stride >= b->n_atoms);
  TS_CHECK_ARG(b->sys_offsets && b->h_sys_offsets && b->system_idx && b->pos && b->cell);
  if (need_vel) TS_CHECK_ARG(b->vel != nullptr);
  const int64_t *o = b->h_sys_offsets;
  TS_CHECK_ARG(o[0] == 0 && o[b->n_systems] == b->n_atoms);
  int64_t mx = 0;
  for (int64_t s = 0; s < b->n_systems; ++s) {
    TS_CHECK_ARG(o[s + 1] >= o[s]);
    mx = o[s + 1] - o[s] > mx ? o[s + 1] - o[s] : mx;
  }
  if (mx > TS_MAX_SYSTEM_ATOMS) return TS_E_CAPACITY;
  if (max_atoms) *max_atoms = mx;
  return TS_OK;
}

int validate_params(const ts_pair_params *pp) {
  TS_CHECK_ARG(pp != nullptr);
  if (pp->kind < TS_LJ || pp->kind > TS_MORSE_SF) return TS_E_UNSUPPORTED;
  if (pp->prec != TS_PAIR_F32 && pp->prec != TS_PAIR_F64) return TS_E_UNSUPPORTED;
  TS_CHECK_ARG(pp->n_species >= 1 && pp->n_species <= TS_MAX_SPECIES);
  TS_CHECK_ARG(std::isfinite(pp->cutoff) && pp->cutoff > 0.0);
  for (int a = 0; a < pp->n_species; ++a)
    for (int b = 0; b < pp->n_species; ++b) {
      const double *p = pp->params[a][b];
      TS_CHECK_ARG(std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]));
      if (pp->kind == TS_LJ || pp->kind == TS_LJ_SF) TS_CHECK_ARG(p[1] > 0.0);
      if (pp->kind == TS_SOFT_SPHERE) TS_CHECK_ARG(p[1] > 0.0);
      if (pp->kind == TS_MORSE || pp->kind == TS_MORSE_SF) TS_CHECK_ARG(p[0] != 0.0 || p[1] != 0.0);
    }
  return TS_OK;
}

int validate_list(const ts_batch *b, const ts_neighbor_list *nl, bool need_workspace) {
  TS_CHECK_ARG(nl != nullptr);
  TS_CHECK_ARG(std::isfinite(nl->cutoff) && nl->cutoff > 0.0);
  TS_CHECK_ARG(std::isfinite(nl->skin) && nl->skin >= 0.0);
  TS_CHECK_ARG(nl->max_nbr >= 1);
  TS_CHECK_ARG(nl->bin_factor >= 1 && nl->bin_factor <= 4);
  TS_CHECK_ARG(nl->lanes_per_atom == 0 || nl->lanes_per_atom == 1 || nl->lanes_per_atom == 2 ||
               nl->lanes_per_atom == 4 || nl->lanes_per_atom == 8);
  TS_CHECK_ARG(nl->group_atoms >= 0 && nl->reserved == 0);
  TS_CHECK_ARG(nl->nbr && nl->n_nbr && nl->ref_pos && nl->ref_cell && nl->status);
  const bool alt = nl->nbr_alt != nullptr;  // the second row buffer: all three pointers or none
  TS_CHECK_ARG((nl->n_nbr_alt != nullptr) == alt && (nl->ref_pos_alt != nullptr) == alt);
  // the pair kernels address the entries with 32-bit byte offsets
  const int64_t stride = b->stride > 0 ? b->stride : b->n_atoms;
  if ((int64_t)((nl->max_nbr + 7) / 8) * (stride > 0 ? stride : 1) * 32 > (int64_t)UINT32_MAX) return TS_E_CAPACITY;
  if (need_workspace) {
    TS_CHECK_ARG(nl->workspace != nullptr);
    TS_CHECK_ARG(nl->workspace_bytes >= ts_neighbor_workspace_bytes(b->n_atoms, b->n_systems));
  }
  return TS_OK;
}

// phi'(r) of the plain LJ (kind TS_LJ) or Morse form and its derivatives by the parameter triple
static double dphi_at(int kind, const double *p, double r, double d[3]) {
  if (kind == TS_LJ) {
    const double s6 = std::pow(p[1] / r, 6), s12 = s6 * s6;
    const double v = 24.0 * p[0] / r * (s6 - 2.0 * s12);
    d[0] = 24.0 / r * (s6 - 2.0 * s12);
    d[1] = 24.0 * p[0] / r * (6.0 * s6 - 24.0 * s12) / p[1];
    d[2] = 0.0;
    return v;
  }
  const double x = std::exp(-p[1] * (r - p[2]));
  const double q = x - x * x, one_m = 1.0 - 2.0 * x;
  d[0] = 2.0 * p[1] * q;
  d[1] = 2.0 * p[0] * q - 2.0 * p[1] * p[0] * one_m * (r - p[2]) * x;
  d[2] = 2.0 * p[1] * p[1] * p[0] * one_m * x;
  return 2.0 * p[1] * p[0] * q;
}

static double phi_at(int kind, const double *p, double r) {
  if (kind == TS_LJ) {
    const double sr6 = std::pow(p[1] / r, 6);
    return 4.0 * p[0] * (sr6 * sr6 - sr6);
  }
  if (kind == TS_MORSE) {
    const double x = std::exp(-p[1] * (r - p[2]));
    return p[0] * (x * x - 2.0 * x);
  }
  return 0.0;
}

PairTable make_table(const ts_pair_params *pp) {
  PairTable t;
  std::memset(&t, 0, sizeof(t));
  t.n_species = pp->n_species;
  t.kind = pp->kind;
  t.cut2 = pp->cutoff * pp->cutoff;
  for (int a = 0; a < TS_MAX_SPECIES; ++a)
    for (int b = 0; b < TS_MAX_SPECIES; ++b) {
      PairCoef &c = t.c[a * TS_MAX_SPECIES + b];
      const double *p = pp->params[a][b];
      c.raw[0] = p[0];
      c.raw[1] = p[1];
      c.raw[2] = p[2];
      c.sig2 = std::numeric_limits<double>::infinity();
      if (a >= pp->n_species || b >= pp->n_species) continue;
      const bool sf = pp->kind == TS_LJ_SF || pp->kind == TS_MORSE_SF;
      const int base = pp->kind == TS_LJ_SF ? TS_LJ : (pp->kind == TS_MORSE_SF ? TS_MORSE : pp->kind);
      if (base == TS_LJ) {
        const double s6 = std::pow(p[1], 6);
        c.a = 4.0 * p[0] * s6 * s6;
        c.b = 4.0 * p[0] * s6;
      } else if (base == TS_MORSE) {
        c.a = p[0];
        c.b = p[1];
        c.c = p[2];
      } else {
        c.a = p[0];
        c.b = p[1];
        c.c = 1.0 / p[1];
        c.sig2 = p[1] * p[1];
      }
      c.shift = ((pp->shift_energy || sf) && base != TS_SOFT_SPHERE) ? phi_at(base, p, pp->cutoff) : 0.0;
      if (sf) {
        c.rc = pp->cutoff;
        c.fs = dphi_at(base, p, pp->cutoff, c.dfs);
      }
    }
  return t;
}

}  // namespace ts

extern "C" int ts_lorentz_berthelot(int32_t n_species, const double *eps, const double *sigma, ts_pair_params *pp) {
  TS_CHECK_ARG(eps && sigma && pp && n_species >= 1 && n_species <= TS_MAX_SPECIES);
  for (int a = 0; a < n_species; ++a)
    TS_CHECK_ARG(std::isfinite(eps[a]) && eps[a] >= 0.0 && std::isfinite(sigma[a]) && sigma[a] > 0.0);
  for (int a = 0; a < TS_MAX_SPECIES; ++a)
    for (int b = 0; b < TS_MAX_SPECIES; ++b) {
      double *p = pp->params[a][b];
      const bool in = a < n_species && b < n_species;
      p[0] = in ? std::sqrt(eps[a] * eps[b]) : 0.0;
      p[1] = in ? 0.5 * (sigma[a] + sigma[b]) : 0.0;
      p[2] = 0.0;
    }
  pp->n_species = n_species;
  return TS_OK;
}

extern "C" const char *ts_strerror(int status) {
  switch (status) {
    case TS_OK: return "ok";
    case TS_NOT_CONVERGED: return "not converged";
    case TS_E_INVALID: return "invalid argument";
    case TS_E_UNSUPPORTED: return "unsupported configuration";
    case TS_E_CAPACITY: return "size exceeds a library limit";
    case TS_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

extern "C" const char *ts_version(void) { return "ts-mi355x 0.1 (gfx950)"; }
