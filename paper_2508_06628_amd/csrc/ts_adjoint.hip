// Adjoint of the pair step and the velocity-Verlet integrator, and the Gaussian-smeared RDF
// observable with its vector-Jacobian product (differentiable simulation, paper Section 2:
// gradients of an RDF computed at the end of a trajectory with respect to potential parameters).
//
// Per pair (i, j, S), with d = r_j - r_i + S cell, r = |d|, g = phi'/r, h = phi'' and
// du = u_j - u_i, the Hessian-vector product added to atom i is
//     K du = (h - g) (d . du) / r^2 d + g du,
// and the parameter term is (dg/dtheta)(u_i . d).  Pair arithmetic in the pair precision,
// accumulators in float64.
#include <mutex>

#include "ts_adjoint.h"
#include "ts_forces.h"
#include "ts_neighbor.h"

namespace ts {

struct AdjArgs {
  int64_t n, stride;
  const int32_t *sys_idx;
  const int64_t *offs;
  const double *pos, *cell, *mass;
  const int32_t *species;
  const uint32_t *nbr;
  const int32_t *n_nbr;
  double *lr;        // adj_pos (in/out)
  const double *lv;  // adj_vel (read)
  double *adj_params;
  double *slots;   // [n_slots][kAdjSlot] partial sums of the parameter gradient
  int64_t n_slots;
  double w, accel;
};

// adj_params[k] += sum over the slots of slots[q][k]
__global__ void k_sum_slots(int64_t n_slots, const double *__restrict__ slots, double *__restrict__ adj_params) {
  const int k = threadIdx.x;
  if (k >= kAdjSlot) return;
  double v = 0.0;
  for (int64_t q = 0; q < n_slots; ++q) v += slots[(int64_t)kAdjSlot * q + k];
  adj_params[k] += v;
}

int launch_sum_slots(int64_t n_slots, const double *slots, double *adj_params, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_slots, dim3(1), dim3(kAdjSlot), 0, st, n_slots, slots, adj_params);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

__global__ void k_adj_drift(int64_t n, int64_t st, const double *__restrict__ lr, double *__restrict__ lv, double dt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) lv[c * st + i] = lv[c * st + i] + dt * lr[c * st + i];
}

template <int KIND, typename T, bool SINGLE>
__global__ void __launch_bounds__(256) k_pair_vjp(PairTable tab, AdjArgs a) {
  __shared__ double acc[TS_MAX_SPECIES * TS_MAX_SPECIES * 3];
  __shared__ PairCoef ltab[TS_MAX_SPECIES * TS_MAX_SPECIES];
  if (!SINGLE) table_to_lds(ltab);
  if (!SINGLE) {
    for (int k = threadIdx.x; k < TS_MAX_SPECIES * TS_MAX_SPECIES * 3; k += blockDim.x) acc[k] = 0.0;
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < a.n;
  double tp0 = 0.0, tp1 = 0.0, tp2 = 0.0;
  if (valid) {
    const int64_t st = a.stride;
    const int s = a.sys_idx[i];
    const int64_t a0 = a.offs[s];
    const double *h = a.cell + 9 * (int64_t)s;
    const double rx = a.pos[i], ry = a.pos[st + i], rz = a.pos[2 * st + i];
    const double sci = a.mass ? a.accel / a.mass[i] : a.accel;
    const double uix = sci * a.lv[i], uiy = sci * a.lv[st + i], uiz = sci * a.lv[2 * st + i];
    const int si = (SINGLE || a.species == nullptr) ? 0 : a.species[i];
    const int nn = a.n_nbr[i];
    double jx = 0.0, jy = 0.0, jz = 0.0;
    const PairCoef pc0 = tab.c[0];
    for (int k = 0; k < nn; ++k) {
      const uint32_t ent = a.nbr[row_index(k, i, st)];
      const int64_t j = a0 + entry_j(ent);
      const double S0 = (double)entry_s0(ent), S1 = (double)entry_s1(ent), S2 = (double)entry_s2(ent);
      const double dx = shift_comp(a.pos[j] - rx, S0, S1, S2, h[0], h[3], h[6]);
      const double dy = shift_comp(a.pos[st + j] - ry, S0, S1, S2, h[1], h[4], h[7]);
      const double dz = shift_comp(a.pos[2 * st + j] - rz, S0, S1, S2, h[2], h[5], h[8]);
      const double r2 = norm2(dx, dy, dz);
      if (!(r2 < tab.cut2)) continue;
      const int sj = (SINGLE || a.species == nullptr) ? 0 : a.species[j];
      const PairCoef &pc = (SINGLE || a.species == nullptr) ? pc0 : ltab[si * TS_MAX_SPECIES + sj];
      if (KIND == TS_SOFT_SPHERE && !(r2 < pc.sig2)) continue;
      const double scj = a.mass ? a.accel / a.mass[j] : a.accel;
      const double dux = scj * a.lv[j] - uix, duy = scj * a.lv[st + j] - uiy, duz = scj * a.lv[2 * st + j] - uiz;
      T g, hh;
      pair_g_h<KIND, T>(pc, (T)r2, r2, &g, &hh);
      const T tx = (T)dx, ty = (T)dy, tz = (T)dz;
      const T ux = (T)dux, uy = (T)duy, uz = (T)duz;
      const T proj = tx * ux + ty * uy + tz * uz;
      const T coef = (hh - g) * proj / (T)r2;
      jx += (double)(coef * tx + g * ux);
      jy += (double)(coef * ty + g * uy);
      jz += (double)(coef * tz + g * uz);
      if (a.adj_params) {
        double dg[3];
        pair_dg_dparams<KIND>(pc, r2, dg);
        const double ud = uix * dx + uiy * dy + uiz * dz;
        if (SINGLE) {
          tp0 += dg[0] * ud;
          tp1 += dg[1] * ud;
          tp2 += dg[2] * ud;
        } else {
          double *q = acc + 3 * (si * TS_MAX_SPECIES + sj);
          atomicAdd(&q[0], a.w * dg[0] * ud);
          atomicAdd(&q[1], a.w * dg[1] * ud);
          atomicAdd(&q[2], a.w * dg[2] * ud);
        }
      }
    }
    a.lr[i] = a.lr[i] + a.w * jx;
    a.lr[st + i] = a.lr[st + i] + a.w * jy;
    a.lr[2 * st + i] = a.lr[2 * st + i] + a.w * jz;
  }
  if (a.adj_params) {
    // workgroup sums go to one of many slots (one word for the whole launch would serialise the
    // atomics of every wavefront); the caller sums the slots afterwards
    double *slot = a.slots + (int64_t)kAdjSlot * (blockIdx.x % a.n_slots);
    if (SINGLE) {
      __shared__ double wsum[256 / kWave][3];
      const double t0 = wave_sum(a.w * tp0), t1 = wave_sum(a.w * tp1), t2 = wave_sum(a.w * tp2);
      if (__lane_id() == 0) {
        wsum[threadIdx.x / kWave][0] = t0;
        wsum[threadIdx.x / kWave][1] = t1;
        wsum[threadIdx.x / kWave][2] = t2;
      }
      __syncthreads();
      if (threadIdx.x < 3) {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 256 / kWave; ++q) v += wsum[q][threadIdx.x];
        atomicAdd(&slot[threadIdx.x], v);
      }
    } else {
      __syncthreads();
      for (int k = threadIdx.x; k < kAdjSlot; k += blockDim.x)
        if (acc[k] != 0.0) atomicAdd(&slot[k], acc[k]);
    }
  }
}

template <int KIND, typename T>
static void launch_vjp(const AdjArgs &a, const PairTable &t, bool single, hipStream_t st) {
  const dim3 g((unsigned)ceil_div(a.n, 256));
  if (single)
    hipLaunchKernelGGL((k_pair_vjp<KIND, T, true>), g, dim3(256), 0, st, t, a);
  else
    hipLaunchKernelGGL((k_pair_vjp<KIND, T, false>), g, dim3(256), 0, st, t, a);
}

// ----------------------------------------------------------------------------- RDF

__device__ inline double cell_volume(const double *h) {
  return fabs(h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
              h[2] * (h[3] * h[7] - h[4] * h[6]));
}

struct RdfArgs {
  int64_t n, stride;
  const int32_t *sys_idx;
  const int64_t *offs;
  const double *pos, *cell;
  const uint32_t *nbr;
  const int32_t *n_nbr;
  int n_bins;
  double dr, sigma, rmax2;
};

// Histogram of exp(-(r_b - r)^2 / 2 sigma^2) over ordered pairs (bins within 10 sigma of r).
__global__ void __launch_bounds__(256) k_rdf_hist(RdfArgs a, double *g) {
  extern __shared__ double lh[];
  const int64_t first = (int64_t)blockIdx.x * blockDim.x;
  const int s_blk = a.sys_idx[first < a.n ? first : a.n - 1];
  for (int b = threadIdx.x; b < a.n_bins; b += blockDim.x) lh[b] = 0.0;
  __syncthreads();
  const int64_t i = first + threadIdx.x;
  if (i < a.n) {
    const int64_t st = a.stride;
    const int s = a.sys_idx[i];
    const int64_t a0 = a.offs[s];
    const double *h = a.cell + 9 * (int64_t)s;
    const double rx = a.pos[i], ry = a.pos[st + i], rz = a.pos[2 * st + i];
    const int nn = a.n_nbr[i];
    const double inv2s2 = 1.0 / (2.0 * a.sigma * a.sigma);
    const double span = 10.0 * a.sigma;
    for (int k = 0; k < nn; ++k) {
      const uint32_t ent = a.nbr[row_index(k, i, st)];
      const int64_t j = a0 + entry_j(ent);
      const double S0 = (double)entry_s0(ent), S1 = (double)entry_s1(ent), S2 = (double)entry_s2(ent);
      const double dx = shift_comp(a.pos[j] - rx, S0, S1, S2, h[0], h[3], h[6]);
      const double dy = shift_comp(a.pos[st + j] - ry, S0, S1, S2, h[1], h[4], h[7]);
      const double dz = shift_comp(a.pos[2 * st + j] - rz, S0, S1, S2, h[2], h[5], h[8]);
      const double r2 = norm2(dx, dy, dz);
      if (!(r2 < a.rmax2)) continue;
      const double r = sqrt(r2);
      int b0 = (int)floor((r - span) / a.dr - 0.5);
      int b1 = (int)ceil((r + span) / a.dr - 0.5);
      b0 = b0 < 0 ? 0 : b0;
      b1 = b1 > a.n_bins - 1 ? a.n_bins - 1 : b1;
      // exp(-x_b^2 k) for x_b = x_0 + (b - b0) dr by the exact recurrence e_{b+1} = e_b q_b,
      // q_{b+1} = q_b c (two exponentials per pair instead of one per bin)
      const double x0 = (b0 + 0.5) * a.dr - r;
      double e = exp(-x0 * x0 * inv2s2), q = exp(-(2.0 * x0 * a.dr + a.dr * a.dr) * inv2s2);
      const double c = exp(-2.0 * a.dr * a.dr * inv2s2);
      for (int b = b0; b <= b1; ++b) {
        if (s == s_blk)
          atomicAdd(&lh[b], e);
        else
          atomicAdd(&g[(int64_t)s * a.n_bins + b], e);
        e *= q;
        q *= c;
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < a.n_bins; b += blockDim.x)
    if (lh[b] != 0.0) atomicAdd(&g[(int64_t)s_blk * a.n_bins + b], lh[b]);
}

// g[s][b] *= 1 / (sqrt(2 pi) sigma 4 pi r_b^2 rho_s N_s)
__global__ void k_rdf_norm(int64_t n_sys, const int64_t *offs, const double *cell, int n_bins, double dr, double sigma,
                           double *g) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_sys * n_bins) return;
  const int64_t s = t / n_bins;
  const int b = (int)(t % n_bins);
  const double na = (double)(offs[s + 1] - offs[s]);
  const double rho = na / cell_volume(cell + 9 * s);
  const double rb = (b + 0.5) * dr;
  const double norm = 1.0 / sqrt(2.0 * M_PI * sigma * sigma);
  g[t] = g[t] * norm / (4.0 * M_PI * rb * rb * rho * na);
}

__global__ void __launch_bounds__(256) k_rdf_loss(const double *g, const double *gt, int64_t m, double inv_m,
                                                  double *loss, double *dl) {
  __shared__ double sh[4];
  double acc = 0.0;
  for (int64_t t = threadIdx.x; t < m; t += blockDim.x) {
    const double e = g[t] - gt[t];
    acc += e * e;
    if (dl) dl[t] = 2.0 * e * inv_m;
  }
  acc = wave_sum(acc);
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0 && loss) *loss = ((sh[0] + sh[1]) + (sh[2] + sh[3])) * inv_m;
}

// grad_i += -2 sum_{(j,S)} [sum_b pref_b dN(r_b - r)/dr] d^
__global__ void __launch_bounds__(256) k_rdf_vjp(RdfArgs a, const double *dl_dg, double *grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int64_t st = a.stride;
  const int s = a.sys_idx[i];
  const int64_t a0 = a.offs[s];
  const double *h = a.cell + 9 * (int64_t)s;
  const double na = (double)(a.offs[s + 1] - a0);
  const double rho = na / cell_volume(h);
  const double norm = 1.0 / sqrt(2.0 * M_PI * a.sigma * a.sigma);
  const double *dg = dl_dg + (int64_t)s * a.n_bins;
  const double rx = a.pos[i], ry = a.pos[st + i], rz = a.pos[2 * st + i];
  const int nn = a.n_nbr[i];
  const double inv2s2 = 1.0 / (2.0 * a.sigma * a.sigma);
  const double invs2 = 1.0 / (a.sigma * a.sigma);
  const double span = 10.0 * a.sigma;
  const double c = exp(-2.0 * a.dr * a.dr * inv2s2);
  const double kpref = norm / (4.0 * M_PI * rho * na);  // per-bin weight dg_b kpref / r_b^2
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int k = 0; k < nn; ++k) {
    const uint32_t ent = a.nbr[row_index(k, i, st)];
    const int64_t j = a0 + entry_j(ent);
    const double S0 = (double)entry_s0(ent), S1 = (double)entry_s1(ent), S2 = (double)entry_s2(ent);
    const double dx = shift_comp(a.pos[j] - rx, S0, S1, S2, h[0], h[3], h[6]);
    const double dy = shift_comp(a.pos[st + j] - ry, S0, S1, S2, h[1], h[4], h[7]);
    const double dz = shift_comp(a.pos[2 * st + j] - rz, S0, S1, S2, h[2], h[5], h[8]);
    const double r2 = norm2(dx, dy, dz);
    if (!(r2 < a.rmax2)) continue;
    const double r = sqrt(r2);
    int b0 = (int)floor((r - span) / a.dr - 0.5);
    int b1 = (int)ceil((r + span) / a.dr - 0.5);
    b0 = b0 < 0 ? 0 : b0;
    b1 = b1 > a.n_bins - 1 ? a.n_bins - 1 : b1;
    // the Gaussian of each bin by the recurrence of k_rdf_hist
    double hs = 0.0;
    const double x0 = (b0 + 0.5) * a.dr - r;
    double e = exp(-x0 * x0 * inv2s2), q = exp(-(2.0 * x0 * a.dr + a.dr * a.dr) * inv2s2);
    for (int b = b0; b <= b1; ++b) {
      const double rb = (b + 0.5) * a.dr;
      const double x = rb - r;
      hs += dg[b] / (rb * rb) * e * x;
      e *= q;
      q *= c;
    }
    hs *= kpref * invs2;
    const double c = -2.0 * hs / r;
    gx += c * dx;
    gy += c * dy;
    gz += c * dz;
  }
  grad[i] += gx;
  grad[st + i] += gy;
  grad[2 * st + i] += gz;
}

static RdfArgs make_rdf_args(const ts_batch *b, const ts_neighbor_list *nl, int n_bins, double r_end, double sigma,
                             double r_max) {
  RdfArgs a;
  a.n = b->n_atoms;
  a.stride = stride_of(b);
  a.sys_idx = b->system_idx;
  a.offs = b->sys_offsets;
  a.pos = b->pos;
  a.cell = b->cell;
  a.nbr = reinterpret_cast<const uint32_t *>(nl->nbr);
  a.n_nbr = nl->n_nbr;
  a.n_bins = n_bins;
  a.dr = r_end / n_bins;
  a.sigma = sigma;
  a.rmax2 = r_max * r_max;
  return a;
}

static int validate_rdf(const ts_batch *b, const ts_neighbor_list *nl, int n_bins, double r_end, double sigma,
                        double r_max) {
  int rc = validate_batch(b, false, nullptr);
  if (rc != TS_OK) return rc;
  rc = validate_list(b, nl);
  if (rc != TS_OK) return rc;
  if (nl->half) return TS_E_UNSUPPORTED;
  TS_CHECK_ARG(n_bins >= 1 && n_bins <= 8192 && r_end > 0.0 && sigma > 0.0 && r_max > 0.0);
  TS_CHECK_ARG(nl->cutoff + nl->skin >= r_max);
  return TS_OK;
}

}  // namespace ts

namespace ts {

// The pair adjoint of both entry points below; the parameter-gradient partial sums go to
// `slots` ([n_slots][kAdjSlot] doubles, cleared here when adj_params is wanted).
static int pair_adjoint(const ts_batch *batch, const ts_neighbor_list *nl, const ts_pair_params *pp, double dt_drift,
                        double w_kick, double accel, double *adj_pos, double *adj_vel, double *adj_params,
                        double *slots, int64_t n_slots, hipStream_t st) {
  if (batch->n_atoms == 0) return TS_OK;
  const int64_t stride = stride_of(batch);
  if (dt_drift != 0.0) {
    hipLaunchKernelGGL(k_adj_drift, dim3((unsigned)ceil_div(batch->n_atoms, 256)), dim3(256), 0, st, batch->n_atoms,
                       stride, adj_pos, adj_vel, dt_drift);
    TS_LAUNCH_CHECK();
  }
  if (w_kick == 0.0) return TS_OK;
  AdjArgs a;
  a.n = batch->n_atoms;
  a.stride = stride;
  a.sys_idx = batch->system_idx;
  a.offs = batch->sys_offsets;
  a.pos = batch->pos;
  a.cell = batch->cell;
  a.mass = batch->mass;
  a.species = batch->species;
  a.nbr = reinterpret_cast<const uint32_t *>(nl->nbr);
  a.n_nbr = nl->n_nbr;
  a.lr = adj_pos;
  a.lv = adj_vel;
  a.adj_params = adj_params;
  a.slots = slots;
  a.n_slots = n_slots;
  a.w = w_kick;
  a.accel = accel;
  if (adj_params) {
    const int rc = fill_async<double>(a.slots, kAdjSlot * a.n_slots, 0.0, st);
    if (rc != TS_OK) return rc;
  }
  const PairTable t = make_table(pp);
  const bool single = t.n_species == 1 || batch->species == nullptr;
  with_kind(t.kind, [&](auto k) {
    constexpr int KIND = decltype(k)::value;
    if (pp->prec == TS_PAIR_F32) launch_vjp<KIND, float>(a, t, single, st);
    else launch_vjp<KIND, double>(a, t, single, st);
  });
  TS_LAUNCH_CHECK();
  if (adj_params) return launch_sum_slots(a.n_slots, a.slots, adj_params, st);
  return TS_OK;
}

// Partial-sum slots of ts_pair_adjoint_noalloc: a library-held array, one copy per GPU (at most
// kNoallocSystems systems, one slot each; 1.5 MiB).  Host code never uses the symbol's name as an
// address: the device address of each GPU's copy comes from hipGetSymbolAddress (noalloc_slots).
constexpr int64_t kNoallocSystems = 4096;
static __device__ __align__(256) double scratch[kNoallocSystems * kAdjSlot];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices];

// Device address of the current GPU's copy of `scratch`, looked up once per device.
static int noalloc_slots(double **out) {
  int dev = 0;
  TS_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return TS_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    TS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double *>(p);
  }
  *out = g_scratch_ptr[dev];
  return TS_OK;
}

}  // namespace ts

extern "C" int ts_pair_adjoint(const ts_batch *batch, const ts_neighbor_list *nl, const ts_pair_params *pp,
                               double dt_drift, double w_kick, double accel, double *adj_pos, double *adj_vel,
                               double *adj_params, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, false);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(adj_pos && adj_vel && std::isfinite(dt_drift) && std::isfinite(w_kick) && std::isfinite(accel) &&
               accel > 0.0);
  const ts::NlWork w = ts::nl_work(nl->workspace, batch->n_atoms, batch->n_systems);
  return ts::pair_adjoint(batch, nl, pp, dt_drift, w_kick, accel, adj_pos, adj_vel, adj_params, w.adj_slots,
                          ts::adj_slot_count(batch->n_systems), ts::as_stream(stream));
}

extern "C" int ts_pair_adjoint_noalloc(const ts_batch *batch, const ts_neighbor_list *nl, const ts_pair_params *pp,
                                       double dt_drift, double w_kick, double accel, double *adj_pos,
                                       double *adj_vel, double *adj_params, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_pair_call(batch, nl, pp, &max_atoms, false, false);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(adj_pos && adj_vel && std::isfinite(dt_drift) && std::isfinite(w_kick) && std::isfinite(accel) &&
               accel > 0.0);
  if (adj_params && batch->n_systems > ts::kNoallocSystems) return TS_E_CAPACITY;
  double *slots = nullptr;
  if (adj_params && w_kick != 0.0 && batch->n_atoms > 0) {  // only launches that accumulate use the array
    rc = ts::noalloc_slots(&slots);
    if (rc != TS_OK) return rc;
  }
  return ts::pair_adjoint(batch, nl, pp, dt_drift, w_kick, accel, adj_pos, adj_vel, adj_params, slots,
                          ts::adj_slot_count(batch->n_systems), ts::as_stream(stream));
}

extern "C" int ts_rdf_smeared(const ts_batch *batch, const ts_neighbor_list *nl, int32_t n_bins, double r_end,
                              double sigma, double r_max, double *g, ts_stream_t stream) {
  int rc = ts::validate_rdf(batch, nl, n_bins, r_end, sigma, r_max);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(g != nullptr);
  hipStream_t st = ts::as_stream(stream);
  const int64_t m = batch->n_systems * (int64_t)n_bins;
  rc = ts::fill_async<double>(g, m, 0.0, st);
  if (rc != TS_OK) return rc;
  const ts::RdfArgs a = ts::make_rdf_args(batch, nl, n_bins, r_end, sigma, r_max);
  if (batch->n_atoms > 0) {
    hipLaunchKernelGGL(ts::k_rdf_hist, dim3((unsigned)ts::ceil_div(batch->n_atoms, 256)), dim3(256),
                       sizeof(double) * n_bins, st, a, g);
    TS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(ts::k_rdf_norm, dim3((unsigned)ts::ceil_div(m, 256)), dim3(256), 0, st, batch->n_systems,
                     batch->sys_offsets, batch->cell, n_bins, r_end / n_bins, sigma, g);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

extern "C" int ts_rdf_loss(const double *g, const double *g_target, int64_t n_systems, int32_t n_bins, double *loss,
                           double *dl_dg, ts_stream_t stream) {
  TS_CHECK_ARG(g && g_target && n_systems >= 1 && n_bins >= 1);
  const int64_t m = n_systems * (int64_t)n_bins;
  hipLaunchKernelGGL(ts::k_rdf_loss, dim3(1), dim3(256), 0, ts::as_stream(stream), g, g_target, m, 1.0 / (double)m,
                     loss, dl_dg);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

extern "C" int ts_rdf_vjp(const ts_batch *batch, const ts_neighbor_list *nl, int32_t n_bins, double r_end,
                          double sigma, double r_max, const double *dl_dg, double *grad_pos, ts_stream_t stream) {
  int rc = ts::validate_rdf(batch, nl, n_bins, r_end, sigma, r_max);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(dl_dg && grad_pos);
  if (batch->n_atoms == 0) return TS_OK;
  const ts::RdfArgs a = ts::make_rdf_args(batch, nl, n_bins, r_end, sigma, r_max);
  hipLaunchKernelGGL(ts::k_rdf_vjp, dim3((unsigned)ts::ceil_div(batch->n_atoms, 256)), dim3(256), 0,
                     ts::as_stream(stream), a, dl_dg, grad_pos);
  TS_LAUNCH_CHECK();
  return TS_OK;
}
