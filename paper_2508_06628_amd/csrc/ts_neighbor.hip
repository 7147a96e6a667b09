// Cell-list neighbor build under triclinic periodic boundaries (the neighbor-list "graph
// construction" the paper names as the main cost difference between models, Section 4).
//
// Per system that needs it: fractional coordinates s = r cell^-1 (float64), wrapped to [0, 1)
// with the integer image offset kept per atom; a counting sort by bin (stable: each bin's atoms
// are sorted by index); then each atom scans the bins within reach along every direction (a
// bin may be visited under several lattice images when the cell is narrower than 2 r_list),
// tests |d|^2 < r_list^2 in float64 and appends (j, S) to its padded row, which is finally sorted
// into the canonical (j, S0, S1, S2) order.
#include "ts_internal.h"
#include "ts_neighbor.h"
#include "ts_step.h"

namespace ts {

// ----------------------------------------------------------------------------- small 3x3 helpers

__device__ inline double det3(const double *h) {
  return h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) + h[2] * (h[3] * h[7] - h[4] * h[6]);
}

__device__ inline void inv3(const double *h, double *inv, double det) {
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

__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

__device__ inline int pack_img(int a, int b, int c) {
  return ((a + 512) & 1023) | (((b + 512) & 1023) << 10) | (((c + 512) & 1023) << 20);
}
__device__ inline void unpack_img(int p, int *a, int *b, int *c) {
  *a = (p & 1023) - 512;
  *b = ((p >> 10) & 1023) - 512;
  *c = ((p >> 20) & 1023) - 512;
}

// ----------------------------------------------------------------------------- kernels

// Validity bound of the list of each system: flag a rebuild when
//   2 |r_i - ref_i M| + r_list ||M - I||_F > skin   (M = ref_cell^-1 cell; M = I if cell unchanged).
__global__ void k_nl_trigger(int64_t n, int64_t stride, const int32_t *__restrict__ sys_idx,
                             const double *__restrict__ pos, const double *__restrict__ ref_pos,
                             const double *__restrict__ cell, const double *__restrict__ ref_cell,
                             int32_t *__restrict__ flags, double skin, double r_list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = sys_idx[i];
  double r[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = pos[c * stride + i];
  // also true for a non-finite position, which the build then reports
  if (list_invalid(r, ref_pos, stride, i, cell + 9 * (int64_t)s, ref_cell + 9 * (int64_t)s, skin, r_list))
    flags[s] = 1;
}

// One thread per system: bin geometry of the systems to rebuild.
__global__ void k_nl_setup(int64_t n_sys, const int64_t *__restrict__ offs, const double *__restrict__ cell,
                           double *__restrict__ ref_cell, int32_t *__restrict__ flags, NlGeom *__restrict__ geom,
                           int force, double r_list, int bin_factor, int64_t *__restrict__ status) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  NlGeom g;
  g.active = (force || flags[s]) ? 1 : 0;
  flags[s] = 0;
  if (!g.active) {
    geom[s].active = 0;
    return;
  }
  const double *h = cell + 9 * s;
  const double det = det3(h);
  bool ok = isfinite(det) && det != 0.0;
  for (int k = 0; k < 9; ++k) ok &= isfinite(h[k]);
  if (!ok) {
    atomicMax((unsigned long long *)&status[TS_STATUS_NONFINITE], 1ull);
    geom[s].active = 0;
    return;
  }
  inv3(h, g.inv, det);
  const double vol = fabs(det);
  const int64_t na = offs[s + 1] - offs[s];
  int nb[3];
  double w[3];
  for (int k = 0; k < 3; ++k) {
    const double *a = h + 3 * ((k + 1) % 3);
    const double *b = h + 3 * ((k + 2) % 3);
    const double cx = a[1] * b[2] - a[2] * b[1], cy = a[2] * b[0] - a[0] * b[2], cz = a[0] * b[1] - a[1] * b[0];
    w[k] = vol / sqrt(cx * cx + cy * cy + cz * cz);
    double q = floor(bin_factor * w[k] / r_list);
    q = q < 1.0 ? 1.0 : (q > 1024.0 ? 1024.0 : q);
    nb[k] = (int)q;
  }
  const int64_t cap = 2 * na + 1;
  while ((int64_t)nb[0] * nb[1] * nb[2] > cap) {
    int k = 0;
    if (nb[1] > nb[k]) k = 1;
    if (nb[2] > nb[k]) k = 2;
    nb[k] -= 1;
  }
  for (int k = 0; k < 3; ++k) {
    g.n[k] = nb[k];
    g.reach[k] = r_list / w[k];
    g.m[k] = (int)ceil(g.reach[k] * nb[k] + 1e-9);
  }
  geom[s] = g;
  for (int k = 0; k < 9; ++k) ref_cell[9 * s + k] = h[k];
  atomicAdd((unsigned long long *)&status[TS_STATUS_REBUILDS], 1ull);
}

__global__ void k_nl_zero(const int64_t *__restrict__ offs, const NlGeom *__restrict__ geom, int32_t *__restrict__ count,
                          int32_t *__restrict__ fill) {
  const int s = blockIdx.y;
  if (!geom[s].active) return;
  const int nb = geom[s].n[0] * geom[s].n[1] * geom[s].n[2];
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t base = 2 * offs[s] + s;
  count[base + b] = 0;
  fill[base + b] = 0;
}

__device__ inline void frac_of(const NlGeom &g, const double r[3], double f[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) f[k] = r[0] * g.inv[k] + r[1] * g.inv[3 + k] + r[2] * g.inv[6 + k];
}

__global__ void k_nl_assign(int64_t n, int64_t stride, const int32_t *__restrict__ sys_idx,
                            const int64_t *__restrict__ offs, const double *__restrict__ pos,
                            double *__restrict__ ref_pos, const NlGeom *__restrict__ geom,
                            int32_t *__restrict__ atom_bin, int32_t *__restrict__ atom_img,
                            int32_t *__restrict__ count, int64_t *__restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = sys_idx[i];
  const NlGeom &g = geom[s];
  if (!g.active) return;
  double r[3], f[3];
  bool fin = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    r[c] = pos[c * stride + i];
    ref_pos[c * stride + i] = r[c];
    fin &= isfinite(r[c]);
  }
  int b[3], im[3];
  if (fin) {
    frac_of(g, r, f);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double fl = floor(f[k]);
      const double wv = f[k] - fl;
      int bk = (int)(wv * g.n[k]);
      b[k] = bk >= g.n[k] ? g.n[k] - 1 : (bk < 0 ? 0 : bk);
      if (fl < -500.0 || fl > 500.0) {
        atomicMax((unsigned long long *)&status[TS_STATUS_SHIFT], 1ull);
        im[k] = 0;
      } else {
        im[k] = (int)fl;
      }
    }
  } else {
    atomicMax((unsigned long long *)&status[TS_STATUS_NONFINITE], 1ull);
    b[0] = b[1] = b[2] = 0;
    im[0] = im[1] = im[2] = 0;
  }
  const int lb = (b[0] * g.n[1] + b[1]) * g.n[2] + b[2];
  atom_bin[i] = lb;
  atom_img[i] = pack_img(im[0], im[1], im[2]);
  atomicAdd(&count[2 * offs[s] + s + lb], 1);
}

// One block per system: exclusive scan of the bin counts -> global start of each bin.
__global__ void __launch_bounds__(256) k_nl_scan(const int64_t *__restrict__ offs, const NlGeom *__restrict__ geom,
                                                 const int32_t *__restrict__ count, int32_t *__restrict__ start) {
  // thread t owns a contiguous segment of the system's bins: segment totals, one block-wide
  // exclusive scan of the 256 totals (wavefront shuffles, one barrier), then each thread writes its
  // segment's starts sequentially
  const int s = blockIdx.x;
  if (!geom[s].active) return;
  const int nb = geom[s].n[0] * geom[s].n[1] * geom[s].n[2];
  const int64_t base = 2 * offs[s] + s;
  const int seg = (nb + 255) / 256;
  const int b0 = min((int)threadIdx.x * seg, nb), b1 = min(b0 + seg, nb);
  int32_t sum = 0;
  for (int b = b0; b < b1; ++b) sum += count[base + b];
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  int32_t incl = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int32_t t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  __shared__ int32_t wtot[4];
  if (lane == kWave - 1) wtot[wave] = incl;
  __syncthreads();
  int32_t ex = (int32_t)offs[s] + incl - sum;
  for (int w = 0; w < wave; ++w) ex += wtot[w];
  for (int b = b0; b < b1; ++b) {
    start[base + b] = ex;
    ex += count[base + b];
  }
}

__global__ void k_nl_scatter(int64_t n, const int32_t *__restrict__ sys_idx, const int64_t *__restrict__ offs,
                             const NlGeom *__restrict__ geom, const int32_t *__restrict__ atom_bin,
                             const int32_t *__restrict__ start, int32_t *__restrict__ fill, int32_t *__restrict__ perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = sys_idx[i];
  if (!geom[s].active) return;
  const int64_t bi = 2 * offs[s] + s + atom_bin[i];
  const int slot = atomicAdd(&fill[bi], 1);
  perm[start[bi] + slot] = (int32_t)i;
}

// One thread per bin: sort the bin's atoms by index (makes the lists deterministic).
__global__ void k_nl_sort(const int64_t *__restrict__ offs, const NlGeom *__restrict__ geom,
                          const int32_t *__restrict__ count, const int32_t *__restrict__ start,
                          int32_t *__restrict__ perm) {
  const int s = blockIdx.y;
  if (!geom[s].active) return;
  const int nb = geom[s].n[0] * geom[s].n[1] * geom[s].n[2];
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nb) return;
  const int64_t bi = 2 * offs[s] + s + b;
  int32_t *p = perm + start[bi];
  const int c = count[bi];
  for (int a = 1; a < c; ++a) {
    const int32_t key = p[a];
    int q = a - 1;
    while (q >= 0 && p[q] > key) {
      p[q + 1] = p[q];
      --q;
    }
    p[q + 1] = key;
  }
}

// One thread per atom: scan the bins within reach and append every (j, S) inside r_list.
__global__ void __launch_bounds__(256) k_nl_enum(int64_t n, int64_t stride, const int32_t *__restrict__ sys_idx,
                                                 const int64_t *__restrict__ offs, const double *__restrict__ pos,
                                                 const double *__restrict__ cell, const NlGeom *__restrict__ geom,
                                                 const int32_t *__restrict__ atom_img,
                                                 const int32_t *__restrict__ count,
                                                 const int32_t *__restrict__ start,
                                                 const int32_t *__restrict__ perm, uint32_t *__restrict__ nbr,
                                                 int32_t *__restrict__ n_nbr, int max_nbr, double r_list,
                                                 int half, int64_t *__restrict__ status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int cnt = 0;
  bool shift_bad = false;
  // no early return: every thread reaches the workgroup-level status update at the end
  if (i < n && geom[sys_idx[i]].active) {
  const int s = sys_idx[i];
  const NlGeom &g = geom[s];
  const int64_t a0 = offs[s];
  const int64_t base = 2 * a0 + s;
  const double *h = cell + 9 * (int64_t)s;
  double r[3], f[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = pos[c * stride + i];
  int imi[3];
  unpack_img(atom_img[i], &imi[0], &imi[1], &imi[2]);
  int lo[3], hi[3];
  const bool fin = isfinite(r[0]) && isfinite(r[1]) && isfinite(r[2]);
  if (fin) {
    frac_of(g, r, f);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double wv = f[k] - floor(f[k]);
      const int bk = min(max((int)(wv * g.n[k]), 0), g.n[k] - 1);
      int l = (int)floor((wv - g.reach[k]) * g.n[k] - 1e-9);
      int u = (int)floor((wv + g.reach[k]) * g.n[k] + 1e-9);
      lo[k] = max(l, bk - g.m[k]);
      hi[k] = min(u, bk + g.m[k]);
    }
  } else {
    lo[0] = lo[1] = lo[2] = 0;
    hi[0] = hi[1] = hi[2] = -1;
  }
  const double rl2 = r_list * r_list;
  for (int v0 = lo[0]; v0 <= hi[0]; ++v0) {
    const int I0 = floor_div(v0, g.n[0]);
    const int b0 = v0 - I0 * g.n[0];
    for (int v1 = lo[1]; v1 <= hi[1]; ++v1) {
      const int I1 = floor_div(v1, g.n[1]);
      const int b1 = v1 - I1 * g.n[1];
      for (int v2 = lo[2]; v2 <= hi[2]; ++v2) {
        const int I2 = floor_div(v2, g.n[2]);
        const int b2 = v2 - I2 * g.n[2];
        const int64_t bi = base + (b0 * g.n[1] + b1) * g.n[2] + b2;
        const int st = start[bi];
        const int ct = count[bi];
        for (int t = 0; t < ct; ++t) {
          const int j = perm[st + t];
          int imj[3];
          unpack_img(atom_img[j], &imj[0], &imj[1], &imj[2]);
          const int S0 = I0 + imi[0] - imj[0];
          const int S1 = I1 + imi[1] - imj[1];
          const int S2 = I2 + imi[2] - imj[2];
          if (j == i && S0 == 0 && S1 == 0 && S2 == 0) continue;
          double d[3];
#pragma unroll
          for (int c = 0; c < 3; ++c)
            d[c] = shift_comp(pos[c * stride + j] - r[c], (double)S0, (double)S1, (double)S2, h[c], h[3 + c], h[6 + c]);
          const double r2 = norm2(d[0], d[1], d[2]);
          if (!(r2 < rl2)) continue;
          if (half) {
            const int first = S0 != 0 ? S0 : (S1 != 0 ? S1 : S2);
            if (!(i < j || (i == j && first > 0))) continue;
          }
          if (S0 < -TS_MAX_IMAGE_SHIFT || S0 > TS_MAX_IMAGE_SHIFT || S1 < -TS_MAX_IMAGE_SHIFT ||
              S1 > TS_MAX_IMAGE_SHIFT || S2 < -TS_MAX_IMAGE_SHIFT || S2 > TS_MAX_IMAGE_SHIFT) {
            shift_bad = true;
            continue;
          }
          if (cnt < max_nbr) nbr[row_index(cnt, i, stride)] = pack_entry((int)(j - a0), S0, S1, S2);
          ++cnt;
        }
      }
    }
  }
  // canonical row order: ascending packed entry = lexicographic (j, S0, S1, S2)
  const int nw = cnt < max_nbr ? cnt : max_nbr;
  for (int a = 1; a < nw; ++a) {
    const uint32_t key = nbr[row_index(a, i, stride)];
    int q = a - 1;
    while (q >= 0 && nbr[row_index(q, i, stride)] > key) {
      nbr[row_index(q + 1, i, stride)] = nbr[row_index(q, i, stride)];
      --q;
    }
    nbr[row_index(q + 1, i, stride)] = key;
  }
  n_nbr[i] = nw;
  }
  block_status(status, cnt, max_nbr, shift_bad, false);
}

// ----------------------------------------------------------------------------- host side

NlWork nl_work(void *ws, int64_t n_atoms, int64_t n_sys) {
  NlWork w;
  // offsets are accumulated as integers: ts_neighbor_workspace_bytes sizes the layout with ws = NULL
  const uintptr_t base = reinterpret_cast<uintptr_t>(ws);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char *q = reinterpret_cast<char *>(base + off);
    off += (bytes + 255) & ~size_t(255);
    return q;
  };
  const int64_t nbins = 2 * n_atoms + n_sys;
  w.geom = reinterpret_cast<NlGeom *>(take(sizeof(NlGeom) * n_sys));
  w.flags = reinterpret_cast<int32_t *>(take(4 * n_sys));
  w.atom_bin = reinterpret_cast<int32_t *>(take(4 * (n_atoms + 1)));
  w.atom_img = reinterpret_cast<int32_t *>(take(4 * (n_atoms + 1)));
  w.count = reinterpret_cast<int32_t *>(take(4 * nbins));
  w.start = reinterpret_cast<int32_t *>(take(4 * nbins));
  w.fill = reinterpret_cast<int32_t *>(take(4 * nbins));
  w.perm = reinterpret_cast<int32_t *>(take(4 * (n_atoms + 1)));
  w.pos_alt = reinterpret_cast<double *>(take(24 * (n_atoms + 1)));
  w.adj_alt = reinterpret_cast<double *>(take(48 * (n_atoms + 1)));
  w.flags3 = reinterpret_cast<int32_t *>(take(4 * (6 * n_sys + 8)));
  w.pos4 = reinterpret_cast<double *>(take(32 * (n_atoms + 1)));
  w.adj_slots = reinterpret_cast<double *>(take(sizeof(double) * kAdjSlot * adj_slot_count(n_sys)));
  w.sel2 = reinterpret_cast<int32_t *>(take(4 * 2 * n_sys));
  w.pflags3 = reinterpret_cast<int32_t *>(take(4 * (6 * n_sys + 8)));
  w.row_geom = reinterpret_cast<double *>(take(sizeof(double) * 14 * n_sys));
  w.bytes = off;
  return w;
}

// Rebuild list of the small-system path: with force every system, else none yet (flags cleared);
// and each system's cell geometry for the row rebuild (one thread per system).
__global__ void __launch_bounds__(256) k_list_init(int64_t n_sys, int force, int32_t *__restrict__ flags,
                                                   int32_t *__restrict__ list, int32_t *__restrict__ count,
                                                   const double *__restrict__ cell, double r_list,
                                                   RowGeom *__restrict__ geom) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) *count = force ? (int32_t)n_sys : 0;
  if (s >= n_sys) return;
  flags[s] = 0;
  if (force) list[s] = (int32_t)s;
  RowGeom g;
  row_geometry(cell + 9 * s, r_list, &g);
  geom[s] = g;
}

// Validity test of every atom; the first atom of a system to exceed the bound appends the system to
// the rebuild list (a plain read skips the exchange once the flag is visibly set).
__global__ void k_nl_trigger_list(int64_t n, int64_t stride, const int32_t *__restrict__ sys_idx,
                                  const double *__restrict__ pos, const double *__restrict__ ref_pos,
                                  const double *__restrict__ cell, const double *__restrict__ ref_cell,
                                  int32_t *__restrict__ flags, int32_t *__restrict__ list, int32_t *__restrict__ count,
                                  double skin, double r_list) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = sys_idx[i];
  double r[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) r[c] = pos[c * stride + i];
  if (!list_invalid(r, ref_pos, stride, i, cell + 9 * (int64_t)s, ref_cell + 9 * (int64_t)s, skin, r_list)) return;
  if (__hip_atomic_load(&flags[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  if (atomicExch(&flags[s], 1) == 0) list[atomicAdd(count, 1)] = s;
}

int nl_update(const ts_batch *b, ts_neighbor_list *nl, int force, int64_t max_atoms, hipStream_t st) {
  const int64_t n = b->n_atoms, S = b->n_systems, stride = stride_of(b);
  NlWork w = nl_work(nl->workspace, n, S);
  const double r_list = nl->cutoff + nl->skin;
  const unsigned ga = (unsigned)ceil_div(n > 0 ? n : 1, 256);
  if (max_atoms <= kLdsMaxAtoms) {
    // systems that fit in LDS: a device list of the systems to rebuild and the row kernel of the
    // fused step loop (canonical rows straight from a wavefront scan, no sort)
    int32_t *list = w.flags3 + 3 * S, *count = w.flags3 + 6 * S + 4;
    RowGeom *geom = reinterpret_cast<RowGeom *>(w.row_geom);
    hipLaunchKernelGGL(k_list_init, dim3((unsigned)ceil_div(S > 0 ? S : 1, 256)), dim3(256), 0, st, S, force, w.flags,
                       list, count, b->cell, r_list, geom);
    TS_LAUNCH_CHECK();
    if (n == 0) return TS_OK;
    if (!force) {
      hipLaunchKernelGGL(k_nl_trigger_list, dim3(ga), dim3(256), 0, st, n, stride, b->system_idx, b->pos,
                         nl->ref_pos, b->cell, nl->ref_cell, w.flags, list, count, nl->skin, r_list);
      TS_LAUNCH_CHECK();
    }
    StepArgs a;
    std::memset(&a, 0, sizeof(a));
    a.offs = b->sys_offsets;
    a.pos_in = b->pos;
    a.st_in = stride;
    a.st_vel = stride;
    a.cell = b->cell;
    a.nbr = reinterpret_cast<uint32_t *>(nl->nbr);
    a.n_nbr = nl->n_nbr;
    a.max_nbr = nl->max_nbr;
    a.half = nl->half;
    a.ref_pos = nl->ref_pos;
    a.ref_cell = nl->ref_cell;
    a.status = nl->status;
    a.r_list = r_list;
    a.skin = nl->skin;
    a.list_cur = list;
    a.count_cur = count;
    a.row_geom = geom;
    return launch_rebuild(a, S, max_atoms, st);
  }
  if (!force && n > 0) {
    hipLaunchKernelGGL(k_nl_trigger, dim3(ga), dim3(256), 0, st, n, stride, b->system_idx, b->pos, nl->ref_pos,
                       b->cell, nl->ref_cell, w.flags, nl->skin, r_list);
    TS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_nl_setup, dim3((unsigned)ceil_div(S, 64)), dim3(64), 0, st, S, b->sys_offsets, b->cell,
                     nl->ref_cell, w.flags, w.geom, force, r_list, nl->bin_factor, nl->status);
  TS_LAUNCH_CHECK();
  if (n == 0) return TS_OK;
  const dim3 gb((unsigned)ceil_div(2 * max_atoms + 1, 256), (unsigned)S);
  hipLaunchKernelGGL(k_nl_zero, gb, dim3(256), 0, st, b->sys_offsets, w.geom, w.count, w.fill);
  TS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_nl_assign, dim3(ga), dim3(256), 0, st, n, stride, b->system_idx, b->sys_offsets, b->pos,
                     nl->ref_pos, w.geom, w.atom_bin, w.atom_img, w.count, nl->status);
  TS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_nl_scan, dim3((unsigned)S), dim3(256), 0, st, b->sys_offsets, w.geom, w.count, w.start);
  TS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_nl_scatter, dim3(ga), dim3(256), 0, st, n, b->system_idx, b->sys_offsets, w.geom,
                     w.atom_bin, w.start, w.fill, w.perm);
  TS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_nl_sort, gb, dim3(256), 0, st, b->sys_offsets, w.geom, w.count, w.start, w.perm);
  TS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_nl_enum, dim3(ga), dim3(256), 0, st, n, stride, b->system_idx, b->sys_offsets, b->pos,
                     b->cell, w.geom, w.atom_img, w.count, w.start, w.perm, reinterpret_cast<uint32_t *>(nl->nbr),
                     nl->n_nbr, nl->max_nbr, r_list, nl->half, nl->status);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

}  // namespace ts

extern "C" size_t ts_neighbor_workspace_bytes(int64_t n_atoms, int64_t n_systems) {
  if (n_atoms < 0 || n_systems < 1) return 0;
  return ts::nl_work(nullptr, n_atoms, n_systems).bytes + 256;
}

extern "C" int ts_neighbor_build(const ts_batch *batch, ts_neighbor_list *nl, int32_t force, ts_stream_t stream) {
  int64_t max_atoms = 0;
  int rc = ts::validate_batch(batch, false, &max_atoms);
  if (rc != TS_OK) return rc;
  rc = ts::validate_list(batch, nl);
  if (rc != TS_OK) return rc;
  return ts::nl_update(batch, nl, force ? 1 : 0, max_atoms, ts::as_stream(stream));
}
