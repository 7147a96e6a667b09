// FIRE relaxation of an uneven batch in one persistent launch (the paper's variable-length,
// in-flight batching idea of Section 3, carried onto the device: a system leaves as soon as it
// has converged and the freed workgroup takes the next one).
//
// Workgroups of 512 threads pop systems from a device work queue ordered largest first.  A
// workgroup keeps its system's positions in LDS and iterates FIRE on it until it converges, reaches
// max_iter or exhausts this call's iteration budget, then writes the system back and pops the next.
// Inside a workgroup an iteration is: list validity bound (block reduction) and, when exceeded, a
// rebuild of the system's rows (one wavefront per atom, canonical (j, S) order); pair forces with
// TL lanes per atom (TL from the system size); block reductions of max |F|^2, g.v, |v|^2, |g|^2,
// energy and virial in a fixed order; the FIRE decision by one thread; the atom (and cell) update.
// No workgroup ever waits for another, so the launch cannot deadlock, and every workgroup exits
// once the queue is empty.
#include "ts_fire.h"
#include "ts_step.h"

namespace ts {

constexpr int kPT = 512;          // threads per workgroup
constexpr int kPW = kPT / kWave;  // wavefronts per workgroup
constexpr int kPR = 16;           // reduced quantities: fmax2 P vv gg E W[9] (2 spare)
constexpr int kPSurv = 2 * kWave;  // survivor queue of a wavefront in the wide-cell rebuild

struct FirePArgs {
  FireArgs f;
  int64_t n_sys;
  const int32_t *species;
  uint32_t *nbr;
  int32_t *n_nbr;
  int max_nbr;
  double *ref_pos;   // list reference positions
  double *ref_lcell; // list reference cells [S][9]
  int64_t *status;
  double r_list, skin;
  double *energy;    // [S] or null
  int32_t *queue;    // [1] head of the work queue (zeroed before launch)
  int32_t *order;    // [S] systems, largest first
  int64_t budget;    // iterations per system in this call (< 0: until converged or max_iter)
  int32_t *idle;     // [1] workgroups that found the queue empty (zeroed before launch)
  int32_t idle_limit;  // > 0: stop iterating once idle >= idle_limit (the tail goes elsewhere)
};

// order[rank] = s with systems ranked by decreasing size (ties by index)
__global__ void k_fire_order(int64_t n_sys, const int64_t *offs, int32_t *order, int32_t *queue) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s == 0) {
    queue[0] = 0;  // head
    queue[1] = 0;  // idle workgroups
  }
  if (s >= n_sys) return;
  const int64_t ns = offs[s + 1] - offs[s];
  int64_t rank = 0;
  for (int64_t t = 0; t < n_sys; ++t) {
    const int64_t nt = offs[t + 1] - offs[t];
    rank += (nt > ns || (nt == ns && t < s)) ? 1 : 0;
  }
  order[rank] = (int32_t)s;
}

__device__ inline void inv3p(const double *h, double *inv) {
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

template <int KIND, typename T, bool CELL>
__global__ void __launch_bounds__(kPT) k_fire_persistent(PairTable tab, FirePArgs a) {
  extern __shared__ double lds[];
  __shared__ PairCoef ltab[TS_MAX_SPECIES * TS_MAX_SPECIES];
  __shared__ double red[kPW * kPR];
  // sh: 0..8 cell, 9..17 cell^-1, 18..20 reach, 21 cv, 22 cg, 23 dt, 24..32 D, 33..41 D^-1 (old),
  //     42..50 D_new, 51 strain term, 52 flags (1 stop, 2 rebuild), 53..61 M = ref^-1 cell, 62 same cell
  __shared__ double sh[64];
  __shared__ int s_sys;
  __shared__ int s_any;
  table_to_lds(ltab);
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const ts_fire_config &cf = a.f.cfg;
  const int64_t st = a.f.stride;
  const bool single = tab.n_species == 1 || a.species == nullptr;
  const double rl2 = a.r_list * a.r_list;
  for (;;) {
    if (tid == 0) {
      const int q = atomicAdd(a.queue, 1);
      s_sys = q < a.n_sys ? a.order[q] : -1;
    }
    __syncthreads();
    const int s = s_sys;
    if (s < 0) {
      if (tid == 0) atomicAdd(a.idle, 1);
      break;
    }
    const int64_t a0 = a.f.offs[s];
    const int ns = (int)(a.f.offs[s + 1] - a0);
    if (a.f.converged[s] || ns == 0) {
      __syncthreads();
      continue;
    }
    // TL lanes per atom: as many as spread the system over the workgroup (1..16)
    int tl = 1;
    while (tl < 16 && tl * 2 * ns <= kPT) tl *= 2;
    const int G = kPT / tl, grp = tid / tl, gl = tid % tl;
    double *lx = lds, *ly = lds + ns, *lz = lds + 2 * ns;
    for (int k = tid; k < ns; k += kPT) {
      lx[k] = a.f.pos[a0 + k];
      ly[k] = a.f.pos[st + a0 + k];
      lz[k] = a.f.pos[2 * st + a0 + k];
    }
    if (tid == 0) {
      for (int k = 0; k < 9; ++k) {
        sh[k] = a.f.cell[9 * (int64_t)s + k];
        sh[24 + k] = CELL ? a.f.deform[9 * (int64_t)s + k] : (k % 4 == 0 ? 1.0 : 0.0);
      }
    }
    __syncthreads();
    int64_t it = 0;
    for (;;) {
      // ---- list validity (cell-aware bound) and rebuild
      if (tid == 0) {
        const double *h = sh, *h0 = a.ref_lcell + 9 * (int64_t)s;
        bool same = true;
        for (int k = 0; k < 9; ++k) same &= (h[k] == h0[k]);
        sh[62] = same ? 1.0 : 0.0;
        double strain = 0.0;
        if (!same) {
          double hi[9];
          inv3p(h0, hi);
          double acc = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int q = 0; q < 3; ++q) {
              const double m = hi[3 * p] * h[q] + hi[3 * p + 1] * h[3 + q] + hi[3 * p + 2] * h[6 + q];
              sh[53 + 3 * p + q] = m;
              const double e = m - (p == q ? 1.0 : 0.0);
              acc += e * e;
            }
          strain = sqrt(acc);
        }
        sh[51] = strain;
        s_any = 0;
      }
      __syncthreads();
      {
        const bool same = sh[62] != 0.0;
        bool bad = false;
        for (int k = tid; k < ns; k += kPT) {
          const int64_t i = a0 + k;
          const double r0x = a.ref_pos[i], r0y = a.ref_pos[st + i], r0z = a.ref_pos[2 * st + i];
          double dx, dy, dz;
          if (same) {
            dx = lx[k] - r0x;
            dy = ly[k] - r0y;
            dz = lz[k] - r0z;
          } else {
            const double *M = sh + 53;
            dx = lx[k] - (r0x * M[0] + r0y * M[3] + r0z * M[6]);
            dy = ly[k] - (r0x * M[1] + r0y * M[4] + r0z * M[7]);
            dz = lz[k] - (r0x * M[2] + r0y * M[5] + r0z * M[8]);
          }
          bad |= bound_exceeded(sqrt(norm2(dx, dy, dz)), same ? 0.0 : sh[51], a.skin, a.r_list);
        }
        if (bad) s_any = 1;
      }
      __syncthreads();
      if (s_any) {
        if (tid == 0) {
          inv3p(sh, sh + 9);
          const double *h = sh;
          const double vol = fabs(h[0] * (h[4] * h[8] - h[5] * h[7]) - h[1] * (h[3] * h[8] - h[5] * h[6]) +
                                  h[2] * (h[3] * h[7] - h[4] * h[6]));
          for (int k = 0; k < 3; ++k) {
            const double *p = h + 3 * ((k + 1) % 3);
            const double *q = h + 3 * ((k + 2) % 3);
            const double cx = p[1] * q[2] - p[2] * q[1], cy = p[2] * q[0] - p[0] * q[2],
                         cz = p[0] * q[1] - p[1] * q[0];
            sh[18 + k] = a.r_list / (vol / sqrt(cx * cx + cy * cy + cz * cz));
          }
          for (int k = 0; k < 9; ++k) a.ref_lcell[9 * (int64_t)s + k] = h[k];
          atomicAdd((unsigned long long *)&a.status[TS_STATUS_REBUILDS], 1ull);
        }
        __syncthreads();
        const double h00 = sh[0], h01 = sh[1], h02 = sh[2], h10 = sh[3], h11 = sh[4], h12 = sh[5], h20 = sh[6],
                     h21 = sh[7], h22 = sh[8];
        // every lattice direction comfortably wider than 2 r_list: one candidate image per pair, and a
        // float32 prefilter on wrapped fractional coordinates ahead of the exact float64 test
        const bool wide = sh[18] < 0.5 - 1e-3 && sh[19] < 0.5 - 1e-3 && sh[20] < 0.5 - 1e-3;
        if (wide) {
          float4 *sf = reinterpret_cast<float4 *>(lds + 3 * ns + (ns & 1));  // 16-byte aligned
          for (int k = tid; k < ns; k += kPT) {
            const double x = lx[k], y = ly[k], z = lz[k];
            const double f0 = x * sh[9] + y * sh[12] + z * sh[15], f1 = x * sh[10] + y * sh[13] + z * sh[16],
                         f2 = x * sh[11] + y * sh[14] + z * sh[17];
            sf[k] = make_float4((float)(f0 - floor(f0)), (float)(f1 - floor(f1)), (float)(f2 - floor(f2)), 0.0f);
          }
          __syncthreads();
          int *surv = reinterpret_cast<int *>(sf + ns) + wave * kPSurv;
          const float g00 = (float)h00, g01 = (float)h01, g02 = (float)h02, g10 = (float)h10, g11 = (float)h11,
                      g12 = (float)h12, g20 = (float)h20, g21 = (float)h21, g22 = (float)h22;
          const double rowsum = sqrt(h00 * h00 + h01 * h01 + h02 * h02) + sqrt(h10 * h10 + h11 * h11 + h12 * h12) +
                                sqrt(h20 * h20 + h21 * h21 + h22 * h22);
          const double rcut = a.r_list + 1e-4 + 4e-6 * rowsum;
          const float rc2f = (float)(rcut * rcut);
          for (int li = wave; li < ns; li += kPW) {
            const int64_t i = a0 + li;
            const double rx = lx[li], ry = ly[li], rz = lz[li];
            const float4 fi = sf[li];
            int cnt = 0, pend = 0;
            auto exact = [&](int n) {  // the first n queued survivors, in queue (= j) order
              __builtin_amdgcn_wave_barrier();
              const int j = lane < n ? surv[lane] : li;
              const double drx = lx[j] - rx, dry = ly[j] - ry, drz = lz[j] - rz;
              const double f0 = drx * sh[9] + dry * sh[12] + drz * sh[15];
              const double f1 = drx * sh[10] + dry * sh[13] + drz * sh[16];
              const double f2 = drx * sh[11] + dry * sh[14] + drz * sh[17];
              constexpr double kRound = 6755399441055744.0;  // f + 1.5 2^52 rounds f like rint
              const double t0 = f0 + kRound, t1 = f1 + kRound, t2 = f2 + kRound;
              const double S0 = kRound - t0, S1 = kRound - t1, S2 = kRound - t2;
              const int s0 = -__double2loint(t0), s1 = -__double2loint(t1), s2 = -__double2loint(t2);
              const double dx = shift_comp(drx, S0, S1, S2, h00, h10, h20);
              const double dy = shift_comp(dry, S0, S1, S2, h01, h11, h21);
              const double dz = shift_comp(drz, S0, S1, S2, h02, h12, h22);
              const bool self = (j == li) & (s0 == 0) & (s1 == 0) & (s2 == 0);
              const bool sok = ((unsigned)(s0 + TS_MAX_IMAGE_SHIFT) <= 2u * TS_MAX_IMAGE_SHIFT) &
                               ((unsigned)(s1 + TS_MAX_IMAGE_SHIFT) <= 2u * TS_MAX_IMAGE_SHIFT) &
                               ((unsigned)(s2 + TS_MAX_IMAGE_SHIFT) <= 2u * TS_MAX_IMAGE_SHIFT);
              const bool in = (lane < n) & (norm2(dx, dy, dz) < rl2) & !self & sok;
              const uint64_t m = __ballot(in);
              const int p = cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
              if (in && p < a.max_nbr) a.nbr[row_index(p, i, st)] = pack_entry(j, s0, s1, s2);
              cnt += __popcll(m);
            };
            for (int j0 = 0; j0 < ns; j0 += kWave) {
              const int j = j0 + lane;
              const float4 fj = sf[j < ns ? j : li];
              float dfx = fj.x - fi.x, dfy = fj.y - fi.y, dfz = fj.z - fi.z;
              dfx -= rintf(dfx);
              dfy -= rintf(dfy);
              dfz -= rintf(dfz);
              const float dx = dfx * g00 + dfy * g10 + dfz * g20;
              const float dy = dfx * g01 + dfy * g11 + dfz * g21;
              const float dz = dfx * g02 + dfy * g12 + dfz * g22;
              const bool pass = (j < ns) & (dx * dx + dy * dy + dz * dz < rc2f);
              const uint64_t m = __ballot(pass);
              const int q = pend + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
              if (pass) surv[q] = j;
              pend += __popcll(m);
              if (pend >= kWave) {
                exact(kWave);
                const int rest = pend - kWave;
                const int moved = lane < rest ? surv[kWave + lane] : 0;
                __builtin_amdgcn_wave_barrier();
                if (lane < rest) surv[lane] = moved;
                __builtin_amdgcn_wave_barrier();
                pend = rest;
              }
            }
            if (pend > 0) exact(pend);
            if (lane == 0) {
              a.n_nbr[i] = cnt < a.max_nbr ? cnt : a.max_nbr;
              a.ref_pos[i] = rx;
              a.ref_pos[st + i] = ry;
              a.ref_pos[2 * st + i] = rz;
              status_raise(a.status, TS_STATUS_MAX_NBR, cnt);
              if (cnt > a.max_nbr) status_raise(a.status, TS_STATUS_OVERFLOW, 1);
            }
          }
        }
        for (int li = wide ? ns : wave; li < ns; li += kPW) {
          const int64_t i = a0 + li;
          const double rx = lx[li], ry = ly[li], rz = lz[li];
          int cnt = 0;
          for (int j0 = 0; j0 < ns; j0 += kWave) {
            const int j = j0 + lane;
            int c = 0;
            uint32_t e1 = 0;
            int lo0 = 0, hi0 = -1, lo1 = 0, hi1 = -1, lo2 = 0, hi2 = -1;
            double drx = 0.0, dry = 0.0, drz = 0.0;
            if (j < ns) {
              drx = lx[j] - rx;
              dry = ly[j] - ry;
              drz = lz[j] - rz;
              const double f0 = drx * sh[9] + dry * sh[12] + drz * sh[15];
              const double f1 = drx * sh[10] + dry * sh[13] + drz * sh[16];
              const double f2 = drx * sh[11] + dry * sh[14] + drz * sh[17];
              bool clipped = false;  // reported like an out-of-range shift (the list is then incomplete)
              image_range(f0, sh[18], &lo0, &hi0, &clipped);
              image_range(f1, sh[19], &lo1, &hi1, &clipped);
              image_range(f2, sh[20], &lo2, &hi2, &clipped);
              if (clipped) status_raise(a.status, TS_STATUS_SHIFT, 1);
              for (int S0 = lo0; S0 <= hi0; ++S0)
                for (int S1 = lo1; S1 <= hi1; ++S1)
                  for (int S2 = lo2; S2 <= hi2; ++S2) {
                    if (j == li && S0 == 0 && S1 == 0 && S2 == 0) continue;
                    const double dx = shift_comp(drx, S0, S1, S2, h00, h10, h20);
                    const double dy = shift_comp(dry, S0, S1, S2, h01, h11, h21);
                    const double dz = shift_comp(drz, S0, S1, S2, h02, h12, h22);
                    if (!(norm2(dx, dy, dz) < rl2)) continue;
                    if (S0 < -TS_MAX_IMAGE_SHIFT || S0 > TS_MAX_IMAGE_SHIFT || S1 < -TS_MAX_IMAGE_SHIFT ||
                        S1 > TS_MAX_IMAGE_SHIFT || S2 < -TS_MAX_IMAGE_SHIFT || S2 > TS_MAX_IMAGE_SHIFT) {
                      status_raise(a.status, TS_STATUS_SHIFT, 1);  // in range but not packable
                      continue;
                    }
                    if (c == 0) e1 = pack_entry(j, S0, S1, S2);
                    ++c;
                  }
            }
            int pre, total;
            if (__ballot(c > 1) == 0) {
              const uint64_t one = __ballot(c == 1);
              pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(one >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)one, 0));
              total = __popcll(one);
            } else {
              int incl = c;
#pragma unroll
              for (int o = 1; o < kWave; o <<= 1) {
                const int t = __shfl_up(incl, o, kWave);
                if (lane >= o) incl += t;
              }
              pre = incl - c;
              total = __shfl(incl, kWave - 1, kWave);
            }
            int pos = cnt + pre;
            if (c == 1) {
              if (pos < a.max_nbr) a.nbr[row_index(pos, i, st)] = e1;
            } else if (c > 1) {
              for (int S0 = lo0; S0 <= hi0; ++S0)
                for (int S1 = lo1; S1 <= hi1; ++S1)
                  for (int S2 = lo2; S2 <= hi2; ++S2) {
                    if (j == li && S0 == 0 && S1 == 0 && S2 == 0) continue;
                    if (S0 < -TS_MAX_IMAGE_SHIFT || S0 > TS_MAX_IMAGE_SHIFT || S1 < -TS_MAX_IMAGE_SHIFT ||
                        S1 > TS_MAX_IMAGE_SHIFT || S2 < -TS_MAX_IMAGE_SHIFT || S2 > TS_MAX_IMAGE_SHIFT)
                      continue;
                    const double dx = shift_comp(drx, S0, S1, S2, h00, h10, h20);
                    const double dy = shift_comp(dry, S0, S1, S2, h01, h11, h21);
                    const double dz = shift_comp(drz, S0, S1, S2, h02, h12, h22);
                    if (!(norm2(dx, dy, dz) < rl2)) continue;
                    if (pos < a.max_nbr) a.nbr[row_index(pos, i, st)] = pack_entry(j, S0, S1, S2);
                    ++pos;
                  }
            }
            cnt += total;
          }
          if (lane == 0) {
            a.n_nbr[i] = cnt < a.max_nbr ? cnt : a.max_nbr;
            a.ref_pos[i] = rx;
            a.ref_pos[st + i] = ry;
            a.ref_pos[2 * st + i] = rz;
            status_raise(a.status, TS_STATUS_MAX_NBR, cnt);
            if (cnt > a.max_nbr) status_raise(a.status, TS_STATUS_OVERFLOW, 1);
          }
        }
        __syncthreads();  // rows are read by other wavefronts below
      }

      // ---- forces, energy, virial and the FIRE scalars
      const double h00 = sh[0], h01 = sh[1], h02 = sh[2], h10 = sh[3], h11 = sh[4], h12 = sh[5], h20 = sh[6],
                   h21 = sh[7], h22 = sh[8];
      double D[9];
#pragma unroll
      for (int k = 0; k < 9; ++k) D[k] = sh[24 + k];
      double q[kPR];
#pragma unroll
      for (int k = 0; k < kPR; ++k) q[k] = 0.0;
      double wv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // sum g d (x) d: xx yy zz xy xz yz
      T *F = static_cast<T *>(a.f.force);
      for (int li0 = 0; li0 < ns; li0 += G) {
        const int li = li0 + grp;
        const bool own = li < ns;
        const int64_t i = a0 + li;
        double fx = 0.0, fy = 0.0, fz = 0.0;
        if (own) {
          const double rx = lx[li], ry = ly[li], rz = lz[li];
          const int si = single ? 0 : a.species[i];
          const int nn = a.n_nbr[i];
          for (int k = gl; k < nn; k += tl) {
            const uint32_t ent = a.nbr[row_index(k, i, st)];
            const int j = entry_j(ent);
            const double S0 = (double)entry_s0(ent), S1 = (double)entry_s1(ent), S2 = (double)entry_s2(ent);
            const double dx = shift_comp(lx[j] - rx, S0, S1, S2, h00, h10, h20);
            const double dy = shift_comp(ly[j] - ry, S0, S1, S2, h01, h11, h21);
            const double dz = shift_comp(lz[j] - rz, S0, S1, S2, h02, h12, h22);
            const double r2 = norm2(dx, dy, dz);
            if (!(r2 < tab.cut2)) continue;
            const PairCoef &pc = ltab[single ? 0 : si * TS_MAX_SPECIES + a.species[a0 + j]];
            if (KIND == TS_SOFT_SPHERE && !(r2 < pc.sig2)) continue;
            T phi = (T)0;
            const double g = (double)pair_g<KIND, T>(pc, (T)r2, r2, &phi, true);
            acc_force(g, dx, dy, dz, fx, fy, fz);
            q[4] += 0.5 * (double)phi;
            acc_virial(g, dx, dy, dz, wv);
          }
        }
        for (int o = 1; o < tl; o <<= 1) {
          fx += __shfl_xor(fx, o, tl);
          fy += __shfl_xor(fy, o, tl);
          fz += __shfl_xor(fz, o, tl);
        }
        if (own && gl == 0) {
          const T Fx = (T)fx, Fy = (T)fy, Fz = (T)fz;
          F[i] = Fx;
          F[st + i] = Fy;
          F[2 * st + i] = Fz;
          const double f0 = (double)Fx, f1 = (double)Fy, f2 = (double)Fz;
          q[0] = fmax(q[0], f0 * f0 + f1 * f1 + f2 * f2);
          double g0 = f0, g1 = f1, g2 = f2;
          if (CELL) {
            g0 = f0 * D[0] + f1 * D[1] + f2 * D[2];
            g1 = f0 * D[3] + f1 * D[4] + f2 * D[5];
            g2 = f0 * D[6] + f1 * D[7] + f2 * D[8];
          }
          const double v0 = a.f.vel[i], v1 = a.f.vel[st + i], v2 = a.f.vel[2 * st + i];
          q[1] += g0 * v0 + g1 * v1 + g2 * v2;
          q[2] += v0 * v0 + v1 * v1 + v2 * v2;
          q[3] += g0 * g0 + g1 * g1 + g2 * g2;
        }
      }
      // virial W = -1/2 sum over ordered pairs g d (x) d (slots xx xy xz . yy yz . . zz)
      q[5] = -0.5 * wv[0];
      q[6] = -0.5 * wv[3];
      q[7] = -0.5 * wv[4];
      q[9] = -0.5 * wv[1];
      q[10] = -0.5 * wv[5];
      q[13] = -0.5 * wv[2];
      // block reduction in a fixed order
#pragma unroll
      for (int k = 0; k < kPR; ++k) {
        double v = q[k];
        if (k == 0) {
#pragma unroll
          for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
        } else {
          v = wave_sum(v);
        }
        if (lane == 0) red[wave * kPR + k] = v;
      }
      __syncthreads();
      if (tid == 0) {
        double R[kPR];
        for (int k = 0; k < kPR; ++k) R[k] = k == 0 ? 0.0 : 0.0;
        for (int w = 0; w < kPW; ++w)
          for (int k = 0; k < kPR; ++k) R[k] = k == 0 ? fmax(R[0], red[w * kPR]) : R[k] + red[w * kPR + k];
        const double W[9] = {R[5], R[6], R[7], R[6], R[9], R[10], R[7], R[10], R[13]};
        if (a.energy) a.energy[s] = R[4];
        if (a.f.virial)
          for (int k = 0; k < 9; ++k) a.f.virial[9 * (int64_t)s + k] = W[k];
        bool conv = sqrt(R[0]) < cf.fmax;
        double Di[9], G[9], V[9];
        if (CELL) {
          inv3p(D, Di);
          double gmax = 0.0;
          for (int p = 0; p < 3; ++p)
            for (int r = 0; r < 3; ++r) {
              const double v = (Di[0 * 3 + p] * W[0 * 3 + r] + Di[1 * 3 + p] * W[1 * 3 + r] +
                                Di[2 * 3 + p] * W[2 * 3 + r]) / (double)ns;
              G[3 * p + r] = v;
              gmax = fmax(gmax, fabs(v));
            }
          conv = conv && gmax < cf.fmax;
          for (int k = 0; k < 9; ++k) V[k] = a.f.deform_vel[9 * (int64_t)s + k];
        }
        double stop = 0.0;
        if (conv) {
          a.f.converged[s] = 1;
          stop = 1.0;
        } else if (a.f.n_iter[s] >= cf.max_iter || (a.budget >= 0 && it >= a.budget) ||
                   (a.idle_limit > 0 &&
                    __hip_atomic_load(a.idle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= a.idle_limit)) {
          stop = 1.0;
        } else {
          double dt = a.f.dt[s], al = a.f.alpha[s];
          int np = a.f.n_pos[s];
          double cv = 1.0, cg = 0.0;
          if (a.f.n_iter[s] > 0) {
            double Pt = R[1], vvt = R[2], ggt = R[3];
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
              if (np > cf.n_min) {
                dt = fmin(dt * cf.f_inc, cf.dt_max);
                al = al * cf.f_alpha;
              }
            } else {
              cv = 0.0;
              cg = 0.0;
              dt = dt * cf.f_dec;
              al = cf.alpha_start;
              np = 0;
            }
          }
          a.f.dt[s] = dt;
          a.f.alpha[s] = al;
          a.f.n_pos[s] = np;
          a.f.n_iter[s] += 1;
          sh[21] = cv;
          sh[22] = cg;
          sh[23] = dt;
          if (CELL) {
            for (int k = 0; k < 9; ++k) {
              V[k] = cv * V[k] + cg * G[k];
              V[k] = V[k] + dt * G[k] / cf.cell_mass;
              const double dn = D[k] + (dt / (double)ns) * V[k];
              a.f.deform_vel[9 * (int64_t)s + k] = V[k];
              a.f.deform[9 * (int64_t)s + k] = dn;
              sh[33 + k] = Di[k];
              sh[42 + k] = dn;
              sh[24 + k] = dn;
            }
            for (int p = 0; p < 3; ++p)
              for (int r = 0; r < 3; ++r) {
                const double c = a.f.ref_cell[9 * (int64_t)s + 3 * p + 0] * sh[42 + r] +
                                 a.f.ref_cell[9 * (int64_t)s + 3 * p + 1] * sh[42 + 3 + r] +
                                 a.f.ref_cell[9 * (int64_t)s + 3 * p + 2] * sh[42 + 6 + r];
                sh[3 * p + r] = c;
                a.f.cell[9 * (int64_t)s + 3 * p + r] = c;
              }
          }
        }
        sh[52] = stop;
      }
      __syncthreads();
      if (sh[52] != 0.0) break;
      // ---- atom (and cell) update
      {
        const double cv = sh[21], cg = sh[22], dt = sh[23];
        for (int k = tid; k < ns; k += kPT) {
          const int64_t i = a0 + k;
          const double f0 = (double)F[i], f1 = (double)F[st + i], f2 = (double)F[2 * st + i];
          double g[3] = {f0, f1, f2};
          if (CELL) {
            g[0] = f0 * D[0] + f1 * D[1] + f2 * D[2];
            g[1] = f0 * D[3] + f1 * D[4] + f2 * D[5];
            g[2] = f0 * D[6] + f1 * D[7] + f2 * D[8];
          }
          const double m = a.f.mass ? a.f.mass[i] : 1.0;
          double v[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            v[c] = cv * a.f.vel[c * st + i] + cg * g[c];
            v[c] = v[c] + dt * g[c] / m;
            a.f.vel[c * st + i] = v[c];
          }
          const double r0 = lx[k], r1 = ly[k], r2 = lz[k];
          if (CELL) {
            const double *Di = sh + 33, *Dn = sh + 42;
            double qq[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) qq[c] = (r0 * Di[c] + r1 * Di[3 + c] + r2 * Di[6 + c]) + dt * v[c];
            lx[k] = qq[0] * Dn[0] + qq[1] * Dn[3] + qq[2] * Dn[6];
            ly[k] = qq[0] * Dn[1] + qq[1] * Dn[4] + qq[2] * Dn[7];
            lz[k] = qq[0] * Dn[2] + qq[1] * Dn[5] + qq[2] * Dn[8];
          } else {
            lx[k] = r0 + dt * v[0];
            ly[k] = r1 + dt * v[1];
            lz[k] = r2 + dt * v[2];
          }
        }
      }
      ++it;
      __syncthreads();
    }
    // write the system back
    for (int k = tid; k < ns; k += kPT) {
      a.f.pos[a0 + k] = lx[k];
      a.f.pos[st + a0 + k] = ly[k];
      a.f.pos[2 * st + a0 + k] = lz[k];
    }
    __syncthreads();
  }
}

template <int KIND, typename T>
static void launch_fp_kt(bool cell, dim3 g, size_t shm, const FirePArgs &a, const PairTable &t, hipStream_t st) {
  if (cell)
    hipLaunchKernelGGL((k_fire_persistent<KIND, T, true>), g, dim3(kPT), shm, st, t, a);
  else
    hipLaunchKernelGGL((k_fire_persistent<KIND, T, false>), g, dim3(kPT), shm, st, t, a);
}

int fire_persistent(const ts_batch *b, const ts_fire_state *fs, const ts_fire_config *cfg, ts_neighbor_list *nl,
                    const ts_pair_params *pp, int64_t n_iter, void *force, double *energy, double *virial,
                    int64_t max_atoms, bool hand_off, bool *handed_off, hipStream_t st) {
  const int64_t S = b->n_systems;
  NlWork w = nl_work(nl->workspace, b->n_atoms, S);
  FirePArgs a;
  std::memset(&a, 0, sizeof(a));
  a.f = make_fire_args(b, fs, cfg, force, virial ? virial : fs->scratch);
  a.n_sys = S;
  a.species = b->species;
  a.nbr = reinterpret_cast<uint32_t *>(nl->nbr);
  a.n_nbr = nl->n_nbr;
  a.max_nbr = nl->max_nbr;
  a.ref_pos = nl->ref_pos;
  a.ref_lcell = nl->ref_cell;
  a.status = nl->status;
  a.r_list = nl->cutoff + nl->skin;
  a.skin = nl->skin;
  a.energy = energy;
  // the work queue and its order live in the fused-loop flag area of the workspace
  a.order = w.flags3;
  a.queue = w.flags3 + 6 * S;
  a.idle = a.queue + 1;
  a.budget = n_iter;
  hipLaunchKernelGGL(k_fire_order, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, S, b->sys_offsets, a.order,
                     a.queue);
  TS_LAUNCH_CHECK();
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int64_t grid = S < 2 * (int64_t)cus ? S : 2 * (int64_t)cus;
  // hand the tail over once at most a quarter of the chip's workgroups are still iterating: the
  // slowest systems then run one per compute unit while the rest of the chip idles
  const int64_t limit = grid - cus / 4;
  a.idle_limit = (hand_off && limit > 0) ? (int32_t)limit : 0;
  if (handed_off) *handed_off = a.idle_limit > 0;
  // positions (3 x float64), wrapped fractional coordinates of the rebuild (float4) and the
  // rebuild's survivor queues
  const size_t shm = (size_t)(3 * sizeof(double) + sizeof(float4)) * (size_t)max_atoms + sizeof(double) +
                     sizeof(int) * kPSurv * kPW;
  const PairTable t = make_table(pp);
  const dim3 g((unsigned)grid);
  with_kind(t.kind, [&](auto k) {
    constexpr int KIND = decltype(k)::value;
    if (pp->prec == TS_PAIR_F32) launch_fp_kt<KIND, float>(cfg->relax_cell != 0, g, shm, a, t, st);
    else launch_fp_kt<KIND, double>(cfg->relax_cell != 0, g, shm, a, t, st);
  });
  TS_LAUNCH_CHECK();
  return TS_OK;
}

}  // namespace ts
