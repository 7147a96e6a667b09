// Fused velocity-Verlet step loop for batches whose systems fit in LDS: two launches per step.
//
// k_rebuild_rows (before step n): rebuilds the neighbor rows of the systems flagged at the end of
//   step n-1.  The flagged systems come as a device-side list, so the launch has no work and exits
//   at once when nothing was flagged.  A workgroup stages one system's positions in LDS and each
//   wavefront builds the row of one atom: its 64 lanes test 64 candidate atoms at a time under every
//   lattice image in reach, and the per-lane counts are combined with a wavefront prefix sum, so
//   the row comes out in the canonical (j, S0, S1, S2) order without a sort.
// k_step (step n): a workgroup owns `rounds` groups of APB = kStepThreads/TL consecutive atoms of
//   one system (TL lanes per atom); it stages the system's positions r_n in LDS once, evaluates the
//   pair forces of its atoms (TL lanes per atom, reduced across lanes), applies the two half kicks that meet at step n and the drift to r_{n+1}
//   (written to the other position buffer) and tests the list validity bound for r_{n+1}, appending
//   the system to the next rebuild list when it is exceeded.  The Langevin modes replace the drift
//   by half drift, O step (per-atom Philox normals), half drift: a BAOAB step.
// Systems never exchange data, so no synchronisation between workgroups is needed beyond the
// kernel boundaries.
#include "ts_forces.h"
#include "ts_neighbor.h"
#include "ts_step.h"

namespace ts {

// Flag system s for a rebuild before the next step, appending it once to that step's list.  Many
// atoms of a system cross the bound in the same step; a plain read skips the exchange once the flag
// is visibly set (same-address atomics serialise), and the exchange still decides who appends.
__device__ inline void flag_system(const StepArgs &a, int s) {
  if (__hip_atomic_load(&a.flag_next[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  if (atomicExch(&a.flag_next[s], 1) == 0) {
    // each system enters a list once per step (the exchange above), so the slot is below n_sys
    // whenever the count was cleared; the bound keeps a stale count from writing past the list
    const int q = atomicAdd(a.count_next, 1);
    if (q < a.n_sys) a.list_next[q] = s;
  }
}

// Pre-flag system s for the deferred rebuild in the next launch (as flag_system, on the pre-flag
// arrays).
__device__ inline void preflag_system(const StepArgs &a, int s) {
  if (__hip_atomic_load(&a.pflag_next[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  if (atomicExch(&a.pflag_next[s], 1) == 0) {
    const int q = atomicAdd(a.pcount_next, 1);
    if (q < a.n_sys) a.plist_next[q] = s;
  }
}

template <int NW, int RPW, bool COMPACT, typename Target>
__device__ void rebuild_rows(const StepArgs &a, int wg, int n_wg, int chunks1, const int32_t *list,
                             const int32_t *count, Target target);

// The deferred-rebuild modes keep at least four waves per SIMD (at most 128 VGPRs): their rebuild
// path shares the kernel's register budget with the pair loop.
template <int KIND, typename T, int TL, int MODE>
__global__ void __launch_bounds__(kStepThreads, MODE == kStepMidDefer || MODE == kStepLangMidDefer ? 4 : 1)
    k_step(PairTable tab, StepArgs a) {
  extern __shared__ double lds[];
  __shared__ PairCoef ltab[TS_MAX_SPECIES * TS_MAX_SPECIES];
  constexpr int APB = kStepThreads / TL;
  constexpr bool LANG = MODE == kStepLangFirst || MODE == kStepLangMid || MODE == kStepLangMidDefer;
  constexpr bool DEFER = MODE == kStepMidDefer || MODE == kStepLangMidDefer;
  constexpr bool MID = MODE == kStepMid || MODE == kStepLangMid || DEFER;
  // Langevin: no launch after the call's last one reads the counter of this call
  if (MODE == kStepLast && a.lang.rng_step && blockIdx.x == 0 && threadIdx.x == 0)
    *a.lang.rng_step += (uint64_t)a.lang_adv;
  if constexpr (DEFER) {
  if ((int)blockIdx.x < a.n_defer_wgs) {
    // deferred rebuild: the systems pre-flagged by the previous launch, from r_n, into the row
    // buffer each of them does not read in this launch (a multiple of kXcds workgroups, so the
    // XCD of every force workgroup below is unchanged)
    rebuild_rows<kStepThreads / kWave, kDeferRowsPerWave, false>(a, blockIdx.x, a.n_defer_wgs, a.defer_chunks1, a.plist_cur,
                                                          a.pcount_cur, [&](int q) { return 1 - a.sel_cur[q]; });
    return;
  }
  }
  const int wg = (int)xcd_order(blockIdx.x - a.n_defer_wgs, gridDim.x - a.n_defer_wgs);
  if (wg >= a.n_work) return;
  // uniform values: keep them in scalar registers (a vector division result would drag every
  // address derived from it into vector registers)
  const int s = __builtin_amdgcn_readfirstlane(wg / a.chunks);
  const int chunk = __builtin_amdgcn_readfirstlane(wg - s * a.chunks);
  // the flags and the list count of step n+2 (those of step n-1, consumed by the rebuild before
  // step n-1) are cleared here, ahead of every early exit: an empty system still clears its flag,
  // and workgroup 0 (system 0, chunk 0) the count, whatever the size of system 0
  // with the deferred rebuild, the buffer of the next launch (switched when this launch rebuilds
  // the system) and the pre-flag arrays of launch n+2 likewise
  // (the last and forces-only modes of a deferred loop read the buffer too)
  const bool defer = a.sel_cur != nullptr;  // uniform
  const int sel = defer ? __builtin_amdgcn_readfirstlane(a.sel_cur[s]) : 0;
  const bool fresh = DEFER && __builtin_amdgcn_readfirstlane(a.pflag_cur[s]) != 0;
  if (MID && chunk == 0 && threadIdx.x == 0) {
    a.flag_clear[s] = 0;
    if (s == 0) *a.count_clear = 0;
    if (DEFER) {
      a.sel_next[s] = fresh ? 1 - sel : sel;
      a.pflag_clear[s] = 0;
      if (s == 0) *a.pcount_clear = 0;
    }
  }
  // this launch's rows, row lengths and reference positions of system s
  const uint32_t *__restrict__ nbr = sel ? a.nbr_alt : a.nbr;
  const int32_t *__restrict__ n_nbr = sel ? a.n_nbr_alt : a.n_nbr;
  const double *__restrict__ ref_pos = sel ? a.ref_pos_alt : a.ref_pos;
  const int64_t a0 = a.offs[s];
  const int ns = (int)(a.offs[s + 1] - a0);
  const int first = chunk * a.span;
  // forces-only modes: the workgroups of a skipped system leave with those past a system's end
  const bool skipped = (MODE == kStepForce || MODE == kStepForceEV) && a.skip != nullptr && a.skip[s] != 0;
  if (first >= ns || skipped) return;
  const int end = first + a.span < ns ? first + a.span : ns;  // this chunk's atoms: [first, end)
  const int tid = threadIdx.x;
  const int grp = tid / TL, lane = tid % TL;
  const double *h = a.cell + 9 * (int64_t)s;

  if (MODE == kStepFirst || MODE == kStepLangFirst) {
    // v += dt/2 a F(r_0); r_1 = r_0 + dt v (Langevin: r += dt/2 v, O step, r += dt/2 v); list
    // validity of r_1 (cell change included)
    const double kT = LANG ? a.lang.kT[s] : 0.0;
    const uint64_t t = LANG ? *a.lang.rng_step + (uint64_t)a.lang_k : 0;
    for (int r = 0; r < a.rounds; ++r) {
      const int li = first + r * APB + grp;
      if (!(li < end && lane == 0)) continue;
      const int64_t i = a0 + li;
      const T *F = static_cast<const T *>(a.force);
      const double sc = a.mass ? a.accel / a.mass[i] : a.accel;
      double rn[3], z[3] = {0.0, 0.0, 0.0};
      if (LANG) atom_normals((uint64_t)i, t, a.lang.key0, a.lang.key1, z);
      const double sd = LANG ? a.lang.c2 * sqrt(kT * sc) : 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double v = fma(a.half_dt * (double)F[c * a.st_vel + i], sc, a.vel[c * a.st_vel + i]);
        const double r0 = a.pos_in[c * a.st_in + i];
        if (a.pos_copy) a.pos_copy[c * a.n_atoms + i] = r0;
        if (LANG) {
          const double rh = fma(a.half_dt, v, r0);
          v = fma(a.lang.c1, v, sd * z[c]);
          rn[c] = fma(a.half_dt, v, rh);
        } else {
          rn[c] = fma(a.dt, v, r0);
        }
        a.vel[c * a.st_vel + i] = v;
        a.pos_out[c * a.st_out + i] = rn[c];
      }
      if (list_invalid(rn, ref_pos, a.st_vel, i, h, a.ref_cell + 9 * (int64_t)s, a.skin, a.r_list))
        flag_system(a, s);
    }
    return;
  }

  const bool single = tab.n_species == 1 || a.species == nullptr;  // uniform
  if (!single) table_to_lds(ltab);
  constexpr bool FORCE_ONLY = MODE == kStepForce || MODE == kStepForceEV;
  const int64_t st = a.st_vel;  // list, reference positions, velocities and forces share the batch stride
  // per-atom values of the first round, loaded ahead of the staging barrier (a barrier also orders
  // memory, so loads after it could not overlap the staging latency)
  struct AtomPre {
    int nn;
    double v[3], sc, ref[3];
  } pre = {};
  {
    const int li = first + grp;
    const bool own = li < end;
    const int64_t i = a0 + li;
    pre.nn = own ? n_nbr[i] : 0;
    if (!FORCE_ONLY && own && lane == 0) {
#pragma unroll
      for (int c = 0; c < 3; ++c) pre.v[c] = a.vel[c * st + i];
      pre.sc = a.mass ? a.accel / a.mass[i] : a.accel;
      if (MID && !DEFER) {
#pragma unroll
        for (int c = 0; c < 3; ++c) pre.ref[c] = ref_pos[c * st + i];
      }
    }
  }
  // 1. stage r_n of the whole system, one (x, y, z) record per atom: a neighbor's three reads share
  // one address (the record offset goes into the read instructions)
  double *lp = lds;
  for (int k = tid; k < ns; k += kStepThreads) {
    lp[3 * k] = a.pos_in[a0 + k];
    lp[3 * k + 1] = a.pos_in[a.st_in + a0 + k];
    lp[3 * k + 2] = a.pos_in[2 * a.st_in + a0 + k];
  }
  __syncthreads();
  const double h00 = h[0], h01 = h[1], h02 = h[2], h10 = h[3], h11 = h[4], h12 = h[5], h20 = h[6], h21 = h[7],
               h22 = h[8];

  // 3. pair forces of this block's atoms, TL lanes per atom
  constexpr bool EV = MODE == kStepLast || MODE == kStepForceEV;
  const double lang_kT = LANG ? a.lang.kT[s] : 0.0;
  const uint64_t lang_t = LANG ? *a.lang.rng_step + (uint64_t)a.lang_k : 0;
  double e = 0.0, w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};  // over all rounds
  for (int r = 0; r < a.rounds; ++r) {
    const int base = first + r * APB;
    if (base >= end) break;  // uniform over the workgroup
    const int li = base + grp;
    const bool own = li < end;
    const int64_t i = a0 + li;
    const double rx = own ? lp[3 * li] : 0.0, ry = own ? lp[3 * li + 1] : 0.0, rz = own ? lp[3 * li + 2] : 0.0;
    const int nn = r == 0 ? pre.nn : (own ? n_nbr[i] : 0);
    // (evaluated after the atom's own loads: this order keeps the register count of the loop low)
    const bool diag = h01 == 0.0 && h02 == 0.0 && h10 == 0.0 && h12 == 0.0 && h20 == 0.0 && h21 == 0.0 &&
                      h00 > 0.0 && h11 > 0.0 && h22 > 0.0;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    {
      // every lane takes part (the row visit is wavefront-wide); lanes without an atom visit the
      // row of the system's first atom with nn = 0, which masks every entry out
      const int64_t irow = own ? i : a0;
      const int si = (single || !own) ? 0 : a.species[i];
      const double cut2 = tab.cut2;
      const int32_t *__restrict__ species = a.species;
      // kStepUnroll entries per lane at a time, evaluated without branches (masked by ok and the
      // cutoff test) so that their LDS loads and float64 chains overlap
      auto rows = [&](auto diag_c, auto multi_c) {
        constexpr bool DIAG = decltype(diag_c)::value, MULTI = decltype(multi_c)::value;
        const PairCoef pc0 = tab.c[0];  // loop-invariant coefficients in registers
        for_row_batched<TL, kStepUnroll>(nbr, st, irow, nn, lane, [&](const uint32_t *ent, const bool *ok) {
          double dx[kStepUnroll], dy[kStepUnroll], dz[kStepUnroll], r2[kStepUnroll];
          int jj[kStepUnroll];
          // all LDS reads first, then the shift vectors (independent of them), then the pair vectors
#pragma unroll
          for (int u = 0; u < kStepUnroll; ++u) {
            const int j = ok[u] ? entry_j(ent[u]) : 0;  // masked visits read a staged atom
            jj[u] = j;
            dx[u] = lp[3 * j];
            dy[u] = lp[3 * j + 1];
            dz[u] = lp[3 * j + 2];
          }
#pragma unroll
          for (int u = 0; u < kStepUnroll; ++u) {
            const double S0 = entry_s0d(ent[u]), S1 = entry_s1d(ent[u]), S2 = entry_s2d(ent[u]);
            if (DIAG) {
              // off-diagonal products are exact zeros: the same value as the general form
              dx[u] = (dx[u] - rx) + S0 * h00;
              dy[u] = (dy[u] - ry) + S1 * h11;
              dz[u] = (dz[u] - rz) + S2 * h22;
            } else {
              dx[u] = shift_comp(dx[u] - rx, S0, S1, S2, h00, h10, h20);
              dy[u] = shift_comp(dy[u] - ry, S0, S1, S2, h01, h11, h21);
              dz[u] = shift_comp(dz[u] - rz, S0, S1, S2, h02, h12, h22);
            }
            r2[u] = norm2(dx[u], dy[u], dz[u]);
          }
#pragma unroll
          for (int u = 0; u < kStepUnroll; ++u) {
            const PairCoef &c = MULTI ? ltab[si * TS_MAX_SPECIES + species[a0 + jj[u]]] : pc0;
            bool in = ok[u] && r2[u] < cut2;
            if (KIND == TS_SOFT_SPHERE) in = in && r2[u] < c.sig2;
            T phi = (T)0;
            const T gt = pair_g<KIND, T>(c, (T)r2[u], r2[u], &phi, EV);
            const double g = in ? (double)gt : 0.0;
            acc_force(g, dx[u], dy[u], dz[u], fx, fy, fz);
            if (EV) {
              e += in ? (double)phi : 0.0;
              acc_virial(g, dx[u], dy[u], dz[u], w);
            }
          }
        });
      };
      using yes = std::true_type;
      using no = std::false_type;
      if (diag) {
        if (single) rows(yes{}, no{});
        else rows(yes{}, yes{});
      } else {
        if (single) rows(no{}, no{});
        else rows(no{}, yes{});
      }
    }
#pragma unroll
    for (int o = 1; o < TL; o <<= 1) {
      fx += __shfl_xor(fx, o, TL);
      fy += __shfl_xor(fy, o, TL);
      fz += __shfl_xor(fz, o, TL);
    }

    // 4. kicks and drift (lane 0 of each atom)
    if (own && lane == 0) {
      T *F = static_cast<T *>(a.force);
      const T Fx = (T)fx, Fy = (T)fy, Fz = (T)fz;
      const double sc = FORCE_ONLY ? 0.0 : (r == 0 ? pre.sc : (a.mass ? a.accel / a.mass[i] : a.accel));
      const double hx = a.half_dt * (double)Fx, hy = a.half_dt * (double)Fy, hz = a.half_dt * (double)Fz;
      double vx = 0.0, vy = 0.0, vz = 0.0;
      if (!FORCE_ONLY) {
        vx = r == 0 ? pre.v[0] : a.vel[i];
        vy = r == 0 ? pre.v[1] : a.vel[st + i];
        vz = r == 0 ? pre.v[2] : a.vel[2 * st + i];
      }
      // explicit fused multiply-adds: every kick and drift rounds the same way in every kernel
      vx = fma(hx, sc, vx);
      vy = fma(hy, sc, vy);
      vz = fma(hz, sc, vz);
      if (FORCE_ONLY) {
        F[i] = Fx;
        F[st + i] = Fy;
        F[2 * st + i] = Fz;
      } else if (MID) {
        vx = fma(hx, sc, vx);
        vy = fma(hy, sc, vy);
        vz = fma(hz, sc, vz);
        double nx, ny, nz;
        if (LANG) {
          // r += dt/2 v; v = c1 v + c2 sqrt(a kT_s / m) xi; r += dt/2 v
          double z[3];
          atom_normals((uint64_t)i, lang_t, a.lang.key0, a.lang.key1, z);
          const double sd = a.lang.c2 * sqrt(lang_kT * sc);
          const double ax = fma(a.half_dt, vx, rx), ay = fma(a.half_dt, vy, ry), az = fma(a.half_dt, vz, rz);
          vx = fma(a.lang.c1, vx, sd * z[0]);
          vy = fma(a.lang.c1, vy, sd * z[1]);
          vz = fma(a.lang.c1, vz, sd * z[2]);
          nx = fma(a.half_dt, vx, ax);
          ny = fma(a.half_dt, vy, ay);
          nz = fma(a.half_dt, vz, az);
        } else {
          nx = fma(a.dt, vx, rx);
          ny = fma(a.dt, vy, ry);
          nz = fma(a.dt, vz, rz);
        }
        a.pos_out[i] = nx;
        a.pos_out[a.st_out + i] = ny;
        a.pos_out[2 * a.st_out + i] = nz;
        // the cell is unchanged since the list was built (a changed cell was flagged by the first step)
        // (rows rebuilt from r_n in this launch have the reference r_n)
        double qx, qy, qz;
        if (DEFER) {
          qx = fresh ? rx : ref_pos[i];
          qy = fresh ? ry : ref_pos[st + i];
          qz = fresh ? rz : ref_pos[2 * st + i];
        } else {
          qx = r == 0 ? pre.ref[0] : ref_pos[i];
          qy = r == 0 ? pre.ref[1] : ref_pos[st + i];
          qz = r == 0 ? pre.ref[2] : ref_pos[2 * st + i];
        }
        const double dref = sqrt(norm2(nx - qx, ny - qy, nz - qz));
        if (bound_exceeded(dref, 0.0, a.skin, a.r_list)) {
          flag_system(a, s);  // the list of the next launch fails: rebuilt before it
        } else if (DEFER && !fresh) {
          // predicted to fail soon (the displacement since the build grows by about one step's
          // displacement per step): rebuilt during the next launch, which still reads valid rows
          const double dstep = sqrt(norm2(nx - rx, ny - ry, nz - rz));
          if (bound_exceeded(dref + a.pre_factor * dstep, 0.0, a.skin, a.r_list)) preflag_system(a, s);
        }
      } else {
        F[i] = Fx;
        F[st + i] = Fy;
        F[2 * st + i] = Fz;
        if (a.pos_final) {
          a.pos_final[i] = rx;
          a.pos_final[st + i] = ry;
          a.pos_final[2 * st + i] = rz;
        }
      }
      if (!FORCE_ONLY) {
        a.vel[i] = vx;
        a.vel[st + i] = vy;
        a.vel[2 * st + i] = vz;
      }
    }
  }  // rounds
  if (EV && (a.epot || a.virial)) {
    // every lane of the block belongs to system s
    const double ev = wave_sum(0.5 * e);
    const double v0 = wave_sum(-0.5 * w[0]), v1 = wave_sum(-0.5 * w[1]), v2 = wave_sum(-0.5 * w[2]);
    const double v3 = wave_sum(-0.5 * w[3]), v4 = wave_sum(-0.5 * w[4]), v5 = wave_sum(-0.5 * w[5]);
    if ((tid % kWave) == 0) {
      if (a.epot) atomicAdd(&a.epot[s], ev);
      if (a.virial) {
        double *W = a.virial + 9 * (int64_t)s;
        atomicAdd(&W[0], v0);
        atomicAdd(&W[4], v1);
        atomicAdd(&W[8], v2);
        atomicAdd(&W[1], v3);
        atomicAdd(&W[3], v3);
        atomicAdd(&W[2], v4);
        atomicAdd(&W[6], v4);
        atomicAdd(&W[5], v5);
        atomicAdd(&W[7], v5);
      }
    }
  }
}

// Rebuild rows: one wavefront per atom; a workgroup of kRebuildWaves wavefronts handles that many
// consecutive atoms of one flagged system ("chunks"; the chunk count per system covers the largest
// system).
constexpr int kRebuildWaves = 4;
constexpr int kRebuildWgsPerCu = 4;            // rebuild workgroups a CU holds at most (four waves per SIMD)
constexpr size_t kRebuildFullLds = 40 * 1024;  // largest LDS use of the full layout (four workgroups per CU)
constexpr int kSurvCap = 3 * kWave;  // survivor queue of a wavefront in the wide path

__device__ inline bool shift_ok(int S0, int S1, int S2) {
  // |S| <= 15 for all three: (S + 15) as unsigned is at most 30
  return ((unsigned)(S0 + TS_MAX_IMAGE_SHIFT) <= 2u * TS_MAX_IMAGE_SHIFT) &
         ((unsigned)(S1 + TS_MAX_IMAGE_SHIFT) <= 2u * TS_MAX_IMAGE_SHIFT) &
         ((unsigned)(S2 + TS_MAX_IMAGE_SHIFT) <= 2u * TS_MAX_IMAGE_SHIFT);
}

// Per-system geometry of a step loop's rebuilds, once per call (the cells do not change in it).
__global__ void __launch_bounds__(256) k_row_geometry(int64_t n_sys, const double *__restrict__ cell, double r_list,
                                                      RowGeom *__restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_sys) return;
  RowGeom g;
  row_geometry(cell + 9 * s, r_list, &g);
  out[s] = g;
}

int launch_row_geometry(int64_t n_sys, const double *cell, double r_list, RowGeom *out, hipStream_t st) {
  if (n_sys <= 0) return TS_OK;
  hipLaunchKernelGGL(k_row_geometry, dim3((unsigned)ceil_div(n_sys, 256)), dim3(256), 0, st, n_sys, cell, r_list, out);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

// The rows of the systems in list[0 .. *count) from positions a.pos_in, built by workgroup wg of
// n_wg (a grid-stride loop over chunks of NW * RPW consecutive atoms of one system; chunks1 =
// ceil(largest system / NW) is the chunk count per system at one row per wavefront).  Each
// system's rows, row lengths and reference positions go to the buffer `target(s)` selects (0: nbr,
// n_nbr, ref_pos; 1: the deferred-rebuild buffers).  COMPACT: for large systems, wide cells keep only the
// float32 fractional coordinates in LDS (16 B per atom instead of 40) and the exact pass reads the
// float64 positions of its survivors from memory, so that more workgroups share a CU.
template <int NW, int RPW, bool COMPACT, typename Target>
__device__ void rebuild_rows(const StepArgs &a, int wg, int n_wg, int chunks1, const int32_t *list,
                             const int32_t *count, Target target) {
  extern __shared__ double lds[];
  // atoms a thread stages: batches of kStageBatch, every load of a batch issued before its stores
  constexpr int kStageBatch = 4;
  constexpr int kStage = (kLdsMaxAtoms + kWave * NW - 1) / (kWave * NW);
  // the flagged-system count and this workgroup's first list slot are loaded together (the slot
  // is read speculatively: the list has room for every system)
  const int chunks_per_sys = (chunks1 + RPW - 1) / RPW;
  const int q0 = wg / chunks_per_sys;
  const int s_spec = q0 < a.n_sys ? list[q0] : 0;
  const int n_cnt = *count;
  const int n_flag = n_cnt < a.n_sys ? n_cnt : a.n_sys;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const double rl2 = a.r_list * a.r_list;
  const int64_t st = a.st_vel;
  const double *__restrict__ pin = a.pos_in;
  for (int chunk = wg; chunk < n_flag * chunks_per_sys; chunk += n_wg) {
    const int s = chunk == wg ? s_spec : list[chunk / chunks_per_sys];
    const int c0 = (chunk % chunks_per_sys) * (NW * RPW);
    const int64_t a0 = a.offs[s];
    const int ns = (int)(a.offs[s + 1] - a0);
    if (c0 >= ns) continue;  // uniform over the workgroup
    const int buf = __builtin_amdgcn_readfirstlane(target(s));
    uint32_t *__restrict__ nbr = buf ? a.nbr_alt : a.nbr;
    int32_t *__restrict__ n_nbr = buf ? a.n_nbr_alt : a.n_nbr;
    double *__restrict__ ref_pos = buf ? a.ref_pos_alt : a.ref_pos;
    const double *__restrict__ h = a.cell + 9 * (int64_t)s;
    if (c0 == 0) {
      if (threadIdx.x < 9) a.ref_cell[9 * (int64_t)s + threadIdx.x] = h[threadIdx.x];
      if (threadIdx.x == 0) atomicAdd((unsigned long long *)&a.status[TS_STATUS_REBUILDS], 1ull);
    }
    // cell, inverse, reach and prefilter bound: from the per-system table (computed once per call by
    // the step loops, per update by the list-init kernel), else uniform values every lane computes
    // itself (no serial section); both come from row_geometry
    const double h00 = h[0], h01 = h[1], h02 = h[2], h10 = h[3], h11 = h[4], h12 = h[5], h20 = h[6], h21 = h[7],
                 h22 = h[8];
    RowGeom geo;
    if (a.row_geom) geo = a.row_geom[s];
    else row_geometry(h, a.r_list, &geo);
    const double i00 = geo.inv[0], i01 = geo.inv[1], i02 = geo.inv[2], i10 = geo.inv[3], i11 = geo.inv[4],
                 i12 = geo.inv[5], i20 = geo.inv[6], i21 = geo.inv[7], i22 = geo.inv[8];
    const double det = geo.det;
    if (c0 == 0 && threadIdx.x == 0 && !(isfinite(det) && det != 0.0)) status_raise(a.status, TS_STATUS_NONFINITE, 1);
    const double re0 = geo.reach[0], re1 = geo.reach[1], re2 = geo.reach[2];
    // every lattice direction comfortably wider than 2 r_list: at most one image of j is within
    // r_list of i, the nearest one, S = -rint(fractional difference) (a tie at |f + S| = 1/2 is out
    // of reach), and the float32 prefilter on wrapped fractional coordinates below is safe
    const bool wide = re0 < 0.5 - 1e-3 && re1 < 0.5 - 1e-3 && re2 < 0.5 - 1e-3;
    __syncthreads();  // the previous chunk's readers are done with lds
    // LDS: float64 positions [3][ns], float4 wrapped fractional coordinates [ns] (16-byte aligned:
    // one padding double when ns is odd) and the wavefronts' survivor queues.  COMPACT: the
    // fractional coordinates alone, where the positions would be (the exact passes read float64
    // positions from memory).
    constexpr bool kCompact = COMPACT;
    constexpr bool lds_pos = !kCompact;
    double *lx = lds, *ly = lds + ns, *lz = lds + 2 * ns;
    float4 *sf = reinterpret_cast<float4 *>(kCompact ? lds : lds + 3 * ns + (ns & 1));
    int *surv = reinterpret_cast<int *>(sf + ns) + wave * kSurvCap;
    const double *__restrict__ gx = pin + a0, *__restrict__ gy = pin + a.st_in + a0, *__restrict__ gz =
                                                                                       pin + 2 * a.st_in + a0;
    {
      // the loads of a batch are issued before its stores (past the end a thread reloads the last
      // atom and stores nothing)
#pragma unroll 1
      for (int u0 = 0; u0 < kStage && u0 * kWave * NW < ns; u0 += kStageBatch) {
      double px[kStageBatch], py[kStageBatch], pz[kStageBatch];
#pragma unroll
      for (int v = 0; v < kStageBatch; ++v) {
        const int k = threadIdx.x + (u0 + v) * kWave * NW;
        const int kc = k < ns ? k : ns - 1;
        px[v] = pin[a0 + kc];
        py[v] = pin[a.st_in + a0 + kc];
        pz[v] = pin[2 * a.st_in + a0 + kc];
      }
#pragma unroll
      for (int v = 0; v < kStageBatch; ++v) {
        const int u = v;
        const int k = threadIdx.x + (u0 + v) * kWave * NW;
        if (k >= ns) break;
        const double x = px[u], y = py[u], z = pz[u];
        if (lds_pos) {
          lx[k] = x;
          ly[k] = y;
          lz[k] = z;
        }
        if (kCompact || wide) {  // the small-system kernel scans the other cells exhaustively
          const double f0 = x * i00 + y * i10 + z * i20, f1 = x * i01 + y * i11 + z * i21,
                       f2 = x * i02 + y * i12 + z * i22;
          sf[k] = make_float4((float)(f0 - floor(f0)), (float)(f1 - floor(f1)), (float)(f2 - floor(f2)), 0.0f);
        }
      }
      }  // batches
    }
    __syncthreads();
    // wavefront w builds rows c0 + w, c0 + w + kRebuildWaves, ... of the chunk
#pragma unroll 1
    for (int rr = 0; rr < RPW; ++rr) {
    const int li = c0 + wave + NW * rr;
    if (li >= ns) break;  // uniform over the wavefront; no block barrier follows before the loop top
    const int64_t i = a0 + li;
    const double rx = lds_pos ? lx[li] : gx[li], ry = lds_pos ? ly[li] : gy[li], rz = lds_pos ? lz[li] : gz[li];
    int cnt = 0;
    bool shift_bad = false;
    // Pass 1, float32 on wrapped fractional coordinates: candidates are queued (in j order) when
    // they may have an image within r_list.  Pass 2, float64: each batch of up to 64 queued
    // candidates takes the exact test and is compacted into the row in queue order.  The float32
    // tests use r_list + delta, where delta bounds their rounding (a few 1e-5 A at most) with a wide
    // margin, so no pair within r_list is lost.
    //  * wide cells (every direction wider than 2 r_list): at most one image of j is within r_list
    //    of i, the nearest one, S = -rint(fractional difference) (a tie at |f + S| = 1/2 is out of
    //    reach); pass 1 is the nearest-image distance and pass 2 tests that image;
    //  * other cells, large systems (COMPACT): any image's distance is at least |d_k| w_k in every
    //    direction k (d the nearest-image fractional difference, w_k the width across the planes of
    //    the other two lattice vectors); pass 1 keeps candidates with max_k |d_k| w_k below the
    //    bound and pass 2 enumerates every image within reach;
    //  * other cells, small systems: every candidate takes pass 2.
    int pend = 0;
    // queue the survivors of two blocks of 64 candidates per iteration (independent chains until
    // their ballots); the queue holds up to 3 x 64 survivors, and every full 64 of them take pass 2
    auto scan = [&](auto pass1, auto pass2) {
      for (int j0 = 0; j0 < ns; j0 += 2 * kWave) {
        const int ja = j0 + lane, jb = j0 + kWave + lane;
        const bool pa = pass1(ja), pb = pass1(jb);
        const uint64_t ma = __ballot(pa), mb = __ballot(pb);
        const int qa = pend + __builtin_amdgcn_mbcnt_hi((uint32_t)(ma >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)ma, 0));
        if (pa) surv[qa] = ja;
        pend += __popcll(ma);
        const int qb = pend + __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0));
        if (pb) surv[qb] = jb;
        pend += __popcll(mb);
        while (pend >= kWave) {
          pass2(kWave);
          // move the overflow (fewer than 2 x 64 entries) to the front of the queue
          const int rest = pend - kWave;
          const int m0 = lane < rest ? surv[kWave + lane] : 0;
          const int m1 = lane + kWave < rest ? surv[2 * kWave + lane] : 0;
          __builtin_amdgcn_wave_barrier();
          if (lane < rest) surv[lane] = m0;
          if (lane + kWave < rest) surv[kWave + lane] = m1;
          __builtin_amdgcn_wave_barrier();
          pend = rest;
        }
      }
      if (pend > 0) pass2(pend);
    };
    if (wide) {
      const float4 fi = sf[li];
      const double rc = geo.bound;
      const float g00 = (float)h00, g01 = (float)h01, g02 = (float)h02, g10 = (float)h10, g11 = (float)h11,
                  g12 = (float)h12, g20 = (float)h20, g21 = (float)h21, g22 = (float)h22;
      const float rc2f = (float)(rc * rc);
      auto exact = [&](int n) {  // the first n queued survivors
        __builtin_amdgcn_wave_barrier();  // queue writes of other lanes before these reads
        const int j = lane < n ? surv[lane] : li;
        const double drx = (lds_pos ? lx[j] : gx[j]) - rx, dry = (lds_pos ? ly[j] : gy[j]) - ry,
                     drz = (lds_pos ? lz[j] : gz[j]) - rz;
        const double f0 = drx * i00 + dry * i10 + drz * i20, f1 = drx * i01 + dry * i11 + drz * i21,
                     f2 = drx * i02 + dry * i12 + drz * i22;
        // nearest integers without rounding or conversion instructions: t = f + 1.5 2^52 rounds f to
        // an integer n (ties to even, like rint) for |f| < 2^51, and the low word of t is n
        constexpr double kRound = 6755399441055744.0;
        const double t0 = f0 + kRound, t1 = f1 + kRound, t2 = f2 + kRound;
        const double S0 = kRound - t0, S1 = kRound - t1, S2 = kRound - t2;  // -rint(f), exact
        const int s0 = -__double2loint(t0), s1 = -__double2loint(t1), s2 = -__double2loint(t2);
        const double dx = shift_comp(drx, S0, S1, S2, h00, h10, h20);
        const double dy = shift_comp(dry, S0, S1, S2, h01, h11, h21);
        const double dz = shift_comp(drz, S0, S1, S2, h02, h12, h22);
        const int fs = s0 != 0 ? s0 : (s1 != 0 ? s1 : s2);
        const bool self = (j == li) & (s0 == 0) & (s1 == 0) & (s2 == 0);
        const bool side = !a.half | (li < j) | ((li == j) & (fs > 0));
        const bool near = (lane < n) & (norm2(dx, dy, dz) < rl2) & !self & side;
        const bool sok = shift_ok(s0, s1, s2);
        shift_bad |= near & !sok;
        const bool in = near & sok;
        const uint64_t m = __ballot(in);
        const int p = cnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
        if (in && p < a.max_nbr) nbr[row_index(p, i, st)] = pack_entry(j, s0, s1, s2);
        cnt += __popcll(m);
      };
      // float32 nearest-image test of candidate j (false past the end); DIAG: a cell whose
      // off-diagonal entries are zero, where the pair vector needs one product per component
      auto near_f32 = [&](int j, auto diag_c) {
        constexpr bool DIAG = decltype(diag_c)::value;
        const float4 fj = sf[j < ns ? j : li];
        float dfx = fj.x - fi.x, dfy = fj.y - fi.y, dfz = fj.z - fi.z;
        dfx -= rintf(dfx);
        dfy -= rintf(dfy);
        dfz -= rintf(dfz);
        const float dx = DIAG ? dfx * g00 : dfx * g00 + dfy * g10 + dfz * g20;
        const float dy = DIAG ? dfy * g11 : dfx * g01 + dfy * g11 + dfz * g21;
        const float dz = DIAG ? dfz * g22 : dfx * g02 + dfy * g12 + dfz * g22;
        return (j < ns) & (dx * dx + dy * dy + dz * dz < rc2f);
      };
      const bool diag = h01 == 0.0 && h02 == 0.0 && h10 == 0.0 && h12 == 0.0 && h20 == 0.0 && h21 == 0.0;
      if (diag) scan([&](int j) { return near_f32(j, std::true_type{}); }, exact);
      else scan([&](int j) { return near_f32(j, std::false_type{}); }, exact);
    } else {
      // every image within r_list of candidate j (one per lane, valid lanes only), compacted into
      // the row in (lane, S0, S1, S2) order
      auto multi = [&](int j, bool valid) {
        int c = 0;
        uint32_t e1 = 0;
        int lo0 = 0, hi0 = -1, lo1 = 0, hi1 = -1, lo2 = 0, hi2 = -1;
        double drx = 0.0, dry = 0.0, drz = 0.0;
        if (valid) {
          drx = (lds_pos ? lx[j] : gx[j]) - rx;
          dry = (lds_pos ? ly[j] : gy[j]) - ry;
          drz = (lds_pos ? lz[j] : gz[j]) - rz;
          image_range(drx * i00 + dry * i10 + drz * i20, re0, &lo0, &hi0, &shift_bad);
          image_range(drx * i01 + dry * i11 + drz * i21, re1, &lo1, &hi1, &shift_bad);
          image_range(drx * i02 + dry * i12 + drz * i22, re2, &lo2, &hi2, &shift_bad);
          if (lo0 == hi0 && lo1 == hi1 && lo2 == hi2) {
            // one candidate image (always the case when the cell is wider than 2 r_list)
            const int S0 = lo0, S1 = lo1, S2 = lo2;
            if (!(j == li && S0 == 0 && S1 == 0 && S2 == 0)) {
              const double dx = shift_comp(drx, S0, S1, S2, h00, h10, h20);
              const double dy = shift_comp(dry, S0, S1, S2, h01, h11, h21);
              const double dz = shift_comp(drz, S0, S1, S2, h02, h12, h22);
              const int fs = S0 != 0 ? S0 : (S1 != 0 ? S1 : S2);
              if (norm2(dx, dy, dz) < rl2 && (!a.half || li < j || (li == j && fs > 0))) {
                if (shift_ok(S0, S1, S2)) {
                  e1 = pack_entry(j, S0, S1, S2);
                  c = 1;
                } else {
                  shift_bad = true;
                }
              }
            }
          } else {
            for (int S0 = lo0; S0 <= hi0; ++S0)
              for (int S1 = lo1; S1 <= hi1; ++S1)
                for (int S2 = lo2; S2 <= hi2; ++S2) {
                  if (j == li && S0 == 0 && S1 == 0 && S2 == 0) continue;
                  const double dx = shift_comp(drx, S0, S1, S2, h00, h10, h20);
                  const double dy = shift_comp(dry, S0, S1, S2, h01, h11, h21);
                  const double dz = shift_comp(drz, S0, S1, S2, h02, h12, h22);
                  if (!(norm2(dx, dy, dz) < rl2)) continue;
                  const int fs = S0 != 0 ? S0 : (S1 != 0 ? S1 : S2);
                  if (a.half && !(li < j || (li == j && fs > 0))) continue;
                  if (!shift_ok(S0, S1, S2)) {
                    shift_bad = true;
                    continue;
                  }
                  if (c == 0) e1 = pack_entry(j, S0, S1, S2);
                  ++c;
                }
          }
        }
        // exclusive prefix of the per-lane counts across the wavefront (ballot + mbcnt when every
        // lane holds at most one entry)
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
          if (pos < a.max_nbr) nbr[row_index(pos, i, st)] = e1;
        } else if (c > 1) {
          for (int S0 = lo0; S0 <= hi0; ++S0)
            for (int S1 = lo1; S1 <= hi1; ++S1)
              for (int S2 = lo2; S2 <= hi2; ++S2) {
                if (j == li && S0 == 0 && S1 == 0 && S2 == 0) continue;
                const double dx = shift_comp(drx, S0, S1, S2, h00, h10, h20);
                const double dy = shift_comp(dry, S0, S1, S2, h01, h11, h21);
                const double dz = shift_comp(drz, S0, S1, S2, h02, h12, h22);
                if (!(norm2(dx, dy, dz) < rl2)) continue;
                const int fs = S0 != 0 ? S0 : (S1 != 0 ? S1 : S2);
                if (a.half && !(li < j || (li == j && fs > 0))) continue;
                if (!shift_ok(S0, S1, S2)) continue;
                if (pos < a.max_nbr) nbr[row_index(pos, i, st)] = pack_entry(j, S0, S1, S2);
                ++pos;
              }
        }
        cnt += total;
      };
      if constexpr (COMPACT) {
        const float4 fi = sf[li];
        const double rc = geo.bound;
        // perpendicular widths w_k = r_list / reach_k
        const float w0 = (float)(a.r_list / re0), w1 = (float)(a.r_list / re1), w2 = (float)(a.r_list / re2);
        const float rcf = (float)rc;
        auto slab_f32 = [&](int j) {  // float32 slab test of candidate j (false past the end)
          const float4 fj = sf[j < ns ? j : li];
          float d0 = fj.x - fi.x, d1 = fj.y - fi.y, d2 = fj.z - fi.z;
          d0 -= rintf(d0);
          d1 -= rintf(d1);
          d2 -= rintf(d2);
          const float m = fmaxf(fabsf(d0) * w0, fmaxf(fabsf(d1) * w1, fabsf(d2) * w2));
          return (j < ns) & (m < rcf);
        };
        // the first n queued candidates
        auto images = [&](int n) {
          __builtin_amdgcn_wave_barrier();  // queue writes of other lanes before these reads
          multi(lane < n ? surv[lane] : li, lane < n);
        };
        scan(slab_f32, images);
      } else {
        // small systems: every candidate takes the exact test (the shorter code keeps the latency
        // of the step loops' rebuild low)
        for (int j0 = 0; j0 < ns; j0 += kWave) multi(j0 + lane, j0 + lane < ns);
      }
    }
    if (lane == 0) {
      n_nbr[i] = cnt < a.max_nbr ? cnt : a.max_nbr;
      ref_pos[i] = rx;
      ref_pos[st + i] = ry;
      ref_pos[2 * st + i] = rz;
      status_raise(a.status, TS_STATUS_MAX_NBR, cnt);
      if (cnt > a.max_nbr) status_raise(a.status, TS_STATUS_OVERFLOW, 1);
      if (!(isfinite(rx) && isfinite(ry) && isfinite(rz))) status_raise(a.status, TS_STATUS_NONFINITE, 1);
    }
    if (__ballot(shift_bad) != 0 && lane == 0) status_raise(a.status, TS_STATUS_SHIFT, 1);
    }  // rows of this wavefront
  }
}

// Rows of the systems flagged for a rebuild before the next step (the list's own buffer of each
// system: the one the step kernel reads next).
template <bool COMPACT>
__global__ void __launch_bounds__(kWave * kRebuildWaves) k_rebuild_rows(StepArgs a, int chunks1) {
  rebuild_rows<kRebuildWaves, 1, COMPACT>(a, blockIdx.x, gridDim.x, chunks1, a.list_cur, a.count_cur,
                                          [&](int s) { return a.sel_cur ? a.sel_cur[s] : 0; });
}

int launch_rebuild(const StepArgs &a, int64_t n_sys, int64_t max_atoms, hipStream_t st) {
  // float64 positions, float4 fractional coordinates (after one alignment double) and the
  // survivor queues; beyond kRebuildFullLds, the compact layout (the fractional coordinates and the
  // queues)
  const size_t queues = sizeof(int) * kSurvCap * kRebuildWaves;
  const size_t full = (size_t)(5 * max_atoms + 1) * sizeof(double) + queues;
  StepArgs b = a;
  b.n_sys = (int)n_sys;
  const bool compact = full > kRebuildFullLds;
  const size_t shm = compact ? (size_t)max_atoms * sizeof(float4) + queues : full;
  // one workgroup per chunk up to what the CUs hold at once (every workgroup then loops over chunks
  // from the start, none waits for a free slot)
  const int chunks1 = (int)ceil_div(max_atoms, kRebuildWaves);
  const int64_t work = n_sys * chunks1;
  const int64_t fit = kLdsBytes / (int64_t)shm;
  const int64_t per_cu = fit < kRebuildWgsPerCu ? fit : kRebuildWgsPerCu;
  const int64_t resident = (int64_t)device_cus() * (per_cu > 0 ? per_cu : 1);
  const unsigned grid = (unsigned)(work < resident ? work : resident);
  if (compact)
    hipLaunchKernelGGL(k_rebuild_rows<true>, dim3(grid), dim3(kWave * kRebuildWaves), shm, st, b, chunks1);
  else
    hipLaunchKernelGGL(k_rebuild_rows<false>, dim3(grid), dim3(kWave * kRebuildWaves), shm, st, b, chunks1);
  TS_LAUNCH_CHECK();
  return TS_OK;
}

template <int KIND, typename T, int TL>
static void launch_step_k(int mode, const StepArgs &a, const PairTable &t, dim3 g, size_t shm, hipStream_t st) {
  if (mode == kStepFirst)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepFirst>), g, dim3(kStepThreads), 0, st, t, a);
  else if (mode == kStepLangFirst)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepLangFirst>), g, dim3(kStepThreads), 0, st, t, a);
  else if (mode == kStepLangMid)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepLangMid>), g, dim3(kStepThreads), shm, st, t, a);
  else if (mode == kStepMid)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepMid>), g, dim3(kStepThreads), shm, st, t, a);
  else if (mode == kStepMidDefer)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepMidDefer>), g, dim3(kStepThreads), shm, st, t, a);
  else if (mode == kStepLangMidDefer)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepLangMidDefer>), g, dim3(kStepThreads), shm, st, t, a);
  else if (mode == kStepLast)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepLast>), g, dim3(kStepThreads), shm, st, t, a);
  else if (mode == kStepForce)
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepForce>), g, dim3(kStepThreads), shm, st, t, a);
  else
    hipLaunchKernelGGL((k_step<KIND, T, TL, kStepForceEV>), g, dim3(kStepThreads), shm, st, t, a);
}

template <int KIND, typename T>
static void launch_step_kt(int tl, int mode, const StepArgs &a, const PairTable &t, dim3 g, size_t shm,
                           hipStream_t st) {
  switch (tl) {
    case 1: launch_step_k<KIND, T, 1>(mode, a, t, g, shm, st); break;
    case 2: launch_step_k<KIND, T, 2>(mode, a, t, g, shm, st); break;
    case 4: launch_step_k<KIND, T, 4>(mode, a, t, g, shm, st); break;
    default: launch_step_k<KIND, T, 8>(mode, a, t, g, shm, st); break;
  }
}

int launch_step(int mode, int tl, int group_atoms, StepArgs a, const PairTable &t, int prec, int64_t n_sys,
                int64_t max_atoms, const int64_t *h_offs, hipStream_t st) {
  const int apb = kStepThreads / tl;
  const int64_t max_rounds = ceil_div(max_atoms, apb);
  int64_t rounds = 1;
  if (group_atoms > 0) {
    rounds = group_atoms / apb;
  } else {
    // one round per workgroup until the launch holds about kStepTargetWgs non-empty workgroups
    int64_t wgs = 0;
    for (int64_t s = 0; s < n_sys; ++s) wgs += ceil_div(h_offs[s + 1] - h_offs[s], apb);
    rounds = wgs / kStepTargetWgs;
  }
  rounds = rounds < 1 ? 1 : (rounds > max_rounds ? max_rounds : rounds);
  a.rounds = (int)rounds;
  a.chunks = (int)ceil_div(max_atoms, apb * rounds);
  // equal shares of the largest system (the last chunk is not left with a remainder)
  a.span = a.chunks > 0 ? (int)ceil_div(max_atoms, a.chunks) : 1;
  a.n_work = n_sys * a.chunks;
  // deferred-rebuild workgroups first (a multiple of kXcds), then the force workgroups
  const int64_t grid = ceil_div(a.n_work, kXcds) * kXcds + a.n_defer_wgs;
  if (grid > 0x7fffffff) return TS_E_CAPACITY;
  const dim3 g((unsigned)grid);
  size_t shm = (size_t)3 * sizeof(double) * (size_t)max_atoms;
  if (a.n_defer_wgs > 0) {
    constexpr int nw = kStepThreads / kWave;
    a.defer_chunks1 = (int)ceil_div(max_atoms, nw);
    const size_t shm_rb = (size_t)(5 * max_atoms + 1) * sizeof(double) + sizeof(int) * kSurvCap * nw;
    shm = shm_rb > shm ? shm_rb : shm;
  }
  with_kind(t.kind, [&](auto k) {
    constexpr int KIND = decltype(k)::value;
    if (prec == TS_PAIR_F32) launch_step_kt<KIND, float>(tl, mode, a, t, g, shm, st);
    else launch_step_kt<KIND, double>(tl, mode, a, t, g, shm, st);
  });
  TS_LAUNCH_CHECK();
  return TS_OK;
}

// After a loop with the deferred rebuild: the rows, row lengths and reference positions of every
// system whose current rows are in the second buffer (sel[s] = 1) are copied back to the list's
// own buffer, where every other entry point reads them (one workgroup per system).
__global__ void __launch_bounds__(256) k_rows_restore(StepArgs a, const int32_t *__restrict__ sel, int n_blocks) {
  const int s = blockIdx.x;
  if (sel[s] == 0) return;
  const int64_t a0 = a.offs[s], ns = a.offs[s + 1] - a0, st = a.st_vel;
  const int64_t n_rows = ns * n_blocks * kRowBlock;
  for (int64_t t = threadIdx.x; t < n_rows; t += blockDim.x) {
    const int64_t w = t % kRowBlock, r = t / kRowBlock;
    const int64_t idx = ((r / ns) * st + a0 + r % ns) * kRowBlock + w;
    a.nbr[idx] = a.nbr_alt[idx];
  }
  for (int64_t k = threadIdx.x; k < ns; k += blockDim.x) {
    const int64_t i = a0 + k;
    a.n_nbr[i] = a.n_nbr_alt[i];
    a.ref_pos[i] = a.ref_pos_alt[i];
    a.ref_pos[st + i] = a.ref_pos_alt[st + i];
    a.ref_pos[2 * st + i] = a.ref_pos_alt[2 * st + i];
  }
}

int launch_rows_restore(const StepArgs &a, const int32_t *sel, int64_t n_sys, hipStream_t st) {
  if (n_sys <= 0) return TS_OK;
  hipLaunchKernelGGL(k_rows_restore, dim3((unsigned)n_sys), dim3(256), 0, st, a, sel,
                     (int)ceil_div(a.max_nbr, kRowBlock));
  TS_LAUNCH_CHECK();
  return TS_OK;
}

}  // namespace ts
