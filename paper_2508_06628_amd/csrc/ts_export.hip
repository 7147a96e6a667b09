// The neighbor list exported as the batch graph of a learned potential: every periodic pair
// within r_graph as an edge (i, j) with its integer image S and vector d = r_j - r_i + S cell, in
// (system, i, j, S) order, with a CSR row pointer over atoms and edge offsets per system.  The
// paper attributes most of the speed differences between learned potentials to this graph
// construction (Section 4).
//
// Four launches: per-atom edge counts (eight lanes per atom row), a scan of the counts inside each
// system (one workgroup per system), a scan of the system totals (one workgroup), and the edge
// writes (one wavefront per atom row, consecutive lanes writing consecutive edges; the row order
// is already the (j, S) order).
#include "ts_internal.h"

namespace ts {

constexpr int kExportThreads = 256;

struct ExportArgs {
  int64_t n, st;
  const int32_t *sys_idx;
  const int64_t *offs;
  const double *pos, *cell;
  const uint32_t *nbr;
  const int32_t *n_nbr;
  double r2;
  int64_t *row_ptr, *edge_offsets, *edge_index;
  int32_t *edge_shift;
  double *edge_vec;
  int64_t capacity;
  int n_sys;
};

// d = r_j - r_i + S cell (rows of cell are the lattice vectors)
__device__ inline void edge_vector(const ExportArgs &a, int64_t i, int64_t j, uint32_t e, const double *h,
                                   double d[3]) {
  const double s0 = entry_s0d(e), s1 = entry_s1d(e), s2 = entry_s2d(e);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    d[c] = fma(s2, h[6 + c], fma(s1, h[3 + c], fma(s0, h[c], a.pos[c * a.st + j] - a.pos[c * a.st + i])));
}

// Edge counts: kRowBlock lanes per atom, one row block (kRowBlock contiguous entries) per step, so
// that a wavefront load covers the same block of eight consecutive atoms: 256 contiguous bytes.
__global__ void __launch_bounds__(kExportThreads) k_edge_count(ExportArgs a) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = t / kRowBlock;
  const int sub = (int)(t % kRowBlock);
  const bool own = i < a.n;
  int c = 0;
  if (own) {
    const int s = a.sys_idx[i];
    const int64_t a0 = a.offs[s];
    const double *h = a.cell + 9 * (int64_t)s;
    const int nn = a.n_nbr[i];
    for (int k = sub; k < nn; k += kRowBlock) {
      const uint32_t e = a.nbr[row_index(k, i, a.st)];
      double d[3];
      edge_vector(a, i, a0 + entry_j(e), e, h, d);
      c += (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < a.r2;
    }
  }
#pragma unroll
  for (int o = 1; o < kRowBlock; o <<= 1) c += __shfl_xor(c, o, kRowBlock);
  if (own && sub == 0) a.row_ptr[i] = c;
}

// Exclusive scan of v over the workgroup; *total receives the sum.
__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t *total) {
  __shared__ int64_t wsum[kExportThreads / kWave];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int64_t y = __shfl_up(x, o, kWave);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[wv] = x;
  __syncthreads();
  int64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kExportThreads / kWave; ++w) {
    before += w < wv ? wsum[w] : 0;
    all += wsum[w];
  }
  __syncthreads();  // wsum is reused by the next call
  *total = all;
  return before + x - v;
}

// row_ptr[i] (count) -> offset of atom i's first edge within its system; edge_offsets[s + 1] = the
// system's edge count
__global__ void __launch_bounds__(kExportThreads) k_edge_scan_system(ExportArgs a) {
  const int s = blockIdx.x;
  const int64_t a0 = a.offs[s], a1 = a.offs[s + 1];
  int64_t carry = 0;
  for (int64_t b = a0; b < a1; b += kExportThreads) {
    const int64_t i = b + threadIdx.x;
    const int64_t v = i < a1 ? a.row_ptr[i] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, &tot);
    if (i < a1) a.row_ptr[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) a.edge_offsets[s + 1] = carry;
}

// edge_offsets[1..S] (system counts) -> prefix sums, edge_offsets[0] = 0, row_ptr[N] = total
__global__ void __launch_bounds__(kExportThreads) k_edge_scan_total(ExportArgs a) {
  int64_t carry = 0;
  for (int b = 0; b < a.n_sys; b += kExportThreads) {
    const int s = b + (int)threadIdx.x;
    const int64_t v = s < a.n_sys ? a.edge_offsets[s + 1] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, &tot);
    if (s < a.n_sys) a.edge_offsets[s + 1] = carry + ex + v;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    a.edge_offsets[0] = 0;
    a.row_ptr[a.n] = carry;
  }
}

// One wavefront per atom: its 64 lanes test 64 row entries at a time (the row is in (j, S) order,
// so a ballot and a population count give each edge its position).
__device__ inline int64_t wave_atom() { return ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; }

__global__ void __launch_bounds__(kExportThreads) k_edge_write(ExportArgs a) {
  const int64_t i = wave_atom();
  if (i >= a.n) return;  // uniform over the wavefront
  const int lane = threadIdx.x % kWave;
  const uint64_t below = (1ull << lane) - 1ull;
  const int s = a.sys_idx[i];
  const int64_t a0 = a.offs[s];
  const double *h = a.cell + 9 * (int64_t)s;
  int64_t p = a.edge_offsets[s] + a.row_ptr[i];
  if (lane == 0) a.row_ptr[i] = p;
  const int nn = a.n_nbr[i];
  for (int k0 = 0; k0 < nn; k0 += kWave) {
    const int k = k0 + lane;
    bool in = false;
    uint32_t e = 0;
    double d[3] = {0.0, 0.0, 0.0};
    if (k < nn) {
      e = a.nbr[row_index(k, i, a.st)];
      edge_vector(a, i, a0 + entry_j(e), e, h, d);
      in = (d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < a.r2;
    }
    const uint64_t mask = __ballot(in);
    const int64_t q = p + __popcll(mask & below);
    if (in && q < a.capacity) {
      a.edge_index[q] = i;
      a.edge_index[a.capacity + q] = a0 + entry_j(e);
      if (a.edge_shift) {
        a.edge_shift[3 * q] = entry_s0(e);
        a.edge_shift[3 * q + 1] = entry_s1(e);
        a.edge_shift[3 * q + 2] = entry_s2(e);
      }
      if (a.edge_vec) {
        a.edge_vec[3 * q] = d[0];
        a.edge_vec[3 * q + 1] = d[1];
        a.edge_vec[3 * q + 2] = d[2];
      }
    }
    p += __popcll(mask);
  }
}

}  // namespace ts

extern "C" int ts_graph_export(const ts_batch *batch, const ts_neighbor_list *nl, double r_graph, int64_t *row_ptr,
                               int64_t *edge_offsets, int64_t *edge_index, int32_t *edge_shift, double *edge_vec,
                               int64_t capacity, ts_stream_t stream) {
  int rc = ts::validate_batch(batch, false, nullptr);
  if (rc != TS_OK) return rc;
  rc = ts::validate_list(batch, nl);
  if (rc != TS_OK) return rc;
  TS_CHECK_ARG(std::isfinite(r_graph) && r_graph > 0.0 && r_graph <= nl->cutoff + nl->skin);
  TS_CHECK_ARG(row_ptr != nullptr && edge_offsets != nullptr && capacity >= 0);
  TS_CHECK_ARG(capacity == 0 || edge_index != nullptr);
  if (batch->n_systems > 0x7fffffff) return TS_E_CAPACITY;
  ts::ExportArgs a;
  a.n = batch->n_atoms;
  a.st = ts::stride_of(batch);
  a.sys_idx = batch->system_idx;
  a.offs = batch->sys_offsets;
  a.pos = batch->pos;
  a.cell = batch->cell;
  a.nbr = reinterpret_cast<const uint32_t *>(nl->nbr);
  a.n_nbr = nl->n_nbr;
  a.r2 = r_graph * r_graph;
  a.row_ptr = row_ptr;
  a.edge_offsets = edge_offsets;
  a.edge_index = edge_index;
  a.edge_shift = edge_shift;
  a.edge_vec = edge_vec;
  a.capacity = capacity;
  a.n_sys = (int)batch->n_systems;
  hipStream_t st = ts::as_stream(stream);
  const int64_t waves_per_block = ts::kExportThreads / ts::kWave;
  if (ts::ceil_div(a.n, waves_per_block) > 0x7fffffff) return TS_E_CAPACITY;
  const dim3 g((unsigned)ts::ceil_div(a.n > 0 ? a.n : 1, waves_per_block)), b(ts::kExportThreads);
  if (a.n > 0) {
    const dim3 gc((unsigned)ts::ceil_div(a.n * ts::kRowBlock, ts::kExportThreads));
    hipLaunchKernelGGL(ts::k_edge_count, gc, b, 0, st, a);
    TS_LAUNCH_CHECK();
  }
  if (a.n_sys > 0) {
    hipLaunchKernelGGL(ts::k_edge_scan_system, dim3((unsigned)a.n_sys), b, 0, st, a);
    TS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(ts::k_edge_scan_total, dim3(1), b, 0, st, a);
  TS_LAUNCH_CHECK();
  if (a.n > 0) {
    hipLaunchKernelGGL(ts::k_edge_write, g, b, 0, st, a);
    TS_LAUNCH_CHECK();
  }
  return TS_OK;
}
