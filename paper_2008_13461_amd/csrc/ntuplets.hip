// n-tuplet search (paper section 3.2: root doublets, depth-first search over
// the cell graph, maximal paths only) and duplicate removal (section 3.3:
// among tracks sharing a hit doublet only those with the most hits stay).
//
// Roots are collected first (cells without outer links are skipped: their
// path has two hits, below any useful minimum).  One thread per root walks
// the graph with an explicit stack of at most max_hits - 1 cells.  Duplicate
// removal is order independent: every row raises the per-cell maximum of its
// length with atomicMax, then a row is kept when it attains the maximum on
// every one of its cells.
#include "pt_internal.h"

namespace pt {
namespace {

constexpr int kBlock = 256;

struct TupIn {
  const uint8_t* layer;
  const int32_t* cell_inner;
  const int32_t* cell_outer;
  const int32_t* cell_count;
  int32_t cells_cap;
  const int32_t* out_start;
  const int32_t* out_count;
  const int32_t* out_cell;
  const uint8_t* has_inner;
  int32_t links_cap;
  int32_t* roots;
  int32_t* n_roots;
  int32_t cap;
  int32_t* hits;
  int32_t* cells;
  uint8_t* n;
  int32_t* count_raw;
  int32_t* kept;
  int32_t* count;
  int32_t* max_n;
  uint32_t* status;
};

// Append `take` items per thread to a global list with one atomic per block.
__device__ inline int block_reserve(int take, int32_t* counter, int32_t* s_scan, int32_t* s_base) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  int v = take;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  if (lane == kWave - 1) s_scan[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      const int x = s_scan[w];
      s_scan[w] = run;
      run += x;
    }
    *s_base = run ? atomicAdd(counter, run) : 0;
  }
  __syncthreads();
  const int pos = *s_base + s_scan[wave] + v - take;
  __syncthreads();
  return pos;
}

__global__ void __launch_bounds__(kBlock) k_roots(DevCfg k, TupIn a) {
  __shared__ int32_t s_scan[kBlock / kWave + 1];
  __shared__ int32_t s_base;
  const int n = min(*a.cell_count, a.cells_cap);
  const int stride = gridDim.x * kBlock;
  const int rounds = (n + stride - 1) / stride;
  for (int r = 0; r < rounds; ++r) {
    const int c = r * stride + blockIdx.x * kBlock + threadIdx.x;
    bool root = false;
    if (c < n && a.out_count[c] > 0) {
      const int L = a.layer[a.cell_inner[c]];
      root = ((k.root_always_mask >> L) & 1u) || (((k.root_if_free_mask >> L) & 1u) && !a.has_inner[c]);
    }
    const int pos = block_reserve(root ? 1 : 0, a.n_roots, s_scan, &s_base);
    if (root) a.roots[pos] = c;
  }
}

__global__ void k_dfs(DevCfg k, TupIn a) {
  const int nr = *a.n_roots;
  uint32_t truncated = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += gridDim.x * blockDim.x) {
    int stack[kMaxHits];   // cells of the current path
    int next[kMaxHits];    // next outer link to follow at each depth
    stack[0] = a.roots[i];
    next[0] = 0;
    int depth = 0;
    while (depth >= 0) {
      const int c = stack[depth];
      const int oc = a.out_count[c];
      if (next[depth] >= oc) {
        --depth;
        continue;
      }
      const int li = a.out_start[c] + next[depth];
      ++next[depth];
      if (li >= a.links_cap) continue;
      const int child = a.out_cell[li];
      const int nh = depth + 3;  // hits of the path root..child
      const int coc = a.out_count[child];
      if (coc == 0 || nh == k.max_hits) {
        if (coc > 0) ++truncated;
        if (nh >= k.min_hits) {
          const int row = atomicAdd(a.count_raw, 1);
          if (row < a.cap) {
            int32_t* H = a.hits + static_cast<int64_t>(row) * kMaxHits;
            int32_t* C = a.cells + static_cast<int64_t>(row) * (kMaxHits - 1);
            H[0] = a.cell_inner[stack[0]];
            for (int d = 0; d <= depth; ++d) {
              H[d + 1] = a.cell_outer[stack[d]];
              C[d] = stack[d];
            }
            H[depth + 2] = a.cell_outer[child];
            C[depth + 1] = child;
            for (int d = depth + 3; d < kMaxHits; ++d) H[d] = -1;
            for (int d = depth + 2; d < kMaxHits - 1; ++d) C[d] = -1;
            a.n[row] = static_cast<uint8_t>(nh);
          }
        }
      } else {
        ++depth;
        stack[depth] = child;
        next[depth] = 0;
      }
    }
  }
  if (truncated) {
    status_add(a.status, PT_ST_TRUNCATED, truncated);
    status_flag(a.status, PT_FLAG_TRUNCATED);
  }
}

__global__ void k_clear_maxn(TupIn a) {
  const int n = min(*a.cell_count, a.cells_cap);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) a.max_n[c] = 0;
}

__global__ void k_maxn(TupIn a) {
  const int rows = min(*a.count_raw, a.cap);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < rows; t += gridDim.x * blockDim.x) {
    const int nh = a.n[t];
    const int32_t* C = a.cells + static_cast<int64_t>(t) * (kMaxHits - 1);
    for (int d = 0; d < nh - 1; ++d) atomicMax(a.max_n + C[d], nh);
  }
}

__global__ void __launch_bounds__(kBlock) k_keep(TupIn a) {
  __shared__ int32_t s_scan[kBlock / kWave + 1];
  __shared__ int32_t s_base;
  const int rows = min(*a.count_raw, a.cap);
  const int stride = gridDim.x * kBlock;
  const int rounds = (rows + stride - 1) / stride;
  for (int r = 0; r < rounds; ++r) {
    const int t = r * stride + blockIdx.x * kBlock + threadIdx.x;
    bool keep = false;
    if (t < rows) {
      keep = true;
      const int nh = a.n[t];
      const int32_t* C = a.cells + static_cast<int64_t>(t) * (kMaxHits - 1);
      for (int d = 0; d < nh - 1; ++d)
        if (a.max_n[C[d]] != nh) keep = false;
    }
    const int pos = block_reserve(keep ? 1 : 0, a.count, s_scan, &s_base);
    if (keep) a.kept[pos] = t;
  }
}

__global__ void k_finish_tuplets(const int32_t* count_raw, int32_t cap, uint32_t* status) {
  if (*count_raw > cap) status_flag(status, PT_FLAG_TUPLETS_OVERFLOW);
}

}  // namespace

size_t ws_ntuplets(int cells_cap, int tuplets_cap) {
  (void)tuplets_cap;
  Carver c(nullptr);
  c.take<int32_t>(cells_cap);  // roots
  c.take<int32_t>(1);          // n_roots
  c.take<int32_t>(cells_cap);  // max_n
  return c.off + 256;
}

pt_err launch_ntuplets(const pt_hits& h, const DevCfg& k, const pt_cells& cells, const pt_links& L,
                       pt_ntuplets& T, uint32_t* status, pt_workspace ws, hipStream_t s) {
  Carver c(ws.ptr);
  int32_t* roots = c.take<int32_t>(cells.cap);
  int32_t* n_roots = c.take<int32_t>(1);
  int32_t* max_n = c.take<int32_t>(cells.cap);
  TupIn a{h.layer, cells.inner, cells.outer, cells.count, cells.cap, L.out_start, L.out_count, L.out_cell,
          L.has_inner, L.cap, roots, n_roots, T.cap, T.hits, T.cells, T.n, T.count_raw, T.kept, T.count,
          max_n, status};
  if (fill_i32(n_roots, 0, 1, s) != hipSuccess) return PT_ERR_DEVICE;
  if (fill_i32(T.count_raw, 0, 1, s) != hipSuccess) return PT_ERR_DEVICE;
  if (fill_i32(T.count, 0, 1, s) != hipSuccess) return PT_ERR_DEVICE;
  k_roots<<<grid_for(cells.cap, kBlock, 16384), kBlock, 0, s>>>(k, a);
  PT_LAUNCH_CHECK();
  void* tok = timing_begin(s);
  k_dfs<<<grid_for(cells.cap, 128, 8192), 128, 0, s>>>(k, a);
  timing_end(tok, "dfs", s);
  PT_LAUNCH_CHECK();
  k_clear_maxn<<<grid_for(cells.cap, 256, 8192), 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  k_maxn<<<grid_for(T.cap, 256, 8192), 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  k_keep<<<grid_for(T.cap, kBlock, 8192), kBlock, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  k_finish_tuplets<<<1, 1, 0, s>>>(T.count_raw, T.cap, status);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
