// n-tuplet search (paper section 3.2: root doublets, depth-first search over
// the cell graph, maximal paths only) and duplicate removal (section 3.3:
// among tracks sharing a hit doublet only those with the most hits stay).
//
// No output position comes from a shared counter (same-address atomics
// serialise on the device):
//  - roots: each block counts the roots of a chunk of cells and keeps their
//    flags as a bit mask, a scan places the chunks, and one wavefront per
//    chunk writes its roots in cell order from the mask;
//  - search: one thread per root walks the graph with an explicit stack of
//    at most max_hits - 1 cells, first counting the paths it emits, then,
//    after a scan over the roots, writing them at their final rows.  Rows
//    therefore come out in root order and, per root, in search order.
// Duplicate removal is order independent: every row raises the per-cell
// maximum of its length with atomicMax, then a row is kept when it attains
// the maximum on every one of its cells.
#include "pt_internal.h"

#include <algorithm>

namespace pt {
namespace {

constexpr int kBlock = 256;

struct TupIn {
  const int32_t* cell_inner;
  const int32_t* cell_outer;
  const uint8_t* cell_pair;
  const int32_t* cell_count;
  int32_t cells_cap;
  const int32_t* out_start;
  const int32_t* out_count;
  const int32_t* out_cell;
  const uint8_t* has_inner;
  int32_t links_cap;
  const int32_t* link_total;  // links found (the end of the last cell's run)
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

constexpr int kRootItems = 16;                   // cells per thread of the root kernels
constexpr int kRootChunk = kBlock * kRootItems;  // cells per block

// Block-wide exclusive prefix of v; *total receives the block sum.
__device__ inline int block_exclusive(int v, int32_t* s_scan, int* total) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  int incl = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  if (lane == kWave - 1) s_scan[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      const int x = s_scan[w];
      s_scan[w] = run;
      run += x;
    }
    s_scan[kBlock / kWave] = run;
  }
  __syncthreads();
  const int ex = s_scan[wave] + incl - v;
  *total = s_scan[kBlock / kWave];
  __syncthreads();
  return ex;
}

// A cell with outer links (a root without any makes a 2-hit path) whose
// inner hit lies on a root layer, or on a layer whose cells are roots when
// no link ends on them; the inner hit's layer is the inner layer of the
// cell's pair.
__device__ inline bool is_root(const DevCfg& k, int out_count, int pair, bool free_) {
  const int L = k.pair_inner[pair];
  return out_count > 0 && (((k.root_always_mask >> L) & 1u) || (((k.root_if_free_mask >> L) & 1u) && free_));
}

// Root flags of the kRootItems cells of this thread in a chunk (cell
// base + i * kBlock + thread), with every load of the chunk issued up front.
__device__ inline void root_flags(const DevCfg& k, const TupIn& a, int64_t base, int n, bool (&f)[kRootItems]) {
  int oc[kRootItems];
  uint8_t pr[kRootItems], free_[kRootItems];
#pragma unroll
  for (int i = 0; i < kRootItems; ++i) {
    const int64_t c = base + i * kBlock + threadIdx.x;
    const int cc = c < n ? static_cast<int>(c) : 0;
    oc[i] = c < n ? a.out_count[cc] : 0;
    pr[i] = a.cell_pair[cc];
    free_[i] = !a.has_inner[cc];
  }
#pragma unroll
  for (int i = 0; i < kRootItems; ++i) f[i] = is_root(k, oc[i], pr[i], free_[i]);
}

// Spreads the low 16 bits of x to bits 0, 4, .., 60.
__device__ inline uint64_t spread4(uint64_t x) {
  x &= 0xFFFFull;
  x = (x | (x << 24)) & 0x000000FF000000FFull;
  x = (x | (x << 12)) & 0x000F000F000F000Full;
  x = (x | (x << 6)) & 0x0303030303030303ull;
  x = (x | (x << 3)) & 0x1111111111111111ull;
  return x;
}

// Counts the roots of a chunk and stores their flags as a bit mask: bit b of
// word w is the flag of cell 64 w + b.
// VEC: out_count, cell_pair and has_inner 16- and 4-byte aligned; the full
// chunks are then read four consecutive cells per thread and load.
constexpr int kRootWords = kRootChunk / kWave;  // mask words per chunk
template <bool VEC>
__global__ void __launch_bounds__(kBlock) k_root_count(DevCfg k, TupIn a, int32_t* __restrict__ chunk_roots,
                                                       uint64_t* __restrict__ bits) {
  constexpr int kWaves = kBlock / kWave;
  static_assert(kRootItems * kWaves == kRootWords, "one mask word per (item, wavefront) group");
  __shared__ uint64_t s_bits[kRootWords];
  __shared__ int32_t s_cnt[kWaves];
  const int n = min(*a.cell_count, a.cells_cap);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kRootChunk;
  if (base >= n) {
    if (threadIdx.x == 0) chunk_roots[blockIdx.x] = 0;
    return;
  }
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  int cnt = 0;
  if (VEC && base + kRootChunk <= n) {
    // group g: cells base + g 4 kBlock + 4 thread + q, q = 0..3
    constexpr int kGroups = kRootItems / 4;
    int4 oc[kGroups];
    uint32_t pr[kGroups], hin[kGroups];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
      const int64_t c0 = base + g * 4 * kBlock + 4 * threadIdx.x;
      oc[g] = *reinterpret_cast<const int4*>(a.out_count + c0);
      pr[g] = *reinterpret_cast<const uint32_t*>(a.cell_pair + c0);
      hin[g] = *reinterpret_cast<const uint32_t*>(a.has_inner + c0);
    }
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
      const int o[4] = {oc[g].x, oc[g].y, oc[g].z, oc[g].w};
      uint64_t m[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        m[q] = __ballot(is_root(k, o[q], (pr[g] >> (8 * q)) & 0xFF, ((hin[g] >> (8 * q)) & 0xFF) == 0));
        cnt += __popcll(m[q]);
      }
      // the wavefront's 256 cells make mask words g 16 + 4 wave + w, word w
      // from lanes 16 w .. 16 w + 15 (four cells each)
      if (lane < 4) {
        uint64_t word = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) word |= spread4(m[q] >> (16 * lane)) << q;
        s_bits[g * 4 * kWaves + 4 * wave + lane] = word;
      }
    }
  } else {
    bool f[kRootItems];
    root_flags(k, a, base, n, f);
#pragma unroll
    for (int i = 0; i < kRootItems; ++i) {
      // item i of this wavefront covers cells base + 64 (i kWaves + wave) + lane
      const uint64_t m = __ballot(f[i]);
      cnt += __popcll(m);
      if (lane == 0) s_bits[i * kWaves + wave] = m;
    }
  }
  if (lane == 0) s_cnt[wave] = cnt;
  __syncthreads();
  if (threadIdx.x < kRootWords) bits[blockIdx.x * static_cast<int64_t>(kRootWords) + threadIdx.x] = s_bits[threadIdx.x];
  if (threadIdx.x == 0) {
    int total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) total += s_cnt[w];
    chunk_roots[blockIdx.x] = total;
  }
}

// Writes the indices whose mask bit is set, in order, one wavefront per
// chunk of kRootChunk indices below min(*n_dev, n_cap): lane l holds word l;
// an index's position is the chunk's offset, plus the set bits of the words
// before its own, plus its rank in its word.  Used for the roots (cells) and
// for the roots that emit rows.
__global__ void __launch_bounds__(kWave) k_mask_write(const int32_t* __restrict__ n_dev, int32_t n_cap,
                                                     const uint64_t* __restrict__ bits,
                                                     const int32_t* __restrict__ chunk_first, int32_t* __restrict__ out) {
  static_assert(kRootWords == kWave, "one mask word per lane");
  const int n = min(*n_dev, n_cap);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kRootChunk;
  if (base >= n) return;
  const int lane = threadIdx.x;
  const uint64_t word = bits[blockIdx.x * static_cast<int64_t>(kRootWords) + lane];
  const int c = __popcll(word);
  int incl = c;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  const int first = chunk_first[blockIdx.x] + incl - c;  // this word's first root
  uint64_t nz = __ballot(word != 0);
  while (nz) {
    const int w = __builtin_ctzll(nz);
    nz &= nz - 1;
    const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(word), w);
    const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(word >> 32), w);
    const uint64_t m = (static_cast<uint64_t>(hi) << 32) | lo;
    const int at = __builtin_amdgcn_readlane(first, w);
    if ((m >> lane) & 1u) out[at + lane_prefix(m)] = static_cast<int>(base + w * kWave + lane);
  }
}

// The roots that emit a row, from the rows each root emits (paths[i], the
// count pass's output): each block scans its chunk of kRootChunk counts
// (16 consecutive ones per thread; the chunk's offset comes from the scan of
// the chunk sums) into first rows, writes the first row of every root that
// emits one below the capacity over its count (the only first rows the
// write pass reads), flags those roots in a bit mask (word w: roots
// base + 64 w .. + 63) and counts them per chunk.  Block 0 writes the total
// number of rows after the last root.
__global__ void __launch_bounds__(kBlock) k_prod_count(TupIn a, int32_t* __restrict__ paths,
                                                       const int32_t* __restrict__ chunk_off,
                                                       int32_t* __restrict__ chunk_count, uint64_t* __restrict__ bits) {
  static_assert(kRootItems == 16 && kBlock / 4 == kRootWords, "four threads' 16-bit masks per mask word");
  __shared__ int32_t s_scan[kBlock / kWave + 1];
  __shared__ uint16_t s_m16[kBlock];
  const int nr = min(*a.n_roots, a.cells_cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) paths[nr] = chunk_off[gridDim.x];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kRootChunk;
  if (base >= nr) {
    if (threadIdx.x == 0) chunk_count[blockIdx.x] = 0;
    return;
  }
  const int64_t at = base + static_cast<int64_t>(threadIdx.x) * kRootItems;
  int c[kRootItems];
  if (base + kRootChunk <= nr && reinterpret_cast<uintptr_t>(paths) % 16 == 0) {
    const int4* p = reinterpret_cast<const int4*>(paths + at);
#pragma unroll
    for (int i = 0; i < kRootItems / 4; ++i) {
      const int4 q = p[i];
      c[4 * i] = q.x;
      c[4 * i + 1] = q.y;
      c[4 * i + 2] = q.z;
      c[4 * i + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kRootItems; ++i) c[i] = at + i < nr ? paths[at + i] : 0;
  }
  int sum = 0;
#pragma unroll
  for (int i = 0; i < kRootItems; ++i) sum += c[i];
  int tot;
  int run = chunk_off[blockIdx.x] + block_exclusive(sum, s_scan, &tot);  // every count is read by now
  uint32_t m16 = 0;
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < kRootItems; ++i) {
    if (c[i] > 0 && run < a.cap) {
      m16 |= 1u << i;
      paths[at + i] = run;
      ++cnt;
    }
    run += c[i];
  }
  s_m16[threadIdx.x] = static_cast<uint16_t>(m16);
  int n_prod;
  block_exclusive(cnt, s_scan, &n_prod);  // its barriers also order the mask writes
  if (threadIdx.x < kRootWords) {
    const int q = 4 * threadIdx.x;
    bits[blockIdx.x * static_cast<int64_t>(kRootWords) + threadIdx.x] =
        static_cast<uint64_t>(s_m16[q]) | (static_cast<uint64_t>(s_m16[q + 1]) << 16) |
        (static_cast<uint64_t>(s_m16[q + 2]) << 32) | (static_cast<uint64_t>(s_m16[q + 3]) << 48);
  }
  if (threadIdx.x == 0) chunk_count[blockIdx.x] = n_prod;
}

// The run of cell c's outer links, [*first, *end): the links are placed in
// cell order, so the run ends where the next cell's starts (at the total
// after the last cell).  Both loads are issued together, so that a child's
// run comes one dependent load after its index instead of two.
__device__ inline void link_run(const TupIn& a, int c, int n_cells, int total, int* first, int* end) {
  const int f = a.out_start[c];
  const int e = a.out_start[min(c + 1, n_cells - 1)];
  *first = f;
  *end = c + 1 < n_cells ? e : total;
}

// Depth-first search from each root.  COUNT: paths[i] = rows root i emits
// (and the truncation count); otherwise the rows are written from row
// first_row[i] on.
template <bool COUNT>
__global__ void k_dfs(DevCfg k, TupIn a, int32_t* __restrict__ paths, const int32_t* __restrict__ prod,
                      const int32_t* __restrict__ n_prod) {
  // the write pass takes only the roots that emit a row below the capacity
  // (most roots emit none: their paths are too short)
  const int nr = COUNT ? *a.n_roots : *n_prod;
  const int n_cells = min(*a.cell_count, a.cells_cap);
  const int links_found = *a.link_total;
  uint32_t truncated = 0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nr; t += gridDim.x * blockDim.x) {
    int stack[kMaxHits];   // cells of the current path
    int next[kMaxHits];    // next outer link to follow at each depth (absolute link index) ...
    int end[kMaxHits];     // ... and the end of that cell's links
    const int i = COUNT ? t : prod[t];
    const int root = a.roots[i];
    stack[0] = root;
    link_run(a, root, n_cells, links_found, &next[0], &end[0]);
    int depth = 0;
    int row = COUNT ? 0 : paths[i];
    while (depth >= 0) {
      if (next[depth] >= end[depth]) {
        --depth;
        continue;
      }
      const int li = next[depth]++;
      if (li >= a.links_cap) continue;
      const int child = a.out_cell[li];
      const int nh = depth + 3;  // hits of the path root..child
      int cf, ce;
      link_run(a, child, n_cells, links_found, &cf, &ce);
      const int coc = ce - cf;
      if (coc == 0 || nh == k.max_hits) {
        if (COUNT && coc > 0) ++truncated;
        if (nh >= k.min_hits) {
          if (!COUNT && row < a.cap) {  // the cells of the path (its hits: k_row_hits)
            int32_t* C = a.cells + static_cast<int64_t>(row) * (kMaxHits - 1);
            for (int d = 0; d <= depth; ++d) C[d] = stack[d];
            C[depth + 1] = child;
            for (int d = depth + 2; d < kMaxHits - 1; ++d) C[d] = -1;
            a.n[row] = static_cast<uint8_t>(nh);
          }
          ++row;
        }
      } else {
        ++depth;
        stack[depth] = child;
        next[depth] = cf;
        end[depth] = ce;
      }
    }
    if (COUNT) paths[i] = row;
  }
  if (COUNT) {
    const uint32_t total = wave_status_add(a.status, PT_ST_TRUNCATED, truncated);
    if (total && __lane_id() == 0) status_flag(a.status, PT_FLAG_TRUNCATED);
  }
}

// The hits of every row from its cells (inner hit of the first cell, then
// the outer hit of each), one thread per row: the search itself stores only
// the cells it holds in registers.
__global__ void k_row_hits(TupIn a) {
  const int rows = min(*a.count_raw, a.cap);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < rows; t += gridDim.x * blockDim.x) {
    const int nh = a.n[t];
    const int32_t* C = a.cells + static_cast<int64_t>(t) * (kMaxHits - 1);
    int h[kMaxHits];
    h[0] = a.cell_inner[C[0]];
#pragma unroll
    for (int d = 0; d < kMaxHits - 1; ++d) h[d + 1] = d < nh - 1 ? a.cell_outer[C[d]] : -1;
    int32_t* H = a.hits + static_cast<int64_t>(t) * kMaxHits;
#pragma unroll
    for (int d = 0; d < kMaxHits; ++d) H[d] = h[d];
  }
}

__global__ void k_copy_total_rows(const int32_t* __restrict__ paths, const int32_t* __restrict__ n_roots,
                                  int32_t* __restrict__ count_raw) {
  *count_raw = paths[*n_roots];
}

// Clears the per-cell maximum of the cells the rows visit (the only ones
// read afterwards), instead of all cells.
__global__ void k_clear_maxn(TupIn a) {
  const int rows = min(*a.count_raw, a.cap);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < rows; t += gridDim.x * blockDim.x) {
    const int nh = a.n[t];
    const int32_t* C = a.cells + static_cast<int64_t>(t) * (kMaxHits - 1);
    for (int d = 0; d < nh - 1; ++d) a.max_n[C[d]] = 0;
  }
}

__global__ void k_maxn(TupIn a) {
  const int rows = min(*a.count_raw, a.cap);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < rows; t += gridDim.x * blockDim.x) {
    const int nh = a.n[t];
    const int32_t* C = a.cells + static_cast<int64_t>(t) * (kMaxHits - 1);
    for (int d = 0; d < nh - 1; ++d) atomicMax(a.max_n + C[d], nh);
  }
}

__device__ inline bool keep_row(const TupIn& a, int t) {
  const int nh = a.n[t];
  const int32_t* C = a.cells + static_cast<int64_t>(t) * (kMaxHits - 1);
  for (int d = 0; d < nh - 1; ++d)
    if (a.max_n[C[d]] != nh) return false;
  return true;
}

// Keep flags of the kRootItems rows of this thread in a chunk (row
// base + i * kBlock + thread), with every load issued before the tests.
__device__ inline void keep_flags(const TupIn& a, int64_t base, int rows, bool (&f)[kRootItems]) {
#pragma unroll
  for (int i = 0; i < kRootItems; ++i) {
    const int64_t t = base + i * kBlock + threadIdx.x;
    f[i] = t < rows && keep_row(a, static_cast<int>(t));
  }
}

__global__ void __launch_bounds__(kBlock) k_keep_count(TupIn a, int32_t* __restrict__ chunk_kept) {
  __shared__ int32_t s_scan[kBlock / kWave + 1];
  const int rows = min(*a.count_raw, a.cap);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kRootChunk;
  if (base >= rows) {
    if (threadIdx.x == 0) chunk_kept[blockIdx.x] = 0;
    return;
  }
  bool f[kRootItems];
  keep_flags(a, base, rows, f);
  int cnt = 0;
#pragma unroll
  for (int i = 0; i < kRootItems; ++i) cnt += f[i] ? 1 : 0;
  int total;
  block_exclusive(cnt, s_scan, &total);
  if (threadIdx.x == 0) chunk_kept[blockIdx.x] = total;
}

// Writes the chunk's kept rows in row order: a row's position is the
// chunk's offset, plus the kept rows of the (item, wavefront) groups before
// its own (one wavefront scan of the group counts), plus its rank in its
// wavefront's ballot.
__global__ void __launch_bounds__(kBlock) k_keep_write(TupIn a, const int32_t* __restrict__ chunk_first) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ int32_t s_grp[kRootItems * kWaves];
  const int rows = min(*a.count_raw, a.cap);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kRootChunk;
  if (base >= rows) return;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int at = chunk_first[blockIdx.x];
  bool f[kRootItems];
  keep_flags(a, base, rows, f);
  int rank[kRootItems];
#pragma unroll
  for (int i = 0; i < kRootItems; ++i) {
    const uint64_t m = __ballot(f[i]);
    rank[i] = lane_prefix(m);
    if (lane == 0) s_grp[i * kWaves + wave] = __popcll(m);
  }
  __syncthreads();
  if (wave == 0) {
    const int v = s_grp[lane];
    int incl = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    s_grp[lane] = incl - v;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kRootItems; ++i)
    if (f[i]) a.kept[at + s_grp[i * kWaves + wave] + rank[i]] = static_cast<int>(base + i * kBlock + threadIdx.x);
}

__global__ void k_copy_total(const int32_t* __restrict__ src, int32_t* __restrict__ dst) { *dst = *src; }

__global__ void k_finish_tuplets(const int32_t* count_raw, int32_t cap, uint32_t* status) {
  if (*count_raw > cap) status_flag(status, PT_FLAG_TUPLETS_OVERFLOW);
}

}  // namespace

size_t ws_ntuplets(int cells_cap, int tuplets_cap) {
  const int64_t chunks = std::max<int64_t>(
      1, std::max<int64_t>((static_cast<int64_t>(cells_cap) + kRootChunk - 1) / kRootChunk,
                           (static_cast<int64_t>(tuplets_cap) + kRootChunk - 1) / kRootChunk));
  const int64_t cells_chunks = std::max<int64_t>(1, (static_cast<int64_t>(cells_cap) + kRootChunk - 1) / kRootChunk);
  const int64_t scan_n = std::max<int64_t>(chunks, cells_cap);
  Carver c(nullptr);
  c.take<int32_t>(cells_cap);      // roots
  c.take<uint64_t>(chunks * kRootWords);  // root flags, one bit per cell (then per root)
  c.take<int32_t>(chunks + 1);     // roots (then kept rows) per chunk -> chunk offsets (+ total)
  c.take<int32_t>(cells_cap);      // roots that emit rows
  c.take<int32_t>(cells_chunks + 1);  // ... per chunk -> chunk offsets (+ total)
  c.take<int32_t>(static_cast<size_t>(cells_cap) + 1);  // paths per root -> first row (+ total)
  c.take<int32_t>(cells_cap);      // max_n
  c.take<int32_t>(scan_tmp_elems(scan_n));
  return c.off + 256;
}

pt_err launch_ntuplets(const pt_hits& h, const DevCfg& k, const pt_cells& cells, const pt_links& L,
                       pt_ntuplets& T, uint32_t* status, pt_workspace ws, hipStream_t s) {
  const int64_t chunks = std::max<int64_t>(1, (static_cast<int64_t>(cells.cap) + kRootChunk - 1) / kRootChunk);
  const int64_t chunks_max = std::max<int64_t>(chunks, (static_cast<int64_t>(T.cap) + kRootChunk - 1) / kRootChunk);
  const int64_t scan_n = std::max<int64_t>(chunks_max, cells.cap);
  Carver c(ws.ptr);
  int32_t* roots = c.take<int32_t>(cells.cap);
  uint64_t* root_bits = c.take<uint64_t>(chunks_max * kRootWords);
  int32_t* chunk_roots = c.take<int32_t>(chunks_max + 1);
  int32_t* prod = c.take<int32_t>(cells.cap);
  int32_t* chunk_prod = c.take<int32_t>(chunks + 1);
  int32_t* paths = c.take<int32_t>(static_cast<size_t>(cells.cap) + 1);
  int32_t* max_n = c.take<int32_t>(cells.cap);
  int32_t* tmp = c.take<int32_t>(scan_tmp_elems(scan_n));
  int32_t* n_roots = chunk_roots + chunks;  // the scan's total
  TupIn a{cells.inner, cells.outer, cells.pair, cells.count, cells.cap, L.out_start, L.out_count, L.out_cell,
          L.has_inner, L.cap, L.count, roots, n_roots, T.cap, T.hits, T.cells, T.n, T.count_raw, T.kept, T.count,
          max_n, status};
  void* tok = timing_begin(s);
  const bool vec = reinterpret_cast<uintptr_t>(L.out_count) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(cells.pair) % 4 == 0 && reinterpret_cast<uintptr_t>(L.has_inner) % 4 == 0;
  if (vec)
    k_root_count<true><<<static_cast<unsigned>(chunks), kBlock, 0, s>>>(k, a, chunk_roots, root_bits);
  else
    k_root_count<false><<<static_cast<unsigned>(chunks), kBlock, 0, s>>>(k, a, chunk_roots, root_bits);
  timing_end(tok, "root_count", s);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(chunk_roots, chunks, tmp, s));
  tok = timing_begin(s);
  k_mask_write<<<static_cast<unsigned>(chunks), kWave, 0, s>>>(cells.count, cells.cap, root_bits, chunk_roots, roots);
  timing_end(tok, "root_write", s);
  PT_LAUNCH_CHECK();
  tok = timing_begin(s);
  k_dfs<true><<<grid_for(cells.cap, 256, 65536), 256, 0, s>>>(k, a, paths, nullptr, nullptr);
  timing_end(tok, "dfs_count", s);
  PT_LAUNCH_CHECK();
  // first rows: the chunk sums of the counts are scanned, then each chunk
  // scans itself (and writes the total rows after the last root)
  static_assert(kRootChunk == kScanTile, "the chunks are the scan's tiles");
  const int32_t* row_off = nullptr;
  PT_HIP_CHECK(scan_tile_offsets(paths, cells.cap, n_roots, tmp, s, &row_off));
  tok = timing_begin(s);
  k_prod_count<<<static_cast<unsigned>(chunks), kBlock, 0, s>>>(a, paths, row_off, chunk_prod, root_bits);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(chunk_prod, chunks, tmp, s));
  k_mask_write<<<static_cast<unsigned>(chunks), kWave, 0, s>>>(n_roots, cells.cap, root_bits, chunk_prod, prod);
  PT_LAUNCH_CHECK();
  k_dfs<false><<<grid_for(cells.cap, 128, 16384), 128, 0, s>>>(k, a, paths, prod, chunk_prod + chunks);
  timing_end(tok, "dfs_write", s);
  PT_LAUNCH_CHECK();
  // rows found = paths[n_roots] (written by k_prod_count)
  k_copy_total_rows<<<1, 1, 0, s>>>(paths, n_roots, T.count_raw);
  PT_LAUNCH_CHECK();
  k_row_hits<<<grid_for(T.cap, 256, 8192), 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  tok = timing_begin(s);
  k_clear_maxn<<<grid_for(T.cap, 256, 8192), 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  k_maxn<<<grid_for(T.cap, 256, 8192), 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  const int64_t row_chunks = std::max<int64_t>(1, (static_cast<int64_t>(T.cap) + kRootChunk - 1) / kRootChunk);
  k_keep_count<<<static_cast<unsigned>(row_chunks), kBlock, 0, s>>>(a, chunk_roots);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(chunk_roots, row_chunks, tmp, s));
  k_keep_write<<<static_cast<unsigned>(row_chunks), kBlock, 0, s>>>(a, chunk_roots);
  PT_LAUNCH_CHECK();
  k_copy_total<<<1, 1, 0, s>>>(chunk_roots + row_chunks, T.count);
  PT_LAUNCH_CHECK();
  timing_end(tok, "dedup", s);
  k_finish_tuplets<<<1, 1, 0, s>>>(T.count_raw, T.cap, status);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
