// Fishbone (paper section 3.3): among the doublets that share their outer
// hit, the longer of two aligned ones is dropped, so that the overlapping
// modules of a layer give one n-tuplet per particle instead of several.
//
// Runs inside pt_build_doublets after the write pass when the Fishbone is on:
//   1. the stored cells are indexed by outer hit (count, scan, fill);
//   2. one wavefront per outer hit tests every cell of the hit (one lane
//      each) against every other cell of the hit (a wave-uniform loop with
//      scalar loads) and clears the cell's keep flag when a shorter aligned
//      one exists;
//   3. the kept cells are compacted in their order (a scan of the flags),
//      through a copy in the workspace, and each inner hit's range of cells
//      is moved with them.
// The test is the one of pixeltrack.h, in double, as parenthesised, without
// contraction, from the hits' coordinates promoted to double.
#include <algorithm>

#include "pt_internal.h"

#pragma clang fp contract(off)

namespace pt {
namespace {

constexpr int kBlock = 256;

template <class T>
struct FbArgs {
  const T* x;
  const T* y;
  const T* z;
  int32_t n_hits;
  double theta2;
  const int32_t* count;   // cells found
  int32_t cap;
  int32_t* inner;
  int32_t* outer;
  uint8_t* pair;
  double* seg;
  int32_t* inner_first;
  int32_t* inner_count;
  // workspace
  int32_t* out_start;     // [n_hits + 1] counts, then starts
  int32_t* cursor;        // [n_hits]
  int32_t* by_outer;      // [cap]
  int32_t* keep;          // [cap + 1] flags, then positions
  int32_t* t_inner;       // [cap] compacted copies
  int32_t* t_outer;
  uint8_t* t_pair;
  double* t_seg;          // [PT_SEG_DOUBLES(cap)]
};

// Cells the Fishbone works on: every stored cell, or none when the cells
// overflowed their capacity (the products are truncated anyway).
template <class T>
__device__ inline int stored(const FbArgs<T>& a) {
  const int c = *a.count;
  return c <= a.cap ? c : 0;
}

template <class T>
__global__ void k_fb_clear(FbArgs<T> a) {
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h <= a.n_hits; h += gridDim.x * blockDim.x) {
    a.out_start[h] = 0;
    if (h < a.n_hits) a.cursor[h] = 0;
  }
}

template <class T>
__global__ void k_fb_count(FbArgs<T> a) {
  const int n = stored(a);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    atomicAdd(a.out_start + a.outer[c], 1);
    a.keep[c] = 1;
  }
}

template <class T>
__global__ void k_fb_fill(FbArgs<T> a) {
  const int n = stored(a);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int h = a.outer[c];
    a.by_outer[a.out_start[h] + atomicAdd(a.cursor + h, 1)] = c;
  }
}

// One wavefront per outer hit.
template <class T>
__global__ void __launch_bounds__(kBlock) k_fb_kill(FbArgs<T> a) {
  const int h = blockIdx.x * (kBlock / kWave) + static_cast<int>(threadIdx.x) / kWave;
  const int lane = __lane_id();
  if (h >= a.n_hits || stored(a) == 0) return;
  const int s0 = a.out_start[h], m = a.out_start[h + 1] - s0;
  if (m < 2) return;
  const double Xh = double(a.x[h]), Yh = double(a.y[h]), Zh = double(a.z[h]);
  for (int c0 = 0; c0 < m; c0 += kWave) {
    const int i = c0 + lane;
    int c = -1;
    double ux = 0.0, uy = 0.0, uz = 0.0, U2 = 0.0;
    if (i < m) {
      c = a.by_outer[s0 + i];
      const int ia = a.inner[c];
      ux = Xh - double(a.x[ia]);
      uy = Yh - double(a.y[ia]);
      uz = Zh - double(a.z[ia]);
      U2 = (ux * ux + uy * uy) + uz * uz;
    }
    bool killed = false;
    for (int j = 0; j < m; ++j) {  // wave-uniform
      const int d = a.by_outer[s0 + j];
      const int ib = a.inner[d];
      const double vx = Xh - double(a.x[ib]), vy = Yh - double(a.y[ib]), vz = Zh - double(a.z[ib]);
      const double V2 = (vx * vx + vy * vy) + vz * vz;
      if (c < 0 || d == c || !(V2 < U2)) continue;
      const double wx = uy * vz - uz * vy, wy = uz * vx - ux * vz, wz = ux * vy - uy * vx;
      const double W2 = (wx * wx + wy * wy) + wz * wz;
      if (W2 <= a.theta2 * (U2 * V2)) killed = true;
    }
    if (c >= 0 && killed) a.keep[c] = 0;
  }
}

template <class T>
__global__ void k_fb_scatter(FbArgs<T> a) {
  const int n = stored(a);
  const int32_t* pos = a.keep;  // scanned
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int p = pos[c];
    if (pos[c + 1] == p) continue;  // dropped
    a.t_inner[p] = a.inner[c];
    a.t_outer[p] = a.outer[c];
    a.t_pair[p] = a.pair[c];
    const int64_t from = seg_at(c), to = seg_at(p);
    a.t_seg[to] = a.seg[from];
    a.t_seg[to + PT_SEG_BLOCK] = a.seg[from + PT_SEG_BLOCK];
    a.t_seg[to + 2 * PT_SEG_BLOCK] = a.seg[from + 2 * PT_SEG_BLOCK];
  }
}

// Copies the compacted cells back and moves each inner hit's range.
template <class T>
__global__ void k_fb_copy_back(FbArgs<T> a) {
  const int n = stored(a);
  if (n == 0) return;
  const int32_t* pos = a.keep;
  const int total = pos[n];
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < total; p += gridDim.x * blockDim.x) {
    a.inner[p] = a.t_inner[p];
    a.outer[p] = a.t_outer[p];
    a.pair[p] = a.t_pair[p];
    const int64_t at = seg_at(p);
    a.seg[at] = a.t_seg[at];
    a.seg[at + PT_SEG_BLOCK] = a.t_seg[at + PT_SEG_BLOCK];
    a.seg[at + 2 * PT_SEG_BLOCK] = a.t_seg[at + 2 * PT_SEG_BLOCK];
  }
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < a.n_hits; h += gridDim.x * blockDim.x) {
    const int cnt = a.inner_count[h];
    if (cnt <= 0) continue;
    const int f = a.inner_first[h];
    const int e = min(f + cnt, n);
    a.inner_first[h] = pos[min(f, n)];
    a.inner_count[h] = pos[e] - pos[min(f, n)];
  }
}

// The new number of cells (a kernel of its own: the others read the old one).
template <class T>
__global__ void k_fb_set_count(FbArgs<T> a, int32_t* count) {
  const int n = stored(a);
  if (n > 0) *count = a.keep[n];
}

template <class T>
pt_err run_fishbone(const pt_hits& h, const DevCfg& k, pt_cells& cells, int32_t* ws_base, hipStream_t s) {
  const int n_hits = h.n_hits;
  const int cap = cells.cap;
  Carver c(ws_base);
  FbArgs<T> a{};
  a.x = static_cast<const T*>(h.x);
  a.y = static_cast<const T*>(h.y);
  a.z = static_cast<const T*>(h.z);
  a.n_hits = n_hits;
  a.theta2 = k.fishbone_theta2;
  a.count = cells.count;
  a.cap = cap;
  a.inner = cells.inner;
  a.outer = cells.outer;
  a.pair = cells.pair;
  a.seg = cells.seg;
  a.inner_first = cells.inner_first;
  a.inner_count = cells.inner_count;
  a.out_start = c.take<int32_t>(static_cast<size_t>(n_hits) + 1);
  a.cursor = c.take<int32_t>(static_cast<size_t>(n_hits));
  a.by_outer = c.take<int32_t>(static_cast<size_t>(cap));
  a.keep = c.take<int32_t>(static_cast<size_t>(cap) + 1);
  a.t_inner = c.take<int32_t>(static_cast<size_t>(cap));
  a.t_outer = c.take<int32_t>(static_cast<size_t>(cap));
  a.t_pair = c.take<uint8_t>(static_cast<size_t>(cap));
  a.t_seg = c.take<double>(PT_SEG_DOUBLES(static_cast<size_t>(cap)));
  int32_t* tmp = c.take<int32_t>(scan_tmp_elems(std::max(cap, n_hits) + 1));
  if (n_hits == 0 || cap == 0) return PT_OK;
  const int gh = grid_for(n_hits + 1, kBlock);
  const int gc = grid_for(cap, kBlock);
  k_fb_clear<T><<<gh, kBlock, 0, s>>>(a);
  k_fb_count<T><<<gc, kBlock, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(a.out_start, n_hits, tmp, s));
  k_fb_fill<T><<<gc, kBlock, 0, s>>>(a);
  k_fb_kill<T><<<static_cast<unsigned>((n_hits + kBlock / kWave - 1) / (kBlock / kWave)), kBlock, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan_dev(a.keep, cap, cells.count, tmp, s));
  k_fb_scatter<T><<<gc, kBlock, 0, s>>>(a);
  k_fb_copy_back<T><<<std::max(gc, gh), kBlock, 0, s>>>(a);
  k_fb_set_count<T><<<1, 1, 0, s>>>(a, cells.count);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace

size_t ws_fishbone(int n_hits, int cells_cap) {
  Carver c(nullptr);
  c.take<int32_t>(static_cast<size_t>(n_hits) + 1);
  c.take<int32_t>(static_cast<size_t>(n_hits));
  c.take<int32_t>(static_cast<size_t>(cells_cap));
  c.take<int32_t>(static_cast<size_t>(cells_cap) + 1);
  c.take<int32_t>(static_cast<size_t>(cells_cap));
  c.take<int32_t>(static_cast<size_t>(cells_cap));
  c.take<uint8_t>(static_cast<size_t>(cells_cap));
  c.take<double>(PT_SEG_DOUBLES(static_cast<size_t>(cells_cap)));
  c.take<int32_t>(scan_tmp_elems(std::max(cells_cap, n_hits) + 1));
  return c.off + 256;
}

pt_err launch_fishbone(const pt_hits& h, const DevCfg& k, pt_cells& cells, void* ws_base, hipStream_t s) {
  void* tok = timing_begin(s);
  const pt_err e = h.dtype == PT_F64 ? run_fishbone<double>(h, k, cells, static_cast<int32_t*>(ws_base), s)
                                     : run_fishbone<float>(h, k, cells, static_cast<int32_t*>(ws_base), s);
  timing_end(tok, "fishbone", s);
  return e;
}

}  // namespace pt
