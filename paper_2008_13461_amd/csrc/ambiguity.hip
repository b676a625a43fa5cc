// Ambiguity resolution among fitted tracks (paper section 3.5).
//
// Tracks sharing a hit doublet (a cell) are ambiguous and only the one with
// the smallest chi^2 stays; then, among the 3-hit tracks that stayed, tracks
// sharing a hit are ambiguous and only the one with the smallest transverse
// impact parameter |d0| stays.  Equal values keep both.  Tracks whose fit
// failed (non-finite chi^2) take no part and are not selected.
//
// Both rules are a minimum per key (cell, then hit) followed by a test of
// each track against the minima of its keys, as the duplicate removal of the
// n-tuplet search does with its maximum per cell.  Values are compared as
// the bit patterns of their magnitudes promoted to double (for non-negative
// doubles the unsigned order of the bits is the numeric order), so one 64-bit
// atomicMin per (track, key) takes each minimum, whatever the fit precision.
// The minima are reset first for the keys the tracks visit, so the cost
// follows the number of tracks, not the capacity of cells or hits.  Selected
// tracks are listed in track order (flags, a scan, a scatter).
#include <algorithm>

#include "pt_internal.h"

namespace pt {
namespace {

constexpr int kBlock = 256;
constexpr uint64_t kNone = ~uint64_t(0);

struct AmbArgs {
  const int32_t* hits;   // rows [cap][kMaxHits]
  const int32_t* cells;  // rows [cap][kMaxHits - 1]
  const uint8_t* n;      // [cap]
  const int32_t* kept;   // track i is row kept[i] (row i when null)
  const int32_t* count;  // number of tracks (device)
  int32_t n_max;
  const void* chi2;      // [n_max], double when dbl else float
  const void* params;    // [n_max][5]
  int32_t dbl;
  int32_t n_hits, n_cells;
  uint64_t* best_cell;   // [n_cells]
  uint64_t* best_hit;    // [n_hits]
  int32_t* flag;         // [n_max]: 0 dropped, 1 kept, 2 triplet kept by the chi2 rule (pass 1)
  int32_t* pos;          // [n_max + 1]
};

__device__ inline int n_tracks(const AmbArgs& a) { return min(*a.count, a.n_max); }

__device__ inline double value(const void* p, int64_t i, int dbl) {
  return dbl ? static_cast<const double*>(p)[i] : double(static_cast<const float*>(p)[i]);
}

// Order key of a magnitude: the bits of |v| as a double.
__device__ inline uint64_t key_of(double v) { return static_cast<uint64_t>(__double_as_longlong(fabs(v))); }

// A track takes part when its fit succeeded and its row indexes valid cells
// and hits.
__device__ inline bool candidate(const AmbArgs& a, int i, int& row, int& nh) {
  row = a.kept ? a.kept[i] : i;
  nh = a.n[row];
  if (nh < 2 || nh > kMaxHits) return false;
  const double c = value(a.chi2, i, a.dbl);
  if (!isfinite(c)) return false;
  const int32_t* C = a.cells + static_cast<int64_t>(row) * (kMaxHits - 1);
  for (int d = 0; d < nh - 1; ++d)
    if (C[d] < 0 || C[d] >= a.n_cells) return false;
  if (nh == 3) {
    const int32_t* H = a.hits + static_cast<int64_t>(row) * kMaxHits;
    for (int d = 0; d < 3; ++d)
      if (H[d] < 0 || H[d] >= a.n_hits) return false;
  }
  return true;
}

__global__ void __launch_bounds__(kBlock) k_amb_reset(AmbArgs a) {
  const int n = n_tracks(a);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int row, nh;
    if (!candidate(a, i, row, nh)) continue;
    const int32_t* C = a.cells + static_cast<int64_t>(row) * (kMaxHits - 1);
    for (int d = 0; d < nh - 1; ++d) a.best_cell[C[d]] = kNone;
    if (nh == 3) {
      const int32_t* H = a.hits + static_cast<int64_t>(row) * kMaxHits;
      for (int d = 0; d < 3; ++d) a.best_hit[H[d]] = kNone;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_amb_cell_min(AmbArgs a) {
  const int n = n_tracks(a);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int row, nh;
    if (!candidate(a, i, row, nh)) continue;
    const uint64_t k = key_of(value(a.chi2, i, a.dbl));
    const int32_t* C = a.cells + static_cast<int64_t>(row) * (kMaxHits - 1);
    for (int d = 0; d < nh - 1; ++d) atomicMin(reinterpret_cast<unsigned long long*>(a.best_cell + C[d]), k);
  }
}

// The chi^2 rule; the triplets that pass it enter the minima of |d0| of
// their hits.
__global__ void __launch_bounds__(kBlock) k_amb_chi2_rule(AmbArgs a) {
  const int n = n_tracks(a);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    int row, nh;
    int f = 0;
    if (candidate(a, i, row, nh)) {
      const uint64_t k = key_of(value(a.chi2, i, a.dbl));
      const int32_t* C = a.cells + static_cast<int64_t>(row) * (kMaxHits - 1);
      bool ok = true;
      for (int d = 0; d < nh - 1; ++d) ok = ok && a.best_cell[C[d]] == k;
      if (ok && nh == 3) {
        const uint64_t t = key_of(value(a.params, static_cast<int64_t>(i) * 5 + 3, a.dbl));
        const int32_t* H = a.hits + static_cast<int64_t>(row) * kMaxHits;
        for (int d = 0; d < 3; ++d) atomicMin(reinterpret_cast<unsigned long long*>(a.best_hit + H[d]), t);
        f = 2;
      } else {
        f = ok ? 1 : 0;
      }
    }
    a.flag[i] = f;
  }
}

// The |d0| rule among the triplets that passed the chi^2 rule.
__global__ void __launch_bounds__(kBlock) k_amb_tip_rule(AmbArgs a) {
  const int n = n_tracks(a);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    if (a.flag[i] != 2) continue;
    const int row = a.kept ? a.kept[i] : i;
    const uint64_t t = key_of(value(a.params, static_cast<int64_t>(i) * 5 + 3, a.dbl));
    const int32_t* H = a.hits + static_cast<int64_t>(row) * kMaxHits;
    bool ok = true;
    for (int d = 0; d < 3; ++d) ok = ok && a.best_hit[H[d]] == t;
    a.flag[i] = ok ? 1 : 0;
  }
}

__global__ void __launch_bounds__(kBlock) k_amb_list(AmbArgs a, int32_t* __restrict__ selected) {
  const int n = n_tracks(a);
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock)
    if (a.flag[i]) selected[a.pos[i]] = i;
}

}  // namespace

size_t ws_ambiguity(int n_hits, int cells_cap, int n_max) {
  Carver c(nullptr);
  c.take<uint64_t>(static_cast<size_t>(cells_cap));
  c.take<uint64_t>(static_cast<size_t>(n_hits));
  c.take<int32_t>(static_cast<size_t>(n_max));
  c.take<int32_t>(static_cast<size_t>(n_max) + 1);
  c.take<int32_t>(scan_tmp_elems(n_max));
  return c.off + 256;
}

pt_err launch_ambiguity(const pt_hits& h, const pt_cells& cells, const pt_ntuplets& T, int precision,
                        const pt_tracks& tracks, int32_t* selected, int32_t* n_selected, pt_workspace ws,
                        hipStream_t s) {
  const int n_max = std::min(T.cap, tracks.cap);
  Carver c(ws.ptr);
  AmbArgs a{};
  a.hits = T.hits;
  a.cells = T.cells;
  a.n = T.n;
  a.kept = T.kept;
  a.count = T.count;
  a.n_max = n_max;
  a.chi2 = tracks.chi2;
  a.params = tracks.params;
  a.dbl = precision == PT_FIT_F64 ? 1 : 0;
  a.n_hits = h.n_hits;
  a.n_cells = cells.cap;
  a.best_cell = c.take<uint64_t>(static_cast<size_t>(cells.cap));
  a.best_hit = c.take<uint64_t>(static_cast<size_t>(h.n_hits));
  a.flag = c.take<int32_t>(static_cast<size_t>(n_max));
  a.pos = c.take<int32_t>(static_cast<size_t>(n_max) + 1);
  int32_t* tmp = c.take<int32_t>(scan_tmp_elems(n_max));
  if (n_max == 0) return fill_i32(n_selected, 0, 1, s) == hipSuccess ? PT_OK : PT_ERR_DEVICE;
  const int g = grid_for(n_max, kBlock, 8192);
  k_amb_reset<<<g, kBlock, 0, s>>>(a);
  k_amb_cell_min<<<g, kBlock, 0, s>>>(a);
  k_amb_chi2_rule<<<g, kBlock, 0, s>>>(a);
  k_amb_tip_rule<<<g, kBlock, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan_to(a.flag, a.pos, n_max, a.count, n_selected, tmp, s));
  k_amb_list<<<g, kBlock, 0, s>>>(a, selected);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
