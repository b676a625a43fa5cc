// Internal declarations shared by the HIP sources of the pixel-track library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/pixeltrack.h"

namespace pt {

constexpr int kWave = 64;
constexpr int kLayers = PT_N_LAYERS;
constexpr int kMaxPairs = PT_MAX_PAIRS;
constexpr int kMaxHits = PT_MAX_HITS;
constexpr int kMaxPairsPerLayer = 8;
constexpr int kRzBuckets = 128;  // direction buckets of the windowed R-Z search, at most

// Constants the kernels use, derived once on the host from pt_config
// (see the expressions documented in pixeltrack.h).
struct DevCfg {
  // doublets
  double tan_dphi[kMaxPairs];
  double zlo[kMaxPairs];
  double zhi[kMaxPairs];
  double z0_max;
  double kappa_max2;
  uint32_t cut_mask;
  int32_t n_pairs;
  int32_t n_bins;                       // azimuth bins per layer
  int32_t bin_shift;                    // log2(n_bins) when a power of two, else -1
  float bin_scale;                      // n_bins / (2 pi)
  int32_t pair_inner[kMaxPairs];
  int32_t pair_outer[kMaxPairs];
  int32_t pair_wbins[kMaxPairs];        // half window in bins (>= n_bins/2: whole layer)
  int32_t inner_pairs[kLayers][kMaxPairsPerLayer];  // pairs whose inner layer is l, -1 padded
  int32_t n_inner_pairs[kLayers];
  // links
  double theta2_barrel, theta2_endcap;
  uint32_t endcap_pairs;  // bit p set when the outer layer of pair p is an end-cap layer
  int32_t rz_buckets;  // direction buckets of the windowed R-Z search (0: every pair is tested)
  double rmax_bpix1, rmax_other;
  uint8_t layer_barrel[kLayers];
  // n-tuplets
  uint32_t root_always_mask, root_if_free_mask;
  int32_t min_hits, max_hits;
  // fit
  double K;          // 0.299792458 B / 100
  double x_over_x0, highland_a, highland_b;
  double VT, VZ_barrel, VR_disk, p_cap;
  double f64_threshold;
  int32_t n_modules;
  int32_t block_doublets;
  // vertices
  int32_t vtx_min_hits, vtx_kmeans_iter;
  double vtx_pt_min, vtx_err_max, vtx_dz_cut, vtx_chi2_max, vtx_split_chi2_ndf, vtx_pt_cap;
  // Fishbone (0: off)
  double fishbone_theta2;
  // adjoint: grad_hits rows are written by one track each
  int32_t exclusive_hits;
};

bool derive_config(const pt_config& c, DevCfg* d);

// ---------------------------------------------------------------------------
// Workspace carving: every region 256-byte aligned.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(void* p) : base(static_cast<char*>(p)) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += n * sizeof(T);
    return p;
  }
};

// Workspace needed by each call (bytes); the public size is their maximum.
size_t ws_doublets(int n_hits, int n_events, int n_bins);
size_t ws_links(int n_hits, int cells_cap);
size_t ws_ntuplets(int cells_cap, int tuplets_cap);
size_t ws_fit(int n_max, int n_modules);
size_t ws_ambiguity(int n_hits, int cells_cap, int n_max);
size_t ws_fishbone(int n_hits, int cells_cap);
// Host-side set-up of the Fishbone's launch shapes (device queries), done
// before a plan captures its graph.
void fishbone_prepare();

// The index of the stored cells by outer hit (links.hip): hit h's cells are
// the entries ent[f .. f + k) (cell, inner hit with bit 31 set when on
// BPix1) of its segments (f, k) = seg[seg_first[h] .. seg_first[h + 1]).
// The cells must not have overflowed their capacity.
struct OuterIndex {
  const int2* ent;
  const int2* seg;
  const int32_t* seg_first;
};
size_t ws_outer_index(int n_hits, int cells_cap);
pt_err build_outer_index(const pt_hits& h, const pt_cells& cells, Carver& c, OuterIndex& out, hipStream_t s);
size_t ws_vertices(int n_events, int n_max);

// Device-wide exclusive scan of n int32 values in place; data[n] receives the
// total.  tmp must hold scan_tmp_elems(n) int32.
size_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan(int32_t* data, int64_t n, int32_t* tmp, hipStream_t s);
// The same over the first min(*n_dev, n) values, n_dev a device count; the
// total goes to data[min(*n_dev, n)].
hipError_t exclusive_scan_dev(int32_t* data, int64_t n, const int32_t* n_dev, int32_t* tmp, hipStream_t s);
// Out of place: dst[i] = src[0] + .. + src[i-1] over the first
// min(*n_dev, n) values (all n when n_dev is null), the total to *total
// (dst[that count] when total is null).  src may equal dst.
hipError_t exclusive_scan_to(const int32_t* src, int32_t* dst, int64_t n, const int32_t* n_dev, int32_t* total,
                             int32_t* tmp, hipStream_t s);
// The first step of such a scan alone, for a kernel that scans its own tile
// of kScanTile values: *offsets (in tmp) receives, for each of the
// ceil(n / kScanTile) tiles, the sum of the values before it, and after them
// the total (the values counted as above).
constexpr int kScanTile = 4096;
hipError_t scan_tile_offsets(const int32_t* src, int64_t n, const int32_t* n_dev, int32_t* tmp, hipStream_t s,
                             const int32_t** offsets);

// Fill helpers (graph-safe: kernels, not hipMemsetAsync).
hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s);

// grid size for grid-stride loops over n items
inline int grid_for(int64_t n, int block, int max_blocks = 65536) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > max_blocks) g = max_blocks;
  return static_cast<int>(g);
}

// Kernel timing hooks (no-ops unless pt_timing_enable(1) and not capturing).
void* timing_begin(hipStream_t s);
void timing_end(void* token, const char* name, hipStream_t s);
extern thread_local bool g_capturing;
extern thread_local bool g_no_timing;  // set by entry points that must not create events

// Device errors: the HIP error behind a PT_ERR_DEVICE is kept per host thread
// (pt_last_device_error).  Entry points clear the thread's HIP error state
// before they launch, so that an error another caller left there (an event
// query's hipErrorNotReady, say) is not taken for one of theirs.
pt_err device_error(hipError_t e);
inline void clear_stale_error() { (void)hipGetLastError(); }

#define PT_HIP_CHECK(expr)                                   \
  do {                                                       \
    const hipError_t pt_e_ = (expr);                         \
    if (pt_e_ != hipSuccess) return ::pt::device_error(pt_e_); \
  } while (0)

#define PT_LAUNCH_CHECK() PT_HIP_CHECK(hipGetLastError())

// ---------------------------------------------------------------------------
// device helpers

__device__ inline void status_flag(uint32_t* st, uint32_t bit) {
  if (st) atomicOr(st + PT_ST_FLAGS, bit);
}
__device__ inline void status_add(uint32_t* st, int word, uint32_t v) {
  if (st && v) atomicAdd(st + word, v);
}

// status_add summed over the wavefront first: one atomic per wavefront.  All
// lanes of the wavefront must call it.
// Returns the wavefront's total.
__device__ inline uint32_t wave_status_add(uint32_t* st, int word, uint32_t v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  if (__lane_id() == 0) status_add(st, word, v);
  return v;
}

// Sum and inclusive prefix sum over the wavefront; all lanes must call them.
__device__ inline int wave_sum(int v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}
__device__ inline float wave_min(float v) {
#pragma unroll
  for (int d = kWave / 2; d > 0; d >>= 1) v = fminf(v, __shfl_xor(v, d, kWave));
  return v;
}
__device__ inline int wave_incl_scan(int v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  return v;
}

// Number of set bits of a wave mask below this lane.
__device__ inline int lane_prefix(uint64_t mask) {
  return static_cast<int>(__builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u)));
}

// Work-group dispatch places consecutive work-group ids on different XCDs
// (round robin over kXcds), each with its own L2.  xcd_block(b, nb) renumbers
// the nb work-groups of a 1-D grid so that each XCD takes one contiguous
// range of the logical ids: neighbouring work-groups, which write
// neighbouring output, then share an L2 and complete its cache lines there.
constexpr int kXcds = 8;
__device__ inline int xcd_block(int b, int nb) {
  const int q = nb / kXcds, r = nb % kXcds;
  const int x = b % kXcds, k = b / kXcds;
  return x * q + min(x, r) + k;
}

// Orders the LDS traffic of one wavefront (its lanes run in lockstep, so a
// compiler barrier is all that is needed between a write and a read by
// another lane).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace pt
