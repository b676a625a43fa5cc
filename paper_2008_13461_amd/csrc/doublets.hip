// Doublet building (paper section 3.2, Table 1).
//
// Hits are first binned per (event, layer, azimuth bin) by a counting sort
// (the "tiled data structure along phi" of the paper), with sorted copies
// of the coordinates (in the input type, converted to double exactly where
// they are used) and of R in double.  Doublets are then built by one wavefront
// per inner hit that loops over the layer pairs starting on its layer and
// scans the outer hits in the azimuth bins around it, one outer hit per lane.
// Two passes -- count, scan, write -- give every inner hit a contiguous,
// deterministic run of cells without any per-cell atomic: the cells come out
// grouped by inner hit in the sorted order (pair order, then window order),
// and (inner_first, inner_count) index them by hit for the linking step.
#include "pt_internal.h"

#include <algorithm>
#include <cmath>

// Every decision below is made in double precision exactly as parenthesised:
// no multiply-add contraction anywhere in this file.
#pragma clang fp contract(off)

namespace pt {

pt_err launch_fishbone(const pt_hits& h, const DevCfg& k, pt_cells& cells, void* ws_base, hipStream_t s);

// The cut predicates of Table 1, as documented in pixeltrack.h (tdphi is
// tan_dphi of the pair, loaded once per pair by the caller).  ALL: PhiW,
// ZIP and PT are all on, and the three are evaluated without branches (a
// divergent early exit costs scalar instructions to mask lanes, and a whole
// wavefront of candidates rarely fails together); the same comparisons of
// the same values, so the same decisions.
constexpr uint32_t kCutsAll = PT_CUT_PHIW | PT_CUT_ZIP | PT_CUT_PT;
template <bool ALL>
__device__ __forceinline__ bool doublet_pass(const DevCfg& k, double tdphi, double Xi, double Yi, double Zi,
                                             double Ri, double Xo, double Yo, double Zo, double Ro) {
  const double D = Xi * Xo + Yi * Yo;
  const double C = Xi * Yo - Yi * Xo;
  if (ALL) {
    const double dR = Ro - Ri;
    const double R2i = Xi * Xi + Yi * Yi;
    const double R2o = Xo * Xo + Yo * Yo;
    const double dx = Xo - Xi;
    const double dy = Yo - Yi;
    const double L2 = dx * dx + dy * dy;
    const bool phiw = D > 0.0 && fabs(C) <= tdphi * D;
    const bool zip = dR > 0.0 && fabs(Zi * Ro - Zo * Ri) <= k.z0_max * dR;
    const bool pt = (4.0 * C) * C <= (k.kappa_max2 * (R2i * R2o)) * L2;
    return static_cast<int>(phiw) & static_cast<int>(zip) & static_cast<int>(pt);
  }
  if (k.cut_mask & PT_CUT_PHIW) {
    if (!(D > 0.0 && fabs(C) <= tdphi * D)) return false;
  }
  if (k.cut_mask & PT_CUT_ZIP) {
    const double dR = Ro - Ri;
    if (!(dR > 0.0 && fabs(Zi * Ro - Zo * Ri) <= k.z0_max * dR)) return false;
  }
  if (k.cut_mask & PT_CUT_PT) {
    const double R2i = Xi * Xi + Yi * Yi;
    const double R2o = Xo * Xo + Yo * Yo;
    const double dx = Xo - Xi;
    const double dy = Yo - Yi;
    const double L2 = dx * dx + dy * dy;
    if (!((4.0 * C) * C <= (k.kappa_max2 * (R2i * R2o)) * L2)) return false;
  }
  return true;
}

namespace {

// Four values of the input type in one vector (one load).
template <class T>
struct Vec4Of;
template <>
struct Vec4Of<float> { using type = float4; };
template <>
struct Vec4Of<double> { using type = double4; };
template <class T>
using Vec4 = typename Vec4Of<T>::type;

template <class T>
struct HitsIn {
  int32_t n_hits, n_events;
  const int32_t* off;
  const T* x;
  const T* y;
  const T* z;
  const uint8_t* layer;
};

// Event of hit h: off[e] <= h < off[e+1]; -1 when h is in no event.
__device__ inline int event_of(const int32_t* off, int n_events, int h) {
  if (n_events <= 0 || h < off[0] || h >= off[n_events]) return -1;
  int lo = 0, hi = n_events;  // invariant: off[lo] <= h < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= h) lo = mid; else hi = mid;
  }
  return lo;
}

template <class T>
__global__ void k_hit_keys(HitsIn<T> in, int n_bins, float bin_scale, int32_t* __restrict__ key,
                           int32_t* __restrict__ rank, int32_t* __restrict__ bin_count,
                           uint32_t* status) {
  uint32_t bad = 0;
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < in.n_hits; h += gridDim.x * blockDim.x) {
    key[h] = -1;
    const int e = event_of(in.off, in.n_events, h);
    if (e < 0) continue;
    const int lay = in.layer[h];
    const double X = static_cast<double>(in.x[h]);
    const double Y = static_cast<double>(in.y[h]);
    const double Z = static_cast<double>(in.z[h]);
    if (lay >= kLayers || !isfinite(X) || !isfinite(Y) || !isfinite(Z)) {
      ++bad;
      continue;
    }
    const float phi = atan2f(static_cast<float>(Y), static_cast<float>(X));
    int b = static_cast<int>((phi + 3.14159265358979f) * bin_scale);
    b = b < 0 ? 0 : (b >= n_bins ? n_bins - 1 : b);
    const int k = (e * kLayers + lay) * n_bins + b;
    key[h] = k;
    rank[h] = atomicAdd(bin_count + k, 1);
  }
  if (bad) {
    status_add(status, PT_ST_BAD_HITS, bad);
    status_flag(status, PT_FLAG_BAD_HITS);
  }
}

// Places every valid hit in its bin (arrival order within the bin, from the
// ranks of k_hit_keys) and clears the per-hit cell counts.
template <class T>
__global__ void k_scatter(HitsIn<T> in, const int32_t* __restrict__ key, const int32_t* __restrict__ rank,
                          const int32_t* __restrict__ bin_start, int32_t* __restrict__ arrived,
                          int32_t* __restrict__ skey, int32_t* __restrict__ inner_count) {
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < in.n_hits; h += gridDim.x * blockDim.x) {
    inner_count[h] = 0;
    const int k = key[h];
    if (k < 0) continue;
    const int pos = bin_start[k] + rank[h];
    arrived[pos] = h;
    skey[pos] = k;
  }
}

// Orders each bin by hit index, so that the sorted order -- and with it the
// order of the cells, links and rows -- does not depend on the order in
// which the atomics of k_hit_keys were served: the hit at position p moves to
// its bin's start plus the number of the bin's hits with a smaller index.
// Then fills the sorted copies (in double) at the new position.
template <class T>
__global__ void k_bin_order(HitsIn<T> in, const int32_t* __restrict__ valid, const int32_t* __restrict__ bin_start,
                            const int32_t* __restrict__ arrived, const int32_t* __restrict__ skey,
                            int32_t* __restrict__ sorted_hit, Vec4<T>* __restrict__ sP, double* __restrict__ sR) {
  const int total = *valid;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < total; p += gridDim.x * blockDim.x) {
    const int k = skey[p];
    const int b0 = bin_start[k], b1 = bin_start[k + 1];
    const int h = arrived[p];
    int r = 0;
    for (int q = b0; q < b1; ++q) r += arrived[q] < h ? 1 : 0;
    const int pos = b0 + r;
    const double X = static_cast<double>(in.x[h]);
    const double Y = static_cast<double>(in.y[h]);
    sorted_hit[pos] = h;
    Vec4<T> q;  // in the input type: converted where used, exactly
    q.x = in.x[h];
    q.y = in.y[h];
    q.z = in.z[h];
    q.w = T(0);
    sP[pos] = q;
    sR[pos] = sqrt(X * X + Y * Y);
  }
}

template <class T>
struct DoubletArgs {
  int32_t n_hits;
  const int32_t* bin_start;
  const int32_t* skey;
  const int32_t* sorted_hit;
  const Vec4<T>* sP;  // sorted (x, y, z, 0) in the input type: one 16-byte load for float hits
  const double* sR;
  int32_t* cnt;            // pass 1: per sorted inner hit
  const int32_t* off;      // pass 2: scanned counts
  int4* chunks;            // [n_hits][kMaskChunks] pass 1: the groups of candidates with a passing one
  int32_t* n_chunks;       // [n_hits] pass 1: how many (-1: more than kMaskChunks)
  int32_t cap;
  int32_t* inner;
  int32_t* outer;
  uint8_t* pair;
  int32_t* inner_first;
  int32_t* inner_count;
};

// The azimuth-bin ranges of the outer layer of pair p scanned for an inner
// hit in bin b: [r0a, r0b) and [r1a, r1b) (the second one non-empty when the
// window wraps around phi = +-pi).
__device__ inline void window_ranges(const DevCfg& k, const int32_t* bin_start, int p, int e, int b,
                                     int& r0a, int& r0b, int& r1a, int& r1b) {
  const int B = k.n_bins;
  const int base = (e * kLayers + k.pair_outer[p]) * B;
  const int w = k.pair_wbins[p];
  r1a = r1b = 0;
  if (2 * w + 1 >= B) {
    r0a = bin_start[base];
    r0b = bin_start[base + B];
    return;
  }
  const int lo = b - w, hi = b + w;
  if (lo < 0) {
    r0a = bin_start[base + lo + B];
    r0b = bin_start[base + B];
    r1a = bin_start[base];
    r1b = bin_start[base + hi + 1];
  } else if (hi >= B) {
    r0a = bin_start[base + lo];
    r0b = bin_start[base + B];
    r1a = bin_start[base];
    r1b = bin_start[base + hi - B + 1];
  } else {
    r0a = bin_start[base + lo];
    r0b = bin_start[base + hi + 1];
  }
}

// One wavefront per sorted inner hit: its coordinates are wave-uniform, the
// lanes take consecutive outer hits of each window (coalesced loads), and the
// passing ones are compacted with a ballot, so that the cells of the inner
// hit are written as one contiguous, coalesced run.  COUNT = false writes the
// cells at the scanned offsets, in pair order then window order.
// Outer hits a wavefront of the write pass gathers in LDS before it stores
// them: its stores come after its loads, so no load of the window scan waits
// for a store's acknowledgement (one counter tracks both on this GPU).
constexpr int kStage = 256;
// Groups of candidates with a passing one that the count pass keeps for the
// write pass, per inner hit: (ballot of the group, first outer hit, pair) in
// one 16-byte record.  A hit with more such groups is tested again by the
// write pass.
constexpr int kMaskChunks = 64;
static_assert(kMaskChunks == kWave, "one kept group per lane");
// Threads per block of the write pass, whatever the count pass takes: four
// single-wavefront hits per block measured fastest for the stores.
constexpr int kWriteBlock = 256;

template <bool WRITE, int WAVES, bool ALL, class T>
__global__ void __launch_bounds__(WAVES * kWave) k_doublets(DevCfg k, DoubletArgs<T> a) {
  __shared__ int32_t s_out[WRITE ? WAVES : 1][WRITE ? kStage : 1];
  __shared__ uint8_t s_pair[WRITE ? WAVES : 1][WRITE ? kStage : 1];
  __shared__ int4 s_chunk[WRITE ? WAVES : 1][WRITE ? kMaskChunks : 1];
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = __lane_id();
  const int j = xcd_block(blockIdx.x, gridDim.x) * WAVES + wave;
  if (j >= a.n_hits) return;
  // count pass: the kept groups of the hit, record t on lane t
  int4 rec = make_int4(0, 0, 0, 0);
  // the write pass's own loads go out with the bound's (j < n_hits: every
  // one is in range), so that its chain of dependent loads is one shorter
  const int first = WRITE ? a.off[j] : 0;
  const int last = WRITE ? a.off[j + 1] : 0;
  const int hit_i = WRITE ? a.sorted_hit[j] : 0;
  const int nst = WRITE ? a.n_chunks[j] : 0;
  const int total = a.bin_start[-1];  // valid (sorted) hits
  if (j >= total) {
    if (!WRITE && lane == 0) {
      a.cnt[j] = 0;
      a.n_chunks[j] = 0;
    }
    return;
  }
  int pos = first;  // uniform: next cell position (write pass) or count
  int staged = 0;   // uniform: staged cells, to be written from pos on
  // stores the staged cells (outer hit, pair), consecutive positions on
  // consecutive lanes
  auto flush = [&]() {
    wave_sync();
    for (int i = lane; i < staged; i += kWave) {
      const int w = pos + i;
      if (w < a.cap) {
        a.inner[w] = hit_i;
        a.outer[w] = s_out[wave][i];
        a.pair[w] = s_pair[wave][i];
      }
    }
    wave_sync();
    pos += staged;
    staged = 0;
  };
  // the write pass takes the groups the count pass kept instead of testing
  // the candidates again
  if (WRITE && nst >= 0) {
    if (lane < nst) s_chunk[wave][lane] = a.chunks[static_cast<int64_t>(j) * kMaskChunks + lane];
    wave_sync();
    // kGroupBatch groups at a time: the gathers of all of them are issued
    // before any is staged
    constexpr int kGroupBatch = 4;
    for (int t0 = 0; t0 < nst; t0 += kGroupBatch) {
      uint64_t m[kGroupBatch];
      int pr[kGroupBatch], hit[kGroupBatch];
#pragma unroll
      for (int u = 0; u < kGroupBatch; ++u) {
        m[u] = 0;
        pr[u] = 0;
        if (t0 + u < nst) {  // uniform
          const int4 d = s_chunk[wave][t0 + u];
          m[u] = (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(d.y))) << 32) |
                 static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(d.x));
          pr[u] = __builtin_amdgcn_readfirstlane(d.w);
          const int o = __builtin_amdgcn_readfirstlane(d.z) + lane;
          if ((m[u] >> lane) & 1u) hit[u] = a.sorted_hit[o];
        }
      }
#pragma unroll
      for (int u = 0; u < kGroupBatch; ++u) {
        if (staged + kWave > kStage) flush();
        if ((m[u] >> lane) & 1u) {
          const int at = staged + lane_prefix(m[u]);
          s_out[wave][at] = hit[u];
          s_pair[wave][at] = static_cast<uint8_t>(pr[u]);
        }
        staged += __popcll(m[u]);
      }
    }
    flush();
    if (lane == 0) {
      a.inner_first[hit_i] = first;
      a.inner_count[hit_i] = last - first;
    }
    return;
  }
  const int B = k.n_bins;
  const int key = a.skey[j];
  const int sh = k.bin_shift;  // log2 B for a power of two: no integer division
  const int b = sh >= 0 ? (key & (B - 1)) : key % B;
  const int el = sh >= 0 ? (key >> sh) : key / B;
  const int lay = el % kLayers;
  const int e = el / kLayers;
  const Vec4<T> Pi = a.sP[j];
  const double Xi = double(Pi.x), Yi = double(Pi.y), Zi = double(Pi.z), Ri = a.sR[j];
  // the count pass, or the write pass of a hit with more groups than kept:
  // every group of candidates, in pair order, then window order
  int kept = 0;  // uniform: groups with a passing candidate (count pass)
  const int np = k.n_inner_pairs[lay];
  for (int q = 0; q < np; ++q) {
    const int p = k.inner_pairs[lay][q];
    if (k.cut_mask & PT_CUT_ZW) {
      if (!(k.zlo[p] <= Zi && Zi <= k.zhi[p])) continue;
    }
    const double tdphi = k.tan_dphi[p];
    int ra[2], rb[2];
    window_ranges(k, a.bin_start, p, e, b, ra[0], rb[0], ra[1], rb[1]);
    for (int r = 0; r < 2; ++r) {
      for (int o0 = ra[r]; o0 < rb[r]; o0 += kWave) {
        const int o = o0 + lane;
        const int oc = min(o, rb[r] - 1);  // lanes past the range test its last hit and are masked out
        const Vec4<T> Po = a.sP[oc];
        const bool pass = static_cast<int>(o < rb[r]) &
                          static_cast<int>(doublet_pass<ALL>(k, tdphi, Xi, Yi, Zi, Ri, double(Po.x), double(Po.y),
                                                             double(Po.z), a.sR[oc]));
        const uint64_t m = __ballot(pass);
        if (WRITE) {
          if (staged + kWave > kStage) flush();
          if (pass) {
            const int at = staged + lane_prefix(m);
            s_out[wave][at] = a.sorted_hit[o];
            s_pair[wave][at] = static_cast<uint8_t>(p);
          }
          staged += __popcll(m);
        } else {
          if (m) {
            if (lane == kept)
              rec = make_int4(static_cast<int>(static_cast<uint32_t>(m)), static_cast<int>(static_cast<uint32_t>(m >> 32)),
                              o0, p);
            ++kept;
          }
          pos += __popcll(m);
        }
      }
    }
  }
  if (WRITE) flush();
  if (!WRITE) {  // the kept groups, after every load of the scan
    const int nk = min(kept, kMaskChunks);
    if (lane < nk) a.chunks[static_cast<int64_t>(j) * kMaskChunks + lane] = rec;
  }
  if (lane == 0) {
    if (!WRITE) {
      a.cnt[j] = pos;
      a.n_chunks[j] = kept <= kMaskChunks ? kept : -1;
    } else {
      a.inner_first[hit_i] = first;
      a.inner_count[hit_i] = last - first;
    }
  }
}

__global__ void k_finish_cells(const int32_t* total, int32_t cap, int32_t* count, uint32_t* status) {
  const int t = *total;
  *count = t;
  if (t > cap) status_flag(status, PT_FLAG_CELLS_OVERFLOW);
}

// bin_start is laid out with one leading word that receives the number of
// valid hits, so that kernels can read it as bin_start[-1].
__global__ void k_copy_total(const int32_t* __restrict__ bin_start, int nb, int32_t* __restrict__ dst) {
  *dst = bin_start[nb];
}

}  // namespace

size_t ws_doublets(int n_hits, int n_events, int n_bins) {
  const size_t nb = static_cast<size_t>(n_events) * kLayers * n_bins;
  Carver c(nullptr);
  c.take<int32_t>(n_hits);        // key
  c.take<int32_t>(n_hits);        // rank
  c.take<int32_t>(nb + 2);        // [total] + bin counts/starts (+ end)
  c.take<int32_t>(n_hits);        // sorted_hit
  c.take<int32_t>(n_hits);        // skey
  c.take<double4>(n_hits);        // sP (x, y, z) in the input type: at most 32 bytes
  c.take<double>(n_hits);         // sR
  c.take<int32_t>(n_hits + 1);    // cnt / off
  c.take<int4>(static_cast<size_t>(n_hits) * kMaskChunks);  // kept groups of candidates
  c.take<int32_t>(n_hits);        // groups per hit
  const size_t t = scan_tmp_elems(std::max<int64_t>(static_cast<int64_t>(nb), n_hits));
  c.take<int32_t>(t);
  return c.off + 256;
}

template <bool WRITE, bool ALL, class T>
static void launch_doublets_as(const DevCfg& k, const DoubletArgs<T>& a, int n, int block, hipStream_t s) {
  const int64_t hits = std::max(n, 1);
  switch (block) {
    case 64:
      k_doublets<WRITE, 1, ALL, T><<<static_cast<unsigned>(hits), 64, 0, s>>>(k, a);
      break;
    case 128:
      k_doublets<WRITE, 2, ALL, T><<<static_cast<unsigned>((hits + 1) / 2), 128, 0, s>>>(k, a);
      break;
    case 512:
      k_doublets<WRITE, 8, ALL, T><<<static_cast<unsigned>((hits + 7) / 8), 512, 0, s>>>(k, a);
      break;
    default:
      k_doublets<WRITE, 4, ALL, T><<<static_cast<unsigned>((hits + 3) / 4), 256, 0, s>>>(k, a);
  }
}

template <bool WRITE, class T>
static void launch_doublets(const DevCfg& k, const DoubletArgs<T>& a, int n, int block, hipStream_t s) {
  if ((k.cut_mask & kCutsAll) == kCutsAll)
    launch_doublets_as<WRITE, true, T>(k, a, n, block, s);
  else
    launch_doublets_as<WRITE, false, T>(k, a, n, block, s);
}

template <class T>
static pt_err run_doublets(const pt_hits& h, const DevCfg& k, pt_cells& cells, uint32_t* status,
                           pt_workspace ws, hipStream_t s) {
  const int n = h.n_hits;
  const int B = k.n_bins;
  const int64_t nb = static_cast<int64_t>(h.n_events) * kLayers * B;
  Carver c(ws.ptr);
  int32_t* key = c.take<int32_t>(n);
  int32_t* rank = c.take<int32_t>(n);
  int32_t* bins = c.take<int32_t>(nb + 2);   // bins[0] = valid hits; bins+1 = counts -> starts
  int32_t* sorted_hit = c.take<int32_t>(n);
  int32_t* skey = c.take<int32_t>(n);
  Vec4<T>* sP = c.take<Vec4<T>>(n);
  double* sR = c.take<double>(n);
  int32_t* cnt = c.take<int32_t>(n + 1);
  int4* chunks = c.take<int4>(static_cast<size_t>(n) * kMaskChunks);
  int32_t* n_chunks = c.take<int32_t>(n);
  int32_t* tmp = c.take<int32_t>(scan_tmp_elems(std::max<int64_t>(nb, n)));
  int32_t* bin_start = bins + 1;

  HitsIn<T> in{n, h.n_events, h.event_offsets, static_cast<const T*>(h.x), static_cast<const T*>(h.y),
               static_cast<const T*>(h.z), h.layer};
  PT_HIP_CHECK(fill_i32(bins, 0, nb + 2, s));
  k_hit_keys<T><<<grid_for(n, 256), 256, 0, s>>>(in, B, k.bin_scale, key, rank, bin_start, status);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(bin_start, nb, tmp, s));
  k_copy_total<<<1, 1, 0, s>>>(bin_start, static_cast<int>(nb), bins);
  PT_LAUNCH_CHECK();
  // the hits in arrival order within their bins, then each bin ordered by
  // hit index
  int32_t* arrived = cnt;  // the per-hit counts are free until the count pass
  k_scatter<T><<<grid_for(n, 256), 256, 0, s>>>(in, key, rank, bin_start, arrived, skey, cells.inner_count);
  PT_LAUNCH_CHECK();
  k_bin_order<T><<<grid_for(n, 256), 256, 0, s>>>(in, bins, bin_start, arrived, skey, sorted_hit, sP, sR);
  PT_LAUNCH_CHECK();

  DoubletArgs<T> a{n, bin_start, skey, sorted_hit, sP, sR, cnt, cnt, chunks, n_chunks, cells.cap, cells.inner,
                cells.outer, cells.pair, cells.inner_first, cells.inner_count};
  // bin_start[-1] holds the number of valid hits (sorted positions).
  const int block = (k.block_doublets == 64 || k.block_doublets == 128 || k.block_doublets == 512)
                        ? k.block_doublets : 256;
  void* tok = timing_begin(s);
  launch_doublets<false, T>(k, a, n, block, s);
  timing_end(tok, "doublets_count", s);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(cnt, n, tmp, s));
  tok = timing_begin(s);
  launch_doublets<true, T>(k, a, n, kWriteBlock, s);
  timing_end(tok, "doublets_write", s);
  PT_LAUNCH_CHECK();
  k_finish_cells<<<1, 1, 0, s>>>(cnt + n, cells.cap, cells.count, status);
  PT_LAUNCH_CHECK();
  // the Fishbone reuses the workspace from its start (the sorted hits are dead)
  if (k.fishbone_theta2 > 0.0) return launch_fishbone(h, k, cells, ws.ptr, s);
  return PT_OK;
}

pt_err launch_doublets(const pt_hits& h, const DevCfg& k, pt_cells& cells, uint32_t* status,
                       pt_workspace ws, hipStream_t s) {
  if (h.dtype == PT_F64) return run_doublets<double>(h, k, cells, status, ws, s);
  return run_doublets<float>(h, k, cells, status, ws, s);
}

}  // namespace pt
