// Broken-line fit and its adjoint on the GPU (paper section 3.4: one thread
// per n-tuplet).
//
// Tracks are first binned by their number of hits, so that each
// instantiation fit<N> runs over a dense list with its own register budget
// (every per-hit quantity of a track lives in registers).  In the
// single-precision mode with the double fallback, tracks whose transverse
// system is too stiff for float (high momentum: the scattering kinks weigh
// far more than the measurements) are put on a list and refitted entirely in
// double by a second kernel.
//
// The adjoint recomputes the forward fit in registers and sweeps it back
// (fit_core.h).  Hit gradients are added with float atomics (hits can be
// shared between tracks); module-offset gradients are accumulated per block in
// LDS in double and written as one partial sum per block, then reduced across
// blocks in a fixed order (no global atomics on the table).  The order of the
// additions within a block still depends on the schedule, so module sums
// agree between runs to the rounding of double, not bit for bit.
#include <mutex>

#include "fit_core.h"
#include "pt_internal.h"

#include <type_traits>

namespace pt {
namespace {

constexpr int kMinN = 3;
constexpr int kNBins = kMaxHits - kMinN + 1;  // N = 3..8
constexpr int kBlock = 256;
constexpr int kBwdBlocks = 256;
constexpr int kRefitBlock = 64;

struct FitArgs {
  int32_t dtype;
  int32_t n_hits;
  const void* x;
  const void* y;
  const void* z;
  const uint8_t* layer;
  const int16_t* module;
  const float* offsets;
  int32_t n_modules;
  const int32_t* tup_hits;
  const uint8_t* tup_n;
  const int32_t* kept;       // may be null: track i is row i
  const int32_t* count;      // number of tracks (device)
  int32_t n_max;             // host bound on the number of tracks
  // binning
  int32_t* bins;             // [kNBins][n_max]
  int32_t* bin_count;        // [kNBins]
  int32_t* redo;             // [n_max] tracks refitted in double
  int32_t* redo_count;
  // forward outputs
  void* params;
  void* chi2;
  uint8_t* track_status;
  void* cov;                 // [n_max][15] or null
  // adjoint
  const void* g_params;       // GT (the type of grad_hits) [n][5]
  const void* g_chi2;         // GT [n], may be null
  void* grad_hits;           // float, or double in the double-precision mode
  double* partials;          // [kBwdBlocks][n_modules * 3]
  uint32_t* status;
};

__host__ __device__ fit::Consts consts_of(const DevCfg& k) {
  fit::Consts c;
  c.K = k.K;
  c.x0 = k.x_over_x0;
  c.ha = k.highland_a;
  c.hb = k.highland_b;
  c.VT = k.VT;
  c.VZb = k.VZ_barrel;
  c.VRd = k.VR_disk;
  c.pcap = k.p_cap;
  c.thr = k.f64_threshold;
  return c;
}

__device__ inline int track_row(const FitArgs& a, int i) { return a.kept ? a.kept[i] : i; }
__device__ inline int n_tracks(const FitArgs& a) { return min(*a.count, a.n_max); }

// Bin tracks by hit count.  Each block owns a contiguous range of tracks:
// it counts its tracks per bin (ballots), takes its base in each bin with
// one atomic per bin, then walks its range again placing the tracks (ranks
// within a wavefront from ballots, per-wave offsets in LDS).  The grid is
// capped (kBinBlocks) so that few atomics meet on each bin counter.
constexpr int kBinBlocks = 1024;

__device__ inline int track_bin(const FitArgs& a, int i, int n) {
  if (i >= n) return -1;
  const int nh = a.tup_n[track_row(a, i)];
  return nh >= kMinN && nh <= kMaxHits ? nh - kMinN : -1;
}

__global__ void __launch_bounds__(kBlock) k_bin(FitArgs a) {
  constexpr int kWaves = kBlock / kWave;
  __shared__ int32_t s_cnt[kWaves][kNBins];
  __shared__ int32_t s_run[kNBins];
  const int n = n_tracks(a);
  const int lane = __lane_id();
  const int w = static_cast<int>(threadIdx.x) / kWave;
  const uint64_t below = (uint64_t(1) << lane) - 1;
  const int per = ((n + gridDim.x - 1) / gridDim.x + kBlock - 1) / kBlock * kBlock;
  const int lo = blockIdx.x * per, hi = min(n, lo + per);
  // pass 1: counts of the block's range
  int cnt[kNBins];
#pragma unroll
  for (int b = 0; b < kNBins; ++b) cnt[b] = 0;
  for (int i0 = lo; i0 < hi; i0 += kBlock) {
    const int bin = track_bin(a, i0 + threadIdx.x, hi);
#pragma unroll
    for (int b = 0; b < kNBins; ++b) cnt[b] += __popcll(__ballot(bin == b));
  }
  if (lane == 0)
    for (int b = 0; b < kNBins; ++b) s_cnt[w][b] = cnt[b];
  __syncthreads();
  if (threadIdx.x < kNBins) {
    const int b = threadIdx.x;
    int c = 0;
    for (int q = 0; q < kWaves; ++q) c += s_cnt[q][b];
    s_run[b] = c ? atomicAdd(a.bin_count + b, c) : 0;
  }
  __syncthreads();
  // pass 2: place the tracks in order of the range
  for (int i0 = lo; i0 < hi; i0 += kBlock) {
    const int i = i0 + threadIdx.x;
    const int bin = track_bin(a, i, hi);
    int rank = 0;
#pragma unroll
    for (int b = 0; b < kNBins; ++b) {
      const uint64_t m = __ballot(bin == b);
      if (bin == b) rank = __popcll(m & below);
      if (lane == 0) s_cnt[w][b] = __popcll(m);
    }
    __syncthreads();
    if (bin >= 0) {
      int off = s_run[bin];
      for (int q = 0; q < w; ++q) off += s_cnt[q][bin];
      a.bins[static_cast<int64_t>(bin) * a.n_max + off + rank] = i;
    }
    __syncthreads();
    if (threadIdx.x < kNBins) {
      int c = 0;
      for (int q = 0; q < kWaves; ++q) c += s_cnt[q][threadIdx.x];
      s_run[threadIdx.x] += c;
    }
    __syncthreads();
  }
}

// Tracks with an invalid hit count get a failed status.
template <class OT>
__global__ void k_reject(FitArgs a) {
  const int n = n_tracks(a);
  uint32_t bad = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int nh = a.tup_n[track_row(a, i)];
    if (nh < kMinN || nh > kMaxHits) {
      OT* P = static_cast<OT*>(a.params) + static_cast<int64_t>(i) * 5;
      for (int q = 0; q < 5; ++q) P[q] = OT(NAN);
      static_cast<OT*>(a.chi2)[i] = OT(NAN);
      if (a.cov)
        for (int q = 0; q < 15; ++q) static_cast<OT*>(a.cov)[static_cast<int64_t>(i) * 15 + q] = OT(NAN);
      a.track_status[i] = fit::ST_FAILED;
      ++bad;
    }
  }
  if (bad) {
    status_add(a.status, PT_ST_FIT_FAILED, bad);
    status_flag(a.status, PT_FLAG_FIT_FAILED);
  }
}

// Gathers the hits of one track (P = hit + module offset, in double).
// Returns false when a hit or module index is out of range.
template <int N, class S, class HT>
__device__ inline bool load_track(const FitArgs& a, const uint8_t* layer_barrel, int row, fit::State<N, S>& f,
                                  int hit[N], int mod[N]) {
  const HT* X = static_cast<const HT*>(a.x);
  const HT* Y = static_cast<const HT*>(a.y);
  const HT* Z = static_cast<const HT*>(a.z);
  const int32_t* H = a.tup_hits + static_cast<int64_t>(row) * kMaxHits;
  double px[N], py[N], pz[N];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < N; ++k) {
    int h = H[k];
    if (h < 0 || h >= a.n_hits) {
      ok = false;
      h = 0;
    }
    hit[k] = h;
    px[k] = double(X[h]);
    py[k] = double(Y[h]);
    pz[k] = double(Z[h]);
    int m = a.module ? a.module[h] : 0;
    if (m < 0 || m >= a.n_modules) {
      ok = false;
      m = 0;
    }
    mod[k] = m;
    if (a.offsets) {
      const float* o = a.offsets + 3 * m;
      px[k] += double(o[0]);
      py[k] += double(o[1]);
      pz[k] += double(o[2]);
    }
    const int L = a.layer[h];
    f.barrel[k] = L < kLayers ? (layer_barrel[L] != 0) : true;
  }
  f.P0x = px[0];
  f.P0y = py[0];
  f.P0z = pz[0];
#pragma unroll
  for (int k = 0; k < N; ++k) {
    f.rx[k] = px[k] - px[0];
    f.ry[k] = py[k] - py[0];
    f.rz[k] = pz[k] - pz[0];
  }
  return ok;
}

// Forward fit of the tracks in bin N (LIST = false) or on the double-refit
// list (LIST = true, any N, dispatched at run time).
template <int N, class S, class HT, class OT, bool COV>
__device__ inline void fit_one(const DevCfg& k, const fit::Consts& C, const FitArgs& a, int i, bool fallback,
                               uint32_t& n_bad, uint32_t& n_fail, uint32_t& n_redo) {
  fit::State<N, S> f;
  int hit[N], mod[N];
  const bool ok = load_track<N, S, HT>(a, k.layer_barrel, track_row(a, i), f, hit, mod);
  if (ok) fit::forward<N, S>(C, f);
  OT* P = static_cast<OT*>(a.params) + static_cast<int64_t>(i) * 5;
  int st = ok ? f.status : fit::ST_FAILED;
  // Stiff systems, and systems whose single-precision solve broke down, are
  // solved again in double.
  if (fallback && ok && (st == fit::ST_FAILED || (st == fit::ST_OK && double(f.cond) > C.thr))) {
    const int slot = atomicAdd(a.redo_count, 1);
    a.redo[slot] = i;
    ++n_redo;
    return;  // written by the double-precision refit
  }
  if (st == fit::ST_OK) {
    P[0] = OT(f.kappa);
    P[1] = OT(f.phi0);
    P[2] = OT(f.cot);
    P[3] = OT(f.d0);
    P[4] = OT(f.z0);
    static_cast<OT*>(a.chi2)[i] = OT(f.chi2);
    if (COV) {
      double cv[15];
      fit::covariance<N, S>(f, cv);
      OT* V = static_cast<OT*>(a.cov) + static_cast<int64_t>(i) * 15;
#pragma unroll
      for (int q = 0; q < 15; ++q) V[q] = OT(cv[q]);
    }
  } else {
    for (int q = 0; q < 5; ++q) P[q] = OT(NAN);
    static_cast<OT*>(a.chi2)[i] = OT(NAN);
    if (COV)
      for (int q = 0; q < 15; ++q) static_cast<OT*>(a.cov)[static_cast<int64_t>(i) * 15 + q] = OT(NAN);
    if (st & fit::ST_BAD_ORDER) ++n_bad; else ++n_fail;
  }
  a.track_status[i] = static_cast<uint8_t>(st);
}

template <class HT>
__device__ inline void flush_counts(const FitArgs& a, uint32_t n_bad, uint32_t n_fail, uint32_t n_redo) {
  if (n_bad) {
    status_add(a.status, PT_ST_FIT_BAD_ORDER, n_bad);
    status_flag(a.status, PT_FLAG_FIT_BAD_ORDER);
  }
  if (n_fail) {
    status_add(a.status, PT_ST_FIT_FAILED, n_fail);
    status_flag(a.status, PT_FLAG_FIT_FAILED);
  }
  if (n_redo) status_add(a.status, PT_ST_FIT_F64, n_redo);
}

// Work item j of the bins NLO..NHI (in bin order) -> (N, track index).
template <int NLO, int NHI>
__device__ inline int bin_item(const FitArgs& a, int j, int& nh) {
  int base = 0;
#pragma unroll
  for (int N = NLO; N <= NHI; ++N) {
    const int c = a.bin_count[N - kMinN];
    if (j < base + c) {
      nh = N;
      return a.bins[static_cast<int64_t>(N - kMinN) * a.n_max + (j - base)];
    }
    base += c;
  }
  nh = 0;
  return -1;
}

template <int NLO, int NHI>
__device__ inline int bin_total(const FitArgs& a) {
  int t = 0;
#pragma unroll
  for (int N = NLO; N <= NHI; ++N) t += a.bin_count[N - kMinN];
  return t;
}

// Forward fit of the tracks with NLO..NHI hits.
template <int NLO, int NHI, class S, class HT, class OT, bool COV>
__global__ void __launch_bounds__(kBlock) k_fit(DevCfg k, FitArgs a, bool fallback) {
  const fit::Consts C = consts_of(k);
  const int m = bin_total<NLO, NHI>(a);
  uint32_t n_bad = 0, n_fail = 0, n_redo = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    int nh;
    const int i = bin_item<NLO, NHI>(a, j, nh);
    if (NLO <= 3 && 3 <= NHI && nh == 3) fit_one<3, S, HT, OT, COV>(k, C, a, i, fallback, n_bad, n_fail, n_redo);
    if (NLO <= 4 && 4 <= NHI && nh == 4) fit_one<4, S, HT, OT, COV>(k, C, a, i, fallback, n_bad, n_fail, n_redo);
    if (NLO <= 5 && 5 <= NHI && nh == 5) fit_one<5, S, HT, OT, COV>(k, C, a, i, fallback, n_bad, n_fail, n_redo);
    if (NLO <= 6 && 6 <= NHI && nh == 6) fit_one<6, S, HT, OT, COV>(k, C, a, i, fallback, n_bad, n_fail, n_redo);
    if (NLO <= 7 && 7 <= NHI && nh == 7) fit_one<7, S, HT, OT, COV>(k, C, a, i, fallback, n_bad, n_fail, n_redo);
    if (NLO <= 8 && 8 <= NHI && nh == 8) fit_one<8, S, HT, OT, COV>(k, C, a, i, fallback, n_bad, n_fail, n_redo);
  }
  flush_counts<HT>(a, n_bad, n_fail, n_redo);
}

// Double-precision refit of the listed tracks; outputs in OT.
template <class HT, class OT>
__global__ void __launch_bounds__(kRefitBlock) k_refit(DevCfg k, FitArgs a) {
  const fit::Consts C = consts_of(k);
  const int m = *a.redo_count;
  uint32_t n_bad = 0, n_fail = 0, n_redo = 0;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    const int i = a.redo[j];
    const int nh = a.tup_n[track_row(a, i)];
    switch (nh) {
      case 3:
        if (a.cov) fit_one<3, double, HT, OT, true>(k, C, a, i, false, n_bad, n_fail, n_redo);
        else fit_one<3, double, HT, OT, false>(k, C, a, i, false, n_bad, n_fail, n_redo);
        break;
      case 4:
        if (a.cov) fit_one<4, double, HT, OT, true>(k, C, a, i, false, n_bad, n_fail, n_redo);
        else fit_one<4, double, HT, OT, false>(k, C, a, i, false, n_bad, n_fail, n_redo);
        break;
      case 5:
        if (a.cov) fit_one<5, double, HT, OT, true>(k, C, a, i, false, n_bad, n_fail, n_redo);
        else fit_one<5, double, HT, OT, false>(k, C, a, i, false, n_bad, n_fail, n_redo);
        break;
      case 6:
        if (a.cov) fit_one<6, double, HT, OT, true>(k, C, a, i, false, n_bad, n_fail, n_redo);
        else fit_one<6, double, HT, OT, false>(k, C, a, i, false, n_bad, n_fail, n_redo);
        break;
      case 7:
        if (a.cov) fit_one<7, double, HT, OT, true>(k, C, a, i, false, n_bad, n_fail, n_redo);
        else fit_one<7, double, HT, OT, false>(k, C, a, i, false, n_bad, n_fail, n_redo);
        break;
      case 8:
        if (a.cov) fit_one<8, double, HT, OT, true>(k, C, a, i, false, n_bad, n_fail, n_redo);
        else fit_one<8, double, HT, OT, false>(k, C, a, i, false, n_bad, n_fail, n_redo);
        break;
      default: break;
    }
    a.track_status[i] |= fit::ST_F64;
  }
  flush_counts<HT>(a, n_bad, n_fail, n_redo);
}

// ---------------------------------------------------------------------------
// adjoint

// The hit gradients of the last track a thread took, added with device-scope
// atomics (or, when no hit is shared, stored as final sums) only once the
// next track's inputs have been loaded: one counter tracks loads, stores and
// atomics alike, so a load issued after them would wait for them to
// complete.
template <class GT>
struct PendingGrad {
  int n = 0;
  int hit[kMaxHits];
  GT g[kMaxHits][3];
};

template <class GT>
__device__ inline void flush_pending(PendingGrad<GT>& p, void* grad_hits, bool exclusive) {
#pragma unroll
  for (int kk = 0; kk < kMaxHits; ++kk) {
    if (kk < p.n) {
      GT* gh = static_cast<GT*>(grad_hits) + static_cast<int64_t>(p.hit[kk]) * 3;
      if (exclusive) {
        gh[0] = p.g[kk][0];
        gh[1] = p.g[kk][1];
        gh[2] = p.g[kk][2];
      } else {
        unsafeAtomicAdd(gh + 0, p.g[kk][0]);
        unsafeAtomicAdd(gh + 1, p.g[kk][1]);
        unsafeAtomicAdd(gh + 2, p.g[kk][2]);
      }
    }
  }
  p.n = 0;
}

template <class GT>
__device__ inline void load_cotangents(const FitArgs& a, int i, GT (&g)[6]) {
  const GT* gp = static_cast<const GT*>(a.g_params) + static_cast<int64_t>(i) * 5;
#pragma unroll
  for (int q = 0; q < 5; ++q) g[q] = gp[q];
  g[5] = a.g_chi2 ? static_cast<const GT*>(a.g_chi2)[i] : GT(0);
}

template <int N, class S, class HT, class GT>
__device__ inline void grad_one(const DevCfg& k, const fit::Consts& C, const FitArgs& a, int i, bool fallback,
                                double* lds_mod, uint32_t& n_redo, PendingGrad<GT>& pend) {
  // deferred in the float adjoint of four or more hits only (the double
  // state leaves no registers for it; three hits keep two wavefronts per SIMD)
  constexpr bool kDefer = std::is_same<S, float>::value && std::is_same<GT, float>::value && N > 3;
  fit::State<N, S> f;
  int hit[N], mod[N];
  const bool ok = load_track<N, S, HT>(a, k.layer_barrel, track_row(a, i), f, hit, mod);
  GT gin[6];
  if (kDefer) load_cotangents(a, i, gin);
  if (kDefer && pend.n) flush_pending(pend, a.grad_hits, k.exclusive_hits);  // the previous track's, after this one's loads
  if (!ok) return;
  fit::forward<N, S>(C, f);
  if (fallback && (f.status == fit::ST_FAILED || (f.status == fit::ST_OK && double(f.cond) > C.thr))) {
    const int slot = atomicAdd(a.redo_count, 1);
    a.redo[slot] = i;
    ++n_redo;
    return;
  }
  if (f.status != fit::ST_OK) return;
  if (!kDefer) load_cotangents(a, i, gin);
  double g[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) g[q] = double(gin[q]);
  S gP[N][3];
  fit::backward<N, S>(C, f, g, gP);
  if (a.grad_hits && k.exclusive_hits) {
    // the row is this track's alone, its hits distinct: every load before
    // the first store, so that no load waits for a store
    GT cur[N][3];
#pragma unroll
    for (int kk = 0; kk < N; ++kk) {
      const GT* gh = static_cast<const GT*>(a.grad_hits) + static_cast<int64_t>(hit[kk]) * 3;
      cur[kk][0] = gh[0];
      cur[kk][1] = gh[1];
      cur[kk][2] = gh[2];
    }
#pragma unroll
    for (int kk = 0; kk < N; ++kk) {
      if (kDefer) {
        pend.hit[kk] = hit[kk];
        pend.g[kk][0] = cur[kk][0] + GT(gP[kk][0]);
        pend.g[kk][1] = cur[kk][1] + GT(gP[kk][1]);
        pend.g[kk][2] = cur[kk][2] + GT(gP[kk][2]);
      } else {
        GT* gh = static_cast<GT*>(a.grad_hits) + static_cast<int64_t>(hit[kk]) * 3;
        gh[0] = cur[kk][0] + GT(gP[kk][0]);
        gh[1] = cur[kk][1] + GT(gP[kk][1]);
        gh[2] = cur[kk][2] + GT(gP[kk][2]);
      }
    }
  }
#pragma unroll
  for (int kk = 0; kk < N; ++kk) {
    if (a.grad_hits && !k.exclusive_hits) {
      if (kDefer) {
        pend.hit[kk] = hit[kk];
        pend.g[kk][0] = GT(gP[kk][0]);
        pend.g[kk][1] = GT(gP[kk][1]);
        pend.g[kk][2] = GT(gP[kk][2]);
      } else {
        GT* gh = static_cast<GT*>(a.grad_hits) + static_cast<int64_t>(hit[kk]) * 3;
        unsafeAtomicAdd(gh + 0, GT(gP[kk][0]));
        unsafeAtomicAdd(gh + 1, GT(gP[kk][1]));
        unsafeAtomicAdd(gh + 2, GT(gP[kk][2]));
      }
    }
    if (lds_mod) {
      double* lm = lds_mod + 3 * mod[kk];
      atomicAdd(lm + 0, double(gP[kk][0]));
      atomicAdd(lm + 1, double(gP[kk][1]));
      atomicAdd(lm + 2, double(gP[kk][2]));
    }
  }
  if (kDefer && a.grad_hits) pend.n = N;
}

__device__ inline void lds_clear(double* lds, int n) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) lds[q] = 0.0;
  __syncthreads();
}

// Writes (FIRST) or adds the block's module sums to its partial row.  Blocks
// that processed no track skip the add.
template <bool FIRST>
__device__ inline void lds_flush(const double* lds, int n, bool any, double* dst) {
  const int busy = __syncthreads_or(any ? 1 : 0);
  if (!FIRST && !busy) return;
  for (int q = threadIdx.x; q < n; q += blockDim.x) {
    if (FIRST) dst[q] = lds[q]; else dst[q] += lds[q];
  }
}

// The adjoint of the tracks with NLO..NHI hits.  Grid: kBwdBlocks persistent
// blocks, block b owning the partial module sums partials[b].  The kernel
// with FIRST = true runs first and initialises every partial row.
template <int NLO, int NHI, bool FIRST, class S, class HT, class GT>
__global__ void __launch_bounds__(kBlock) k_grad(DevCfg k, FitArgs a, bool fallback) {
  extern __shared__ double lds_mod[];
  const fit::Consts C = consts_of(k);
  const int nm3 = a.partials ? a.n_modules * 3 : 0;
  if (nm3) lds_clear(lds_mod, nm3);
  double* lm = nm3 ? lds_mod : nullptr;
  const int m = bin_total<NLO, NHI>(a);
  uint32_t n_redo = 0;
  bool any = false;
  PendingGrad<GT> pend;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    int nh;
    const int i = bin_item<NLO, NHI>(a, j, nh);
    any = true;
    if (NLO <= 3 && 3 <= NHI && nh == 3) grad_one<3, S, HT, GT>(k, C, a, i, fallback, lm, n_redo, pend);
    if (NLO <= 4 && 4 <= NHI && nh == 4) grad_one<4, S, HT, GT>(k, C, a, i, fallback, lm, n_redo, pend);
    if (NLO <= 5 && 5 <= NHI && nh == 5) grad_one<5, S, HT, GT>(k, C, a, i, fallback, lm, n_redo, pend);
    if (NLO <= 6 && 6 <= NHI && nh == 6) grad_one<6, S, HT, GT>(k, C, a, i, fallback, lm, n_redo, pend);
    if (NLO <= 7 && 7 <= NHI && nh == 7) grad_one<7, S, HT, GT>(k, C, a, i, fallback, lm, n_redo, pend);
    if (NLO <= 8 && 8 <= NHI && nh == 8) grad_one<8, S, HT, GT>(k, C, a, i, fallback, lm, n_redo, pend);
  }
  if (pend.n) flush_pending(pend, a.grad_hits, k.exclusive_hits);
  if (nm3) lds_flush<FIRST>(lds_mod, nm3, any, a.partials + static_cast<int64_t>(blockIdx.x) * nm3);
}

template <class HT>
__global__ void __launch_bounds__(kBlock) k_regrad(DevCfg k, FitArgs a) {
  extern __shared__ double lds_mod[];
  const fit::Consts C = consts_of(k);
  const int nm3 = a.partials ? a.n_modules * 3 : 0;
  if (nm3) lds_clear(lds_mod, nm3);
  const int m = *a.redo_count;
  uint32_t n_redo = 0;
  double* lm = nm3 ? lds_mod : nullptr;
  bool any = false;
  PendingGrad<float> pend;
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    const int i = a.redo[j];
    any = true;
    switch (a.tup_n[track_row(a, i)]) {
      case 3: grad_one<3, double, HT, float>(k, C, a, i, false, lm, n_redo, pend); break;
      case 4: grad_one<4, double, HT, float>(k, C, a, i, false, lm, n_redo, pend); break;
      case 5: grad_one<5, double, HT, float>(k, C, a, i, false, lm, n_redo, pend); break;
      case 6: grad_one<6, double, HT, float>(k, C, a, i, false, lm, n_redo, pend); break;
      case 7: grad_one<7, double, HT, float>(k, C, a, i, false, lm, n_redo, pend); break;
      case 8: grad_one<8, double, HT, float>(k, C, a, i, false, lm, n_redo, pend); break;
      default: break;
    }
  }
  if (pend.n) flush_pending(pend, a.grad_hits, k.exclusive_hits);
  if (nm3) lds_flush<false>(lds_mod, nm3, any, a.partials + static_cast<int64_t>(blockIdx.x) * nm3);
}

// grad_offsets[q] += sum over blocks of partials[b][q]: each of the
// kRedWaves wavefronts of a block sums the rows b = w, w + kRedWaves, ... of
// 64 consecutive q in order, and the wavefronts' sums are added in order
// (a fixed order, the same on every run).
constexpr int kRedWaves = 16;

__global__ void __launch_bounds__(kRedWaves * kWave) k_reduce_modules(const double* __restrict__ partials, int nm3,
                                                                      int nblocks, double* __restrict__ out) {
  __shared__ double s_part[kRedWaves][kWave];
  const int lane = __lane_id();
  const int w = static_cast<int>(threadIdx.x) / kWave;
  const int q = blockIdx.x * kWave + lane;
  double s = 0.0;
  if (q < nm3)
    for (int b = w; b < nblocks; b += kRedWaves) s += partials[static_cast<int64_t>(b) * nm3 + q];
  s_part[w][lane] = s;
  __syncthreads();
  if (w == 0 && q < nm3) {
    double t = 0.0;
    for (int v = 0; v < kRedWaves; ++v) t += s_part[v][lane];
    out[q] += t;
  }
}

int fit_grid(int n_max) { return grid_for(n_max, kBlock, 4096); }

}  // namespace

// Workspace of the forward fit (with_partials = false) or of the adjoint.
static size_t fit_scratch_bytes(int n_max, int n_modules, bool with_partials) {
  Carver c(nullptr);
  c.take<int32_t>(static_cast<size_t>(kNBins) * n_max);
  c.take<int32_t>(kNBins);
  c.take<int32_t>(n_max);
  c.take<int32_t>(1);
  if (with_partials) c.take<double>(static_cast<size_t>(kBwdBlocks) * n_modules * 3);
  return c.off + 256;
}

size_t ws_fit(int n_max, int n_modules) { return fit_scratch_bytes(n_max, n_modules, true); }

static FitArgs make_args(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, const float* offsets,
                         int n_max, pt_workspace ws, uint32_t* status, bool with_partials = true) {
  Carver c(ws.ptr);
  FitArgs a{};
  a.dtype = h.dtype;
  a.n_hits = h.n_hits;
  a.x = h.x;
  a.y = h.y;
  a.z = h.z;
  a.layer = h.layer;
  a.module = h.module;
  a.offsets = offsets;
  a.n_modules = k.n_modules;
  a.tup_hits = T.hits;
  a.tup_n = T.n;
  a.kept = T.kept;
  a.count = T.count;
  a.n_max = n_max;
  a.bins = c.take<int32_t>(static_cast<size_t>(kNBins) * n_max);
  a.bin_count = c.take<int32_t>(kNBins);
  a.redo = c.take<int32_t>(n_max);
  a.redo_count = c.take<int32_t>(1);
  a.partials = with_partials ? c.take<double>(static_cast<size_t>(kBwdBlocks) * k.n_modules * 3) : nullptr;
  a.status = status;
  return a;
}

static pt_err prepare(FitArgs& a, hipStream_t s) {
  PT_HIP_CHECK(fill_i32(a.bin_count, 0, kNBins, s));
  PT_HIP_CHECK(fill_i32(a.redo_count, 0, 1, s));
  k_bin<<<std::min(fit_grid(a.n_max), kBinBlocks), kBlock, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

template <class S, class HT, class OT>
static pt_err run_fit(const DevCfg& k, FitArgs& a, bool fallback, hipStream_t s) {
  const int g = fit_grid(a.n_max);
  k_reject<OT><<<g, kBlock, 0, s>>>(a);
  if (a.cov) {
    k_fit<4, 6, S, HT, OT, true><<<g, kBlock, 0, s>>>(k, a, fallback);
    k_fit<3, 3, S, HT, OT, true><<<g, kBlock, 0, s>>>(k, a, fallback);
    k_fit<7, 8, S, HT, OT, true><<<g, kBlock, 0, s>>>(k, a, fallback);
  } else {
    k_fit<4, 6, S, HT, OT, false><<<g, kBlock, 0, s>>>(k, a, fallback);
    k_fit<3, 3, S, HT, OT, false><<<g, kBlock, 0, s>>>(k, a, fallback);
    k_fit<7, 8, S, HT, OT, false><<<g, kBlock, 0, s>>>(k, a, fallback);
  }
  PT_LAUNCH_CHECK();
  if (fallback) {
    // one thread per refitted track (a few percent of the tracks)
    k_refit<HT, OT><<<grid_for(a.n_max / 16 + 1, kRefitBlock, 1024), kRefitBlock, 0, s>>>(k, a);
    PT_LAUNCH_CHECK();
  }
  return PT_OK;
}

pt_err launch_fit(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, const float* offsets, int precision,
                  pt_tracks& out, uint32_t* status, pt_workspace ws, hipStream_t s) {
  const int n_max = std::min(T.cap, out.cap);
  FitArgs a = make_args(h, k, T, offsets, n_max, ws, status, false);
  a.params = out.params;
  a.chi2 = out.chi2;
  a.track_status = out.status;
  a.cov = out.cov;
  // one timing region over every kernel of the forward fit
  void* tok = timing_begin(s);
  pt_err e = prepare(a, s);
  if (e == PT_OK) {
    const bool f64in = h.dtype == PT_F64;
    const bool fb = precision == PT_FIT_F32_F64SOLVE;
    if (precision == PT_FIT_F64)
      e = f64in ? run_fit<double, double, double>(k, a, false, s) : run_fit<double, float, double>(k, a, false, s);
    else
      e = f64in ? run_fit<float, double, float>(k, a, fb, s) : run_fit<float, float, float>(k, a, fb, s);
  }
  timing_end(tok, "fit_fwd", s);
  return e;
}

template <class S, class HT, class GT>
static pt_err run_grad(const DevCfg& k, FitArgs& a, bool fallback, double* grad_offsets, hipStream_t s) {
  const size_t lds = a.partials ? static_cast<size_t>(a.n_modules) * 3 * sizeof(double) : 0;
  const int nm3 = a.n_modules * 3;
  k_grad<4, 6, true, S, HT, GT><<<kBwdBlocks, kBlock, lds, s>>>(k, a, fallback);
  k_grad<3, 3, false, S, HT, GT><<<kBwdBlocks, kBlock, lds, s>>>(k, a, fallback);
  k_grad<7, 8, false, S, HT, GT><<<kBwdBlocks, kBlock, lds, s>>>(k, a, fallback);
  PT_LAUNCH_CHECK();
  if (fallback) {
    k_regrad<HT><<<kBwdBlocks, kBlock, lds, s>>>(k, a);
    PT_LAUNCH_CHECK();
  }
  if (a.partials) {
    k_reduce_modules<<<(nm3 + kWave - 1) / kWave, kRedWaves * kWave, 0, s>>>(a.partials, nm3, kBwdBlocks,
                                                                         grad_offsets);
    PT_LAUNCH_CHECK();
  }
  return PT_OK;
}

pt_err launch_fit_bwd(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, const float* offsets, int precision,
                      const void* g_params, const void* g_chi2, void* grad_hits, double* grad_offsets,
                      int n_max, uint32_t* status, pt_workspace ws, hipStream_t s) {
  FitArgs a = make_args(h, k, T, offsets, n_max, ws, status);
  a.g_params = g_params;
  a.g_chi2 = g_chi2;
  a.grad_hits = grad_hits;
  if (!grad_offsets) a.partials = nullptr;
  // one timing region over every kernel of the adjoint
  void* tok = timing_begin(s);
  pt_err e = prepare(a, s);
  if (e == PT_OK) {
    const bool f64in = h.dtype == PT_F64;
    const bool fb = precision == PT_FIT_F32_F64SOLVE;
    if (precision == PT_FIT_F64)
      e = f64in ? run_grad<double, double, double>(k, a, false, grad_offsets, s)
                : run_grad<double, float, double>(k, a, false, grad_offsets, s);
    else
      e = f64in ? run_grad<float, double, float>(k, a, fb, grad_offsets, s)
                : run_grad<float, float, float>(k, a, fb, grad_offsets, s);
  }
  timing_end(tok, "fit_bwd", s);
  return e;
}

// ---------------------------------------------------------------------------
// The forward fit without a caller workspace, for callers that cannot
// allocate (graph capture, tight serving loops).  Its scratch (track bins and
// the double-refit list) is a file-scope device array of fixed size, one per
// GPU, held until the process ends.  Calls on one GPU share it: calls that
// overlap in time on one GPU race.  The counters it must start from zero are
// cleared by fill kernels at the start of every call.

constexpr size_t kStaticScratchBytes = 7340800;  // >= fit_scratch_bytes(PT_NOALLOC_FIT_MAX_TRACKS, -, false)
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of this GPU's scratch array (looked up once per device,
// with that device current).  Null on failure.
static void* static_scratch(hipError_t* err) {
  int dev = 0;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

pt_err launch_fit_noalloc(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, const float* offsets,
                         int precision, pt_tracks& out, uint32_t* status, hipStream_t s) {
  const int n_max = std::min(T.cap, out.cap);
  if (n_max > PT_NOALLOC_FIT_MAX_TRACKS) return PT_ERR_TOO_LARGE;
  static_assert(kStaticScratchBytes >= 6 * 4 * size_t(PT_NOALLOC_FIT_MAX_TRACKS) + 4 * size_t(PT_NOALLOC_FIT_MAX_TRACKS),
                "scratch smaller than the forward fit needs");
  if (fit_scratch_bytes(n_max, k.n_modules, false) > kStaticScratchBytes) return PT_ERR_TOO_LARGE;
  hipError_t err = hipSuccess;
  void* p = static_scratch(&err);
  if (!p) return device_error(err);
  const bool was = g_no_timing;
  g_no_timing = true;  // timing records create events: not here
  const pt_err e = launch_fit(h, k, T, offsets, precision, out, status, pt_workspace{p, kStaticScratchBytes}, s);
  g_no_timing = was;
  return e;
}

}  // namespace pt
