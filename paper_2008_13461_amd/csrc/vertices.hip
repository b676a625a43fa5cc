// Pixel vertices (paper section 3.6): clusters of the fitted tracks in z0.
//
// Tracks take part when they were selected by the ambiguity resolution, have
// at least vtx_min_hits hits, p_T above vtx_pt_min and a finite z0 with a
// positive variance (the (z0, z0) element of their covariance).  Per event:
//   * the local density of a track (computed only when its sigma(z0) is at
//     most vtx_err_max): the other tracks within vtx_dz_cut in z0 whose
//     compatibility (dz)^2 / (var_i + var_j) is below vtx_chi2_max;
//   * each track links to the nearest track of higher rank (density, then
//     track index) within the same window with compatibility at most
//     vtx_chi2_max; links climb in rank, so they form trees;
//   * a tree whose root has density > 1 (a seed) and at least 2 tracks is a
//     vertex: weighted mean of z0 (weights 1/var), its variance and chi2;
//   * a vertex with chi2/ndf > vtx_split_chi2_ndf is split in two by 1-D
//     two-means (centres from its extreme members, at most vtx_kmeans_iter
//     rounds); parts of one track are dropped;
//   * the event's vertices are ordered by the sum of min(p_T, vtx_pt_cap)^2
//     of their tracks, largest (the primary) first.
// All sums run over a vertex's members in the order of (z0, track index),
// sequentially in one thread, in double without contraction, so that the
// result is reproducible and the decisions of the split are exact.
//
// GPU layout: the tracks of each event are gathered into a contiguous list
// (count, scan, scatter), then one work-group per event sorts its list by
// (z0, track index) -- a bitonic sort in LDS, or in global scratch for
// events with more tracks than the LDS holds -- so that every window in z0
// is a contiguous range of the sorted list.  Everything after the sort is
// flat over the sorted positions of all events at once: densities and
// links one thread per position over its window, roots by following the
// links, one thread per tree for its fit (and split).  A second work-group
// per event orders its vertices by their key, and the writes are flat again.
#include <algorithm>

#include "pt_internal.h"

#pragma clang fp contract(off)

namespace pt {
namespace {

constexpr int kBlock = 1024;
constexpr int kLdsSort = 8192;  // entries sorted in LDS (12 bytes each: 96 KB)

struct VtxArgs {
  // tracks
  const int32_t* hits;   // rows [cap][kMaxHits]
  const uint8_t* n;
  const int32_t* kept;
  const int32_t* count;
  int32_t n_max;
  const void* params;    // [n_max][5]
  const void* cov;       // [n_max][15]
  int32_t dbl;
  const int32_t* selected;    // may be null: every track
  const int32_t* n_selected;
  // events
  const int32_t* event_offsets;
  int32_t n_events;
  int32_t n_hits;
  // settings
  int32_t min_hits, kmeans_iter;
  double pt_min, err_max, dz_cut, chi2_max, split, pt_cap, K;
  // scratch, [n_max] unless noted
  uint8_t* use;
  int32_t* ev_of;        // event of each track, -1 when it takes no part
  int32_t* ev_count;     // [n_events + 1], scanned in place into the starts
  int32_t* ev_cursor;    // [n_events]
  int32_t* list;         // tracks grouped by event
  uint64_t* skey;        // [2 n_max] sort keys (padded per event)
  int32_t* sval;         // [2 n_max]
  double* sz;            // sorted z0
  double* sv;            // sorted variance
  int32_t* sidx;         // sorted track index
  int32_t* pev;          // event of each sorted position
  int32_t* rho;
  int32_t* parent;
  int32_t* root;
  int32_t* tsize;        // tree size, per root position
  int32_t* tlo;          // first member position, per root
  int32_t* thi;          // last member position, per root
  uint8_t* side;
  // per event vertex records (at the event's list offset, at most one per track)
  double* rz;
  double* rvar;
  double* rchi2;
  double* rsum;
  int32_t* rndf;
  int32_t* rn;
  int32_t* rfirst;       // first member position (identifies the record)
  int32_t* rslot;        // per position: event-local slot of the record whose first member it is
  int32_t* rrank;        // per record slot: rank of the vertex in its event
  int32_t* rec0;         // per root position: record slot of the whole tree, -1
  int32_t* rec1;         // per root position: record slots of the two parts of a split tree, -1
  int32_t* rec2;
  int32_t* vlocal;       // per position: rank of the track's vertex in its event, -1
  int32_t* ev_nvtx;      // [n_events + 1] records per event, scanned into the first vertex of each event
  // outputs
  double *oz, *ovar, *ochi2, *osum;
  int32_t *ondf, *on;
  int32_t* event_first;  // [n_events + 1]
  int32_t* n_vertices;   // [1]
  int32_t* track_vertex; // [n_max]
  int32_t cap;
  uint32_t* status;
};

__device__ inline int n_tracks(const VtxArgs& a) { return min(*a.count, a.n_max); }

__device__ inline double val(const void* p, int64_t i, int dbl) {
  return dbl ? static_cast<const double*>(p)[i] : double(static_cast<const float*>(p)[i]);
}

// Key whose unsigned order is the numeric order of the double.
__device__ inline uint64_t order_key(double v) {
  const uint64_t b = static_cast<uint64_t>(__double_as_longlong(v));
  return (b >> 63) ? ~b : (b | (uint64_t(1) << 63));
}

// ---------------------------------------------------------------------------
// tracks -> events

// Adds the active lanes with key e >= 0 to cnt[e], one atomic per distinct
// key in the wavefront (tracks come grouped by event, so mostly one), and
// returns each lane's slot (the old count plus its rank among the lanes of
// its key), -1 for e < 0.  Called by every active lane of the wavefront.
__device__ inline int wave_add(int32_t* cnt, int e) {
  const int lane = __lane_id();
  int slot = -1;
  uint64_t todo = __ballot(e >= 0);
  while (todo) {  // wave-uniform
    const int leader = __builtin_ctzll(todo);
    const int e0 = __shfl(e, leader);
    const uint64_t grp = __ballot(e == e0) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(cnt + e0, __popcll(grp));
    base = __shfl(base, leader);
    if ((grp >> lane) & 1) slot = base + __popcll(grp & ((uint64_t(1) << lane) - 1));
    todo &= ~grp;
  }
  return slot;
}

__global__ void k_vtx_clear(VtxArgs a) {
  const int n = a.n_max;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    a.use[i] = a.selected ? 0 : 1;
    a.track_vertex[i] = -1;
  }
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e <= a.n_events; e += gridDim.x * blockDim.x) {
    a.ev_count[e] = 0;
    a.ev_nvtx[e] = 0;
    if (e < a.n_events) a.ev_cursor[e] = 0;
  }
}

__global__ void k_vtx_mark(VtxArgs a) {
  const int m = min(*a.n_selected, a.n_max);
  const int n = n_tracks(a);
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < m; j += gridDim.x * blockDim.x) {
    const int i = a.selected[j];
    if (i >= 0 && i < n) a.use[i] = 1;
  }
}

__global__ void k_vtx_events(VtxArgs a) {
  const int n = n_tracks(a);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int e = -1;
    const int row = a.kept ? a.kept[i] : i;
    const int nh = a.n[row];
    const double kap = val(a.params, static_cast<int64_t>(i) * 5 + 0, a.dbl);
    const double z = val(a.params, static_cast<int64_t>(i) * 5 + 4, a.dbl);
    const double v = val(a.cov, static_cast<int64_t>(i) * 15 + 14, a.dbl);
    const double pt = a.K / fabs(kap);
    const int h0 = a.hits[static_cast<int64_t>(row) * kMaxHits];
    if (a.use[i] && nh >= a.min_hits && pt > a.pt_min && isfinite(z) && isfinite(v) && v > 0.0 && h0 >= 0 &&
        h0 < a.n_hits) {
      // the event owning the first hit: the last e with event_offsets[e] <= h0
      int lo = 0, hi = a.n_events - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.event_offsets[mid] <= h0) lo = mid; else hi = mid - 1;
      }
      if (a.n_events > 0 && a.event_offsets[lo] <= h0 && h0 < a.event_offsets[lo + 1]) e = lo;
    }
    a.ev_of[i] = e;
    wave_add(a.ev_count, e);
  }
}

__global__ void k_vtx_scatter(VtxArgs a) {
  const int n = n_tracks(a);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int e = a.ev_of[i];
    const int slot = wave_add(a.ev_cursor, e);
    if (e >= 0) a.list[a.ev_count[e] + slot] = i;
  }
}

// ---------------------------------------------------------------------------
// one work-group per event

// Ascending bitonic sort of (key, val) pairs, P a power of two, by the whole
// block; key and val may point to LDS or to global memory.
__device__ void bitonic(uint64_t* key, int32_t* v, int P) {
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < P / 2; t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t kl = key[lo], kh = key[hi];
        const int32_t vl = v[lo], vh = v[hi];
        const bool gt = kl > kh || (kl == kh && vl > vh);
        if (gt == asc) {
          key[lo] = kh;
          key[hi] = kl;
          v[lo] = vh;
          v[hi] = vl;
        }
      }
      __syncthreads();
    }
  }
}

__device__ inline int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// Sorts the n pairs at (key, v) (room for the padding to a power of two
// given), in LDS when they fit.
__device__ void sort_pairs(uint64_t* key, int32_t* v, int n, uint64_t* lkey, int32_t* lval) {
  const int P = pow2_at_least(max(n, 2));
  for (int k = n + threadIdx.x; k < P; k += blockDim.x) {
    key[k] = ~uint64_t(0);
    v[k] = 0x7fffffff;
  }
  __syncthreads();
  if (P <= kLdsSort) {
    for (int k = threadIdx.x; k < P; k += blockDim.x) {
      lkey[k] = key[k];
      lval[k] = v[k];
    }
    __syncthreads();
    bitonic(lkey, lval, P);
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
      key[k] = lkey[k];
      v[k] = lval[k];
    }
  } else {
    bitonic(key, v, P);
  }
  __syncthreads();
}

// Fit of the members of tree r (positions lo..hi whose root is r, and, for
// part p > 0, whose side is p - 1) by one wavefront: lanes scan 64
// consecutive positions at a time and the sums run over the members in
// position order (each member's term taken from its lane in turn), the same
// additions in the same order as one thread walking the members.
struct VFit {
  double z, var, chi2, sum;
  int n, first;
};

__device__ inline bool member(const VtxArgs& a, int q, int hi, int r, int part) {
  return q <= hi && a.root[q] == r && (part == 0 || a.side[q] == part - 1);
}

__device__ inline VFit wave_fit(const VtxArgs& a, int r, int lo, int hi, int part, int lane) {
  VFit f;
  f.n = 0;
  f.first = -1;
  double W = 0.0, S = 0.0;
  for (int c = lo; c <= hi; c += kWave) {
    const int q = c + lane;
    const bool m = member(a, q, hi, r, part);
    double w = 0.0, wz = 0.0;
    if (m) {
      w = 1.0 / a.sv[q];
      wz = w * a.sz[q];
    }
    uint64_t bits = __ballot(m);
    if (bits && f.first < 0) f.first = c + __builtin_ctzll(bits);
    f.n += __popcll(bits);
    while (bits) {
      const int l = __builtin_ctzll(bits);
      bits &= bits - 1;
      W = W + __shfl(w, l);
      S = S + __shfl(wz, l);
    }
  }
  f.z = S / W;
  f.var = 1.0 / W;
  double c2 = 0.0, s2 = 0.0;
  for (int c = lo; c <= hi; c += kWave) {
    const int q = c + lane;
    const bool m = member(a, q, hi, r, part);
    double tc = 0.0, tp = 0.0;
    if (m) {
      const double d = a.sz[q] - f.z;
      tc = (d * d) / a.sv[q];
      const int i = a.sidx[q];
      const double pt = a.K / fabs(val(a.params, static_cast<int64_t>(i) * 5 + 0, a.dbl));
      const double p = pt < a.pt_cap ? pt : a.pt_cap;
      tp = p * p;
    }
    uint64_t bits = __ballot(m);
    while (bits) {
      const int l = __builtin_ctzll(bits);
      bits &= bits - 1;
      c2 = c2 + __shfl(tc, l);
      s2 = s2 + __shfl(tp, l);
    }
  }
  f.chi2 = c2;
  f.sum = s2;
  return f;
}

__device__ inline void put_record(const VtxArgs& a, int64_t slot, const VFit& f) {
  a.rz[slot] = f.z;
  a.rvar[slot] = f.var;
  a.rchi2[slot] = f.chi2;
  a.rsum[slot] = f.sum;
  a.rndf[slot] = f.n - 1;
  a.rn[slot] = f.n;
  a.rfirst[slot] = f.first;
}

// ---- one work-group per event: sort its tracks by (z0, track index)
__global__ void __launch_bounds__(kBlock) k_vtx_sort(VtxArgs a) {
  __shared__ uint64_t lkey[kLdsSort];
  __shared__ int32_t lval[kLdsSort];
  const int e = blockIdx.x;
  const int64_t b = a.ev_count[e];             // the event's first list entry
  const int n = a.ev_count[e + 1] - a.ev_count[e];
  if (n == 0) return;
  uint64_t* key = a.skey + 2 * b;
  int32_t* sv = a.sval + 2 * b;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int i = a.list[b + k];
    key[k] = order_key(val(a.params, static_cast<int64_t>(i) * 5 + 4, a.dbl));
    sv[k] = i;
  }
  __syncthreads();
  sort_pairs(key, sv, n, lkey, lval);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    const int i = sv[k];
    const int64_t p = b + k;
    a.sidx[p] = i;
    a.sz[p] = val(a.params, static_cast<int64_t>(i) * 5 + 4, a.dbl);
    a.sv[p] = val(a.cov, static_cast<int64_t>(i) * 15 + 14, a.dbl);
    a.pev[p] = e;
    a.tsize[p] = 0;
    a.tlo[p] = 0x7fffffff;
    a.thi[p] = -1;
    a.rec0[p] = -1;
    a.rec1[p] = -1;
    a.rec2[p] = -1;
  }
}

// ---- flat over the sorted positions of every event

__device__ inline int positions(const VtxArgs& a) { return a.ev_count[a.n_events]; }

__global__ void k_vtx_density(VtxArgs a) {
  const int total = positions(a);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < total; p += gridDim.x * blockDim.x) {
    const int e = a.pev[p];
    const int lo = a.ev_count[e], hi = a.ev_count[e + 1];
    const double zk = a.sz[p], vk = a.sv[p];
    int c = 0;
    if (sqrt(vk) <= a.err_max) {
      for (int j = p - 1; j >= lo; --j) {
        const double d = zk - a.sz[j];
        if (!(fabs(d) < a.dz_cut)) break;
        if (d * d < a.chi2_max * (vk + a.sv[j])) ++c;
      }
      for (int j = p + 1; j < hi; ++j) {
        const double d = zk - a.sz[j];
        if (!(fabs(d) < a.dz_cut)) break;
        if (d * d < a.chi2_max * (vk + a.sv[j])) ++c;
      }
    }
    a.rho[p] = c;
  }
}

// Link to the nearest higher-ranked compatible track (-1: none).
__global__ void k_vtx_parent(VtxArgs a) {
  const int total = positions(a);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < total; p += gridDim.x * blockDim.x) {
    const int e = a.pev[p];
    const int lo = a.ev_count[e], hi = a.ev_count[e + 1];
    const double zk = a.sz[p], vk = a.sv[p];
    const int rk = a.rho[p], ik = a.sidx[p];
    int best = -1, ib = 0;
    double bd = 0.0;
    for (int dir = -1; dir <= 1; dir += 2) {
      for (int j = p + dir; j >= lo && j < hi; j += dir) {
        const double d = zk - a.sz[j];
        if (!(fabs(d) < a.dz_cut)) break;
        const int rj = a.rho[j], ij = a.sidx[j];
        const bool higher = rj > rk || (rj == rk && ij > ik);
        if (!higher || !(d * d <= a.chi2_max * (vk + a.sv[j]))) continue;
        const double ad = fabs(d);
        if (best < 0 || ad < bd || (ad == bd && ij < ib)) {
          best = j;
          bd = ad;
          ib = ij;
        }
      }
    }
    a.parent[p] = best;
  }
}

// Root of each position's tree (links climb in rank, so the walk ends), and
// each tree's size and range of positions.
__global__ void k_vtx_root(VtxArgs a) {
  const int total = positions(a);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < total; p += gridDim.x * blockDim.x) {
    const int e = a.pev[p];
    const int steps = a.ev_count[e + 1] - a.ev_count[e];
    int r = p;
    for (int s = 0; s < steps; ++s) {
      const int q = a.parent[r];
      if (q < 0) break;
      r = q;
    }
    a.root[p] = r;
    atomicAdd(a.tsize + r, 1);
    atomicMin(a.tlo + r, p);
    atomicMax(a.thi + r, p);
  }
}

// One wavefront per tree (the trees rooted in each run of 64 positions in
// turn): fit, split, records (in the event's record slots, taken by lane 0).
__device__ inline void record(const VtxArgs& a, int e, int64_t eb, const VFit& f, int32_t* rec, int r, int lane) {
  if (lane == 0) {
    const int64_t slot = eb + atomicAdd(a.ev_nvtx + e, 1);
    put_record(a, slot, f);
    rec[r] = static_cast<int32_t>(slot);
  }
}

__device__ inline void wave_tree(const VtxArgs& a, int r, int lane) {
  const double* z = a.sz;
  const double* v = a.sv;
  const int e = a.pev[r];
  const int64_t eb = a.ev_count[e];
  const int lo = a.tlo[r], hi = a.thi[r];
  const VFit f = wave_fit(a, r, lo, hi, 0, lane);
  if (!(f.chi2 / (f.n - 1) > a.split)) {
    record(a, e, eb, f, a.rec0, r, lane);
    return;
  }
  // two-means from the extreme members
  double c1 = z[lo], c2 = z[hi];
  bool empty = false, first_round = true;
  for (int it = 0; it < a.kmeans_iter; ++it) {
    bool moved = first_round;
    double W1 = 0.0, S1 = 0.0, W2 = 0.0, S2 = 0.0;
    for (int c = lo; c <= hi; c += kWave) {
      const int q = c + lane;
      const bool m = member(a, q, hi, r, 0);
      uint8_t sd = 0;
      bool mv = false;
      double w = 0.0, wz = 0.0;
      if (m) {
        sd = fabs(z[q] - c1) <= fabs(z[q] - c2) ? 0 : 1;
        mv = !first_round && sd != a.side[q];
        a.side[q] = sd;
        w = 1.0 / v[q];
        wz = w * z[q];
      }
      if (__ballot(mv)) moved = true;
      uint64_t b0 = __ballot(m && sd == 0), b1 = __ballot(m && sd == 1);
      while (b0) {
        const int l = __builtin_ctzll(b0);
        b0 &= b0 - 1;
        W1 = W1 + __shfl(w, l);
        S1 = S1 + __shfl(wz, l);
      }
      while (b1) {
        const int l = __builtin_ctzll(b1);
        b1 &= b1 - 1;
        W2 = W2 + __shfl(w, l);
        S2 = S2 + __shfl(wz, l);
      }
    }
    first_round = false;
    if (!moved) break;
    if (W1 == 0.0 || W2 == 0.0) {
      empty = true;
      break;
    }
    c1 = S1 / W1;
    c2 = S2 / W2;
  }
  if (empty) {
    record(a, e, eb, f, a.rec0, r, lane);
    return;
  }
  for (int part = 1; part <= 2; ++part) {
    const VFit g = wave_fit(a, r, lo, hi, part, lane);
    if (g.n >= 2) record(a, e, eb, g, part == 1 ? a.rec1 : a.rec2, r, lane);
  }
}

__global__ void __launch_bounds__(256) k_vtx_trees(VtxArgs a) {
  const int total = positions(a);
  const int lane = __lane_id();
  const int w = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int nw = static_cast<int>(gridDim.x * blockDim.x / kWave);
  for (int base = w * kWave; base < total; base += nw * kWave) {
    const int p = base + lane;
    const bool cand = p < total && a.root[p] == p && a.rho[p] > 1 && a.tsize[p] >= 2;
    uint64_t todo = __ballot(cand);
    while (todo) {
      const int r = base + __builtin_ctzll(todo);
      todo &= todo - 1;
      wave_tree(a, r, lane);
    }
  }
}

// ---- one work-group per event: its records by sum of p_T^2 (descending),
// then first member
__global__ void __launch_bounds__(kBlock) k_vtx_order(VtxArgs a) {
  __shared__ uint64_t lkey[kLdsSort];
  __shared__ int32_t lval[kLdsSort];
  const int e = blockIdx.x;
  const int64_t b = a.ev_count[e];
  const int nr = a.ev_nvtx[e];
  if (nr == 0) return;
  uint64_t* key = a.skey + 2 * b;
  int32_t* sv = a.sval + 2 * b;
  for (int k = threadIdx.x; k < nr; k += blockDim.x) {
    key[k] = ~order_key(a.rsum[b + k]);
    sv[k] = a.rfirst[b + k];
    a.rslot[a.rfirst[b + k]] = k;
  }
  __syncthreads();
  sort_pairs(key, sv, nr, lkey, lval);
  for (int k = threadIdx.x; k < nr; k += blockDim.x) a.rrank[b + a.rslot[sv[k]]] = k;
}

// Each track's vertex rank in its event (-1: none).
__global__ void k_vtx_members(VtxArgs a) {
  const int total = positions(a);
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < total; p += gridDim.x * blockDim.x) {
    const int r = a.root[p];
    int slot = a.rec0[r];
    if (slot < 0) {
      const int s1 = a.rec1[r], s2 = a.rec2[r];
      if (s1 >= 0 || s2 >= 0) slot = a.side[p] == 0 ? s1 : s2;   // a split tree
    }
    a.vlocal[p] = slot >= 0 ? a.rrank[slot] : -1;
  }
}

// Writes each event's ordered vertices at event_first[e] and the tracks'
// vertex indices.
__global__ void k_vtx_write(VtxArgs a) {
  const int total = positions(a);
  uint32_t over = 0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < total; p += gridDim.x * blockDim.x) {
    const int e = a.pev[p];
    const int base = a.event_first[e];
    const int nr = a.event_first[e + 1] - base;
    if (p - a.ev_count[e] < nr) {   // a record slot
      const int at = base + a.rrank[p];
      if (at >= a.cap) {
        ++over;
      } else {
        a.oz[at] = a.rz[p];
        a.ovar[at] = a.rvar[p];
        a.ochi2[at] = a.rchi2[p];
        a.osum[at] = a.rsum[p];
        a.ondf[at] = a.rndf[p];
        a.on[at] = a.rn[p];
      }
    }
    const int l = a.vlocal[p];
    if (l >= 0) a.track_vertex[a.sidx[p]] = base + l;
  }
  if (over) status_flag(a.status, PT_FLAG_VERTICES_OVERFLOW);
}

// event_first from the scanned vertex counts, and the total.
__global__ void k_vtx_event_first(VtxArgs a) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e <= a.n_events; e += gridDim.x * blockDim.x) {
    a.event_first[e] = a.ev_nvtx[e];
    if (e == a.n_events) *a.n_vertices = a.ev_nvtx[e];
  }
}

}  // namespace

size_t ws_vertices(int n_events, int n_max) {
  Carver c(nullptr);
  const size_t n = static_cast<size_t>(n_max) + 1, E = static_cast<size_t>(n_events) + 1;
  c.take<uint8_t>(n);        // use
  c.take<int32_t>(n);        // ev_of
  c.take<int32_t>(E);        // ev_count
  c.take<int32_t>(E);        // ev_cursor
  c.take<int32_t>(n);        // list
  c.take<uint64_t>(2 * n);   // skey
  c.take<int32_t>(2 * n);    // sval
  c.take<double>(n);         // sz
  c.take<double>(n);         // sv
  for (int q = 0; q < 6; ++q) c.take<int32_t>(n);  // sidx rho parent root tsize tlo
  c.take<int32_t>(n);        // thi
  c.take<uint8_t>(n);        // side
  for (int q = 0; q < 4; ++q) c.take<double>(n);   // rz rvar rchi2 rsum
  for (int q = 0; q < 5; ++q) c.take<int32_t>(n);  // rndf rn rfirst rslot vlocal
  for (int q = 0; q < 5; ++q) c.take<int32_t>(n);  // pev rrank rec0 rec1 rec2
  c.take<int32_t>(E);        // ev_nvtx
  c.take<int32_t>(scan_tmp_elems(static_cast<int64_t>(E)));
  return c.off + 256;
}

pt_err launch_vertices(const pt_hits& h, const DevCfg& k, const pt_ntuplets& T, int precision,
                       const pt_tracks& tracks, const int32_t* selected, const int32_t* n_selected,
                       pt_vertices& out, uint32_t* status, pt_workspace ws, hipStream_t s) {
  const int n_max = std::min(T.cap, tracks.cap);
  const size_t n = static_cast<size_t>(n_max) + 1, E = static_cast<size_t>(h.n_events) + 1;
  Carver c(ws.ptr);
  VtxArgs a{};
  a.hits = T.hits;
  a.n = T.n;
  a.kept = T.kept;
  a.count = T.count;
  a.n_max = n_max;
  a.params = tracks.params;
  a.cov = tracks.cov;
  a.dbl = precision == PT_FIT_F64 ? 1 : 0;
  a.selected = selected;
  a.n_selected = n_selected;
  a.event_offsets = h.event_offsets;
  a.n_events = h.n_events;
  a.n_hits = h.n_hits;
  a.min_hits = k.vtx_min_hits;
  a.kmeans_iter = k.vtx_kmeans_iter;
  a.pt_min = k.vtx_pt_min;
  a.err_max = k.vtx_err_max;
  a.dz_cut = k.vtx_dz_cut;
  a.chi2_max = k.vtx_chi2_max;
  a.split = k.vtx_split_chi2_ndf;
  a.pt_cap = k.vtx_pt_cap;
  a.K = k.K;
  a.use = c.take<uint8_t>(n);
  a.ev_of = c.take<int32_t>(n);
  a.ev_count = c.take<int32_t>(E);
  a.ev_cursor = c.take<int32_t>(E);
  a.list = c.take<int32_t>(n);
  a.skey = c.take<uint64_t>(2 * n);
  a.sval = c.take<int32_t>(2 * n);
  a.sz = c.take<double>(n);
  a.sv = c.take<double>(n);
  a.sidx = c.take<int32_t>(n);
  a.rho = c.take<int32_t>(n);
  a.parent = c.take<int32_t>(n);
  a.root = c.take<int32_t>(n);
  a.tsize = c.take<int32_t>(n);
  a.tlo = c.take<int32_t>(n);
  a.thi = c.take<int32_t>(n);
  a.side = c.take<uint8_t>(n);
  a.rz = c.take<double>(n);
  a.rvar = c.take<double>(n);
  a.rchi2 = c.take<double>(n);
  a.rsum = c.take<double>(n);
  a.rndf = c.take<int32_t>(n);
  a.rn = c.take<int32_t>(n);
  a.rfirst = c.take<int32_t>(n);
  a.rslot = c.take<int32_t>(n);
  a.vlocal = c.take<int32_t>(n);
  a.pev = c.take<int32_t>(n);
  a.rrank = c.take<int32_t>(n);
  a.rec0 = c.take<int32_t>(n);
  a.rec1 = c.take<int32_t>(n);
  a.rec2 = c.take<int32_t>(n);
  a.ev_nvtx = c.take<int32_t>(E);
  int32_t* tmp = c.take<int32_t>(scan_tmp_elems(static_cast<int64_t>(E)));
  a.oz = out.z;
  a.ovar = out.var;
  a.ochi2 = out.chi2;
  a.osum = out.sum_pt2;
  a.ondf = out.ndf;
  a.on = out.n_tracks;
  a.event_first = out.event_first;
  a.n_vertices = out.count;
  a.track_vertex = out.track_vertex;
  a.cap = out.cap;
  a.status = status;
  const int g = grid_for(std::max<int64_t>(n_max, h.n_events + 1), 256, 8192);
  k_vtx_clear<<<g, 256, 0, s>>>(a);
  if (selected) k_vtx_mark<<<g, 256, 0, s>>>(a);
  k_vtx_events<<<g, 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(a.ev_count, h.n_events, tmp, s));
  k_vtx_scatter<<<g, 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  const int gp = grid_for(n_max, 256, 16384);   // flat over the sorted positions
  if (h.n_events > 0) {
    k_vtx_sort<<<h.n_events, kBlock, 0, s>>>(a);
    PT_LAUNCH_CHECK();
  }
  k_vtx_density<<<gp, 256, 0, s>>>(a);
  k_vtx_parent<<<gp, 256, 0, s>>>(a);
  k_vtx_root<<<gp, 256, 0, s>>>(a);
  k_vtx_trees<<<gp, 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  if (h.n_events > 0) {
    k_vtx_order<<<h.n_events, kBlock, 0, s>>>(a);
    PT_LAUNCH_CHECK();
  }
  k_vtx_members<<<gp, 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(a.ev_nvtx, h.n_events, tmp, s));
  k_vtx_event_first<<<grid_for(h.n_events + 1, 256), 256, 0, s>>>(a);
  k_vtx_write<<<gp, 256, 0, s>>>(a);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

}  // namespace pt
