// Cell linking (paper section 3.2: doublets that share a hit are tested for
// a compatible triplet).
//
// The candidates are all pairs (c', c) of cells meeting on a middle hit h1:
// c' = (h0, h1) ends there, c = (h1, h2) starts there.  At pileup 200 there
// are billions of them and only about 2% pass the R-Z alignment test, so the
// step is organised around that test:
//
//  1. k_hit_table: (X, Y, Z, R) of every hit in double, one 32-byte entry.
//     Each cell's R-Z segment (dr, dz) is rebuilt from it with the
//     operations of the doublet step, and the class (barrel or end-cap) of
//     the out-cell's outer hit h2, which selects theta, comes from the cell's
//     layer pair.
//  2. k_cell_index: each chunk of cells is grouped by outer hit in an LDS
//     hash table and written to the index grouped that way.
//  3. exclusive scan of the per-hit segment counts, then k_seg_scatter:
//     each hit's in-cells as a list of segments of the index (8 bytes per
//     cell: cell, inner hit), one segment per chunk of k_cell_index.
//  4. k_link_hits: one wavefront per middle hit.  Lanes hold the in-cells.
//     The hit's out-cells (a contiguous run, grouped by inner hit by the
//     doublet step) are binned in LDS by the direction of their R-Z segment,
//     in bins at least as wide as the cut angle, so that each in-cell is
//     tested only against the out-cells of its own and the neighbouring bins
//     (a few percent of the pairs), the examined pairs dealt out 64 at a
//     time over the lanes.  Hits with too many out-cells for the LDS lists,
//     and wide cuts, sweep every out-cell in a uniform loop whose loads are
//     wave-uniform, so the R-Z test of 64 pairs costs a handful of
//     double-precision instructions.  Pairs that pass are queued in LDS and
//     the beam-spot test (divisions, square roots) runs on full waves of
//     queued pairs.  Each in-cell's link count is recorded, with its links
//     when there are at most kLocal of them, and the hit's out-cells that
//     gained an inner link are flagged (has_inner) in one coalesced run.
//  5. the counts are recorded straight into out_count; their scan into
//     out_start places every in-cell's links, in cell order (no shared
//     counter: same-address atomics serialise): after a scan of the counts'
//     tile sums, k_link_place scans each tile, writes out_start and the
//     links of the cells with at most kLocal, and k_links_overflow
//     recomputes the few in-cells with more.
#include "pt_internal.h"

#include <algorithm>

// Every decision below is made in double precision exactly as parenthesised.
#pragma clang fp contract(off)

namespace pt {
namespace {

constexpr int kLocal = 8;        // links an in-cell keeps in LDS before the overflow path
constexpr int kRow = kLocal;     // record of an in-cell with links (by cell): up to kLocal links
constexpr int kUnroll = 4;       // out-cells tested per step of the sweep
constexpr int kSegment = 1 << 24;  // out-cells per queue segment (offsets fit beside the lane)
constexpr int kSegWin = 64;        // in-cell segments of a hit handled per window (one per lane)
constexpr int kHinBits = 2048;     // out-cells of a hit whose has_inner flag is gathered in LDS
constexpr int kWinCap = 224;       // out-cells of the windowed search, with the copies at both ends

// Index entry of an in-cell c' = (h0, h1): its cell index, and its inner hit
// with the BPix1 flag in the top bit.  The triplet tests rebuild the R-Z
// segment from the hit table with the same operations as the doublet step.
struct InCell {
  int32_t cell;
  int32_t h0b;
};
constexpr int32_t kBpix1Bit = static_cast<int32_t>(0x80000000u);

// The R-Z test, with the out-cell's segment (br, bz) and length Lb.
__device__ __forceinline__ bool rz_pass(double ar, double az, double La, double br, double bz, double Lb,
                                        double theta2) {
  const double A = ar * bz - az * br;
  return A * A <= theta2 * (La * Lb);
}

// Class of a cell's outer hit from its layer pair: true for an end-cap layer.
__device__ __forceinline__ bool endcap_outer(const DevCfg& k, int pair) {
  return (k.endcap_pairs >> pair) & 1u;
}

// Direction key of an R-Z segment, in [-1, 1]: the diamond angle
// dz / (|dr| + |dz|) of the segment turned to dr >= 0 (the R-Z test does not
// depend on the orientation).  As a function of the polar angle of the
// undirected line its slope is at most 1, and its ends -1 and +1 are the
// same direction, so two segments at an angle d (mod pi) have keys at most d
// apart on a circle of length 2.  NaN for a zero-length or non-finite
// segment.
__device__ __forceinline__ float rz_key(double dr, double dz) {
  const float r = static_cast<float>(dr < 0.0 ? -dr : dr);
  const float z = static_cast<float>(dr < 0.0 ? -dz : dz);
  return z / (r + fabsf(z));
}

// Bucket of a key: B buckets of width 2 / B over [-1, 1], the last one
// closed.  Keys at most one bucket width apart (on the circle) fall in the
// same or neighbouring buckets (B - 1 and 0 are neighbours).
__device__ __forceinline__ int rz_bucket(float key, int B) {
  const int b = static_cast<int>((key + 1.0f) * (0.5f * static_cast<float>(B)));
  return min(max(b, 0), B - 1);
}

// The value of v in lane i (i wave-uniform).
__device__ __forceinline__ double lane_value(double v, int i) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), i);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), i);
  return __hiloint2double(hi, lo);
}

// The beam-spot test of the circle through the three hits.
__device__ __forceinline__ bool beam_pass(double X0, double Y0, double X1, double Y1, double X2, double Y2,
                                          double rmax) {
  const double ux = X1 - X0, uy = Y1 - Y0;
  const double vx = X2 - X0, vy = Y2 - Y0;
  const double Dd = 2.0 * (ux * vy - uy * vx);
  if (Dd == 0.0) {
    const double cr = X0 * vy - Y0 * vx;
    return cr * cr <= (rmax * rmax) * (vx * vx + vy * vy);
  }
  const double U2 = ux * ux + uy * uy;
  const double V2 = vx * vx + vy * vy;
  const double cx = (U2 * vy - V2 * uy) / Dd;
  const double cy = (V2 * ux - U2 * vx) / Dd;
  const double rho2 = cx * cx + cy * cy;
  const double Cx = X0 + cx, Cy = Y0 + cy;
  const double c2 = Cx * Cx + Cy * Cy;
  return fabs(sqrt(c2) - sqrt(rho2)) <= rmax;
}

// Hit table: (X, Y, Z, R) in double, one 32-byte entry per hit, R = sqrt(X X + Y Y).
template <class T>
__global__ void k_hit_table(int n, const T* __restrict__ x, const T* __restrict__ y, const T* __restrict__ z,
                            double4* __restrict__ hx) {
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < n; h += gridDim.x * blockDim.x) {
    const double X = static_cast<double>(x[h]);
    const double Y = static_cast<double>(y[h]);
    hx[h] = make_double4(X, Y, static_cast<double>(z[h]), sqrt(X * X + Y * Y));
  }
}

struct IndexArgs {
  const int32_t* cell_count;
  int32_t cells_cap;
  const int32_t* inner;
  const int32_t* outer;
  const uint8_t* layer;
  InCell* ent;         // the block's cells grouped by outer hit, in the block's own range
  int4* grp;           // per block: its groups (outer hit, first entry, cells, slot in the hit's list)
  int32_t* n_grp;      // per block: number of groups
  int32_t* n_seg;      // [n_hits + 1] groups ending on each hit
  int32_t* out_count;  // cleared here (link counts of the cells)
  uint8_t* has_inner;
};

constexpr int kIndexBlock = 1024;
constexpr int kIndexItems = 4;
constexpr int kIndexChunk = kIndexBlock * kIndexItems;  // cells per block; also the hash table size
static_assert((kIndexChunk & (kIndexChunk - 1)) == 0, "hash table size must be a power of two");

// The index of cells by outer hit.  Each block takes a
// chunk of kIndexChunk consecutive cells (neighbouring inner hits, which share
// most outer hits), groups them by outer hit in an LDS hash table, and writes
// them as index entries grouped by outer hit into the chunk's own range of
// `ent` (staged in LDS, then written contiguously).  Each group becomes one
// segment of its outer hit's in-cell list: the hit's segment count is taken
// with one global atomic per group, and the segment itself is placed by
// k_seg_scatter once the counts are scanned.  has_inner and the link counts
// are cleared here (when given).
//
// Every global load and atomic of the block is issued before its first
// global store: on this architecture one counter tracks loads and stores
// alike, so a load issued after a store would wait for the store's write
// acknowledgement as well.
__global__ void __launch_bounds__(kIndexBlock) k_cell_index(IndexArgs a) {
  __shared__ int32_t s_key[kIndexChunk];      // outer hit of the slot, -1 when free
  __shared__ int32_t s_pos[kIndexChunk + 1];  // cells in the slot; after the scan its first entry
                                             // << 16 | its group index
  __shared__ int32_t s_cell[kIndexChunk];     // per cell: slot | rank in the slot << 12
  __shared__ int32_t s_h0b[kIndexChunk];      // per cell: inner hit | BPix1 bit
  __shared__ int32_t s_scan[kIndexBlock / kWave + 1];
  static_assert(kIndexChunk <= 4096, "slot and rank are packed in 12 bits each");
  const int n = min(*a.cell_count, a.cells_cap);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kIndexChunk;
  if (base >= n) return;
  const int m = static_cast<int>(min<int64_t>(kIndexChunk, n - base));
  for (int i = threadIdx.x; i < kIndexChunk; i += kIndexBlock) {
    s_key[i] = -1;
    s_pos[i] = 0;
  }
  // loads of the block's cells, item u = cell base + u * kIndexBlock + thread
  int h0[kIndexItems], h1[kIndexItems];
#pragma unroll
  for (int u = 0; u < kIndexItems; ++u) {
    const int loc = u * kIndexBlock + threadIdx.x;
    const int c = static_cast<int>(base) + (loc < m ? loc : 0);
    h0[u] = a.inner[c];
    h1[u] = a.outer[c];
  }
  int32_t h0b[kIndexItems];
#pragma unroll
  for (int u = 0; u < kIndexItems; ++u) h0b[u] = h0[u] | (a.layer[h0[u]] == 0 ? kBpix1Bit : 0);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kIndexItems; ++u) {
    const int loc = u * kIndexBlock + threadIdx.x;
    if (loc >= m) break;
    // linear probing; the table has a slot for every cell of the block
    const int key = h1[u];
    int slot = static_cast<int>((static_cast<uint32_t>(key) * 2654435761u) >> 20) & (kIndexChunk - 1);
    while (true) {
      const int prev = atomicCAS(&s_key[slot], -1, key);
      if (prev == -1 || prev == key) break;
      slot = (slot + 1) & (kIndexChunk - 1);
    }
    const int r = atomicAdd(&s_pos[slot], 1);
    s_cell[loc] = slot | (r << 12);
    s_h0b[loc] = h0b[u];
  }
  __syncthreads();
  // one scan gives every slot its first entry (high half) and its group
  // index (low half): kIndexItems consecutive slots per thread
  int ngroups;
  {
    const int t0 = threadIdx.x * kIndexItems;
    int v[kIndexItems];
    int sum = 0;
#pragma unroll
    for (int i = 0; i < kIndexItems; ++i) {
      v[i] = (s_pos[t0 + i] << 16) | (s_key[t0 + i] >= 0 ? 1 : 0);
      sum += v[i];
    }
    const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
    int incl = sum;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(incl, d, kWave);
      if (lane >= d) incl += o;
    }
    if (lane == kWave - 1) s_scan[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
      int run = 0;
      for (int w = 0; w < kIndexBlock / kWave; ++w) {
        const int x = s_scan[w];
        s_scan[w] = run;
        run += x;
      }
      s_scan[kIndexBlock / kWave] = run;
      s_pos[kIndexChunk] = run;
    }
    __syncthreads();
    int run = s_scan[wave] + incl - sum;
#pragma unroll
    for (int i = 0; i < kIndexItems; ++i) {
      s_pos[t0 + i] = run;  // each thread rewrites only the slots it read
      run += v[i];
    }
    ngroups = s_scan[kIndexBlock / kWave] & 0xFFFF;
  }
  __syncthreads();
  // the segment slots of the block's groups (stored with the rest at the end)
  int key[kIndexItems], slot_in_list[kIndexItems], pv[kIndexItems], cells[kIndexItems];
#pragma unroll
  for (int u = 0; u < kIndexItems; ++u) {
    const int i = u * kIndexBlock + threadIdx.x;
    key[u] = s_key[i];
    slot_in_list[u] = key[u] >= 0 ? atomicAdd(a.n_seg + key[u], 1) : 0;
    pv[u] = s_pos[i];
    cells[u] = (s_pos[i + 1] >> 16) - (pv[u] >> 16);  // empty slots add nothing
  }
  __syncthreads();  // the hash keys are dead: their array stages the entry order
  for (int loc = threadIdx.x; loc < m; loc += kIndexBlock) {
    const int v = s_cell[loc];
    s_key[(s_pos[v & (kIndexChunk - 1)] >> 16) + (v >> 12)] = loc;
  }
  __syncthreads();
  // every atomic result is taken here, so that no store below waits for another
  static_assert(kIndexItems == 4, "one operand per item");
  asm volatile("" ::"v"(slot_in_list[0]), "v"(slot_in_list[1]), "v"(slot_in_list[2]), "v"(slot_in_list[3]));
#pragma unroll
  for (int u = 0; u < kIndexItems; ++u) {
    if (key[u] >= 0)
      a.grp[base + (pv[u] & 0xFFFF)] =
          make_int4(key[u], static_cast<int>(base) + (pv[u] >> 16), cells[u], slot_in_list[u]);
  }
  if (threadIdx.x == 0) a.n_grp[blockIdx.x] = ngroups;
  for (int i = threadIdx.x; i < m; i += kIndexBlock) {  // the chunk's entries, contiguous
    const int loc = s_key[i];
    InCell e;
    e.cell = static_cast<int>(base) + loc;
    e.h0b = s_h0b[loc];
    a.ent[base + i] = e;
  }
  if (a.has_inner) {
#pragma unroll
    for (int u = 0; u < kIndexItems; ++u) {
      const int loc = u * kIndexBlock + threadIdx.x;
      if (loc >= m) break;
      const int c = static_cast<int>(base) + loc;
      a.has_inner[c] = 0;
      a.out_count[c] = 0;
    }
  }
}

// Places every group as a segment (first entry, cells) of its outer hit's
// list, at the hit's scanned segment offset plus the group's slot.  One block
// per index chunk; 1024 threads spread its groups' scattered stores over
// more wavefronts (0.30 ms against 0.48 ms with 256).
constexpr int kScatterBlock = 1024;
__global__ void k_seg_scatter(const int32_t* __restrict__ cell_count, int32_t cells_cap,
                              const int4* __restrict__ grp, const int32_t* __restrict__ n_grp,
                              const int32_t* __restrict__ seg_first, int2* __restrict__ seg) {
  const int n = min(*cell_count, cells_cap);
  const int64_t base = static_cast<int64_t>(blockIdx.x) * kIndexChunk;
  if (base >= n) return;
  const int g_n = n_grp[blockIdx.x];
  // kBatch groups per thread and round, their loads issued before any store
  constexpr int kBatch = 8;
  for (int g0 = 0; g0 < g_n; g0 += kBatch * blockDim.x) {
    int4 e[kBatch];
    int at[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int g = g0 + u * blockDim.x + threadIdx.x;
      if (g < g_n) e[u] = grp[base + g];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int g = g0 + u * blockDim.x + threadIdx.x;
      if (g < g_n) at[u] = seg_first[e[u].x] + e[u].w;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int g = g0 + u * blockDim.x + threadIdx.x;
      if (g < g_n) seg[at[u]] = make_int2(e[u].y, e[u].z);
    }
  }
}

// Per-wave LDS of k_link_hits.
template <class T>
struct alignas(16) WaveLds {
  int32_t queue[2 * kWave];      // queued pairs: out-cell offset << 6 | in-cell lane
  int32_t cnt[kWave];            // links found per in-cell lane
  uint16_t found[kWave * kLocal];  // their out-cells' offsets in the hit's out-cells (windowed search)
  int32_t sfirst[kSegWin];       // a window of the hit's segments: first entry ...
  int32_t spre[kSegWin + 1];     // ... and the in-cells before each (exclusive prefix)
  int32_t segat[kWave];          // segment starting at each in-cell of a pass, or -1
  uint32_t hin[kHinBits / 32];   // out-cells of the hit with an inner link (first kHinBits)
  // windowed search: the hit's out-cells by bucket (segment, offset | end-cap
  // bit << 15), bucket B - 1 copied in front and bucket 0 behind, and where
  // each bucket starts
  double wdr[kWinCap];
  T wz2[kWinCap];  // the outer hit's z (dz = z2 - Z1 as the doublet step computes it)
  uint16_t wj[kWinCap];
  uint16_t bst[kRzBuckets + 1];
  // and the outer hits' x and y, by out-cell offset (values of the input
  // type, which the hit table holds exactly)
  T wx2[kWinCap];
  T wy2[kWinCap];
};
static_assert(kRzBuckets <= 2 * kWave, "the bucket counts use the queue, two buckets per lane");
static_assert(kWinCap * sizeof(int32_t) <= sizeof(WaveLds<float>::found) && kWinCap <= 0x8000,
              "staging uses the found array; offsets fit 15 bits");

template <class T>
struct HitArgs {
  int32_t n_hits;
  const double4* hx;
  const int32_t* cell_count;
  int32_t cells_cap;
  const int32_t* outer;
  const uint8_t* pair;
  const int32_t* inner_first;
  const int32_t* inner_count;
  const int32_t* seg_first;  // [n_hits + 1] first segment of each hit's in-cell list
  const int2* seg;           // segments: (first entry, entries)
  const InCell* ent;         // index entries
  int32_t* out_count;  // [cells_cap] links of each cell, zero on entry (scanned afterwards)
  int32_t* spill;     // per in-cell with links: its out-cells (at most kLocal), the first four
                      // at [cell][4], the others at [cells_cap + cell][4]
  int32_t* ovf;       // in-cells with more than kLocal links
  int32_t* ovf_count;
  uint8_t* has_inner;  // set for every out-cell with a link (zero on entry)
};

// Beam-spot test of the first nq queued pairs, one per lane; cb is the first
// out-cell of the segment the queued offsets refer to, hb its offset in the
// hit's out-cells (for the has_inner bits).  The in-cells' inner hits (X0,
// Y0, BPix1 flag, cell) are read from the lanes that hold them; all lanes
// call it.  The windowed search (staged) keeps the links in LDS as offsets
// in the hit's out-cells; the sweeps of larger hits write them straight to
// the in-cell's record.
template <class T>
__device__ __forceinline__ void beam_batch(const DevCfg& k, const HitArgs<T>& a, WaveLds<T>& L, int nq, int cb,
                                           int hb, double X1, double Y1, double X0l, double Y0l, int bpix1l,
                                           int celll, bool staged) {
  const int lane = __lane_id();
  const int e = lane < nq ? L.queue[lane] : 0;
  const int j = e >> 6;
  const int li = e & (kWave - 1);
  const double X0 = __shfl(X0l, li, kWave), Y0 = __shfl(Y0l, li, kWave);
  const int bpix1 = __shfl(bpix1l, li, kWave);
  const int cl = __shfl(celll, li, kWave);
  if (lane < nq) {
    double X2, Y2;
    if (staged) {  // the windowed search staged the outer hits
      X2 = static_cast<double>(L.wx2[j]);
      Y2 = static_cast<double>(L.wy2[j]);
    } else {
      const double4 P2 = a.hx[a.outer[cb + j]];
      X2 = P2.x;
      Y2 = P2.y;
    }
    const double rmax = bpix1 ? k.rmax_bpix1 : k.rmax_other;
    if (beam_pass(X0, Y0, X1, Y1, X2, Y2, rmax)) {
      const int slot = atomicAdd(&L.cnt[li], 1);
      if (slot < kLocal) {
        if (staged) {
          L.found[li * kLocal + slot] = static_cast<uint16_t>(hb + j);
        } else {
          const int64_t row = slot < 4 ? cl : static_cast<int64_t>(a.cells_cap) + cl;
          a.spill[row * 4 + (slot & 3)] = cb + j;
        }
      }
      const int bit = hb + j;
      if (bit < kHinBits)
        atomicOr(&L.hin[bit >> 5], 1u << (bit & 31));
      else
        a.has_inner[cb + j] = 1;
    }
  }
}

// Stages the hit's nb out-cells (from cb on) for the windowed search, sorted
// by bucket into wdr / wz2 / wj, and the bucket starts into bst; (R1, Z1)
// is the middle hit.  Returns false (wave-uniform) when an out-cell has no
// key or the list with its copies does not fit; the hit is then swept pair
// by pair.
template <class T>
__device__ bool stage_window(const DevCfg& k, const HitArgs<T>& a, WaveLds<T>& L, int cb, int nb, double R1,
                             double Z1) {
  const int lane = __lane_id();
  const int B = k.rz_buckets;
  int32_t* hist = L.queue;  // bucket counts (the queue is empty between passes)
  int32_t* tmp = reinterpret_cast<int32_t*>(L.found);  // per out-cell: bucket | rank in the bucket << 8
  for (int b = lane; b < B; b += kWave) hist[b] = 0;
  wave_sync();
  bool bad = false;
  // out-cell j = r kWave + lane; its segment stays in registers
  constexpr int kRounds = (kWinCap + kWave - 1) / kWave;
  double sdr[kRounds];
  T sz2[kRounds];
  bool send[kRounds];
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const int j = r * kWave + lane;
    sdr[r] = 0.0;
    sz2[r] = T(0);
    send[r] = false;
    if (j < nb) {
      const double4 P2 = a.hx[a.outer[cb + j]];
      sdr[r] = P2.w - R1;  // as the doublet step computes dr and dz
      sz2[r] = static_cast<T>(P2.z);  // exact: the hit table holds values of the input type
      send[r] = endcap_outer(k, a.pair[cb + j]);
      const float key = rz_key(sdr[r], P2.z - Z1);
      bad |= !(key == key);
      const int b = key == key ? rz_bucket(key, B) : 0;
      tmp[j] = b | (atomicAdd(&hist[b], 1) << 8);
      L.wx2[j] = static_cast<T>(P2.x);
      L.wy2[j] = static_cast<T>(P2.y);
    }
  }
  if (__ballot(bad)) return false;
  wave_sync();
  // bucket starts: exclusive scan of the counts, two buckets per lane
  const int h0 = 2 * lane < B ? hist[2 * lane] : 0;
  const int h1 = 2 * lane + 1 < B ? hist[2 * lane + 1] : 0;
  int incl = h0 + h1;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int o = __shfl_up(incl, d, kWave);
    if (lane >= d) incl += o;
  }
  const int front = hist[B - 1], back = hist[0];  // copies before and after the list
  if (front + nb + back > kWinCap) return false;   // uniform
  const int ex = incl - h0 - h1;
  if (2 * lane < B) L.bst[2 * lane] = static_cast<uint16_t>(front + ex);
  if (2 * lane + 1 < B) L.bst[2 * lane + 1] = static_cast<uint16_t>(front + ex + h0);
  if (lane == 0) L.bst[B] = static_cast<uint16_t>(front + nb);
  wave_sync();
#pragma unroll
  for (int q = 0; q < kRounds; ++q) {
    const int j = q * kWave + lane;
    if (j >= nb) continue;
    const double dr = sdr[q];
    const T z2 = sz2[q];
    const int v = tmp[j];
    const int b = v & 0xFF, r = v >> 8;
    const uint16_t jv = static_cast<uint16_t>(j | (send[q] ? 0x8000 : 0));
    const int at = L.bst[b] + r;
    L.wdr[at] = dr;
    L.wz2[at] = z2;
    L.wj[at] = jv;
    if (b == B - 1 || b == 0) {  // its copy at the other end
      const int c = b == B - 1 ? r : front + nb + r;
      L.wdr[c] = dr;
      L.wz2[c] = z2;
      L.wj[c] = jv;
    }
  }
  wave_sync();
  return true;
}

// One wavefront per middle hit; WAVES independent wavefronts per block.
template <class T, int WAVES>
__global__ void __launch_bounds__(WAVES * kWave)
    k_link_hits(DevCfg k, HitArgs<T> a) {
  __shared__ WaveLds<T> lds[WAVES];
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = __lane_id();
  WaveLds<T>& L = lds[wave];
  const int h1 = blockIdx.x * WAVES + wave;
  if (h1 >= a.n_hits) return;
  // every load of the hit's own entries at once (all in range for h1 < n_hits)
  const int sb = a.seg_first[h1];
  const int se = a.seg_first[h1 + 1];
  const int cell_count = *a.cell_count;
  const int cb = a.inner_first[h1];
  const int icount = a.inner_count[h1];
  const double4 P1 = a.hx[h1];
  if (se <= sb) return;
  const int n_cells = min(cell_count, a.cells_cap);
  const int nb = min(cb + icount, n_cells) - cb;
  if (icount <= 0 || nb <= 0) return;  // no out-cells: no links (counts are zero)
  const double X1 = P1.x, Y1 = P1.y, Z1 = P1.z, R1 = P1.w;
  const double th2b = k.theta2_barrel, th2e = k.theta2_endcap;
  const int nh = min(nb, kHinBits);  // out-cells whose has_inner bit is kept in LDS
  for (int w = lane; w < (nh + 31) / 32; w += kWave) L.hin[w] = 0;
  // the first window of the hit's in-cell segments, loaded before the staging
  int2 seg0 = make_int2(0, 0);
  if (lane < min(kSegWin, se - sb)) seg0 = a.seg[sb + lane];
  // the out-cells by direction bucket, when the search can be windowed
  const bool win = k.rz_buckets > 0 && nb <= kWinCap && stage_window(k, a, L, cb, nb, R1, Z1);

  for (int sw = sb; sw < se; sw += kSegWin) {
    // a window of the hit's segments and the prefix of their sizes
    const int wn = min(kSegWin, se - sw);
    int c0 = 0;
    if (lane < wn) {
      const int2 g = sw == sb ? seg0 : a.seg[sw + lane];
      L.sfirst[lane] = g.x;
      c0 = g.y;
    }
    int i0 = c0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o0 = __shfl_up(i0, d, kWave);
      if (lane >= d) i0 += o0;
    }
    const int aw = __builtin_amdgcn_readfirstlane(__shfl(i0, kWave - 1, kWave));  // in-cells of the window
    L.spre[lane] = i0 - c0;
    wave_sync();
    if (lane == 0) L.spre[wn] = aw;
    wave_sync();

    for (int base = 0; base < aw; base += kWave) {
      const int m = min(kWave, aw - base);
      // in-cell of this lane (NaN makes the R-Z test fail for idle lanes)
      double ar = __builtin_nan(""), az = __builtin_nan(""), La = __builtin_nan("");
      double X0 = 0.0, Y0 = 0.0;  // its inner hit, for the beam-spot test
      int bpix1 = 0;
      int cell = -1;
      int r = -1;  // its index entry
      // segment of each lane's in-cell: every segment overlapping the pass
      // marks its first in-cell in it, then a prefix maximum over the lanes
      L.segat[lane] = -1;
      wave_sync();
      if (lane < wn) {
        const int lo = L.spre[lane] - base, hi = L.spre[lane + 1] - base;
        if (hi > 0 && lo < kWave) L.segat[lo > 0 ? lo : 0] = lane;
      }
      wave_sync();
      int sg = L.segat[lane];
#pragma unroll
      for (int d = 1; d < kWave; d <<= 1) {
        const int o = __shfl_up(sg, d, kWave);
        if (lane >= d) sg = max(sg, o);
      }
      if (lane < m) {
        const int idx = base + lane;
        r = L.sfirst[sg] + (idx - L.spre[sg]);
        const InCell e = a.ent[r];
        const double4 P0 = a.hx[e.h0b & ~kBpix1Bit];
        ar = R1 - P0.w;  // as the doublet step computes dr
        az = Z1 - P0.z;
        La = ar * ar + az * az;
        cell = e.cell;
        X0 = P0.x;
        Y0 = P0.y;
        bpix1 = (e.h0b & kBpix1Bit) ? 1 : 0;
      }
      L.cnt[lane] = 0;
      // A partial pass with few in-cells sweeps the other way round: lanes over
      // the out-cells, the in-cells (read from their lanes) in a wave-uniform loop.
      const int out_blocks = (nb + kWave - 1) / kWave;
      const bool transposed = m < kWave && static_cast<int64_t>(m) * out_blocks < nb;
      wave_sync();

      // Sweep the out-cells in segments short enough for the packed queue
      // entries (offset << 6 | lane).
      for (int jb = 0; jb < nb; jb += kSegment) {
        const int cs = cb + jb;
        const int ns = min(kSegment, nb - jb);
        int qn = 0;  // queued pairs (uniform)
        // Queues the passing lanes of out-cell j; runs a beam batch when a full
        // wave of pairs is waiting.
        auto append = [&](int j, int li, bool pass, uint64_t mk) {
          if (pass) L.queue[qn + lane_prefix(mk)] = (j << 6) | li;
          qn += __popcll(mk);
          if (qn >= kWave) {
            wave_sync();
            beam_batch(k, a, L, kWave, cs, jb, X1, Y1, X0, Y0, bpix1, cell, win);
            qn -= kWave;
            const int t = (lane < qn) ? L.queue[kWave + lane] : 0;
            wave_sync();
            if (lane < qn) L.queue[lane] = t;
            wave_sync();
          }
        };
        if (win) {
          // Windowed: each in-cell meets only the out-cells of its own and the
          // neighbouring buckets, a contiguous range of the staged list.  The
          // ranges of all lanes are laid end to end and dealt out 64 pairs at
          // a time, pair f going to the last lane whose range starts at or
          // before f.
          static_assert(kWinCap < kSegment, "the staged list is one segment");
          const int B = k.rz_buckets;
          int wstart = 0, wlen = 0;
          if (lane < m) {
            const float key = rz_key(ar, az);
            if (key == key) {
              const int b = rz_bucket(key, B);
              wstart = b == 0 ? 0 : L.bst[b - 1];
              const int wend = b == B - 1 ? L.bst[B] + (L.bst[1] - L.bst[0]) : L.bst[b + 2];
              wlen = wend - wstart;
            } else {  // no key: every out-cell once
              wstart = L.bst[0];
              wlen = nb;
            }
          }
          int incl = wlen;
#pragma unroll
          for (int d = 1; d < kWave; d <<= 1) {
            const int o = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += o;
          }
          const int P = incl - wlen;  // first pair of this lane's range
          const int npairs = __builtin_amdgcn_readfirstlane(__shfl(incl, kWave - 1, kWave));
          // the pass set-up's segment marks are free now: they hold the
          // lane whose range starts at each place of a step, and a bit set
          // of those places
          uint8_t* starter = reinterpret_cast<uint8_t*>(L.segat);
          uint32_t* starts = reinterpret_cast<uint32_t*>(L.segat) + kWave / 4;
          static_assert(kWave / 4 + 2 <= kWave, "both fit the segment marks");
          int carry = 0;  // the lane owning the last pair of the previous step
          for (int f0 = 0; f0 < npairs; f0 += kWave) {
            const int f = f0 + lane;
            if (lane < 2) starts[lane] = 0;
            wave_sync();
            const int rel = P - f0;
            if (wlen > 0 && rel >= 0 && rel < kWave) {
              starter[rel] = static_cast<uint8_t>(lane);
              atomicOr(&starts[rel >> 5], 1u << (rel & 31));
            }
            wave_sync();
            // the last range starting at or before f: the highest start at or
            // below this place, else the range running on from the previous step
            const uint64_t sm = (static_cast<uint64_t>(starts[1]) << 32) | starts[0];
            const uint64_t below = sm & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1));
            const int o = below ? starter[63 - __builtin_clzll(below)] : carry;
            carry = __builtin_amdgcn_readlane(o, kWave - 1);
            const double oar = __shfl(ar, o, kWave), oaz = __shfl(az, o, kWave), oLa = __shfl(La, o, kWave);
            const int at = __shfl(wstart, o, kWave) + (f - __shfl(P, o, kWave));
            bool pass = false;
            int j = 0;
            if (f < npairs) {
              const double br = L.wdr[at], bz = static_cast<double>(L.wz2[at]) - Z1;
              const int jv = L.wj[at];
              pass = rz_pass(oar, oaz, oLa, br, bz, br * br + bz * bz, (jv & 0x8000) ? th2e : th2b);
              j = jv & 0x7FFF;
            }
            const uint64_t mk = __ballot(pass);
            if (mk) append(j, o, pass, mk);
          }
          if (qn > 0) {
            wave_sync();
            beam_batch(k, a, L, qn, cs, jb, X1, Y1, X0, Y0, bpix1, cell, win);
          }
          wave_sync();
          continue;
        }
        if (transposed) {
          for (int ob = 0; ob < ns; ob += kWave) {
            const int j = ob + lane;
            const bool valid = j < ns;
            double br = 0.0, bz = 0.0, Lb = 0.0, theta2 = 0.0;
            if (valid) {
              const double4 P2 = a.hx[a.outer[cs + j]];
              br = P2.w - R1;
              bz = P2.z - Z1;
              Lb = br * br + bz * bz;
              theta2 = endcap_outer(k, a.pair[cs + j]) ? th2e : th2b;
            }
            for (int i = 0; i < m; ++i) {
              const bool pass =
                  valid && rz_pass(lane_value(ar, i), lane_value(az, i), lane_value(La, i), br, bz, Lb, theta2);
              const uint64_t mk = __ballot(pass);
              if (mk) append(j, i, pass, mk);
            }
          }
          if (qn > 0) {
            wave_sync();
            beam_batch(k, a, L, qn, cs, jb, X1, Y1, X0, Y0, bpix1, cell, win);
          }
          wave_sync();
          continue;
        }
        // One out-cell at a time, wave-uniform, its segment rebuilt from the
        // hit table; the loads of the next kUnroll out-cells are issued before
        // the tests of the current ones.
        auto load_out = [&](int j, double& br, double& bz, bool& ec) {
          const double4 P2 = a.hx[a.outer[cs + j]];
          br = P2.w - R1;
          bz = P2.z - Z1;
          ec = endcap_outer(k, a.pair[cs + j]);
        };
        double pbr[kUnroll], pbz[kUnroll];
        bool pec[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
          pbr[u] = pbz[u] = 0.0;
          pec[u] = false;
          if (u < ns) load_out(u, pbr[u], pbz[u], pec[u]);
        }
        for (int j = 0; j < ns; j += kUnroll) {
          double cbr[kUnroll], cbz[kUnroll];
          bool cec[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            cbr[u] = pbr[u];
            cbz[u] = pbz[u];
            cec[u] = pec[u];
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
            if (j + kUnroll + u < ns) load_out(j + kUnroll + u, pbr[u], pbz[u], pec[u]);
          bool pass[kUnroll];
          uint64_t mk[kUnroll];
          uint64_t any = 0;
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            pass[u] = j + u < ns &&
                      rz_pass(ar, az, La, cbr[u], cbz[u], cbr[u] * cbr[u] + cbz[u] * cbz[u], cec[u] ? th2e : th2b);
            mk[u] = __ballot(pass[u]);
            any |= mk[u];
          }
          if (any) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u)
              if (mk[u]) append(j + u, lane, pass[u], mk[u]);
          }
        }
        if (qn > 0) {
          wave_sync();
          beam_batch(k, a, L, qn, cs, jb, X1, Y1, X0, Y0, bpix1, cell, win);
        }
        wave_sync();
      }

      // record the link count of each in-cell, and its links when they fit
      // the spill row; positions come from a scan afterwards
      const int n = (lane < m) ? L.cnt[lane] : 0;
      if (n > 0) {
        a.out_count[cell] = n;
        if (n > kLocal) {
          const int slot = atomicAdd(a.ovf_count, 1);
          a.ovf[slot] = cell;
        }
      }
      if (win && n > 0 && n <= kLocal) {  // the links are sorted by k_link_place
        static_assert(kRow == 8 && kLocal == 8, "a record is two 16-byte vectors");
        // two halves of 16 bytes per cell, so that the records of the cells
        // with at most four links (nearly all) are dense; places past n are
        // never read.  (The sweeps wrote their records as they went.)
        int4* sp = reinterpret_cast<int4*>(a.spill);
        const uint16_t* fl = L.found + lane * kLocal;
        sp[cell] = make_int4(cb + fl[0], cb + fl[1], cb + fl[2], cb + fl[3]);
        if (n > 4) sp[static_cast<int64_t>(a.cells_cap) + cell] = make_int4(cb + fl[4], cb + fl[5], cb + fl[6], cb + fl[7]);
      }
      wave_sync();
    }
  }
  // the hit's out-cells with an inner link, one coalesced run of flags
  for (int j = lane; j < nh; j += kWave) a.has_inner[cb + j] = (L.hin[j >> 5] >> (j & 31)) & 1u;
}

// Places the links of every cell at its scanned position: the links come out
// ordered by in-cell (each cell's run sorted by out-cell), so that the runs of
// neighbouring cells -- the children of one cell in the n-tuplet search -- are
// adjacent.
struct EmitArgs {
  const int32_t* cell_count;
  int32_t cells_cap;
  const int32_t* out_start;  // first link of each cell (scanned counts)
  const int32_t* out_count;  // links of each cell
  const int32_t* spill;      // per in-cell with 1..kLocal links: its out-cells (two halves)
  int32_t links_cap;
  int32_t* in_cell;
  int32_t* out_cell;
};

__device__ __forceinline__ void cmp_swap(int& x, int& y) {
  const int lo = min(x, y), hi = max(x, y);
  x = lo;
  y = hi;
}

// One thread per cell; its loads (range, record) come before its stores, so
// no load waits for a store's acknowledgement.
// Writes the links of cell c (cnt of them, 1..kLocal, from link pos on): its
// record (q0, and q1 when cnt > 4) sorted by out-cell.
__device__ __forceinline__ void emit_cell(const EmitArgs& a, int c, int cnt, int pos, int4 q0, int4 q1) {
  static_assert(kRow == 8, "one record is two 16-byte vectors, one sorting network for eight keys");
  // the sweep records links in the order their beam-spot tests finished:
  // sort them by out-cell (empty places sort last)
  int f[kRow];
  const int v[kRow] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
  for (int q = 0; q < kRow; ++q) f[q] = q < cnt ? v[q] : INT_MAX;
  // Batcher's odd-even merge sort of eight keys (19 compare-exchanges)
  cmp_swap(f[0], f[1]); cmp_swap(f[2], f[3]); cmp_swap(f[4], f[5]); cmp_swap(f[6], f[7]);
  cmp_swap(f[0], f[2]); cmp_swap(f[1], f[3]); cmp_swap(f[4], f[6]); cmp_swap(f[5], f[7]);
  cmp_swap(f[1], f[2]); cmp_swap(f[5], f[6]);
  cmp_swap(f[0], f[4]); cmp_swap(f[1], f[5]); cmp_swap(f[2], f[6]); cmp_swap(f[3], f[7]);
  cmp_swap(f[2], f[4]); cmp_swap(f[3], f[5]);
  cmp_swap(f[1], f[2]); cmp_swap(f[3], f[4]); cmp_swap(f[5], f[6]);
#pragma unroll
  for (int q = 0; q < kLocal; ++q) {
    if (q >= cnt) break;
    if (pos + q < a.links_cap) {
      a.in_cell[pos + q] = c;
      a.out_cell[pos + q] = f[q];
    }
  }
}

// Places the links: each block takes one tile of kScanTile cells, scans
// their link counts (the tile's offset comes from the scan of the tile sums)
// into out_start, and writes the links of its cells with 1..kLocal of them
// from their records.  Cells with more than kLocal links are written by
// k_links_overflow.  The counts are read once, the positions never read
// back: each thread scans kEmitItems consecutive counts (16-byte vectors),
// the positions go through LDS (a count is the difference of two), and the
// records are then taken one cell per thread and round, consecutive cells
// on consecutive lanes.
constexpr int kEmitBlock = 256;
constexpr int kEmitItems = kScanTile / kEmitBlock;
static_assert(kEmitItems % 4 == 0, "counts are read as 16-byte vectors");

__global__ void __launch_bounds__(kEmitBlock) k_link_place(EmitArgs a, const int32_t* __restrict__ tile_off,
                                                          int32_t* __restrict__ out_start, int32_t* __restrict__ total) {
  __shared__ int32_t s_pos[kScanTile + 1];  // positions; a cell's count is the difference to the next
  __shared__ int32_t s_wave[kEmitBlock / kWave + 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) *total = tile_off[gridDim.x];
  const int n = min(*a.cell_count, a.cells_cap);
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kScanTile;
  if (first >= n) return;
  const int m = static_cast<int>(min<int64_t>(kScanTile, n - first));  // cells of this tile
  const int t = threadIdx.x;
  const int lane = __lane_id(), wave = t / kWave;
  // the counts of cells t * kEmitItems .. + kEmitItems of the tile
  int v[kEmitItems];
  const int at = t * kEmitItems;
  const bool vec = m == kScanTile && reinterpret_cast<uintptr_t>(a.out_count) % 16 == 0 &&
                   reinterpret_cast<uintptr_t>(out_start) % 16 == 0;
  if (vec) {
    const int4* p = reinterpret_cast<const int4*>(a.out_count + first + at);
#pragma unroll
    for (int i = 0; i < kEmitItems / 4; ++i) {
      const int4 q = p[i];
      v[4 * i] = q.x;
      v[4 * i + 1] = q.y;
      v[4 * i + 2] = q.z;
      v[4 * i + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i) v[i] = at + i < m ? a.out_count[first + at + i] : 0;
  }
  // exclusive prefix of the thread sums over the block
  int sum = 0;
#pragma unroll
  for (int i = 0; i < kEmitItems; ++i) sum += v[i];
  const int incl = wave_incl_scan(sum);
  if (lane == kWave - 1) s_wave[wave] = incl;
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int w = 0; w < kEmitBlock / kWave; ++w) {
      const int c = s_wave[w];
      s_wave[w] = run;
      run += c;
    }
  }
  __syncthreads();
  int run = tile_off[blockIdx.x] + s_wave[wave] + incl - sum;
  int pos[kEmitItems];
#pragma unroll
  for (int i = 0; i < kEmitItems; ++i) {
    pos[i] = run;
    run += v[i];
    s_pos[at + i] = pos[i];
  }
  if (t == kEmitBlock - 1) s_pos[kScanTile] = run;  // the tile's end (cells past m count nothing)
  if (vec) {
    int4* p = reinterpret_cast<int4*>(out_start + first + at);
#pragma unroll
    for (int i = 0; i < kEmitItems / 4; ++i) p[i] = make_int4(pos[4 * i], pos[4 * i + 1], pos[4 * i + 2], pos[4 * i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < kEmitItems; ++i)
      if (at + i < m) out_start[first + at + i] = pos[i];
  }
  __syncthreads();
  // the links of the cells with 1..kLocal, four rounds of cells at a time:
  // every record load of the rounds before any store
  const int4* sp = reinterpret_cast<const int4*>(a.spill);
  constexpr int kBatch = 4;
  for (int r0 = 0; r0 < kEmitItems; r0 += kBatch) {
    int cnt[kBatch], ps[kBatch];
    int4 q0[kBatch], q1[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int c = (r0 + u) * kEmitBlock + t;
      ps[u] = c < m ? s_pos[c] : 0;
      cnt[u] = c < m ? s_pos[c + 1] - ps[u] : 0;
      q0[u] = q1[u] = make_int4(0, 0, 0, 0);
      if (cnt[u] > 0 && cnt[u] <= kLocal) {
        q0[u] = sp[first + c];
        if (cnt[u] > 4) q1[u] = sp[a.cells_cap + first + c];
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (cnt[u] > 0 && cnt[u] <= kLocal)
        emit_cell(a, static_cast<int>(first + (r0 + u) * kEmitBlock + t), cnt[u], ps[u], q0[u], q1[u]);
  }
}

// In-cells with more than kLocal links: one wavefront each recomputes its
// links, lanes over the out-cells of its middle hit (in order, so the
// compacted links come out sorted), staged in LDS and written at the
// position the scan gave the in-cell once the sweep's loads are done.
constexpr int kOvfWaves = 4;
constexpr int kOvfStage = 256;

template <class T>
__global__ void __launch_bounds__(kOvfWaves * kWave)
    k_links_overflow(DevCfg k, HitArgs<T> a, const int32_t* __restrict__ inner, const uint8_t* __restrict__ layer,
                     const int32_t* __restrict__ out_start, int32_t links_cap,
                     int32_t* __restrict__ in_cell, int32_t* __restrict__ out_cell) {
  __shared__ int32_t s_link[kOvfWaves][kOvfStage];
  const int wave = __builtin_amdgcn_readfirstlane(static_cast<int>(threadIdx.x) / kWave);
  const int lane = __lane_id();
  const int m = *a.ovf_count;
  const int n_cells = min(*a.cell_count, a.cells_cap);
  for (int i = blockIdx.x * kOvfWaves + wave; i < m; i += gridDim.x * kOvfWaves) {
    const int cp = a.ovf[i];
    const int h0 = inner[cp];
    const int h1 = a.outer[cp];
    const double4 P0 = a.hx[h0], P1 = a.hx[h1];
    const double ar = P1.w - P0.w, az = P1.z - P0.z;  // as the doublet step computes dr and dz
    const double La = ar * ar + az * az;
    const double X0 = P0.x, Y0 = P0.y, X1 = P1.x, Y1 = P1.y;
    const double rmax = layer[h0] == 0 ? k.rmax_bpix1 : k.rmax_other;
    const int first = a.inner_first[h1];
    const int last = min(first + a.inner_count[h1], n_cells);
    int w = out_start[cp];  // uniform: position of the next link to write
    int staged = 0;         // uniform
    auto flush = [&]() {
      wave_sync();
      for (int q = lane; q < staged; q += kWave) {
        const int c = s_link[wave][q];
        if (w + q < links_cap) {
          in_cell[w + q] = cp;
          out_cell[w + q] = c;
        }
      }
      wave_sync();
      w += staged;
      staged = 0;
    };
    for (int c0 = first; c0 < last; c0 += kWave) {
      const int c = c0 + lane;
      bool pass = false;
      if (c < last) {
        const double4 P2 = a.hx[a.outer[c]];
        const double br = P2.w - P1.w, bz = P2.z - P1.z;
        const double theta2 = endcap_outer(k, a.pair[c]) ? k.theta2_endcap : k.theta2_barrel;
        pass = rz_pass(ar, az, La, br, bz, br * br + bz * bz, theta2) && beam_pass(X0, Y0, X1, Y1, P2.x, P2.y, rmax);
      }
      const uint64_t mk = __ballot(pass);
      if (staged + kWave > kOvfStage) flush();
      if (pass) s_link[wave][staged + lane_prefix(mk)] = c;
      staged += __popcll(mk);
    }
    flush();
  }
}

__global__ void k_finish_links(const int32_t* count, int32_t cap, uint32_t* status) {
  if (*count > cap) status_flag(status, PT_FLAG_LINKS_OVERFLOW);
}

}  // namespace

// The index of the stored cells by outer hit alone (for the Fishbone), in
// the workspace from its start; returns the bytes it takes.
static size_t carve_outer_index(Carver& c, int n_hits, int cells_cap, OuterIndex* out, InCell** ent, int4** grp,
                                int32_t** n_grp, int32_t** tmp) {
  const int64_t scan_n = std::max<int64_t>(n_hits, cells_cap);
  const int64_t chunks = std::max<int64_t>(1, (static_cast<int64_t>(cells_cap) + kIndexChunk - 1) / kIndexChunk);
  InCell* e = c.take<InCell>(cells_cap);
  int4* g = c.take<int4>(cells_cap);
  int32_t* ng = c.take<int32_t>(chunks);
  int32_t* sf = c.take<int32_t>(static_cast<size_t>(n_hits) + 1);
  int2* sg = c.take<int2>(cells_cap);
  int32_t* t = c.take<int32_t>(scan_tmp_elems(scan_n));
  if (out) {
    out->ent = reinterpret_cast<const int2*>(e);
    out->seg = sg;
    out->seg_first = sf;
    *ent = e;
    *grp = g;
    *n_grp = ng;
    *tmp = t;
  }
  return c.off;
}

size_t ws_outer_index(int n_hits, int cells_cap) {
  Carver c(nullptr);
  return carve_outer_index(c, n_hits, cells_cap, nullptr, nullptr, nullptr, nullptr, nullptr);
}

pt_err build_outer_index(const pt_hits& h, const pt_cells& cells, Carver& c, OuterIndex& out, hipStream_t s) {
  const int n = h.n_hits;
  const int64_t chunks = std::max<int64_t>(1, (static_cast<int64_t>(cells.cap) + kIndexChunk - 1) / kIndexChunk);
  InCell* ent = nullptr;
  int4* grp = nullptr;
  int32_t *n_grp = nullptr, *tmp = nullptr;
  carve_outer_index(c, n, cells.cap, &out, &ent, &grp, &n_grp, &tmp);
  int32_t* seg_first = const_cast<int32_t*>(out.seg_first);
  PT_HIP_CHECK(fill_i32(seg_first, 0, static_cast<int64_t>(n) + 1, s));
  IndexArgs g{cells.count, cells.cap, cells.inner, cells.outer, h.layer, ent, grp, n_grp, seg_first, nullptr,
              nullptr};
  k_cell_index<<<static_cast<unsigned>(chunks), kIndexBlock, 0, s>>>(g);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(seg_first, n, tmp, s));
  k_seg_scatter<<<static_cast<unsigned>(chunks), kScatterBlock, 0, s>>>(cells.count, cells.cap, grp, n_grp, seg_first,
                                                                       const_cast<int2*>(out.seg));
  PT_LAUNCH_CHECK();
  return PT_OK;
}

size_t ws_links(int n_hits, int cells_cap) {
  const int64_t scan_n = std::max<int64_t>(n_hits, cells_cap);
  const int64_t chunks = std::max<int64_t>(1, (static_cast<int64_t>(cells_cap) + kIndexChunk - 1) / kIndexChunk);
  Carver c(nullptr);
  c.take<double4>(n_hits);                  // hit table
  c.take<InCell>(cells_cap);                // index entries
  c.take<int4>(cells_cap);                  // groups of each block
  c.take<int32_t>(chunks);                  // groups per block
  c.take<int32_t>(static_cast<size_t>(n_hits) + 1);     // segments per hit -> first segment
  c.take<int2>(cells_cap);                  // segments
  c.take<int32_t>(scan_tmp_elems(scan_n));
  c.take<int32_t>(static_cast<size_t>(cells_cap) * kRow);  // records of the cells with links (two halves)
  c.take<int32_t>(cells_cap);               // overflow list
  c.take<int32_t>(1);                       // overflow count
  return c.off + 256;
}

template <class T, int WAVES>
static void launch_hits(const DevCfg& k, const HitArgs<T>& a, hipStream_t s) {
  const int64_t blocks = (static_cast<int64_t>(a.n_hits) + WAVES - 1) / WAVES;
  k_link_hits<T, WAVES><<<static_cast<unsigned>(blocks < 1 ? 1 : blocks), WAVES * kWave, 0, s>>>(k, a);
}

template <class T>
static pt_err run_links(const pt_hits& h, const DevCfg& k, const pt_cells& cells, pt_links& L,
                        uint32_t* status, pt_workspace ws, hipStream_t s, int block) {
  const int n = h.n_hits;
  const int64_t scan_n = std::max<int64_t>(n, cells.cap);
  const int64_t chunks = std::max<int64_t>(1, (static_cast<int64_t>(cells.cap) + kIndexChunk - 1) / kIndexChunk);
  Carver c(ws.ptr);
  double4* hx = c.take<double4>(n);
  InCell* ent = c.take<InCell>(cells.cap);
  int4* grp = c.take<int4>(cells.cap);
  int32_t* n_grp = c.take<int32_t>(chunks);
  int32_t* seg_first = c.take<int32_t>(static_cast<size_t>(n) + 1);
  int2* seg = c.take<int2>(cells.cap);
  int32_t* tmp = c.take<int32_t>(scan_tmp_elems(scan_n));
  int32_t* spill = c.take<int32_t>(static_cast<size_t>(cells.cap) * kRow);
  int32_t* ovf = c.take<int32_t>(cells.cap);
  int32_t* ovf_count = c.take<int32_t>(1);
  const T* x = static_cast<const T*>(h.x);
  const T* y = static_cast<const T*>(h.y);
  const T* z = static_cast<const T*>(h.z);

  PT_HIP_CHECK(fill_i32(ovf_count, 0, 1, s));
  PT_HIP_CHECK(fill_i32(seg_first, 0, static_cast<int64_t>(n) + 1, s));
  if (n > 0) {
    k_hit_table<T><<<grid_for(n, 256), 256, 0, s>>>(n, x, y, z, hx);
    PT_LAUNCH_CHECK();
  }
  void* tok = timing_begin(s);
  IndexArgs g{cells.count, cells.cap, cells.inner, cells.outer, h.layer, ent, grp, n_grp, seg_first,
              L.out_count, L.has_inner};
  k_cell_index<<<static_cast<unsigned>(chunks), kIndexBlock, 0, s>>>(g);
  timing_end(tok, "cell_index", s);
  PT_LAUNCH_CHECK();
  PT_HIP_CHECK(exclusive_scan(seg_first, n, tmp, s));
  tok = timing_begin(s);
  k_seg_scatter<<<static_cast<unsigned>(chunks), kScatterBlock, 0, s>>>(cells.count, cells.cap, grp, n_grp, seg_first, seg);
  timing_end(tok, "link_segments", s);
  PT_LAUNCH_CHECK();

  HitArgs<T> a{n, hx, cells.count, cells.cap, cells.outer, cells.pair, cells.inner_first, cells.inner_count,
               seg_first, seg, ent, L.out_count, spill, ovf, ovf_count, L.has_inner};
  tok = timing_begin(s);
  if (n > 0) {
    if (block == 128)
      launch_hits<T, 2>(k, a, s);
    else if (block == 256)
      launch_hits<T, 4>(k, a, s);
    else
      launch_hits<T, 1>(k, a, s);
    PT_LAUNCH_CHECK();
  }
  timing_end(tok, "links", s);
  // first link of each cell and the links: the tile sums of the counts are
  // scanned, then each tile scans itself and places its links
  const int32_t* tile_off = nullptr;
  PT_HIP_CHECK(scan_tile_offsets(L.out_count, cells.cap, cells.count, tmp, s, &tile_off));
  tok = timing_begin(s);
  EmitArgs e{cells.count, cells.cap, L.out_start, L.out_count, spill, L.cap, L.in_cell, L.out_cell};
  {
    const int64_t tiles = std::max<int64_t>(1, (static_cast<int64_t>(cells.cap) + kScanTile - 1) / kScanTile);
    k_link_place<<<static_cast<unsigned>(tiles), kEmitBlock, 0, s>>>(e, tile_off, L.out_start, L.count);
  }
  timing_end(tok, "link_emit", s);
  PT_LAUNCH_CHECK();
  k_links_overflow<T><<<1024, kOvfWaves * kWave, 0, s>>>(k, a, cells.inner, h.layer, L.out_start, L.cap, L.in_cell,
                                                         L.out_cell);
  PT_LAUNCH_CHECK();
  k_finish_links<<<1, 1, 0, s>>>(L.count, L.cap, status);
  PT_LAUNCH_CHECK();
  return PT_OK;
}

pt_err launch_links(const pt_hits& h, const DevCfg& k, const pt_cells& cells, pt_links& L,
                    uint32_t* status, pt_workspace ws, hipStream_t s, int block) {
  if (h.dtype == PT_F64) return run_links<double>(h, k, cells, L, status, ws, s, block);
  return run_links<float>(h, k, cells, L, status, ws, s, block);
}

}  // namespace pt
