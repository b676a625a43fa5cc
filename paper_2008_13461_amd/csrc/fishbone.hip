// Fishbone (paper section 3.3): among the doublets that share their outer
// hit, the longer of two aligned ones is dropped, so that the overlapping
// modules of a layer give one n-tuplet per particle instead of several.
//
// Runs inside pt_build_doublets after the write pass when the Fishbone is on:
//   1. the stored cells are indexed by outer hit with the index of the link
//      step (blocks of consecutive cells grouped by outer hit in LDS, one
//      segment per block and hit; no per-cell atomic);
//   2. one wavefront per outer hit gathers the hit's cells into LDS (cell,
//      inner hit's coordinates), counting-sorted by a polar-direction key of
//      the vector to the outer hit into buckets at least as wide as the cut
//      angle, and tests each cell (one lane each) only against the cells of
//      its own and the neighbouring buckets (and of those around its negated
//      key: nearly opposite vectors); the exact test, in double, decides and
//      clears the cell's keep flag.  Hits with more cells than a wavefront
//      stages are listed and done by one work-group each;
//   3. the kept cells are compacted in their order (a scan of the flags),
//      through a copy in the workspace, and each inner hit's range of cells
//      is moved with them.
// The test is the one of pixeltrack.h, in double, as parenthesised, without
// contraction, from the hits' coordinates promoted to double.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>

#include "pt_internal.h"

#pragma clang fp contract(off)

namespace pt {
namespace {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / kWave;
constexpr int kCapSmall = 256;  // cells per outer hit staged in LDS by the first kernel
constexpr int kCap = 512;       // by the second (the hits with more than kCapSmall)
constexpr int kNB = 256;       // most key buckets
constexpr int32_t kHitMask = 0x7fffffff;

template <class T>
struct FbArgs {
  const T* x;
  const T* y;
  const T* z;
  int32_t n_hits;
  double theta2;
  int32_t nb;             // key buckets: each at least the cut angle wide
  float kwin;             // key window: asin(theta) with a margin, 2 when theta >= 1
  float phwin;            // azimuth window of vectors at least kS0 transverse, > pi: none
  const int32_t* count;   // cells found
  int32_t cap;
  int32_t* inner;
  int32_t* outer;
  uint8_t* pair;
  int32_t* inner_first;
  int32_t* inner_count;
  OuterIndex idx;
  // workspace
  int32_t* keep;          // [cap + 1] flags, then positions
  int32_t* mid;           // [n_hits] outer hits with more than kCapSmall cells
  int32_t* n_mid;
  int32_t* big;           // [n_hits] outer hits with more than kCap cells
  int32_t* n_big;
  int32_t* t_inner;       // [cap] compacted copies
  int32_t* t_outer;
  uint8_t* t_pair;
};

// Cells the Fishbone works on: every stored cell, or none when the cells
// overflowed their capacity (the products are truncated anyway).
template <class T>
__device__ inline int stored(const FbArgs<T>& a) {
  const int c = *a.count;
  return c <= a.cap ? c : 0;
}

// Polar-direction key of a vector: uz / (|u_T| + |uz|), in [-1, 1].  As a
// function of the angle to the z axis its slope is at most 1, and two
// vectors at an angle a differ in that angle by at most a, so their keys
// differ by at most a (for nearly opposite vectors, at an angle pi - a, the
// sum of their keys is at most a in magnitude).
__device__ inline float polar_key(double ux, double uy, double uz) {
  const float t = sqrtf(float(ux * ux + uy * uy));
  const float l = t + fabsf(float(uz));
  return l > 0.f ? float(uz) / l : 0.f;
}

// Azimuth of a vector whose transverse part is at least kS0 of its length,
// else kNoPhi.  Two such vectors at an angle a <= kS0 have transverse parts
// at most a apart, hence azimuths at most asin(a / kS0) apart (for nearly
// opposite vectors, pi minus that).
constexpr float kS0 = 0.2f;
constexpr float kNoPhi = 10.f;
__device__ inline float azimuth(double ux, double uy, double uz) {
  const float t2 = float(ux * ux + uy * uy), l2 = t2 + float(uz * uz);
  return t2 >= (kS0 * kS0) * l2 ? atan2f(float(uy), float(ux)) : kNoPhi;
}

// Azimuths are staged as 16-bit quanta of 2 pi / 65535 (kNoPhiQ: none).
// The test on quanta accepts every pair whose float azimuths are within the
// window (a quantum is the floor of the scaled azimuth, so two are at most
// one quantum further apart than the azimuths, and the window is widened by
// two quanta): it stays a filter in front of the exact test.
constexpr float kPhiScale = 65535.f / 6.28318531f;
constexpr int kNoPhiQ = 0xFFFF;
__device__ inline uint16_t phi_quantum(float phi) {
  if (phi == kNoPhi) return kNoPhiQ;
  const int q = static_cast<int>((phi + 3.14159265f) * kPhiScale);
  return static_cast<uint16_t>(min(max(q, 0), kNoPhiQ - 1));
}
// The window in quanta (the whole circle when the azimuth test is off).
__device__ inline int phi_window_q(float win) {
  return win >= 3.2f ? 65535 : static_cast<int>(ceilf(win * kPhiScale)) + 2;
}
// Whether two azimuths allow an angle within the cut (opp: nearly opposite).
__device__ inline bool phi_ok(int qi, int qj, int wq, bool opp) {
  if (qi == kNoPhiQ || qj == kNoPhiQ) return true;
  int d = abs(qi - qj);
  d = min(d, 65535 - d);
  return opp ? 2 * d >= 65535 - 2 * wq : d <= wq;
}

// Bucket of a key in [-1, 1] among nb buckets of width 2 / nb.
__device__ inline int bucket(float k, int nb) {
  const int b = static_cast<int>((k + 1.f) * (0.5f * static_cast<float>(nb)));
  return b < 0 ? 0 : (b >= nb ? nb - 1 : b);
}

// The exact test: the cell with vector u (length^2 U2) is dropped by a
// shorter cell of vector v when they are aligned.
__device__ inline bool kills(double ux, double uy, double uz, double U2, double vx, double vy, double vz,
                             double V2, double theta2) {
  if (!(V2 < U2)) return false;
  const double wx = uy * vz - uz * vy, wy = uz * vx - ux * vz, wz = ux * vy - uy * vx;
  const double W2 = (wx * wx + wy * wy) + wz * wz;
  return W2 <= theta2 * (U2 * V2);
}

template <class T>
__device__ inline void vec(const FbArgs<T>& a, double Xh, double Yh, double Zh, int i, double& ux, double& uy,
                           double& uz, double& U2) {
  ux = Xh - double(a.x[i]);
  uy = Yh - double(a.y[i]);
  uz = Zh - double(a.z[i]);
  U2 = (ux * ux + uy * uy) + uz * uz;
}

template <class T>
__global__ void k_fb_flags(FbArgs<T> a) {
  const int n = stored(a);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) a.keep[c] = 1;
}

// One wavefront per outer hit.
// CAP cells per wavefront, WAVES wavefronts per block.  Every outer hit (one
// wavefront each) when LISTED is false, else the hits listed in a.mid (a
// persistent grid); hits with more than CAP cells are listed for the next
// kernel (a.mid, then a.big).
template <class T, int CAP, int WAVES, bool LISTED>
__global__ void __launch_bounds__(WAVES * kWave) k_fb_kill(FbArgs<T> a) {
  __shared__ int32_t s_bin[WAVES][kNB + 1];   // cells per key bucket, then first position
  // per staged cell: bucket | rank in it << kBkShift (16 bits when both fit 8)
  constexpr int kBkShift = CAP <= 256 ? 8 : 16;
  static_assert(kNB <= 256 && CAP <= 0x10000, "buckets fit 8 bits, ranks the rest");
  using Bk = std::conditional_t<CAP <= 256, uint16_t, int32_t>;
  __shared__ Bk s_bk[WAVES][CAP];
  __shared__ uint16_t s_val[WAVES][CAP];      // staged cells in bucket order (16 bits: five work-groups fit per CU)
  __shared__ int32_t s_cell[WAVES][CAP];
  __shared__ uint16_t s_phi[WAVES][CAP];      // azimuth quanta
  __shared__ T s_x[WAVES][CAP];               // the inner hit's coordinates
  __shared__ T s_y[WAVES][CAP];
  __shared__ T s_z[WAVES][CAP];
  const int w = static_cast<int>(threadIdx.x) / kWave;
  const int lane = __lane_id();
  if (stored(a) == 0) return;
  const int n_items = LISTED ? *a.n_mid : a.n_hits;
  for (int item = blockIdx.x * WAVES + w; item < n_items; item += LISTED ? gridDim.x * WAVES : n_items) {
  const int h = LISTED ? a.mid[item] : item;
  const int sb = a.idx.seg_first[h], se = a.idx.seg_first[h + 1];
  // the hit's cells: segment descriptors 64 at a time, then their entries
  // 64 at a time (each lane finds its entry's segment among the 64)
  int m = 0;
  for (int s0 = sb; s0 < se; s0 += kWave) {
    const int n = s0 + lane < se ? a.idx.seg[s0 + lane].y : 0;
    m += wave_sum(n);
  }
  if (m < 2) continue;
  const double Xh = double(a.x[h]), Yh = double(a.y[h]), Zh = double(a.z[h]);
  if (m > CAP) {  // more cells than this kernel stages: listed for the next
    if (lane == 0) {
      if (LISTED) a.big[atomicAdd(a.n_big, 1)] = h;
      else a.mid[atomicAdd(a.n_mid, 1)] = h;
    }
    continue;
  }
  const float win = a.kwin;
  const double rh = sqrt(Xh * Xh + Yh * Yh);
  const double nx = rh > 0.0 ? Xh / rh : 0.0, ny = rh > 0.0 ? Yh / rh : 0.0;
  const float zs = Zh < 0.0 ? -1.f : 1.f;
  float rmin = 2.f, zmin = 2.f;  // smallest radial and z-side keys of the lane's cells
  wave_sync();  // the previous hit's LDS is no longer read
  for (int b = lane; b <= a.nb; b += kWave) s_bin[w][b] = 0;
  wave_sync();
  int at = 0;
  for (int s0 = sb; s0 < se; s0 += kWave) {
    const int2 g = s0 + lane < se ? a.idx.seg[s0 + lane] : make_int2(0, 0);
    const int incl = wave_incl_scan(g.y);
    const int excl = incl - g.y;
    const int tot = __shfl(incl, kWave - 1);
    for (int f0 = 0; f0 < tot; f0 += kWave) {  // wave-uniform: every lane takes part in the shuffles
      const int f = f0 + lane;
      // the last lane whose segment starts at or before f
      int j = 0;
#pragma unroll
      for (int step = kWave / 2; step > 0; step >>= 1) {
        const int e = __shfl(excl, j + step);
        if (e <= f) j += step;
      }
      const int first = __shfl(g.x, j) + (f - __shfl(excl, j));
      if (f >= tot) continue;
      const int2 en = a.idx.ent[first];
      const int ih = en.y & kHitMask;
      s_cell[w][at + f] = en.x;
      const T hx = a.x[ih], hy = a.y[ih], hz = a.z[ih];
      s_x[w][at + f] = hx;
      s_y[w][at + f] = hy;
      s_z[w][at + f] = hz;
      const double ux = Xh - double(hx), uy = Yh - double(hy), uz = Zh - double(hz);
      s_phi[w][at + f] = phi_quantum(azimuth(ux, uy, uz));
      const float kz = polar_key(ux, uy, uz);
      const int b = bucket(kz, a.nb);
      s_bk[w][at + f] = static_cast<Bk>(b | (atomicAdd(&s_bin[w][b], 1) << kBkShift));
      // key of the vector about the outer hit's transverse direction
      const double ur = ux * nx + uy * ny;
      const double ox = ux - ur * nx, oy = uy - ur * ny;
      const float lr = sqrtf(float(ox * ox + oy * oy + uz * uz)) + fabsf(float(ur));
      rmin = fminf(rmin, lr > 0.f ? float(ur) / lr : 0.f);
      zmin = fminf(zmin, kz * zs);
    }
    at += tot;
  }
  // nearly opposite partners are possible only when neither family of keys
  // stays above the cut angle for every cell of the hit (two nearly opposite
  // vectors cannot both point away from the beam line, or both along the
  // outer hit's side of z, by more than the cut angle)
  const bool mirror = wave_min(rmin) <= win && wave_min(zmin) <= win;
  wave_sync();
  // counting sort by bucket: first positions (a scan over the buckets), then
  // each staged cell at its bucket's first position plus its rank
  {
    int carry = 0;
    for (int b0 = 0; b0 < a.nb; b0 += kWave) {
      const int b = b0 + lane;
      const int c = b < a.nb ? s_bin[w][b] : 0;
      const int incl = wave_incl_scan(c);
      if (b < a.nb) s_bin[w][b] = carry + incl - c;
      carry += __shfl(incl, kWave - 1);
    }
    if (lane == 0) s_bin[w][a.nb] = carry;
  }
  wave_sync();
  for (int i = lane; i < m; i += kWave) {
    const int v = s_bk[w][i];
    s_val[w][s_bin[w][v & ((1 << kBkShift) - 1)] + (v >> kBkShift)] = static_cast<uint16_t>(i);
  }
  wave_sync();
  // each cell against the cells of its bucket and the two next to it, and of
  // the buckets around its negated key (nearly opposite vectors); the
  // azimuth test first, the exact test from the staged coordinates last
  const int wq = phi_window_q(a.phwin);
  for (int i = lane; i < m; i += kWave) {
    const double ux = Xh - double(s_x[w][i]), uy = Yh - double(s_y[w][i]), uz = Zh - double(s_z[w][i]);
    const double U2 = (ux * ux + uy * uy) + uz * uz;
    bool killed = false;
    const int nb = a.nb;
    const float ki = polar_key(ux, uy, uz);  // the staged key, recomputed
    const int pi = s_phi[w][i];
    for (int pass = 0; pass < (mirror ? 2 : 1) && !killed; ++pass) {
      const int c = bucket(pass == 0 ? ki : -ki, nb);
      const int q0 = s_bin[w][max(c - 1, 0)], q1 = s_bin[w][min(c + 2, nb)];
      for (int q = q0; q < q1 && !killed; ++q) {
        const int j = s_val[w][q];
        if (j == i || !phi_ok(pi, s_phi[w][j], wq, pass == 1)) continue;
        const double vx = Xh - double(s_x[w][j]), vy = Yh - double(s_y[w][j]), vz = Zh - double(s_z[w][j]);
        const double V2 = (vx * vx + vy * vy) + vz * vz;
        killed = kills(ux, uy, uz, U2, vx, vy, vz, V2, a.theta2);
      }
    }
    if (killed) a.keep[s_cell[w][i]] = 0;
  }
  }
}

// The outer hits with more than kCap cells, one work-group each (a
// persistent grid over the list): the hit's cells are staged in LDS (up to
// kBigCap; beyond, from global memory) and each thread tests its cells
// against all the others of the hit whose key is within the cut angle of
// its own or of its negative.
constexpr int kBigBlock = 1024;
constexpr int kBigCap = 3072;
constexpr int kBigSegs = 1024;

template <class T>
__global__ void __launch_bounds__(kBigBlock) k_fb_kill_big(FbArgs<T> a) {
  __shared__ T s_x[kBigCap], s_y[kBigCap], s_z[kBigCap];
  __shared__ float s_k[kBigCap];
  __shared__ int32_t s_cell[kBigCap];
  __shared__ int32_t s_start[kBigSegs + 1];
  const int nbig = *a.n_big;
  const float win = a.kwin;
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int h = a.big[b];
    const int sb = a.idx.seg_first[h], ns = a.idx.seg_first[h + 1] - sb;
    const double Xh = double(a.x[h]), Yh = double(a.y[h]), Zh = double(a.z[h]);
    __syncthreads();  // the previous hit's LDS is no longer read
    if (threadIdx.x == 0) {
      int run = 0;
      for (int q = 0; q < ns && q < kBigSegs; ++q) {
        s_start[q] = run;
        run += a.idx.seg[sb + q].y;
      }
      s_start[min(ns, kBigSegs)] = run;
    }
    __syncthreads();
    const int m = s_start[min(ns, kBigSegs)];
    if (ns <= kBigSegs && m <= kBigCap) {
      for (int f = threadIdx.x; f < m; f += kBigBlock) {
        int l = 0, r = ns - 1;  // the last segment starting at or before f
        while (l < r) {
          const int mid = (l + r + 1) >> 1;
          if (s_start[mid] <= f) l = mid; else r = mid - 1;
        }
        const int2 en = a.idx.ent[a.idx.seg[sb + l].x + (f - s_start[l])];
        const int ih = en.y & kHitMask;
        const T hx = a.x[ih], hy = a.y[ih], hz = a.z[ih];
        s_cell[f] = en.x;
        s_x[f] = hx;
        s_y[f] = hy;
        s_z[f] = hz;
        s_k[f] = polar_key(Xh - double(hx), Yh - double(hy), Zh - double(hz));
      }
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += kBigBlock) {
        const double ux = Xh - double(s_x[i]), uy = Yh - double(s_y[i]), uz = Zh - double(s_z[i]);
        const double U2 = (ux * ux + uy * uy) + uz * uz;
        const float ki = s_k[i];
        bool killed = false;
        for (int j = 0; j < m && !killed; ++j) {
          const float kj = s_k[j];
          if (j == i || (fabsf(kj - ki) > win && fabsf(kj + ki) > win)) continue;
          const double vx = Xh - double(s_x[j]), vy = Yh - double(s_y[j]), vz = Zh - double(s_z[j]);
          const double V2 = (vx * vx + vy * vy) + vz * vz;
          killed = kills(ux, uy, uz, U2, vx, vy, vz, V2, a.theta2);
        }
        if (killed) a.keep[s_cell[i]] = 0;
      }
    } else {
      // beyond the LDS: every pair from global memory, threads over the
      // hit's cells segment by segment
      for (int s = 0; s < ns; ++s) {
        const int2 gi = a.idx.seg[sb + s];
        for (int e = threadIdx.x; e < gi.y; e += kBigBlock) {
          const int2 en = a.idx.ent[gi.x + e];
          double ux, uy, uz, U2;
          vec(a, Xh, Yh, Zh, en.y & kHitMask, ux, uy, uz, U2);
          bool killed = false;
          for (int t = 0; t < ns && !killed; ++t) {
            const int2 gj = a.idx.seg[sb + t];
            for (int f = 0; f < gj.y && !killed; ++f) {
              const int2 ej = a.idx.ent[gj.x + f];
              if (ej.x == en.x) continue;
              double vx, vy, vz, V2;
              vec(a, Xh, Yh, Zh, ej.y & kHitMask, vx, vy, vz, V2);
              killed = kills(ux, uy, uz, U2, vx, vy, vz, V2, a.theta2);
            }
          }
          if (killed) a.keep[en.x] = 0;
        }
      }
    }
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

// Workspace after the outer-hit index: the flags, the copies, the scan's.
template <class T>
void carve_rest(Carver& c, FbArgs<T>* a, int cap, int n_hits, int32_t** tmp) {
  a->keep = c.take<int32_t>(static_cast<size_t>(cap) + 1);
  a->mid = c.take<int32_t>(static_cast<size_t>(n_hits));
  a->n_mid = c.take<int32_t>(1);
  a->big = c.take<int32_t>(static_cast<size_t>(n_hits));
  a->n_big = c.take<int32_t>(1);
  a->t_inner = c.take<int32_t>(static_cast<size_t>(cap));
  a->t_outer = c.take<int32_t>(static_cast<size_t>(cap));
  a->t_pair = c.take<uint8_t>(static_cast<size_t>(cap));
  *tmp = c.take<int32_t>(scan_tmp_elems(std::max(cap, n_hits) + 1));
}

// Work-groups of the listed kernel that are resident at once on this GPU:
// its grid is persistent, so more would only queue behind the first ones and
// fewer would leave wavefront slots empty (1536 against 1024 work-groups:
// 26.5 against 29.1 ms on the PU200 overlap batch).  Looked up once per
// device and input type, never while a graph is being captured (a plan looks
// it up when it is created); 1024 when unknown.
constexpr int kMaxDevices = 64;
std::mutex g_grid_mu;
int g_listed_grid[2][kMaxDevices] = {};

template <class T>
int listed_grid() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return 1024;
  std::lock_guard<std::mutex> g(g_grid_mu);
  int& v = g_listed_grid[sizeof(T) == sizeof(double)][dev];
  if (v == 0 && !g_capturing) {
    int cus = 0, per = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_fb_kill<T, kCap, 2, true>, 2 * kWave, 0) == hipSuccess &&
        cus > 0 && per > 0)
      v = cus * per;
    else
      (void)hipGetLastError();
  }
  return v > 0 ? v : 1024;
}

template <class T>
pt_err run_fishbone(const pt_hits& h, const DevCfg& k, pt_cells& cells, void* ws_base, hipStream_t s) {
  const int n_hits = h.n_hits;
  const int cap = cells.cap;
  if (n_hits == 0 || cap == 0) return PT_OK;
  Carver c(ws_base);
  FbArgs<T> a{};
  a.x = static_cast<const T*>(h.x);
  a.y = static_cast<const T*>(h.y);
  a.z = static_cast<const T*>(h.z);
  a.n_hits = n_hits;
  a.theta2 = k.fishbone_theta2;
  {
    // buckets at least 1% wider than the largest angle of two aligned
    // vectors (plus a margin far above the float rounding of the keys), so
    // that keys within that angle fall in the same or neighbouring buckets
    const double th = std::sqrt(k.fishbone_theta2);
    const double win = th >= 1.0 ? 2.0 : std::asin(th) + 1e-5;
    a.nb = static_cast<int32_t>(std::min<double>(kNB, std::max(1.0, std::floor(2.0 / (win * 1.01)))));
    a.kwin = static_cast<float>(win * 1.001);
    a.phwin = win < 0.9 * kS0 ? static_cast<float>(std::asin(win / kS0) * 1.01 + 1e-5) : 4.f;
  }
  a.count = cells.count;
  a.cap = cap;
  a.inner = cells.inner;
  a.outer = cells.outer;
  a.pair = cells.pair;
  a.inner_first = cells.inner_first;
  a.inner_count = cells.inner_count;
  const pt_err e = build_outer_index(h, cells, c, a.idx, s);
  if (e != PT_OK) return e;
  int32_t* tmp = nullptr;
  carve_rest(c, &a, cap, n_hits, &tmp);
  const int gc = grid_for(cap, kBlock);
  const int gh = grid_for(n_hits + 1, kBlock);
  PT_HIP_CHECK(fill_i32(a.n_big, 0, 1, s));
  PT_HIP_CHECK(fill_i32(a.n_mid, 0, 1, s));
  k_fb_flags<T><<<gc, kBlock, 0, s>>>(a);
  k_fb_kill<T, kCapSmall, kWaves, false><<<static_cast<unsigned>((n_hits + kWaves - 1) / kWaves), kBlock, 0, s>>>(a);
  k_fb_kill<T, kCap, 2, true><<<listed_grid<T>(), 2 * kWave, 0, s>>>(a);
  k_fb_kill_big<T><<<256, kBigBlock, 0, s>>>(a);
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
  c.off = ws_outer_index(n_hits, cells_cap);
  FbArgs<float> a{};
  int32_t* tmp = nullptr;
  carve_rest(c, &a, cells_cap, n_hits, &tmp);
  return c.off + 256;
}

void fishbone_prepare() {
  (void)listed_grid<float>();
  (void)listed_grid<double>();
}

pt_err launch_fishbone(const pt_hits& h, const DevCfg& k, pt_cells& cells, void* ws_base, hipStream_t s) {
  void* tok = timing_begin(s);
  const pt_err e = h.dtype == PT_F64 ? run_fishbone<double>(h, k, cells, ws_base, s)
                                     : run_fishbone<float>(h, k, cells, ws_base, s);
  timing_end(tok, "fishbone", s);
  return e;
}

}  // namespace pt
