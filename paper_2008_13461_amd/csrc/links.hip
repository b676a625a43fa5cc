// Cell linking (paper section 3.2: doublets that share a hit are tested for
// a compatible triplet).
//
// One thread per inner cell c' = (h0, h1).  Its candidates are the cells that
// start on h1, a contiguous run thanks to the grouping of the doublet step.
// The cheap division-free R-Z alignment test runs first; the circle test
// (divisions and square roots) only for the few candidates that pass it.  A
// thread keeps up to kLocal links in registers; the block then reserves space
// for all of its links with one atomic, so that every cell's outer links are
// contiguous (out_start, out_count) without a global sort.  Cells with more
// than kLocal links are finished by a second, rarely used kernel.
#include "pt_internal.h"

// Every decision below is made in double precision exactly as parenthesised.
#pragma clang fp contract(off)

namespace pt {
namespace {

constexpr int kLocal = 8;

template <class T>
struct LinkIn {
  int32_t n_hits;
  const T* x;
  const T* y;
  const T* z;
  const uint8_t* layer;
  const double* R;          // per hit, sqrt(X X + Y Y)
  const int32_t* cell_inner;
  const int32_t* cell_outer;
  const int32_t* cell_count;
  int32_t cells_cap;
  const int32_t* inner_first;
  const int32_t* inner_count;
  int32_t links_cap;
  int32_t* in_cell;
  int32_t* out_cell;
  int32_t* links_count;
  int32_t* out_start;
  int32_t* out_count;
  uint8_t* has_inner;
  int32_t* ovf;             // cells with more than kLocal links
  int32_t* ovf_count;
  uint32_t* status;
};

template <class T>
__global__ void k_radius(LinkIn<T> a, double* __restrict__ R) {
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < a.n_hits; h += gridDim.x * blockDim.x) {
    const double X = static_cast<double>(a.x[h]);
    const double Y = static_cast<double>(a.y[h]);
    R[h] = sqrt(X * X + Y * Y);
  }
}

__global__ void k_clear_has_inner(const int32_t* cell_count, int32_t cap, uint8_t* __restrict__ has_inner) {
  const int n = min(*cell_count, cap);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) has_inner[c] = 0;
}

// The triplet predicates documented in pixeltrack.h.  The R-Z part uses the
// per-hit radii; the beam-spot part the transverse coordinates.
struct Triplet {
  double X0, Y0, Z0, R0, X1, Y1, Z1, R1;
  double ar, az, La;  // R-Z segment h0 -> h1 and its squared length
  double rmax;
};

__device__ __forceinline__ bool rz_pass(const Triplet& t, double theta2, double R2, double Z2) {
  const double br = R2 - t.R1;
  const double bz = Z2 - t.Z1;
  const double A = t.ar * bz - t.az * br;
  return A * A <= theta2 * (t.La * (br * br + bz * bz));
}

__device__ __forceinline__ bool beam_pass(const Triplet& t, double X2, double Y2) {
  const double ux = t.X1 - t.X0, uy = t.Y1 - t.Y0;
  const double vx = X2 - t.X0, vy = Y2 - t.Y0;
  const double Dd = 2.0 * (ux * vy - uy * vx);
  if (Dd == 0.0) {
    const double cr = t.X0 * vy - t.Y0 * vx;
    return cr * cr <= (t.rmax * t.rmax) * (vx * vx + vy * vy);
  }
  const double U2 = ux * ux + uy * uy;
  const double V2 = vx * vx + vy * vy;
  const double cx = (U2 * vy - V2 * uy) / Dd;
  const double cy = (V2 * ux - U2 * vx) / Dd;
  const double rho2 = cx * cx + cy * cy;
  const double Cx = t.X0 + cx, Cy = t.Y0 + cy;
  const double c2 = Cx * Cx + Cy * Cy;
  return fabs(sqrt(c2) - sqrt(rho2)) <= t.rmax;
}

template <class T>
__device__ __forceinline__ bool link_pass(const DevCfg& k, const LinkIn<T>& a, const Triplet& t, int c) {
  const int h2 = a.cell_outer[c];
  const double Z2 = static_cast<double>(a.z[h2]);
  const double R2 = a.R[h2];
  const double theta2 = k.layer_barrel[a.layer[h2]] ? k.theta2_barrel : k.theta2_endcap;
  if (!rz_pass(t, theta2, R2, Z2)) return false;
  return beam_pass(t, static_cast<double>(a.x[h2]), static_cast<double>(a.y[h2]));
}

template <class T>
__device__ __forceinline__ void load_triplet(const DevCfg& k, const LinkIn<T>& a, int cp, Triplet& t,
                                             int& first, int& last) {
  const int h0 = a.cell_inner[cp];
  const int h1 = a.cell_outer[cp];
  t.X0 = static_cast<double>(a.x[h0]);
  t.Y0 = static_cast<double>(a.y[h0]);
  t.Z0 = static_cast<double>(a.z[h0]);
  t.R0 = a.R[h0];
  t.X1 = static_cast<double>(a.x[h1]);
  t.Y1 = static_cast<double>(a.y[h1]);
  t.Z1 = static_cast<double>(a.z[h1]);
  t.R1 = a.R[h1];
  t.ar = t.R1 - t.R0;
  t.az = t.Z1 - t.Z0;
  t.La = t.ar * t.ar + t.az * t.az;
  t.rmax = (a.layer[h0] == 0) ? k.rmax_bpix1 : k.rmax_other;
  first = a.inner_first[h1];
  last = min(first + a.inner_count[h1], a.cells_cap);
}

template <class T, int BLOCK>
__global__ void __launch_bounds__(BLOCK) k_links(DevCfg k, LinkIn<T> a) {
  __shared__ int32_t s_scan[BLOCK / kWave + 1];
  __shared__ int32_t s_base;
  const int n = min(*a.cell_count, a.cells_cap);
  const int stride = gridDim.x * BLOCK;
  const int rounds = (n + stride - 1) / stride;
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
  for (int r = 0; r < rounds; ++r) {
    const int cp = r * stride + blockIdx.x * BLOCK + threadIdx.x;
    int buf[kLocal];
    int cnt = 0;
    bool overflow = false;
    if (cp < n) {
      Triplet t;
      int first, last;
      load_triplet(k, a, cp, t, first, last);
      for (int c = first; c < last; ++c) {
        if (link_pass(k, a, t, c)) {
          if (cnt < kLocal) buf[cnt] = c;
          ++cnt;
        }
      }
      if (cnt > kLocal) {
        overflow = true;
        const int slot = atomicAdd(a.ovf_count, 1);
        a.ovf[slot] = cp;
        a.out_count[cp] = 0;
      }
    }
    const int mine = overflow ? 0 : cnt;
    // block-wide exclusive prefix of `mine`
    int v = mine;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int o = __shfl_up(v, d, kWave);
      if (lane >= d) v += o;
    }
    if (lane == kWave - 1) s_scan[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      int run = 0;
      for (int w = 0; w < BLOCK / kWave; ++w) {
        const int x = s_scan[w];
        s_scan[w] = run;
        run += x;
      }
      s_base = run ? atomicAdd(a.links_count, run) : 0;
    }
    __syncthreads();
    const int pos = s_base + s_scan[wave] + v - mine;
    __syncthreads();
    if (cp < n && !overflow) {
      a.out_start[cp] = pos;
      a.out_count[cp] = cnt;
      for (int i = 0; i < cnt; ++i) {
        const int c = buf[i];
        a.has_inner[c] = 1;
        if (pos + i < a.links_cap) {
          a.in_cell[pos + i] = cp;
          a.out_cell[pos + i] = c;
        }
      }
    }
  }
}

// Cells with more than kLocal outer links: count, reserve, then write.
template <class T>
__global__ void k_links_overflow(DevCfg k, LinkIn<T> a) {
  const int m = *a.ovf_count;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const int cp = a.ovf[i];
    Triplet t;
    int first, last;
    load_triplet(k, a, cp, t, first, last);
    int cnt = 0;
    for (int c = first; c < last; ++c) cnt += link_pass(k, a, t, c) ? 1 : 0;
    const int pos = atomicAdd(a.links_count, cnt);
    a.out_start[cp] = pos;
    a.out_count[cp] = cnt;
    int w = pos;
    for (int c = first; c < last; ++c) {
      if (link_pass(k, a, t, c)) {
        a.has_inner[c] = 1;
        if (w < a.links_cap) {
          a.in_cell[w] = cp;
          a.out_cell[w] = c;
        }
        ++w;
      }
    }
  }
}

__global__ void k_finish_links(const int32_t* count, int32_t cap, uint32_t* status) {
  if (*count > cap) status_flag(status, PT_FLAG_LINKS_OVERFLOW);
}

}  // namespace

size_t ws_links(int n_hits, int cells_cap) {
  Carver c(nullptr);
  c.take<double>(n_hits);
  c.take<int32_t>(cells_cap);
  c.take<int32_t>(1);
  return c.off + 256;
}

template <class T>
static pt_err run_links(const pt_hits& h, const DevCfg& k, const pt_cells& cells, pt_links& L,
                        uint32_t* status, pt_workspace ws, hipStream_t s, int block) {
  Carver c(ws.ptr);
  double* R = c.take<double>(h.n_hits);
  int32_t* ovf = c.take<int32_t>(cells.cap);
  int32_t* ovf_count = c.take<int32_t>(1);
  LinkIn<T> a{h.n_hits, static_cast<const T*>(h.x), static_cast<const T*>(h.y), static_cast<const T*>(h.z),
              h.layer, R, cells.inner, cells.outer, cells.count, cells.cap, cells.inner_first,
              cells.inner_count, L.cap, L.in_cell, L.out_cell, L.count, L.out_start, L.out_count,
              L.has_inner, ovf, ovf_count, status};
  if (fill_i32(L.count, 0, 1, s) != hipSuccess) return PT_ERR_DEVICE;
  if (fill_i32(ovf_count, 0, 1, s) != hipSuccess) return PT_ERR_DEVICE;
  k_radius<T><<<grid_for(h.n_hits, 256), 256, 0, s>>>(a, R);
  PT_LAUNCH_CHECK();
  k_clear_has_inner<<<grid_for(cells.cap, 256, 8192), 256, 0, s>>>(cells.count, cells.cap, L.has_inner);
  PT_LAUNCH_CHECK();
  void* tok = timing_begin(s);
  if (block == 128)
    k_links<T, 128><<<grid_for(cells.cap, 128, 32768), 128, 0, s>>>(k, a);
  else if (block == 512)
    k_links<T, 512><<<grid_for(cells.cap, 512, 8192), 512, 0, s>>>(k, a);
  else
    k_links<T, 256><<<grid_for(cells.cap, 256, 16384), 256, 0, s>>>(k, a);
  timing_end(tok, "links", s);
  PT_LAUNCH_CHECK();
  k_links_overflow<T><<<64, 64, 0, s>>>(k, a);
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
