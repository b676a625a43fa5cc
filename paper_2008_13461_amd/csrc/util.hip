// Device-wide exclusive scan and fill kernels.
#include "pt_internal.h"

namespace pt {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr int kTile = kScanBlock * kScanItems;
static_assert(kTile == kScanTile, "the tile of the declared scan steps");

// Inclusive scan of one int32 per thread across the block; returns the
// inclusive value and writes the block total to *total.
__device__ inline int32_t block_inclusive_scan(int32_t v, int32_t* lds, int32_t* total) {
  const int lane = threadIdx.x % kWave;
  const int wave = threadIdx.x / kWave;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t o = __shfl_up(v, d, kWave);
    if (lane >= d) v += o;
  }
  if (lane == kWave - 1) lds[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) {
      const int32_t t = lds[w];
      lds[w] = run;
      run += t;
    }
    lds[kScanBlock / kWave] = run;
  }
  __syncthreads();
  v += lds[wave];
  *total = lds[kScanBlock / kWave];
  __syncthreads();
  return v;
}

// n_dev, when given, holds the number of items actually present (<= n).
__device__ inline int64_t items(int64_t n, const int32_t* n_dev) {
  if (!n_dev) return n;
  const int64_t m = *n_dev;
  return m < 0 ? 0 : (m < n ? m : n);
}

// Sum of each tile (the order does not matter: consecutive threads read
// consecutive items).
__global__ void __launch_bounds__(kScanBlock) k_tile_sums(const int32_t* __restrict__ data, int64_t n,
                                                          const int32_t* __restrict__ n_dev,
                                                          int32_t* __restrict__ sums) {
  __shared__ int32_t lds[kScanBlock / kWave + 1];
  n = items(n, n_dev);
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kTile;
  if (first >= n) {  // a tile past the end
    if (threadIdx.x == 0) sums[blockIdx.x] = 0;
    return;
  }
  int32_t s = 0;
  if (first + kTile <= n) {
    int32_t v[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] = data[first + i * kScanBlock + threadIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) s += v[i];
  } else {
    for (int i = 0; i < kScanItems; ++i) {
      const int64_t at = first + i * kScanBlock + threadIdx.x;
      if (at < n) s += data[at];
    }
  }
  int32_t total;
  block_inclusive_scan(s, lds, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Scan of each tile plus its offset; each thread takes kScanItems
// consecutive items, read and written as 16-byte vectors when VEC (data
// 16-byte aligned) and the tile is full.
// src may equal dst.  The total goes to *total_out, or to dst[n] when
// total_out is null.
template <bool VEC>
__global__ void __launch_bounds__(kScanBlock) k_tile_scan(const int32_t* src, int32_t* dst, int64_t n,
                                                          const int32_t* __restrict__ n_dev,
                                                          const int32_t* __restrict__ offsets,
                                                          int32_t* __restrict__ total_out) {
  __shared__ int32_t lds[kScanBlock / kWave + 1];
  n = items(n, n_dev);
  const int64_t first = static_cast<int64_t>(blockIdx.x) * kTile;
  // the block holding the last item (block 0 when there is none) writes the total
  const int64_t last_block = n > 0 ? (n - 1) / kTile : 0;
  if (static_cast<int64_t>(blockIdx.x) > last_block) return;
  const int64_t base = first + threadIdx.x * kScanItems;
  const bool full = VEC && first + kTile <= n;
  int32_t v[kScanItems];
  if (full) {
    const int4* p = reinterpret_cast<const int4*>(src + base);
#pragma unroll
    for (int i = 0; i < kScanItems / 4; ++i) {
      const int4 q = p[i];
      v[4 * i] = q.x;
      v[4 * i + 1] = q.y;
      v[4 * i + 2] = q.z;
      v[4 * i + 3] = q.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) v[i] = (base + i < n) ? src[base + i] : 0;
  }
  int32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) s += v[i];
  int32_t total;
  const int32_t incl = block_inclusive_scan(s, lds, &total);
  int32_t run = incl - s + (offsets ? offsets[blockIdx.x] : 0);
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int32_t x = v[i];
    v[i] = run;
    run += x;
  }
  if (full) {
    int4* p = reinterpret_cast<int4*>(dst + base);
#pragma unroll
    for (int i = 0; i < kScanItems / 4; ++i) p[i] = make_int4(v[4 * i], v[4 * i + 1], v[4 * i + 2], v[4 * i + 3]);
  } else {
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
      if (base + i < n) dst[base + i] = v[i];
  }
  if (static_cast<int64_t>(blockIdx.x) == last_block && threadIdx.x == 0)
    (total_out ? *total_out : dst[n]) = total + (offsets ? offsets[blockIdx.x] : 0);
}

template <class T>
__global__ void k_fill(T* __restrict__ p, T v, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

}  // namespace

size_t scan_tmp_elems(int64_t n) {
  size_t total = 0;
  while (n > kTile) {
    const int64_t nb = (n + kTile - 1) / kTile;
    total += nb + 1;
    n = nb;
  }
  return total + 1;
}

hipError_t exclusive_scan_to(const int32_t* src, int32_t* dst, int64_t n, const int32_t* n_dev, int32_t* total,
                             int32_t* tmp, hipStream_t s) {
  if (n <= 0) {
    k_fill<int32_t><<<1, 1, 0, s>>>(total ? total : dst, 0, 1);
    return hipGetLastError();
  }
  const int64_t nb = (n + kTile - 1) / kTile;
  const bool vec = reinterpret_cast<uintptr_t>(src) % 16 == 0 && reinterpret_cast<uintptr_t>(dst) % 16 == 0;
  const int32_t* offsets = nullptr;
  if (nb > 1) {
    k_tile_sums<<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(src, n, n_dev, tmp);
    const hipError_t e = exclusive_scan_dev(tmp, nb, nullptr, tmp + nb + 1, s);
    if (e != hipSuccess) return e;
    offsets = tmp;
  }
  if (vec)
    k_tile_scan<true><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(src, dst, n, n_dev, offsets, total);
  else
    k_tile_scan<false><<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(src, dst, n, n_dev, offsets, total);
  return hipGetLastError();
}

hipError_t scan_tile_offsets(const int32_t* src, int64_t n, const int32_t* n_dev, int32_t* tmp, hipStream_t s,
                             const int32_t** offsets) {
  const int64_t nb = n > 0 ? (n + kTile - 1) / kTile : 1;
  *offsets = tmp;
  if (n <= 0) return fill_i32(tmp, 0, 2, s);
  k_tile_sums<<<static_cast<unsigned>(nb), kScanBlock, 0, s>>>(src, n, n_dev, tmp);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return exclusive_scan_dev(tmp, nb, nullptr, tmp + nb + 1, s);
}

hipError_t exclusive_scan_dev(int32_t* data, int64_t n, const int32_t* n_dev, int32_t* tmp, hipStream_t s) {
  return exclusive_scan_to(data, data, n, n_dev, nullptr, tmp, s);
}

hipError_t exclusive_scan(int32_t* data, int64_t n, int32_t* tmp, hipStream_t s) {
  return exclusive_scan_dev(data, n, nullptr, tmp, s);
}

hipError_t fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<int32_t><<<grid_for(n, 256, 4096), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

hipError_t fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill<uint8_t><<<grid_for(n, 256, 4096), 256, 0, s>>>(p, v, n);
  return hipGetLastError();
}

}  // namespace pt
