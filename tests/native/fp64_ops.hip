// Test kernel: double-precision division and square root on the GPU, for a
// bit-for-bit comparison with the host's IEEE results.  The set-defining
// predicates of the library (doublet and link cuts) use only + - * / and
// sqrt on doubles; the first three are single hardware instructions, while
// division and square root are instruction sequences chosen by the
// compiler, so the test checks that those sequences round correctly, built
// with the library's own compiler flags.  Test infrastructure only.
#include <hip/hip_runtime.h>

#include <cstdint>

__global__ void k_div_sqrt(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ q,
                           double* __restrict__ r, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    q[i] = a[i] / b[i];
    r[i] = sqrt(a[i]);
  }
}

// q[i] = a[i] / b[i], r[i] = sqrt(a[i]) for i < n (device pointers), on
// `stream`.  Returns 0 on success, 1 on a launch error.
extern "C" int fp64_div_sqrt(const double* a, const double* b, double* q, double* r, int64_t n, void* stream) {
  if (n <= 0) return 0;
  int64_t g = (n + 255) / 256;
  if (g > 65536) g = 65536;
  k_div_sqrt<<<static_cast<int>(g), 256, 0, static_cast<hipStream_t>(stream)>>>(a, b, q, r, n);
  return hipGetLastError() == hipSuccess ? 0 : 1;
}
