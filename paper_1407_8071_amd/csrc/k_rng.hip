// k_rng.hip -- bulk Philox4x32-10 words and Box-Muller normals for the
// random-number parity hook: element i comes from counter (i/4, c1, c2, c3),
// lane i%4.
#include "pf_internal.h"

namespace pfk {
namespace {

__global__ void __launch_bounds__(256)
k_philox_stream(Key key, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                uint32_t *__restrict__ bits, float *__restrict__ z) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i0 = g * 4;
  if (i0 >= n) return;
  const uint4 w = philox((uint32_t)g, c1, c2, c3, key);
  float zz[4];
  normals4(w, zz);
  const uint32_t ww[4] = {w.x, w.y, w.z, w.w};
  for (int l = 0; l < 4 && i0 + l < n; ++l) {
    if (bits) bits[i0 + l] = ww[l];
    if (z) z[i0 + l] = zz[l];
  }
}

}  // namespace

hipError_t launch_philox_stream(uint64_t seed, uint32_t c1, uint32_t c2, uint32_t c3, int64_t n,
                                uint32_t *bits, float *z, hipStream_t s) {
  const int64_t calls = (n + 3) / 4;
  const unsigned blocks = (unsigned)((calls + 255) / 256);
  if (blocks > 0)
    k_philox_stream<<<blocks, 256, 0, s>>>(make_key(seed), c1, c2, c3, n, bits, z);
  return hipGetLastError();
}

}  // namespace pfk
