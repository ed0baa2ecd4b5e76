// valu_rates.hip -- issue rate of VALU instruction classes on gfx950 (the
// rates behind the slot weights of the VALU roofline).  Every thread runs
// ITER iterations of 8 independent register chains and writes one word.
// Build and run: hipcc -O3 --offload-arch=gfx950 valu_rates.hip -o valu_rates
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdint>
constexpr int ITER = 2048;
#define CHAINS 8
#define DEFK(NAME, T, INIT, BODY)                                              \
__global__ void __launch_bounds__(256) NAME(uint32_t *out, uint32_t seed) {    \
  T a[CHAINS]; uint32_t b = seed ^ threadIdx.x, c = seed * 7u + 1u;           \
  (void)b; (void)c;                                                            \
  for (int i = 0; i < CHAINS; ++i) a[i] = INIT;                               \
  for (int it = 0; it < ITER; ++it) {                                          \
    _Pragma("unroll") for (int i = 0; i < CHAINS; ++i) { BODY; }              \
  }                                                                            \
  uint32_t r = 0;                                                              \
  for (int i = 0; i < CHAINS; ++i) r ^= (uint32_t)a[i];                       \
  out[blockIdx.x * 256 + threadIdx.x] = r;                                     \
}
DEFK(k_fma32, float, (float)(threadIdx.x + i), asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(a[i]) : "v"((float)b), "v"((float)c)))
DEFK(k_xor, uint32_t, threadIdx.x + i, asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[i]) : "v"(b)))
DEFK(k_xor3, uint32_t, threadIdx.x + i, asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(a[i]) : "v"(b), "v"(c)))
DEFK(k_alignbit, uint32_t, threadIdx.x + i, asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(a[i]) : "v"(b)))
DEFK(k_mulhi, uint32_t, threadIdx.x + i, asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b)))
DEFK(k_mullo, uint32_t, threadIdx.x + i, asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b)))
DEFK(k_mad64, uint64_t, threadIdx.x + i, {uint64_t cc; asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(a[i]), "=s"(cc) : "v"(b), "v"(c)); (void)cc;})
DEFK(k_sin, float, (float)(threadIdx.x + i) * 1e-3f, asm volatile("v_sin_f32 %0, %0" : "+v"(a[i])))
DEFK(k_log, float, (float)(threadIdx.x + i) + 2.f, asm volatile("v_log_f32 %0, %0" : "+v"(a[i])))
DEFK(k_sqrt, float, (float)(threadIdx.x + i) + 2.f, asm volatile("v_sqrt_f32 %0, %0" : "+v"(a[i])))
DEFK(k_fma64, double, (double)(threadIdx.x + i), asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(a[i]) : "v"((double)b), "v"((double)c)))
DEFK(k_cvt, float, (float)(threadIdx.x + i), asm volatile("v_cvt_f32_u32 %0, %1" : "=v"(a[i]) : "v"(b + (uint32_t)i)))

typedef void (*K)(uint32_t *, uint32_t);
int main() {
  const int blocks = 256 * 32, threads = 256;
  uint32_t *out;
  if (hipMalloc(&out, sizeof(uint32_t) * blocks * threads) != hipSuccess) return 1;
  struct { const char *n; K k; } ks[] = {{"v_fma_f32", k_fma32}, {"v_xor_b32", k_xor},
    {"v_bitop3_b32", k_xor3}, {"v_alignbit_b32", k_alignbit},
    {"v_mul_hi_u32", k_mulhi}, {"v_mul_lo_u32", k_mullo}, {"v_mad_u64_u32", k_mad64}, {"v_sin_f32", k_sin},
    {"v_log_f32", k_log}, {"v_sqrt_f32", k_sqrt}, {"v_fma_f64", k_fma64}, {"v_cvt_f32_u32", k_cvt}};
  hipEvent_t e0, e1; hipEventCreate(&e0); hipEventCreate(&e1);
  for (auto &k : ks) {
    hipLaunchKernelGGL(k.k, dim3(blocks), dim3(threads), 0, 0, out, 1u);
    hipEventRecord(e0);
    for (int r = 0; r < 3; ++r) hipLaunchKernelGGL(k.k, dim3(blocks), dim3(threads), 0, 0, out, 1u);
    hipEventRecord(e1); hipEventSynchronize(e1);
    float ms; hipEventElapsedTime(&ms, e0, e1);
    double ops = 3.0 * blocks * threads * (double)ITER * CHAINS;
    printf("%-16s %8.3f ms  %7.2f T lane-ops/s  (%.2f of 256x64x2.4G)\n", k.n, ms, ops / (ms * 1e-3) / 1e12,
           ops / (ms * 1e-3) / (256.0 * 64 * 2.4e9));
  }
  if (hipDeviceSynchronize() != hipSuccess) return 2;
  hipFree(out);
  return 0;
}
