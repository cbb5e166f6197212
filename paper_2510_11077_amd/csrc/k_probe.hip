// Sustained FP64 FMA rate and shader clock of the device under full load: a
// diagnostic for roofline reports, not part of the method. The published
// FP64 peak assumes the maximum engine clock; with every SIMD issuing FP64
// FMAs the clock settles lower, so the rate this kernel sustains is the
// attainable ceiling for the FP64-VALU filter kernels.
//
// Every wave runs four independent FMA chains per lane (enough independent
// work for one wave to issue an FMA every cycle it may) and records, from
// lane 0, the shader-clock cycles (s_memtime) and the constant-rate wall
// clock (s_memrealtime) around its loop.
#include <algorithm>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

__device__ __forceinline__ unsigned long long shader_clock() {
  unsigned long long t;
  asm volatile("s_memtime %0\n\ts_waitcnt lgkmcnt(0)" : "=s"(t));
  return t;
}
__device__ __forceinline__ unsigned long long wall_clock() {
  unsigned long long t;
  asm volatile("s_memrealtime %0\n\ts_waitcnt lgkmcnt(0)" : "=s"(t));
  return t;
}

constexpr int kUnroll = 64;

// stamps[4 w + 0..3] = shader cycles, wall ticks, wall start, wall end of wave w
__global__ void k_fma_rate(double a, double b, int iters, double* sink,
                           unsigned long long* stamps) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  double x0 = 1.0 + 1e-3 * lane, x1 = x0 + 1.0, x2 = x0 + 2.0, x3 = x0 + 3.0;
  const unsigned long long c0 = shader_clock(), r0 = wall_clock();
  // the chains start after the first stamps
  asm volatile("" : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3), "+v"(a), "+v"(b));
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      x0 = __builtin_fma(x0, a, b);
      x1 = __builtin_fma(x1, a, b);
      x2 = __builtin_fma(x2, a, b);
      x3 = __builtin_fma(x3, a, b);
    }
  }
  const double x = (x0 + x1) + (x2 + x3);
  // the last stamps wait for the chains (a wave-uniform copy of their sum)
  const int dep = __builtin_amdgcn_readfirstlane((int)__builtin_bit_cast(unsigned long long, x));
  asm volatile("" ::"s"(dep));
  const unsigned long long c1 = shader_clock(), r1 = wall_clock();
  sink[blockIdx.x * blockDim.x + threadIdx.x] = x;
  if (lane == 0) {
    stamps[4 * w] = c1 - c0;
    stamps[4 * w + 1] = r1 - r0;
    stamps[4 * w + 2] = r0;
    stamps[4 * w + 3] = r1;
  }
}

}  // namespace

int fp64_rate(int waves_per_simd, int iters, double* tflops, double* clock_mhz,
              hipStream_t st) {
  int dev = 0, n_cu = 0, wall_khz = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, dev));
  if (n_cu <= 0 || wall_khz <= 0) return fail(ARGUS_E_HIP, "device attributes unavailable");
  const int block = 4 * kWave * waves_per_simd;  // one block per CU, waves on its 4 SIMDs
  const int64_t threads = (int64_t)n_cu * block, waves = threads / kWave;
  DevBuf sink, stamps;
  int rc = sink.alloc((size_t)threads * sizeof(double));
  if (!rc) rc = stamps.alloc((size_t)waves * 4 * sizeof(unsigned long long));
  if (rc) return rc;
  // a short launch first (clocks ramp up), then the measured one
  hipLaunchKernelGGL(k_fma_rate, dim3(n_cu), dim3(block), 0, st, 0.999999, 1e-9, iters / 16 + 1,
                     sink.as<double>(), stamps.as<unsigned long long>());
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_fma_rate, dim3(n_cu), dim3(block), 0, st, 0.999999, 1e-9, iters,
                     sink.as<double>(), stamps.as<unsigned long long>());
  HIPCHK(hipGetLastError());
  std::vector<unsigned long long> h((size_t)waves * 4);
  HIPCHK(hipMemcpyAsync(h.data(), stamps.p, h.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  double cyc = 0.0, ticks = 0.0;
  unsigned long long t0 = ~0ull, t1 = 0;
  for (int64_t w = 0; w < waves; ++w) {
    cyc += (double)h[4 * w];
    ticks += (double)h[4 * w + 1];
    t0 = std::min(t0, h[4 * w + 2]);
    t1 = std::max(t1, h[4 * w + 3]);
  }
  if (!(t1 > t0) || !(ticks > 0.0)) return fail(ARGUS_E_HIP, "clock stamps not advancing");
  const double span_s = (double)(t1 - t0) / (wall_khz * 1e3);
  const double flop = 2.0 * 4.0 * kUnroll * (double)iters * (double)threads;
  *tflops = flop / span_s / 1e12;
  *clock_mhz = cyc / ticks * (wall_khz * 1e-3);
  return ARGUS_OK;
}

}  // namespace argus
