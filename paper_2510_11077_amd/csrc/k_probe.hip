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

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Matrix-core rate: independent accumulator chains per wave of
// v_mfma_f64_16x16x4f64 (KIND 1: eight chains, 2,048 FLOP each) or
// v_mfma_f32_32x32x16_bf16 (KIND 2: four chains of 16 accumulators, 32,768
// FLOP each), so the accumulators fit in registers; stamps as above.
constexpr int kMfmaChains64 = 8, kMfmaChains16 = 4;
template <int KIND>
__global__ void __launch_bounds__(1024)
    k_mfma_rate(double a, int iters, double* sink, unsigned long long* stamps) {
  const int lane = threadIdx.x & (kWave - 1);
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const double av = a + 1e-3 * lane, bv = 1.0 - 1e-3 * lane;
  double t = 0.0;
  unsigned long long c0, r0;
  if constexpr (KIND == 1) {
    f64x4 c[kMfmaChains64];
#pragma unroll
    for (int j = 0; j < kMfmaChains64; ++j) c[j] = f64x4{0.0, 0.0, 0.0, 0.0};
    double x = av, y = bv;
    c0 = shader_clock();
    r0 = wall_clock();
    asm volatile("" : "+v"(x), "+v"(y));
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < kMfmaChains64; ++j)
        c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < kMfmaChains64; ++j) t += c[j][0];
  } else {
    f32x16 c[kMfmaChains16];
    bf16x8 a16, b16;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a16[e] = (__bf16)(float)(av + e);
      b16[e] = (__bf16)(float)(bv - e);
    }
#pragma unroll
    for (int j = 0; j < kMfmaChains16; ++j)
#pragma unroll
      for (int e = 0; e < 16; ++e) c[j][e] = 0.0f;
    c0 = shader_clock();
    r0 = wall_clock();
    asm volatile("" : "+v"(a16), "+v"(b16));
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int j = 0; j < kMfmaChains16; ++j)
        c[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a16, b16, c[j], 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < kMfmaChains16; ++j) t += (double)c[j][0];
  }
  const int dep = __builtin_amdgcn_readfirstlane((int)__builtin_bit_cast(unsigned long long, t));
  asm volatile("" ::"s"(dep));
  const unsigned long long c1 = shader_clock(), r1 = wall_clock();
  sink[blockIdx.x * blockDim.x + threadIdx.x] = t;
  if (lane == 0) {
    stamps[4 * w] = c1 - c0;
    stamps[4 * w + 1] = r1 - r0;
    stamps[4 * w + 2] = r0;
    stamps[4 * w + 3] = r1;
  }
}

}  // namespace

// kind 0: FP64 FMA (vector ALU); 1: FP64 MFMA; 2: BF16 MFMA
int device_rate(int kind, int waves_per_simd, int iters, double* tflops, double* clock_mhz,
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
  for (const int n : {iters / 16 + 1, iters}) {
    if (kind == 0)
      hipLaunchKernelGGL(k_fma_rate, dim3(n_cu), dim3(block), 0, st, 0.999999, 1e-9, n,
                         sink.as<double>(), stamps.as<unsigned long long>());
    else if (kind == 1)
      hipLaunchKernelGGL(k_mfma_rate<1>, dim3(n_cu), dim3(block), 0, st, 0.5, n, sink.as<double>(),
                         stamps.as<unsigned long long>());
    else
      hipLaunchKernelGGL(k_mfma_rate<2>, dim3(n_cu), dim3(block), 0, st, 0.5, n, sink.as<double>(),
                         stamps.as<unsigned long long>());
    HIPCHK(hipGetLastError());
  }
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
  const double per_wave_iter = kind == 0 ? 2.0 * 4.0 * kUnroll * kWave  // FMA chains, all lanes
                              : kind == 1 ? kMfmaChains64 * 2048.0       // MFMA 16x16x4 FP64
                                          : kMfmaChains16 * 32768.0;     // MFMA 32x32x16 BF16
  const double flop = per_wave_iter * (double)iters * (double)waves;
  *tflops = flop / span_s / 1e12;
  *clock_mhz = cyc / ticks * (wall_khz * 1e-3);
  return ARGUS_OK;
}

}  // namespace argus
