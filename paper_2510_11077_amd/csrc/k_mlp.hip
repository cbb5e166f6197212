// Learned surrogate of the log-likelihood: an MLP d -> w -> w -> w -> 1 with
// SiLU hidden layers, inference and training (forward, backward, Adam), and
// the delayed-acceptance screening kernels that use it. (The paper's
// inference integrates the likelihood with samplers, Functionality,
// "Sampler Integration"; the surrogate screens proposals so that the exact
// filter runs only on stage-1 survivors, Christen & Fox 2005.)
//
// Arithmetic: hidden-layer weights, inputs and activations in BF16, products
// on the matrix cores (v_mfma_f32_32x32x16_bf16) with FP32 accumulation;
// biases, the 1-unit output layer, gradients and Adam state in FP32.
//
// Every GEMM is written C[m][n] = sum_k X[m][k] Y[n][k] with both operands
// K-contiguous, so each lane feeds the MFMA with one 16-B load per operand:
//   forward   Z_l  = A_{l-1} W_l^T       X = A_{l-1} [B x in],  Y = W_l [out x in]
//   backward  dA   = dZ_l W_l            X = dZ_l [B x out],    Y = W_l^T [in x out]
//   weights   dW_l = dZ_l^T A_{l-1}      X = dZ_l^T [out x B],  Y = A_{l-1}^T [in x B]
// so the forward and backward epilogues also write transposed copies.
// MFMA 32x32x16 lane layout (checked on the device): A row l%32, k
// 8(l/32)..+7; B column l%32, same k; accumulator r of lane l is row
// 8(r/4) + 4(l/32) + r%4, column l%32.
#include <algorithm>
#include <cmath>
#include <type_traits>
#include <vector>

#include "argus_host.h"
#include "argus_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

namespace argus {

namespace {

enum { EPI_FWD = 0, EPI_BWD = 1, EPI_WGRAD = 2 };

struct GemmArgs {
  const __bf16* X;
  const __bf16* Y;
  int ldx, ldy, M, N, K;
  const float* bias;  // FWD [N]
  float* zout;        // FWD [M x N] pre-activation, nullable
  __bf16* out;        // FWD/BWD [M x ldo], nullable
  __bf16* outT;       // FWD/BWD [N x ldoT], nullable
  int ldo, ldoT;
  const float* zin;   // BWD [M x N] pre-activation of the layer being entered
  float* C;           // WGRAD [M x ldc]
  int ldc;
  float* part;        // WGRAD split over K: partial products [gridDim.z][M x N]
  int kchunk;         // K per workgroup along z (a multiple of 16)
};

// logistic function with the fast exponential and the hardware reciprocal
// (errors of a few FP32 ulp, far below the BF16 rounding of every use)
__device__ __forceinline__ float sigm(float z) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
  const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m0 = blockIdx.x * 64 + (w >> 1) * 32;
  const int n0 = blockIdx.y * 64 + (w & 1) * 32;
  // rows/columns past the edge are clamped for the loads, never stored
  const int mr = min(m0 + (l & 31), g.M - 1);
  const int nr = min(n0 + (l & 31), g.N - 1);
  const int kk = (l >> 5) * 8;
  const __bf16* xp = g.X + (size_t)mr * g.ldx + kk;
  const __bf16* yp = g.Y + (size_t)nr * g.ldy + kk;
  f32x16 acc = {};
  const int kb = blockIdx.z * g.kchunk, ke = min(g.K, kb + g.kchunk);
  for (int k = kb; k < ke; k += 16) {
    const bf16x8 a = *reinterpret_cast<const bf16x8*>(xp + k);
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(yp + k);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
  }
  const int col = n0 + (l & 31);
  if (col >= g.N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = m0 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    if (row >= g.M) continue;
    const float v = acc[r];
    if (EPI == EPI_WGRAD) {
      if (g.part)
        g.part[((size_t)blockIdx.z * g.M + row) * g.N + col] = v;
      else
        g.C[(size_t)row * g.ldc + col] = v;
    } else {
      float o;
      if (EPI == EPI_FWD) {
        const float z = v + g.bias[col];
        if (g.zout) g.zout[(size_t)row * g.N + col] = z;
        o = z * sigm(z);  // SiLU
      } else {
        const float z = g.zin[(size_t)row * g.N + col];
        const float s = sigm(z);
        o = v * (s * (1.0f + z * (1.0f - s)));  // dA * SiLU'(z)
      }
      const __bf16 ob = (__bf16)o;
      if (g.out) g.out[(size_t)row * g.ldo + col] = ob;
      if (g.outT) g.outT[(size_t)col * g.ldoT + row] = ob;
    }
  }
}

// Sum of the split-K partial products in split order (deterministic).
__global__ void __launch_bounds__(256) k_sum_parts(const float* part, int nsplit, int M, int N,
                                                   float* C, int ldc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  const int64_t mn = (int64_t)M * N;
  float acc = part[i];
  for (int s2 = 1; s2 < nsplit; ++s2) acc += part[s2 * mn + i];
  const int64_t row = i / N, col = i - row * N;
  C[row * ldc + col] = acc;
}

// Inputs through the affine input map x = T (theta - c) (T row-major d x d;
// the box map is T = diag(2 / (hi - lo)), c = (lo + hi) / 2), evaluated in
// FP64 with the products summed in index order, rounded to FP32 and then to
// BF16, padded with zero columns to kKin; optional transposed copy and
// standardised targets.
constexpr int kKin = 32;

__device__ __forceinline__ double map_input(const double* th_row, int d, int k, const double* c,
                                            const double* T) {
  double acc = 0.0;
  for (int j = 0; j < d; ++j) acc = fma(T[k * d + j], th_row[j] - c[j], acc);
  return acc;
}

__global__ void k_prep(const double* theta, int64_t B, int d_in, const double* c,
                       const double* T, __bf16* x0, __bf16* x0T, int ldT,
                       const double* target, double mu, double sd, float* t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * kKin) return;
  const int64_t m = i / kKin;
  const int k = (int)(i - m * kKin);
  float v = 0.0f;
  if (k < d_in) v = (float)map_input(theta + m * d_in, d_in, k, c, T);
  const __bf16 b = (__bf16)v;
  x0[m * kKin + k] = b;
  if (x0T) x0T[(int64_t)k * ldT + m] = b;
  if (t && k == 0) t[m] = (float)((target[m] - mu) / sd);
}

// Output layer in FP32: o = sum_n a3[m][n] W4[n] + b4 (index order).
__device__ __forceinline__ float out_row(const __bf16* a3, int width, const float* W4,
                                         float b4) {
  float acc = 0.0f;
  for (int n = 0; n < width; n += 8) {
    const bf16x8 v = *reinterpret_cast<const bf16x8*>(a3 + n);
#pragma unroll
    for (int j = 0; j < 8; ++j) acc = fmaf((float)v[j], W4[n + j], acc);
  }
  return acc + b4;
}

__global__ void k_out_eval(const __bf16* a3, int64_t Q, int width, const float* W4,
                           const float* b4, double mu, double sd, double* out) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= Q) return;
  const float o = out_row(a3 + m * width, width, W4, b4[0]);
  out[m] = (double)o * sd + mu;
}

// Fused inference for width W <= 256: one persistent block of W / 32 waves
// per CU. Wave w owns output columns [32 w, 32 w + 32) of every hidden layer
// and keeps those columns of W1, W2, W3 in registers as MFMA B fragments for
// the whole launch; 64-row chunks of queries go through standardisation,
// the three hidden layers (activations in LDS, BF16, ping-pong) and the FP32
// output layer. Same rounding as the unfused path: inputs, weights and each
// activation in BF16, FP32 accumulation, bias and SiLU in FP32.
//
// Within a layer a wave runs the MFMA chain of 32-row block 1 interleaved
// with the SiLU epilogue of block 0 (two transcendentals per element), so
// that the matrix core and the vector unit can work at the same time. Two
// waves share each SIMD: 64 columns per wave would halve the LDS reads of
// the A fragments, but its weight fragments need one wave per SIMD, which
// then stalls on every LDS read and MFMA result (measured 1.7x slower).
constexpr int kFusedRows = 64;
struct FusedArgs {
  const double* theta;   // [Q x d_in]
  const double* c;       // [d_in] input map centre
  const double* T;       // [d_in x d_in] input map matrix
  const __bf16* W1;      // [W x kKin]
  const __bf16* W2F;     // [W x W] in fragment order (frag_index)
  const __bf16* W3F;
  const float* p32;      // packed FP32 parameters (biases, W4, b4)
  double* out;           // [Q]
  int64_t Q;
  int d_in;
  double mu, sd;
};

template <int W>
__global__ void __launch_bounds__(W * 2) k_mlp_fused(FusedArgs f) {
  constexpr int NW = W / 32;     // waves
  constexpr int KS = W / 16;     // K steps of a hidden layer
  constexpr int R = kFusedRows;  // query rows per chunk
  constexpr int RB = R / 32;      // 32-row MFMA blocks per chunk
  constexpr int LDA = W + 8;     // activation row stride (16-B pad: b128 reads spread over banks)
  constexpr int LDX = kKin + 8;
  __shared__ __bf16 s_x[R * LDX];
  __shared__ __bf16 s_a[2][R * LDA];
  __shared__ float s_o[NW][R];
  __shared__ double s_th[R * kKin];   // a chunk's theta rows minus c, d per row
  __shared__ double s_T[kKin * kKin];  // input map matrix (d x d)
  __shared__ double s_c[kKin];         // input map centre
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int ncol = 32 * w + (l & 31);     // B-fragment / accumulator column
  const int kh = 8 * (l >> 5);            // this lane's K half within a step
  const int d = f.d_in;
  // a chunk's theta rows (R x d doubles, contiguous) loaded into registers
  // one chunk ahead, flat and coalesced (rows past Q read as zero)
  constexpr int NT = NW * 64, PF = (R * kKin + NT - 1) / NT;
  double pf[PF];
  auto fetch = [&](int64_t row0) {
    const int64_t base = row0 * d;
    const int64_t end = (row0 + R < f.Q ? row0 + R : f.Q) * d;
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int i = t + j * NT;
      pf[j] = (i < R * d && base + i < end) ? f.theta[base + i] : 0.0;
    }
  };
  // the first chunk's inputs before the weights, so that its wait does not
  // also wait for the weight fragments
  fetch((int64_t)blockIdx.x * R);
  for (int i = t; i < d * d; i += NT) s_T[i] = f.T[i];
  if (t < d) s_c[t] = f.c[t];
  bf16x8 w1[2], w2[KS], w3[KS];
#pragma unroll
  for (int ks = 0; ks < 2; ++ks)
    w1[ks] = *reinterpret_cast<const bf16x8*>(f.W1 + (size_t)ncol * kKin + 16 * ks + kh);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    // 1 KB contiguous per wave and K step
    const size_t fo = ((size_t)(w * KS + ks) * 64 + l) * 8;
    w2[ks] = *reinterpret_cast<const bf16x8*>(f.W2F + fo);
    w3[ks] = *reinterpret_cast<const bf16x8*>(f.W3F + fo);
  }
  const float* b1 = f.p32 + (int64_t)W * d;
  const float* b2 = b1 + W + (int64_t)W * W;
  const float* b3 = b2 + W + (int64_t)W * W;
  const float* W4 = b3 + W;
  const float bias1 = b1[ncol], bias2 = b2[ncol], bias3 = b3[ncol], b4 = W4[W];

  // one hidden layer: src rows (stride lds) x this wave's 32 columns -> dst;
  // ksn carries the number of K steps as a type (2 for the input layer).
  // Accumulator element r of 32-row block rb is row rb*32 + 8(r/4) + 4(l/32)
  // + r%4 of column ncol.
  auto layer = [&](auto ksn, const __bf16* src, int lds, const bf16x8* wf, float bias,
                   __bf16* dst) {
    constexpr int KSN = decltype(ksn)::value;
    const __bf16* ap0 = src + (l & 31) * lds + kh;
    auto epi = [&](const f32x16& acc, int rb, int r) {
      const int row = rb * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
      const float z = acc[r] + bias;
      dst[row * LDA + ncol] = (__bf16)(z * sigm(z));
    };
    f32x16 cur = {};
#pragma unroll
    for (int ks = 0; ks < KSN; ++ks) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap0 + 16 * ks);
      cur = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, wf[ks], cur, 0, 0, 0);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      if (rb + 1 < RB) {
        // chain of block rb + 1, one K step at a time, with the epilogue
        // elements of block rb spread evenly between its MFMAs
        f32x16 nxt = {};
        const __bf16* ap = ap0 + (rb + 1) * 32 * lds;
#pragma unroll
        for (int ks = 0; ks < KSN; ++ks) {
          const bf16x8 a = *reinterpret_cast<const bf16x8*>(ap + 16 * ks);
          nxt = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, wf[ks], nxt, 0, 0, 0);
#pragma unroll
          for (int r = ks * 16 / KSN; r < (ks + 1) * 16 / KSN; ++r) epi(cur, rb, r);
        }
        cur = nxt;
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) epi(cur, rb, r);
      }
    }
  };

  __syncthreads();  // s_T, s_c
  for (int64_t c = blockIdx.x; c * R < f.Q; c += gridDim.x) {
    const int64_t row0 = c * R;
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int i = t + j * NT;
      if (i < R * d) s_th[i] = pf[j] - s_c[i % d];
    }
    fetch(row0 + (int64_t)gridDim.x * R);
    __syncthreads();
    // mapped inputs x = T (theta - c) in FP64, summed in index order, then
    // FP32 and BF16 (as map_input); a thread's column k = t mod kKin is the
    // same for all of its elements
#pragma unroll
    for (int j = 0; j < PF; ++j) {
      const int i = t + j * NT;
      const int m = i / kKin, k = i - m * kKin;
      if (i < R * kKin) {
        double acc = 0.0;
        if (k < d)
          for (int jj = 0; jj < d; ++jj) acc = fma(s_T[k * d + jj], s_th[m * d + jj], acc);
        s_x[m * LDX + k] = (__bf16)(float)acc;
      }
    }
    __syncthreads();
    layer(std::integral_constant<int, 2>{}, s_x, LDX, w1, bias1, s_a[0]);
    __syncthreads();
    layer(std::integral_constant<int, KS>{}, s_a[0], LDA, w2, bias2, s_a[1]);
    __syncthreads();
    layer(std::integral_constant<int, KS>{}, s_a[1], LDA, w3, bias3, s_a[0]);
    __syncthreads();
    // output layer in FP32: wave w sums its 32 columns for rows l + 64 h
#pragma unroll
    for (int hr = 0; hr < R / 64; ++hr) {
      const __bf16* ar = s_a[0] + (l + 64 * hr) * LDA + 32 * w;
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < 32; j += 8) {
        const bf16x8 v = *reinterpret_cast<const bf16x8*>(ar + j);
#pragma unroll
        for (int i = 0; i < 8; ++i) acc = fmaf((float)v[i], W4[32 * w + j + i], acc);
      }
      s_o[w][l + 64 * hr] = acc;
    }
    __syncthreads();
    static_assert(2 * W >= R, "one thread per output row");
    if (t < R && row0 + t < f.Q) {
      float o = 0.0f;
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) o += s_o[ww][t];
      f.out[row0 + t] = (double)(o + b4) * f.sd + f.mu;
    }
  }
}

// Training head: o, residual, dout = 2 (o - t) / B, squared residual.
__global__ void k_out_train(const __bf16* a3, int64_t B, int width, const float* W4,
                            const float* b4, const float* t, float* dout, float* sq) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= B) return;
  const float o = out_row(a3 + m * width, width, W4, b4[0]);
  const float d = o - t[m];
  dout[m] = 2.0f * d / (float)B;
  sq[m] = d * d;
}

// dZ3[m][n] = bf16(dout[m] W4[n] SiLU'(z3[m][n])), both layouts.
__global__ void k_dz_last(const float* dout, const float* W4, const float* z3, int64_t B,
                          int width, __bf16* dz, __bf16* dzT, int ldT) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= B * width) return;
  const int64_t m = i / width;
  const int n = (int)(i - m * width);
  const float z = z3[i];
  const float s = sigm(z);
  const __bf16 b = (__bf16)(dout[m] * W4[n] * (s * (1.0f + z * (1.0f - s))));
  dz[i] = b;
  dzT[(int64_t)n * ldT + m] = b;
}

// Fixed-order block reduction of 256 per-thread partial sums (deterministic).
__device__ __forceinline__ float block_sum(float v, float* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const float r = sh[0];
  __syncthreads();
  return r;
}

// Row sums of a [rows x ld] bf16 matrix over its first B columns (the bias
// gradients, from the transposed dZ): one block per row, each thread sums a
// strided slice, then a fixed-order tree.
__global__ void __launch_bounds__(256) k_rowsum_bf16(const __bf16* a, int rows, int64_t B,
                                                     int64_t ld, float* out) {
  __shared__ float sh[256];
  const int r = blockIdx.x;
  const __bf16* p = a + r * ld;
  float acc = 0.0f;
  for (int64_t m = threadIdx.x; m < B; m += 256) acc += (float)p[m];
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) out[r] = acc;
}

// Output-layer gradients and the loss: block n < width computes
// gW4[n] = sum_m dout[m] a3T[n][m]; block `width` computes gb4 = sum_m dout[m]
// and loss = sum_m sq[m] / B. Fixed-order reductions.
__global__ void __launch_bounds__(256) k_head_grad(const float* dout, const float* sq,
                                                   const __bf16* a3T, int64_t ldT, int64_t B,
                                                   int width, float* gW4, float* gb4,
                                                   float* loss) {
  __shared__ float sh[256];
  const int n = blockIdx.x;
  if (n < width) {
    const __bf16* p = a3T + n * ldT;
    float acc = 0.0f;
    for (int64_t m = threadIdx.x; m < B; m += 256) acc = fmaf(dout[m], (float)p[m], acc);
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) gW4[n] = acc;
    return;
  }
  float a = 0.0f, q = 0.0f;
  for (int64_t m = threadIdx.x; m < B; m += 256) {
    a += dout[m];
    q += sq[m];
  }
  a = block_sum(a, sh);
  q = block_sum(q, sh);
  if (threadIdx.x == 0) {
    *gb4 = a;
    *loss = q / (float)B;
  }
}

// Fragment order of a [W x W] hidden weight (W a multiple of 32) for the
// fused inference kernel, where wave w = n / 32 holds rows [32 w, 32 w + 32)
// as B fragments of v_mfma_f32_32x32x16_bf16: lane n % 32 + 32 ((k % 16) / 8)
// of K step k / 16 holds 8 consecutive k, so each wave reads 1 KB contiguous
// per K step.
constexpr int kFusedMaxWidth = 256;
__device__ __forceinline__ int64_t frag_index(int64_t n, int64_t k, int64_t W) {
  const int64_t w = n >> 5, c = n & 31, ks = k >> 4, h = (k >> 3) & 1, e = k & 7;
  return (((w * (W >> 4) + ks) << 6) + c + 32 * h) * 8 + e;
}

struct AdamArgs {
  float* master;
  float* m;
  float* v;
  const float* g;
  float* p32;             // the handle's FP32 copy (biases, output layer)
  __bf16 *w1, *w2, *w3;   // BF16 hidden weights [w x kKin], [w x w], [w x w]
  __bf16 *w2T, *w3T;      // transposed copies
  __bf16 *w2F, *w3F;      // fragment-ordered copies for the fused kernels, or null
  __bf16 *w2TF, *w3TF;    // fragment-ordered copies of the transposes (fused training), or null
  int64_t n;
  int d_in, width;
  // 1 - beta is formed in double on the host: 1.0f - 0.999f is 1.3e-5 off
  float lr, b1, b2, omb1, omb2, eps, c1, c2;  // c1 = 1/(1-b1^t), c2 = 1/(1-b2^t)
  int do_update;                  // 0: only refresh the copies from master
};

__device__ __forceinline__ void scatter_copy(const AdamArgs& a, int64_t i, float w) {
  a.p32[i] = w;
  const int64_t dW = a.width, o1 = 0, o2 = (int64_t)dW * a.d_in + dW,
                o3 = o2 + dW * dW + dW;
  const __bf16 b = (__bf16)w;
  if (i < o1 + dW * a.d_in) {
    const int64_t n = (i - o1) / a.d_in, k = (i - o1) % a.d_in;
    a.w1[n * kKin + k] = b;
  } else if (i >= o2 && i < o2 + dW * dW) {
    const int64_t n = (i - o2) / dW, k = (i - o2) % dW;
    a.w2[n * dW + k] = b;
    a.w2T[k * dW + n] = b;
    if (a.w2F) a.w2F[frag_index(n, k, dW)] = b;
    if (a.w2TF) a.w2TF[frag_index(k, n, dW)] = b;
  } else if (i >= o3 && i < o3 + dW * dW) {
    const int64_t n = (i - o3) / dW, k = (i - o3) % dW;
    a.w3[n * dW + k] = b;
    a.w3T[k * dW + n] = b;
    if (a.w3F) a.w3F[frag_index(n, k, dW)] = b;
    if (a.w3TF) a.w3TF[frag_index(k, n, dW)] = b;
  }
}

__global__ void k_adam(AdamArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  float w = a.master[i];
  if (a.do_update) {
    const float g = a.g[i];
    const float m = a.b1 * a.m[i] + a.omb1 * g;
    const float v = a.b2 * a.v[i] + a.omb2 * g * g;
    a.m[i] = m;
    a.v[i] = v;
    w -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
    a.master[i] = w;
  }
  scatter_copy(a, i, w);
}

// ------------------------------------------------------ fused training
// Training step for W <= 256 in two launches, with the arithmetic of the
// general path (the same BF16 roundings: inputs, hidden weights, hidden
// activations and the pre-activation gradients dz; FP32 accumulation;
// biases, output layer and optimiser state in FP32):
//
// k_train_rows: one workgroup of W/32 waves per 32-row chunk of the batch.
// Rows are gathered through an index list (a shuffled epoch reads the
// training set in place), mapped to inputs, and taken through the three
// hidden layers (wave w owns output columns [32 w, 32 w + 32); the B
// fragments of each layer are loaded into registers one layer ahead, so the
// chain of a chunk waits on global memory once, in its input stage), keeping
// SiLU'(z) of every element in registers; then the output layer, the
// residual, dz of the last layer, and two backward-data products
// (dz_l W_l, B fragments from the transposed copies) down to dz_1. The
// chunk writes its inputs, a_1, a_2 and dz_1..3 transposed (rows of the
// weight-gradient products, 16-B stores), and per-chunk partial sums of
// dz_l (bias gradients), dout a_3 (output weights), dout and the squared
// residual.
//
// The transposed activations (rows: units of a layer; columns: batch rows)
// pass between the two kernels in K-step fragment order: element (n, m) of
// an NR-row matrix sits at
//   ((m / 32) (NR / 32) + n / 32) 1024 + ((m / 16) % 2) 512
//     + (n % 32 + 32 ((m / 8) % 2)) 8 + m % 8,
// so that the MFMA operand of 32 rows and one K step (16 batch rows) is one
// 1-KB run, lane l reading 16 B at l * 16 B, and each 32-row chunk of the
// batch is one contiguous block.
//
// k_train_update: one block per 32 x 32 tile of dW_l = dz_l^T a_{l-1} over
// the whole batch (its eight waves split the batch rows, partial tiles added
// in wave order), and one lane per remaining parameter, whose block's eight
// waves split the chunk partials (sums added in wave order); each
// parameter's gradient is formed by exactly one lane, which then applies
// Adam and refreshes the handle's FP32 and BF16 copies (row-major,
// transposed, fragment order).
constexpr int kTrainRows = 32;
struct TrainRowsArgs {
  const double* theta;   // [N x d] training inputs
  const double* target;  // [N]
  const int32_t* idx;    // [B] rows of this batch, or null for rows 0..B-1
  int d;
  const double* c;       // input map centre [d]
  const double* T;       // input map matrix [d x d]
  double mu, sd;
  const __bf16* W1;      // [W x kKin]
  const __bf16* W2F;     // fragment order
  const __bf16* W3F;
  const __bf16* W2TF;    // the transposes W2^T, W3^T in fragment order
  const __bf16* W3TF;
  const float* p32;      // biases, W4, b4
  float inv_b;           // 1 / B
  __bf16* x0T;           // [kKin x B], K-step fragment order
  __bf16* a1T;           // [W x B], K-step fragment order
  __bf16* a2T;
  __bf16* dz1T;
  __bf16* dz2T;
  __bf16* dz3T;
  float* part;           // [chunks x (4 W + 2)]
};

template <int W>
__global__ void __launch_bounds__(W * 2) k_train_rows(TrainRowsArgs f) {
  constexpr int NW = W / 32, KS = W / 16, R = kTrainRows;
  constexpr int LDA = W + 8, LDX = kKin + 8, NT = NW * 64, NP = 4 * W + 2;
  __shared__ __bf16 s_x[R * LDX];
  __shared__ __bf16 s_a[2][R * LDA];
  __shared__ float s_o[NW][R];
  __shared__ double s_th[R * kKin];
  __shared__ double s_T[kKin * kKin];
  __shared__ double s_c[kKin];
  __shared__ float s_w4[W + 1];  // output weights, then the output bias
  __shared__ float s_t[R], s_dout[R], s_sq[R];
  __shared__ float s_ds1[16 * NT];  // SiLU'(z_1), element r of thread t at r NT + t
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int ncol = 32 * w + (l & 31), kh = 8 * (l >> 5);
  const int d = f.d;
  const int64_t row0 = (int64_t)blockIdx.x * R;
  float* part = f.part + (int64_t)blockIdx.x * NP;
  const float* b1 = f.p32 + (int64_t)W * d;
  const float* b2 = b1 + W + (int64_t)W * W;
  const float* b3 = b2 + W + (int64_t)W * W;
  const float* W4 = b3 + W;

  // Weight fragments are loaded ahead into two register sets: fb holds W1,
  // then W3, then W2^T (loaded once the last layer's SiLU' is used up), fa
  // holds W2, then W3^T, all in fragment order (one 1-KB run per wave and
  // K step). W1 and this lane's biases are loaded with the inputs, W2 while
  // the inputs are mapped.
  bf16x8 fa[KS], fb[KS];
  float bias1, bias2, bias3;

  // inputs, standardised targets and output weights of the chunk: every
  // load is issued (row numbers first, then the rows) before any LDS store,
  // with out-of-range slots reading element 0 and storing nothing
  constexpr int NI = (R * kKin + NT - 1) / NT, NTI = (kKin * kKin + NT - 1) / NT;
  {
    int64_t src[NI], trow;
    const int tr = t < R ? t : 0;
    if (f.idx) {
#pragma unroll
      for (int it = 0; it < NI; ++it) {
        const int i = t + it * NT;
        src[it] = f.idx[row0 + (i < R * d ? i / d : 0)];
      }
      trow = f.idx[row0 + tr];
    } else {
#pragma unroll
      for (int it = 0; it < NI; ++it) {
        const int i = t + it * NT;
        src[it] = row0 + (i < R * d ? i / d : 0);
      }
      trow = row0 + tr;
    }
    double tv[NTI];
#pragma unroll
    for (int it = 0; it < NTI; ++it) {
      const int i = t + it * NT;
      tv[it] = f.T[i < d * d ? i : 0];
    }
    const double cv = f.c[t < d ? t : 0];
    const float w4v = W4[t <= W ? t : W];  // NT = 2 W threads cover W4 and b4
    double thv[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int i = t + it * NT, m = i < R * d ? i / d : 0, j = i < R * d ? i - m * d : 0;
      thv[it] = f.theta[src[it] * d + j];
    }
    const double tg = f.target[trow];
    // after the input loads, so that waiting for those does not wait for these
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
      fb[ks] = *reinterpret_cast<const bf16x8*>(f.W1 + (size_t)ncol * kKin + 16 * ks + kh);
    bias1 = b1[ncol];
    bias2 = b2[ncol];
    bias3 = b3[ncol];
#pragma unroll
    for (int it = 0; it < NTI; ++it)
      if (t + it * NT < d * d) s_T[t + it * NT] = tv[it];
    if (t < d) s_c[t] = cv;
    if (t <= W) s_w4[t] = w4v;
    if (t < R) s_t[t] = (float)((tg - f.mu) / f.sd);
#pragma unroll
    for (int it = 0; it < NI; ++it)
      if (t + it * NT < R * d) s_th[t + it * NT] = thv[it];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      fa[ks] = *reinterpret_cast<const bf16x8*>(f.W2F + ((size_t)(w * KS + ks) * 64 + l) * 8);
  }
  __syncthreads();
  // x = T (theta - c) for the R x d inputs (four terms' operands read
  // ahead, terms added in order), zeros in columns d .. kKin - 1
#pragma unroll
  for (int it = 0; it < NI; ++it) {
    const int i = t + it * NT;
    if (i < R * d) {
      const int m = i / d, k = i - m * d;
      const double* Tk = s_T + k * d;
      const double* th = s_th + m * d;
      double acc = 0.0;
      int jj = 0;
      for (; jj + 4 <= d; jj += 4) {
        double tq[4], xq[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          tq[e] = Tk[jj + e];
          xq[e] = th[jj + e] - s_c[jj + e];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = fma(tq[e], xq[e], acc);
      }
      for (; jj < d; ++jj) acc = fma(Tk[jj], th[jj] - s_c[jj], acc);
      s_x[m * LDX + k] = (__bf16)(float)acc;
    }
  }
  for (int i = t; i < R * (kKin - d); i += NT) {
    const int m = i / (kKin - d);
    s_x[m * LDX + d + (i - m * (kKin - d))] = (__bf16)0.0f;
  }
  __syncthreads();

  // columns [0, ncols) of the chunk's R x ld LDS matrix into dstT, in
  // K-step fragment order: each thread gathers 8 consecutive rows of one
  // column into one 16-B unit, and consecutive threads write consecutive
  // units
  auto store_T = [&](const __bf16* src, int ld, int ncols, __bf16* dstT) {
    __bf16* base = dstT + (int64_t)blockIdx.x * ncols * R;
    for (int i = t; i < ncols * (R / 8); i += NT) {
      const int ln = i & 63, s16 = (i >> 6) & 1, nb = i >> 7;
      const int n = 32 * nb + (ln & 31), m8 = 16 * s16 + 8 * (ln >> 5);
      bf16x8 v;
#pragma unroll
      for (int e = 0; e < 8; ++e) v[e] = src[(m8 + e) * ld + n];
      *reinterpret_cast<bf16x8*>(base + (int64_t)i * 8) = v;
    }
  };
  // per-column sums over the chunk's rows of an R x LDA LDS matrix (rows in order)
  auto col_sums = [&](const __bf16* src, float* out) {
    for (int n = t; n < W; n += NT) {
      float acc = 0.0f;
#pragma unroll 8
      for (int m = 0; m < R; ++m) acc += (float)src[m * LDA + n];
      out[n] = acc;
    }
  };
  // The chunk's rows (src, stride lds) times this wave's 32 columns of Y
  // (B fragments bf[ks]). Element r is row 8(r/4) + 4(l/32) + r%4, column ncol.
  auto product = [&](auto ksn, const __bf16* src, int lds, const bf16x8* bf) {
    constexpr int KSN = decltype(ksn)::value;
    const __bf16* ap = src + (l & 31) * lds + kh;
    f32x16 a = {};
#pragma unroll
    for (int ks = 0; ks < KSN; ++ks)
      a = __builtin_amdgcn_mfma_f32_32x32x16_bf16(*reinterpret_cast<const bf16x8*>(ap + 16 * ks),
                                                  bf[ks], a, 0, 0, 0);
    return a;
  };
  auto row_of = [&](int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); };
  // a = bf16(SiLU(z)) into dst and SiLU'(z) into dsl, z = acc + bias
  auto silu_out = [&](const f32x16& acc, float bias, __bf16* dst, f32x16& dsl) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float z = acc[r] + bias, sg = sigm(z);
      dst[row_of(r) * LDA + ncol] = (__bf16)(z * sg);
      dsl[r] = sg * (1.0f + z * (1.0f - sg));
    }
  };

  f32x16 ds[3];  // SiLU'(z_l) of this lane's elements (that of layer 1 kept in LDS)
  f32x16 acc;
  // ---- layer 1
  acc = product(std::integral_constant<int, 2>{}, s_x, LDX, fb);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
    fb[ks] = *reinterpret_cast<const bf16x8*>(f.W3F + ((size_t)(w * KS + ks) * 64 + l) * 8);
  silu_out(acc, bias1, s_a[0], ds[0]);
#pragma unroll
  for (int r = 0; r < 16; ++r) s_ds1[r * NT + t] = ds[0][r];
  store_T(s_x, LDX, kKin, f.x0T);
  __syncthreads();
  // ---- layer 2
  acc = product(std::integral_constant<int, KS>{}, s_a[0], LDA, fa);
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
    fa[ks] = *reinterpret_cast<const bf16x8*>(f.W3TF + ((size_t)(w * KS + ks) * 64 + l) * 8);
  silu_out(acc, bias2, s_a[1], ds[1]);
  store_T(s_a[0], LDA, W, f.a1T);
  __syncthreads();
  // ---- layer 3
  acc = product(std::integral_constant<int, KS>{}, s_a[1], LDA, fb);
  silu_out(acc, bias3, s_a[0], ds[2]);
  store_T(s_a[1], LDA, W, f.a2T);
  __syncthreads();
  // a_3 is in s_a[0]. ---- output layer: wave w sums its 32 columns, 16 per lane half
  {
    const int c0 = 32 * w + 16 * (l >> 5);
    const __bf16* ar = s_a[0] + (l & 31) * LDA + c0;
    float o = 0.0f;
#pragma unroll
    for (int j = 0; j < 16; j += 8) {
      const bf16x8 v = *reinterpret_cast<const bf16x8*>(ar + j);
#pragma unroll
      for (int e = 0; e < 8; ++e) o = fmaf((float)v[e], s_w4[c0 + j + e], o);
    }
    o += __shfl_xor(o, 32);
    if (l < 32) s_o[w][l] = o;
  }
  __syncthreads();
  if (t < R) {
    float o = 0.0f;
#pragma unroll
    for (int ww = 0; ww < NW; ++ww) o += s_o[ww][t];
    const float res = o + s_w4[W] - s_t[t];
    s_dout[t] = 2.0f * res * f.inv_b;
    s_sq[t] = res * res;
  }
  __syncthreads();
  // output-layer partials: dout a_3 per column, dout and squared residual
  for (int n = t; n < W; n += NT) {
    float acc1 = 0.0f;
#pragma unroll 8
    for (int m = 0; m < R; ++m) acc1 = fmaf(s_dout[m], (float)s_a[0][m * LDA + n], acc1);
    part[3 * W + n] = acc1;
  }
  if (t == 0) {
    float sd = 0.0f, sq = 0.0f;
#pragma unroll 8
    for (int m = 0; m < R; ++m) {
      sd += s_dout[m];
      sq += s_sq[m];
    }
    part[4 * W] = sd;
    part[4 * W + 1] = sq;
  }
  // ---- dz_3 = bf16(dout W4 SiLU'(z_3)) into s_a[1]
  {
    const float w4 = s_w4[ncol];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = row_of(r);
      s_a[1][row * LDA + ncol] = (__bf16)(s_dout[row] * w4 * ds[2][r]);
    }
  }
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
    fb[ks] = *reinterpret_cast<const bf16x8*>(f.W2TF + ((size_t)(w * KS + ks) * 64 + l) * 8);
  __syncthreads();
  // ---- backward-data products: dz_L = bf16((dz_{L+1} W_{L+1}) SiLU'(z_L)),
  // dz_3 in s_a[1] -> dz_2 in s_a[0] (W3^T in fa) -> dz_1 in s_a[1] (W2^T in fb)
  col_sums(s_a[1], part + 2 * W);
  store_T(s_a[1], LDA, W, f.dz3T);
  acc = product(std::integral_constant<int, KS>{}, s_a[1], LDA, fa);
#pragma unroll
  for (int r = 0; r < 16; ++r) s_a[0][row_of(r) * LDA + ncol] = (__bf16)(acc[r] * ds[1][r]);
  __syncthreads();
  col_sums(s_a[0], part + W);
  store_T(s_a[0], LDA, W, f.dz2T);
  acc = product(std::integral_constant<int, KS>{}, s_a[0], LDA, fb);
#pragma unroll
  for (int r = 0; r < 16; ++r) s_a[1][row_of(r) * LDA + ncol] = (__bf16)(acc[r] * s_ds1[r * NT + t]);
  __syncthreads();
  col_sums(s_a[1], part);
  store_T(s_a[1], LDA, W, f.dz1T);
}

struct TrainUpdArgs {
  const __bf16* x0T;
  const __bf16* a1T;
  const __bf16* a2T;
  const __bf16* dz1T;
  const __bf16* dz2T;
  const __bf16* dz3T;
  const float* part;
  int chunks;
  int64_t B;
  float inv_b;
  float* g;       // [n] gradient (packed)
  float* loss;    // [1] mean squared residual, or null
  AdamArgs adam;  // do_update 0: gradient only, copies untouched
};

// Adam on parameter i from its gradient gv and loaded state (m0, v0, w0):
// stores the new moments and master weight and refreshes the copies.
__device__ __forceinline__ void adam_store(const AdamArgs& a, int64_t i, float gv, float m0,
                                           float v0, float w0) {
  const float m = a.b1 * m0 + a.omb1 * gv;
  const float v = a.b2 * v0 + a.omb2 * gv * gv;
  a.m[i] = m;
  a.v[i] = v;
  const float w = w0 - a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
  a.master[i] = w;
  scatter_copy(a, i, w);
}

// k_train_update: one block of 8 waves per 32 x 32 weight-gradient tile.
// The batch's K steps (16 rows each) are cut into groups of 4; wave q sums
// groups [q G/8, (q+1) G/8) with up to 16 K steps of loads issued together
// (each a 1-KB run of the fragment-ordered activations), so that all the
// blocks together keep the whole operand traffic in flight. The eight
// partial tiles meet in LDS, where each of the 512 threads adds two elements
// in wave order and applies the update; blocks after the tiles take the
// remaining parameters and the loss, 64 at a time.
template <int W>
__global__ void __launch_bounds__(512) k_train_update(TrainUpdArgs u) {
  constexpr int NTL = W / 32, NP = 4 * W + 2;
  __shared__ float s_tile[8][32 * 33];
  const int l = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int d = u.adam.d_in;
  const int64_t oW2 = (int64_t)W * d + W, oW3 = oW2 + (int64_t)W * W + W;
  const int tiles_big = NTL * NTL, tiles = 2 * tiles_big + NTL;
  const int unit = blockIdx.x;
  if (unit < tiles) {
    // dW[n][k] = sum over the batch of dzT[n][m] aT[k][m]
    int layer, tile;
    if (unit < tiles_big) {
      layer = 3;
      tile = unit;
    } else if (unit < 2 * tiles_big) {
      layer = 2;
      tile = unit - tiles_big;
    } else {
      layer = 1;
      tile = unit - 2 * tiles_big;
    }
    const int nt_k = layer == 1 ? 1 : NTL;
    const int nb = tile / nt_k, kb = tile % nt_k;
    const __bf16* X = layer == 3 ? u.dz3T : (layer == 2 ? u.dz2T : u.dz1T);
    const __bf16* Y = layer == 3 ? u.a2T : (layer == 2 ? u.a1T : u.x0T);
    const int ynb = layer == 1 ? kKin / 32 : NTL;  // 32-row blocks of Y
    // K step g (chunk g / 2, half g % 2) of row block b of a matrix with nbk
    // row blocks starts at ((g / 2) nbk + b) 1024 + (g % 2) 512 elements
    const __bf16* xp = X + (int64_t)nb * 1024 + l * 8;
    const __bf16* yp = Y + (int64_t)kb * 1024 + l * 8;
    const int64_t xstep = (int64_t)NTL * 1024, ystep = (int64_t)ynb * 1024;
    const int64_t G = u.B / 64, g0 = G * q / 8, g1 = G * (q + 1) / 8;
    // this thread's two parameters' Adam state, read now so that its latency
    // hides behind the products
    const int kin = layer == 1 ? d : W;
    const int64_t off = layer == 3 ? oW3 : (layer == 2 ? oW2 : 0);
    const int n0 = 32 * nb, k0 = 32 * kb;
    const int kl = threadIdx.x & 31, nl = threadIdx.x >> 5;  // elements (nl, kl), (nl + 16, kl)
    const bool own = k0 + kl < kin;
    int64_t ix[2];
    float mo[2] = {0.0f, 0.0f}, vo[2] = {0.0f, 0.0f}, wo[2] = {0.0f, 0.0f};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      ix[h] = off + (int64_t)(n0 + nl + 16 * h) * kin + k0 + kl;
      if (own && u.adam.do_update) {
        mo[h] = u.adam.m[ix[h]];
        vo[h] = u.adam.v[ix[h]];
        wo[h] = u.adam.master[ix[h]];
      }
    }
    // the K steps in groups of up to 16, software-pipelined: each operand
    // register is refilled with the next group's step as soon as its MFMA
    // has been issued, so that 16 steps' loads stay in flight
    f32x16 acc = {};
    bf16x8 xa[16], yb[16];
    auto load = [&](int64_t g, int ng, int e) {
      if ((e >> 2) < ng) {
        const int64_t st = 4 * g + e, c = st >> 1, h = st & 1;
        xa[e] = *reinterpret_cast<const bf16x8*>(xp + c * xstep + h * 512);
        yb[e] = *reinterpret_cast<const bf16x8*>(yp + c * ystep + h * 512);
      }
    };
    if (g0 < g1) {
      const int ng0 = (int)(g1 - g0 < 4 ? g1 - g0 : 4);
#pragma unroll
      for (int e = 0; e < 16; ++e) load(g0, ng0, e);
    }
    for (int64_t g = g0; g < g1; g += 4) {
      const int ng = (int)(g1 - g < 4 ? g1 - g : 4);
      const int64_t gn = g + 4;
      const int ngn = gn < g1 ? (int)(g1 - gn < 4 ? g1 - gn : 4) : 0;
#pragma unroll
      for (int e = 0; e < 16; ++e)
        if ((e >> 2) < ng) {
          acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[e], yb[e], acc, 0, 0, 0);
          load(gn, ngn, e);
        }
    }
    // the eight partial tiles meet in LDS; each thread then forms two of the
    // tile's gradients (partials added in wave order) and updates them
#pragma unroll
    for (int r = 0; r < 16; ++r)
      s_tile[q][(8 * (r >> 2) + 4 * (l >> 5) + (r & 3)) * 33 + (l & 31)] = acc[r];
    __syncthreads();
    if (!own) return;
    float gv[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = (nl + 16 * h) * 33 + kl;
      float sum = s_tile[0][e];
#pragma unroll
      for (int qq = 1; qq < 8; ++qq) sum += s_tile[qq][e];
      gv[h] = sum;
    }
    const AdamArgs& a = u.adam;
    if (a.do_update) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        u.g[ix[h]] = gv[h];
        adam_store(a, ix[h], gv[h], mo[h], vo[h], wo[h]);
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) u.g[ix[h]] = gv[h];
    }
    return;
  }
  const int tiles_end = tiles;
  // the remaining parameters and the loss, 64 per block (one per lane): the
  // eight waves sum consecutive ranges of the chunk partials, in chunk order,
  // and wave 0 adds the eight sums in wave order
  __shared__ float s_vp[8][64];
  const int j = (unit - tiles_end) * 64 + l;
  const bool live = j <= 4 * W || (j == 4 * W + 1 && u.loss);
  const int c0 = u.chunks * q / 8, c1 = u.chunks * (q + 1) / 8;
  float acc = 0.0f;
  if (live) {
    int c = c0;
    for (; c + 16 <= c1; c += 16) {
      float v[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = u.part[(int64_t)(c + e) * NP + j];
#pragma unroll
      for (int e = 0; e < 16; ++e) acc += v[e];
    }
    for (; c < c1; ++c) acc += u.part[(int64_t)c * NP + j];
  }
  s_vp[q][l] = acc;
  __syncthreads();
  if (q > 0 || !live) return;
#pragma unroll
  for (int qq = 1; qq < 8; ++qq) acc += s_vp[qq][l];
  if (j == 4 * W + 1) {
    *u.loss = acc * u.inv_b;
    return;
  }
  int64_t i;
  if (j < W)
    i = (int64_t)W * d + j;                      // b1
  else if (j < 2 * W)
    i = oW2 + (int64_t)W * W + (j - W);          // b2
  else if (j < 3 * W)
    i = oW3 + (int64_t)W * W + (j - 2 * W);      // b3
  else
    i = oW3 + (int64_t)W * W + W + (j - 3 * W);  // W4, then b4
  u.g[i] = acc;
  const AdamArgs& a = u.adam;
  if (a.do_update) adam_store(a, i, acc, a.m[i], a.v[i], a.master[i]);
}

// ------------------------------------------------- delayed acceptance
// Stage 1 for chain i: a proposal outside the prior box is rejected; else
// accepted when log u1 < lhat_prop - lhat_cur. Accepted chain indices are
// compacted in increasing order (per-block counts, one-block scan, then
// per-block ordered writes).
constexpr int kScanBlock = 256;

__device__ __forceinline__ bool stage1_ok(int64_t i, const double* theta_prop, int d,
                                          const double* lo, const double* hi,
                                          const double* lh_cur, const double* lh_prop,
                                          const double* logu1) {
  // every test evaluated without an early exit, so that all the row's loads
  // are in flight together (a NaN fails both comparisons, as before)
  const double* t = theta_prop + i * d;
  bool in = logu1[i] < lh_prop[i] - lh_cur[i];
#pragma unroll 4
  for (int k = 0; k < d; ++k) {
    const double x = t[k];
    in = in & (x >= lo[k]) & (x <= hi[k]);
  }
  return in;
}

struct DA1Args {
  const double *theta_prop, *lo, *hi, *lh_cur, *lh_prop, *logu1;
  int64_t Q;
  int d;
  int32_t* block_cnt;   // [nblocks]
  int32_t* idx;         // [Q] compacted survivors
  int32_t* count;       // [1]
  int32_t* flag1;       // [Q] stage-1 decision
};

// Stage-1 compaction in two launches: per block, the survivors' count from
// one ballot per wave; then per block, its offset as the sum of the earlier
// blocks' counts (all threads of the block share the loads; an integer sum,
// so its order does not matter), and each survivor's slot is that offset
// plus the survivors in earlier waves of the block plus those in lower
// lanes of its own wave (mbcnt). The last block also writes the total. The
// order of the survivors is their chain order.
constexpr int kScanWaves = kScanBlock / 64;

__device__ __forceinline__ int lanes_below(uint64_t m) {
  return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__global__ void __launch_bounds__(kScanBlock) k_da1_count(DA1Args a) {
  __shared__ int s_cnt[kScanWaves];
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
  int ok = 0;
  if (i < a.Q) {
    ok = stage1_ok(i, a.theta_prop, a.d, a.lo, a.hi, a.lh_cur, a.lh_prop, a.logu1);
    a.flag1[i] = ok;
  }
  const uint64_t m = __builtin_amdgcn_ballot_w64(ok != 0);
  if ((threadIdx.x & 63) == 0) s_cnt[threadIdx.x >> 6] = __builtin_popcountll(m);
  __syncthreads();
  if (threadIdx.x == 0) {
    int c = 0;
    for (int w = 0; w < kScanWaves; ++w) c += s_cnt[w];
    a.block_cnt[blockIdx.x] = c;
  }
}

__global__ void __launch_bounds__(kScanBlock) k_da1_write(DA1Args a, int nblocks) {
  __shared__ int s_cnt[kScanWaves], s_part[kScanWaves];
  const int t = threadIdx.x, w = t >> 6;
  int part = 0;
  for (int b = t; b < (int)blockIdx.x; b += kScanBlock) part += a.block_cnt[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, 64);
  const int64_t i = (int64_t)blockIdx.x * kScanBlock + t;
  const int ok = i < a.Q ? a.flag1[i] : 0;
  const uint64_t m = __builtin_amdgcn_ballot_w64(ok != 0);
  if ((t & 63) == 0) {
    s_part[w] = part;
    s_cnt[w] = __builtin_popcountll(m);
  }
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int q = 0; q < kScanWaves; ++q) off += s_part[q];
  if ((int)blockIdx.x == nblocks - 1 && t == 0) {
    int tot = off;
    for (int q = 0; q < kScanWaves; ++q) tot += s_cnt[q];
    *a.count = tot;
  }
  if (!ok) return;
  int before = off + lanes_below(m);
  for (int q = 0; q < w; ++q) before += s_cnt[q];
  a.idx[before] = (int32_t)i;
}

__global__ void k_da1_none(int32_t* count) { *count = 0; }

__global__ void k_gather_rows(const double* src, const int32_t* idx, const int32_t* count,
                              int64_t cap, int d, double* dst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = *count;
  if (j >= cap * d) return;
  const int64_t r = j / d, k = j - r * d;
  // rows past the survivor count repeat the last survivor (padding)
  const int64_t rr = n > 0 ? (r < n ? r : n - 1) : 0;
  dst[j] = n > 0 ? src[(int64_t)idx[rr] * d + k] : 0.0;
}

struct DA2Args {
  const int32_t* idx;
  const int32_t* count;
  const double* ll_prop;   // [>= count] exact logL of the gathered survivors
  const double* lh_prop;   // [Q]
  const double* logu2;     // [Q]
  const double* theta_prop;
  double* theta_cur;       // [Q x d] updated in place
  double* ll_cur;          // [Q]
  double* lh_cur;          // [Q]
  int32_t* acc;            // [Q] accepted-move counters
  int d;
};

__global__ void k_da2(DA2Args a) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= *a.count) return;
  const int64_t i = a.idx[j];
  const double la = (a.ll_prop[j] - a.ll_cur[i]) - (a.lh_prop[i] - a.lh_cur[i]);
  if (a.logu2[i] < la) {
    // the row in chunks of 8: all of a chunk's loads, then its stores (an
    // element-wise copy would wait for each store before the next load)
    const double* src = a.theta_prop + i * a.d;
    double* dst = a.theta_cur + i * a.d;
    for (int k0 = 0; k0 < a.d; k0 += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q < a.d) v[q] = src[k0 + q];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (k0 + q < a.d) dst[k0 + q] = v[q];
    }
    a.ll_cur[i] = a.ll_prop[j];
    a.lh_cur[i] = a.lh_prop[i];
    a.acc[i] += 1;
  }
}

}  // namespace
}  // namespace argus

// ================================================================ host side
struct argus_mlp {
  int d_in = 0, width = 0;
  int64_t n = 0, max_batch = 0;
  int device = 0, n_cu = 256;
  argus::DevBuf p32, w1, w2, w3, w2T, w3T, w2F, w3F, w2TF, w3TF;
  argus::DevBuf ic, iT;  // input map x = T (theta - c): c [d_in], T [d_in x d_in]
  double mu = 0.0, sd = 1.0;
  bool loaded = false;
  // inference buffers (grown on demand)
  argus::DevBuf e_x0, e_a, e_b;
  int64_t e_cap = 0;
  // captured inference sequence, replayed for pointers seen on two
  // consecutive calls
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t e_exec{};
  bool e_has_graph = false;
  const void *e_theta = nullptr, *e_out = nullptr, *l_theta = nullptr, *l_out = nullptr;
  int64_t e_Q = -1, l_Q = -1;
  ~argus_mlp() {
    if (e_has_graph) (void)hipGraphExecDestroy(e_exec);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  // training buffers
  argus::DevBuf x0, x0T, z[3], a[3], aT[3], dz[3], dzT[3], t, dout, sq, g;
  argus::DevBuf wpart;  // split-K partial weight gradients
  argus::DevBuf tpart;  // fused training: per-chunk partial sums [max_batch/32 x (4 w + 2)]
};

namespace argus {
namespace {

int64_t mlp_params(int d, int w) { return (int64_t)w * d + 2LL * w * w + 4LL * w + 1; }

constexpr int kWgradSplits = 16;

int launch_gemm(int epi, GemmArgs g, hipStream_t st, int nsplit = 1) {
  if (g.kchunk <= 0) g.kchunk = g.K;
  dim3 grid((g.M + 63) / 64, (g.N + 63) / 64, nsplit);
  if (epi == EPI_FWD)
    hipLaunchKernelGGL(k_gemm<EPI_FWD>, grid, dim3(256), 0, st, g);
  else if (epi == EPI_BWD)
    hipLaunchKernelGGL(k_gemm<EPI_BWD>, grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL(k_gemm<EPI_WGRAD>, grid, dim3(256), 0, st, g);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

GemmArgs gemm(const __bf16* X, int ldx, const __bf16* Y, int ldy, int M, int N, int K) {
  GemmArgs g{};
  g.X = X;
  g.Y = Y;
  g.ldx = ldx;
  g.ldy = ldy;
  g.M = M;
  g.N = N;
  g.K = K;
  return g;
}

unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Forward of the three hidden layers for B rows from standardised inputs x0.
// train = store pre-activations and transposed activations.
int hidden_forward(argus_mlp* h, const __bf16* x0, int64_t B, __bf16* a1, __bf16* a2, __bf16* a3,
                   bool train, hipStream_t st) {
  const int w = h->width;
  const float* p = h->p32.as<float>();
  const float* b[3] = {p + (int64_t)w * h->d_in, p + (int64_t)w * h->d_in + w + (int64_t)w * w,
                       p + (int64_t)w * h->d_in + 2 * (w + (int64_t)w * w)};
  const __bf16* Ws[3] = {h->w1.as<__bf16>(), h->w2.as<__bf16>(), h->w3.as<__bf16>()};
  const __bf16* in[3] = {x0, a1, a2};
  __bf16* outs[3] = {a1, a2, a3};
  for (int l = 0; l < 3; ++l) {
    const int K = l == 0 ? kKin : w;
    GemmArgs g = gemm(in[l], K, Ws[l], K, (int)B, w, K);
    g.bias = b[l];
    g.out = outs[l];
    g.ldo = w;
    if (train) {
      g.zout = h->z[l].as<float>();
      g.outT = h->aT[l].as<__bf16>();
      g.ldoT = (int)h->max_batch;
    }
    int rc = launch_gemm(EPI_FWD, g, st);
    if (rc) return rc;
  }
  return ARGUS_OK;
}

int check_mlp(const argus_mlp* h) {
  if (!h) return fail(ARGUS_E_INVAL, "mlp handle is NULL");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != h->device) return fail(ARGUS_E_INVAL, "mlp handle belongs to another device");
  return ARGUS_OK;
}

// forward + backward into h->g (packed FP32 gradient) and loss_out
int mlp_backprop(argus_mlp* h, const double* theta, const double* target, int64_t B,
                 float* loss_out, hipStream_t st) {
  const int w = h->width, d = h->d_in;
  const int64_t ldT = h->max_batch;
  hipLaunchKernelGGL(k_prep, dim3(blocks(B * kKin, 256)), dim3(256), 0, st, theta, B, d,
                     h->ic.as<double>(), h->iT.as<double>(), h->x0.as<__bf16>(),
                     h->x0T.as<__bf16>(), (int)ldT, target, h->mu, h->sd, h->t.as<float>());
  HIPCHK(hipGetLastError());
  __bf16* A[3] = {h->a[0].as<__bf16>(), h->a[1].as<__bf16>(), h->a[2].as<__bf16>()};
  int rc = hidden_forward(h, h->x0.as<__bf16>(), B, A[0], A[1], A[2], true, st);
  if (rc) return rc;
  const float* p = h->p32.as<float>();
  const int64_t oW2 = (int64_t)w * d + w, oW3 = oW2 + (int64_t)w * w + w,
                oW4 = oW3 + (int64_t)w * w + w;
  float* g = h->g.as<float>();
  hipLaunchKernelGGL(k_out_train, dim3(blocks(B, 256)), dim3(256), 0, st, A[2], B, w, p + oW4,
                     p + oW4 + w, h->t.as<float>(), h->dout.as<float>(), h->sq.as<float>());
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_head_grad, dim3(w + 1), dim3(256), 0, st, h->dout.as<float>(),
                     h->sq.as<float>(), h->aT[2].as<__bf16>(), ldT, B, w, g + oW4, g + oW4 + w,
                     loss_out);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_dz_last, dim3(blocks(B * w, 256)), dim3(256), 0, st, h->dout.as<float>(),
                     p + oW4, h->z[2].as<float>(), B, w, h->dz[2].as<__bf16>(),
                     h->dzT[2].as<__bf16>(), (int)ldT);
  HIPCHK(hipGetLastError());
  const int64_t oW[3] = {0, oW2, oW3};
  const __bf16* WT[3] = {nullptr, h->w2T.as<__bf16>(), h->w3T.as<__bf16>()};
  for (int l = 2; l >= 0; --l) {
    // weight gradient dW_l = dZ_l^T A_{l-1}
    const int K_in = l == 0 ? kKin : w;
    const __bf16* AinT = l == 0 ? h->x0T.as<__bf16>() : h->aT[l - 1].as<__bf16>();
    const int Nw = l == 0 ? d : w;
    GemmArgs gw = gemm(h->dzT[l].as<__bf16>(), (int)ldT, AinT, (int)ldT, w, Nw, (int)B);
    (void)K_in;
    // K = batch is long and M x N small: split K so that the launch fills the
    // chip, then sum the partials in split order
    const int nsplit = (int)std::min<int64_t>(kWgradSplits, B / 64);
    gw.kchunk = (int)(((B + nsplit - 1) / nsplit + 63) / 64 * 64);
    const int nsp = (int)((B + gw.kchunk - 1) / gw.kchunk);
    gw.part = h->wpart.as<float>();
    if ((rc = launch_gemm(EPI_WGRAD, gw, st, nsp))) return rc;
    hipLaunchKernelGGL(k_sum_parts, dim3(blocks((int64_t)w * Nw, 256)), dim3(256), 0, st,
                       h->wpart.as<float>(), nsp, w, Nw, g + oW[l], Nw);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_rowsum_bf16, dim3(w), dim3(256), 0, st,
                       h->dzT[l].as<__bf16>(), w, B, ldT, g + oW[l] + (int64_t)w * (l == 0 ? d : w));
    HIPCHK(hipGetLastError());
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l) * SiLU'(Z_{l-1})
      GemmArgs gb = gemm(h->dz[l].as<__bf16>(), w, WT[l], w, (int)B, w, w);
      gb.zin = h->z[l - 1].as<float>();
      gb.out = h->dz[l - 1].as<__bf16>();
      gb.ldo = w;
      gb.outT = h->dzT[l - 1].as<__bf16>();
      gb.ldoT = (int)ldT;
      if ((rc = launch_gemm(EPI_BWD, gb, st))) return rc;
    }
  }
  return ARGUS_OK;
}

AdamArgs adam_args(argus_mlp* h, float* master, float* m, float* v, bool update, float lr,
                   int64_t step) {
  AdamArgs a{};
  a.master = master;
  a.m = m;
  a.v = v;
  a.g = h->g.as<float>();
  a.p32 = h->p32.as<float>();
  a.w1 = h->w1.as<__bf16>();
  a.w2 = h->w2.as<__bf16>();
  a.w3 = h->w3.as<__bf16>();
  a.w2T = h->w2T.as<__bf16>();
  a.w3T = h->w3T.as<__bf16>();
  a.w2F = h->w2F.p ? h->w2F.as<__bf16>() : nullptr;
  a.w3F = h->w3F.p ? h->w3F.as<__bf16>() : nullptr;
  a.w2TF = h->w2TF.p ? h->w2TF.as<__bf16>() : nullptr;
  a.w3TF = h->w3TF.p ? h->w3TF.as<__bf16>() : nullptr;
  a.n = h->n;
  a.d_in = h->d_in;
  a.width = h->width;
  a.lr = lr;
  a.b1 = 0.9f;
  a.b2 = 0.999f;
  a.omb1 = (float)(1.0 - 0.9);
  a.omb2 = (float)(1.0 - 0.999);
  a.eps = 1e-8f;
  a.c1 = update ? (float)(1.0 / (1.0 - std::pow(0.9, (double)step))) : 1.0f;
  a.c2 = update ? (float)(1.0 / (1.0 - std::pow(0.999, (double)step))) : 1.0f;
  a.do_update = update ? 1 : 0;
  return a;
}

// Adam on the handle's gradient buffer (update), or only the copies from
// master (no update)
int refresh(argus_mlp* h, float* master, float* m, float* v, bool update, float lr,
            int64_t step, hipStream_t st) {
  const AdamArgs a = adam_args(h, master, m, v, update, lr, step);
  hipLaunchKernelGGL(k_adam, dim3(blocks(h->n, 256)), dim3(256), 0, st, a);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

// One fused training step (width <= 256): rows of theta/target through idx
// (or 0..B-1), gradient into gout, loss into loss (or null), Adam when update.
int train_fused(argus_mlp* h, const double* theta, const double* target, const int32_t* idx,
                int64_t B, float* master, float* m, float* v, bool update, float lr,
                int64_t step, float* gout, float* loss, hipStream_t st) {
  const int w = h->width;
  TrainRowsArgs f{};
  f.theta = theta;
  f.target = target;
  f.idx = idx;
  f.d = h->d_in;
  f.c = h->ic.as<double>();
  f.T = h->iT.as<double>();
  f.mu = h->mu;
  f.sd = h->sd;
  f.W1 = h->w1.as<__bf16>();
  f.W2F = h->w2F.as<__bf16>();
  f.W3F = h->w3F.as<__bf16>();
  f.W2TF = h->w2TF.as<__bf16>();
  f.W3TF = h->w3TF.as<__bf16>();
  f.p32 = h->p32.as<float>();
  f.inv_b = (float)(1.0 / (double)B);
  f.x0T = h->x0T.as<__bf16>();
  f.a1T = h->aT[0].as<__bf16>();
  f.a2T = h->aT[1].as<__bf16>();
  f.dz1T = h->dzT[0].as<__bf16>();
  f.dz2T = h->dzT[1].as<__bf16>();
  f.dz3T = h->dzT[2].as<__bf16>();
  f.part = h->tpart.as<float>();
  const dim3 rows_grid((unsigned)(B / kTrainRows)), rows_block(2 * w);
  switch (w) {
    case 64: hipLaunchKernelGGL(k_train_rows<64>, rows_grid, rows_block, 0, st, f); break;
    case 128: hipLaunchKernelGGL(k_train_rows<128>, rows_grid, rows_block, 0, st, f); break;
    case 192: hipLaunchKernelGGL(k_train_rows<192>, rows_grid, rows_block, 0, st, f); break;
    default: hipLaunchKernelGGL(k_train_rows<256>, rows_grid, rows_block, 0, st, f); break;
  }
  HIPCHK(hipGetLastError());
  TrainUpdArgs u{};
  u.x0T = f.x0T;
  u.a1T = f.a1T;
  u.a2T = f.a2T;
  u.dz1T = f.dz1T;
  u.dz2T = f.dz2T;
  u.dz3T = f.dz3T;
  u.part = f.part;
  u.chunks = (int)(B / kTrainRows);
  u.B = B;
  u.inv_b = f.inv_b;
  u.g = gout;
  u.loss = loss;
  u.adam = adam_args(h, master, m, v, update, lr, step);
  const int nt = w / 32;
  const int units = 2 * nt * nt + nt + (4 * w + 2 + 63) / 64;
  const dim3 upd_grid((unsigned)units), upd_block(512);
  switch (w) {
    case 64: hipLaunchKernelGGL(k_train_update<64>, upd_grid, upd_block, 0, st, u); break;
    case 128: hipLaunchKernelGGL(k_train_update<128>, upd_grid, upd_block, 0, st, u); break;
    case 192: hipLaunchKernelGGL(k_train_update<192>, upd_grid, upd_block, 0, st, u); break;
    default: hipLaunchKernelGGL(k_train_update<256>, upd_grid, upd_block, 0, st, u); break;
  }
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

int eval_seq(argus_mlp* h, const double* theta, int64_t Q, double* logl_hat, hipStream_t st) {
  if (h->width <= kFusedMaxWidth) {
    FusedArgs f{theta, h->ic.as<double>(), h->iT.as<double>(), h->w1.as<__bf16>(),
                h->w2F.as<__bf16>(), h->w3F.as<__bf16>(), h->p32.as<float>(), logl_hat, Q,
                h->d_in, h->mu, h->sd};
    const unsigned grid =
        (unsigned)std::min<int64_t>(h->n_cu, (Q + kFusedRows - 1) / kFusedRows);
    const dim3 block(h->width * 2);
    switch (h->width) {
      case 64: hipLaunchKernelGGL(k_mlp_fused<64>, dim3(grid), block, 0, st, f); break;
      case 128: hipLaunchKernelGGL(k_mlp_fused<128>, dim3(grid), block, 0, st, f); break;
      case 192: hipLaunchKernelGGL(k_mlp_fused<192>, dim3(grid), block, 0, st, f); break;
      default: hipLaunchKernelGGL(k_mlp_fused<256>, dim3(grid), block, 0, st, f); break;
    }
    HIPCHK(hipGetLastError());
    return ARGUS_OK;
  }
  hipLaunchKernelGGL(k_prep, dim3(blocks(Q * kKin, 256)), dim3(256), 0, st, theta, Q, h->d_in,
                     h->ic.as<double>(), h->iT.as<double>(), h->e_x0.as<__bf16>(), nullptr, 0,
                     nullptr, 0.0, 1.0, nullptr);
  HIPCHK(hipGetLastError());
  __bf16* A = h->e_a.as<__bf16>();
  __bf16* Bb = h->e_b.as<__bf16>();
  // a1 -> A, a2 -> B, a3 -> A
  int rc = hidden_forward(h, h->e_x0.as<__bf16>(), Q, A, Bb, A, false, st);
  if (rc) return rc;
  const int w = h->width;
  const float* p = h->p32.as<float>();
  const int64_t oW4 = (int64_t)w * h->d_in + w + 2 * ((int64_t)w * w + w);
  hipLaunchKernelGGL(k_out_eval, dim3(blocks(Q, 256)), dim3(256), 0, st, A, Q, w, p + oW4,
                     p + oW4 + w, h->mu, h->sd, logl_hat);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

}  // namespace
}  // namespace argus

using namespace argus;

extern "C" {

int argus_mlp_create(int32_t d_in, int32_t width, int64_t max_batch, argus_mlp_t* out) {
  if (!out) return fail(ARGUS_E_INVAL, "out is NULL");
  *out = nullptr;
  if (d_in < 1 || d_in > kKin) return fail(ARGUS_E_UNSUPPORTED, "d_in must be in [1, 32]");
  if (width < 64 || width > 1024 || width % 64)
    return fail(ARGUS_E_UNSUPPORTED, "width must be a multiple of 64 in [64, 1024]");
  if (max_batch < 64 || max_batch % 64 || max_batch > (1LL << 24))
    return fail(ARGUS_E_UNSUPPORTED, "max_batch must be a multiple of 64 in [64, 2^24]");
  auto h = std::make_unique<argus_mlp>();
  h->d_in = d_in;
  h->width = width;
  h->n = mlp_params(d_in, width);
  h->max_batch = max_batch;
  HIPCHK(hipGetDevice(&h->device));
  HIPCHK(hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device));
  const int64_t w = width, B = max_batch;
  int rc;
  if ((rc = h->p32.alloc(h->n * 4)) || (rc = h->w1.alloc(w * kKin * 2)) ||
      (rc = h->w2.alloc(w * w * 2)) || (rc = h->w3.alloc(w * w * 2)) ||
      (rc = h->w2T.alloc(w * w * 2)) || (rc = h->w3T.alloc(w * w * 2)) ||
      (rc = h->ic.alloc(kKin * 8)) || (rc = h->iT.alloc(kKin * kKin * 8)) ||
      (rc = h->x0.alloc(B * kKin * 2)) || (rc = h->x0T.alloc(B * kKin * 2)) ||
      (rc = h->t.alloc(B * 4)) || (rc = h->dout.alloc(B * 4)) || (rc = h->sq.alloc(B * 4)) ||
      (rc = h->g.alloc(h->n * 4)) || (rc = h->wpart.alloc(kWgradSplits * w * w * 4)) ||
      (rc = h->tpart.alloc((B / kTrainRows) * (4 * w + 2) * 4)))
    return rc;
  if (w <= kFusedMaxWidth &&
      ((rc = h->w2F.alloc(w * w * 2)) || (rc = h->w3F.alloc(w * w * 2)) ||
       (rc = h->w2TF.alloc(w * w * 2)) || (rc = h->w3TF.alloc(w * w * 2))))
    return rc;
  for (int l = 0; l < 3; ++l)
    if ((rc = h->z[l].alloc(B * w * 4)) || (rc = h->a[l].alloc(B * w * 2)) ||
        (rc = h->aT[l].alloc(B * w * 2)) || (rc = h->dz[l].alloc(B * w * 2)) ||
        (rc = h->dzT[l].alloc(B * w * 2)))
      return rc;
  // zero padding columns of W1 and unused tails once
  HIPCHK(hipMemset(h->w1.p, 0, w * kKin * 2));
  HIPCHK(hipMemset(h->g.p, 0, h->n * 4));
  HIPCHK(hipDeviceSynchronize());
  *out = h.release();
  return ARGUS_OK;
}

int argus_mlp_destroy(argus_mlp_t h) {
  if (!h) return ARGUS_OK;
  (void)hipDeviceSynchronize();
  delete h;
  return ARGUS_OK;
}

int argus_mlp_n_params(argus_mlp_t h, int64_t* n) {
  if (!h || !n) return fail(ARGUS_E_INVAL, "NULL argument");
  *n = h->n;
  return ARGUS_OK;
}

int argus_mlp_load_affine(argus_mlp_t h, const float* master, const double* center,
                          const double* T, double out_mu, double out_sd, void* stream) {
  int rc = check_mlp(h);
  if (rc) return rc;
  if (!master || !center || !T) return fail(ARGUS_E_INVAL, "NULL argument");
  if (!(out_sd > 0.0) || !std::isfinite(out_sd) || !std::isfinite(out_mu))
    return fail(ARGUS_E_INVAL, "bad standardisation");
  const int d = h->d_in;
  for (int k = 0; k < d; ++k)
    if (!std::isfinite(center[k])) return fail(ARGUS_E_INVAL, "input map centre must be finite");
  for (int k = 0; k < d * d; ++k)
    if (!std::isfinite(T[k])) return fail(ARGUS_E_INVAL, "input map matrix must be finite");
  hipStream_t st = (hipStream_t)stream;
  HIPCHK(hipMemcpyAsync(h->ic.p, center, d * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->iT.p, T, (size_t)d * d * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  h->mu = out_mu;
  h->sd = out_sd;
  if (h->e_has_graph) {  // the captured output kernel holds mu and sd by value
    HIPCHK(hipGraphExecDestroy(h->e_exec));
    h->e_has_graph = false;
  }
  if ((rc = refresh(h, const_cast<float*>(master), nullptr, nullptr, false, 0.f, 0, st)))
    return rc;
  h->loaded = true;
  return ARGUS_OK;
}

int argus_mlp_load(argus_mlp_t h, const float* master, const double* in_lo, const double* in_hi,
                   double out_mu, double out_sd, void* stream) {
  int rc = check_mlp(h);
  if (rc) return rc;
  if (!master || !in_lo || !in_hi) return fail(ARGUS_E_INVAL, "NULL argument");
  const int d = h->d_in;
  std::vector<double> c(d), T((size_t)d * d, 0.0);
  for (int k = 0; k < d; ++k) {
    if (!(in_hi[k] > in_lo[k]) || !std::isfinite(in_hi[k] - in_lo[k]))
      return fail(ARGUS_E_INVAL, "input box must be finite with hi > lo");
    c[k] = 0.5 * (in_lo[k] + in_hi[k]);
    T[(size_t)k * d + k] = 2.0 / (in_hi[k] - in_lo[k]);
  }
  return argus_mlp_load_affine(h, master, c.data(), T.data(), out_mu, out_sd, stream);
}

int argus_surrogate_eval(argus_mlp_t h, const double* theta, int64_t Q, double* logl_hat,
                         void* stream) {
  int rc = check_mlp(h);
  if (rc) return rc;
  if (!h->loaded) return fail(ARGUS_E_INVAL, "weights not loaded");
  if (Q < 0) return fail(ARGUS_E_INVAL, "Q must be >= 0");
  if (Q == 0) return ARGUS_OK;
  if (!theta || !logl_hat) return fail(ARGUS_E_INVAL, "NULL argument");
  if (Q > h->e_cap) {
    const int64_t cap = ((Q + 63) / 64) * 64;
    if ((rc = h->e_x0.alloc(cap * kKin * 2)) || (rc = h->e_a.alloc(cap * h->width * 2)) ||
        (rc = h->e_b.alloc(cap * h->width * 2)))
      return rc;
    h->e_cap = cap;
    if (h->e_has_graph) {
      HIPCHK(hipGraphExecDestroy(h->e_exec));
      h->e_has_graph = false;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const bool stable = h->l_theta == theta && h->l_out == logl_hat && h->l_Q == Q;
  h->l_theta = theta;
  h->l_out = logl_hat;
  h->l_Q = Q;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(st, &cs));
  if (!stable || cs != hipStreamCaptureStatusNone) return eval_seq(h, theta, Q, logl_hat, st);
  if (!h->e_has_graph || h->e_theta != theta || h->e_out != logl_hat || h->e_Q != Q) {
    if (h->e_has_graph) {
      HIPCHK(hipGraphExecDestroy(h->e_exec));
      h->e_has_graph = false;
    }
    if (!h->cap_stream) HIPCHK(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = eval_seq(h, theta, Q, logl_hat, h->cap_stream);
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (rc) return rc;
    if (e != hipSuccess) return fail(ARGUS_E_HIP, "hipStreamEndCapture failed");
    e = hipGraphInstantiate(&h->e_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(ARGUS_E_HIP, "hipGraphInstantiate failed");
    h->e_has_graph = true;
    h->e_theta = theta;
    h->e_out = logl_hat;
    h->e_Q = Q;
  }
  HIPCHK(hipGraphLaunch(h->e_exec, st));
  return ARGUS_OK;
}

int argus_mlp_grad(argus_mlp_t h, const double* theta, const double* target, int64_t B,
                   float* grad_out, float* loss_out, void* stream) {
  int rc = check_mlp(h);
  if (rc) return rc;
  if (!h->loaded) return fail(ARGUS_E_INVAL, "weights not loaded");
  if (B < 64 || B % 64 || B > h->max_batch)
    return fail(ARGUS_E_INVAL, "batch must be a multiple of 64 and <= max_batch");
  if (!theta || !target || !loss_out) return fail(ARGUS_E_INVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  if (h->width <= kFusedMaxWidth)
    return train_fused(h, theta, target, nullptr, B, nullptr, nullptr, nullptr, false, 0.f, 0,
                       grad_out ? grad_out : h->g.as<float>(), loss_out, st);
  if ((rc = mlp_backprop(h, theta, target, B, loss_out, st))) return rc;
  if (grad_out)
    HIPCHK(hipMemcpyAsync(grad_out, h->g.p, h->n * 4, hipMemcpyDeviceToDevice, st));
  return ARGUS_OK;
}

int argus_surrogate_train_step(argus_mlp_t h, float* master, float* adam_m, float* adam_v,
                               const double* theta, const double* target, int64_t B, float lr,
                               int64_t step, float* loss_out, void* stream) {
  int rc = check_mlp(h);
  if (rc) return rc;
  if (!master || !adam_m || !adam_v) return fail(ARGUS_E_INVAL, "NULL argument");
  if (step < 1) return fail(ARGUS_E_INVAL, "step counts from 1");
  if (h->width <= kFusedMaxWidth) {
    if (!h->loaded) return fail(ARGUS_E_INVAL, "weights not loaded");
    if (B < 64 || B % 64 || B > h->max_batch)
      return fail(ARGUS_E_INVAL, "batch must be a multiple of 64 and <= max_batch");
    if (!theta || !target || !loss_out) return fail(ARGUS_E_INVAL, "NULL argument");
    return train_fused(h, theta, target, nullptr, B, master, adam_m, adam_v, true, lr, step,
                       h->g.as<float>(), loss_out, (hipStream_t)stream);
  }
  if ((rc = argus_mlp_grad(h, theta, target, B, nullptr, loss_out, stream))) return rc;
  return refresh(h, master, adam_m, adam_v, true, lr, step, (hipStream_t)stream);
}

int argus_surrogate_train_epoch(argus_mlp_t h, float* master, float* adam_m, float* adam_v,
                                const double* theta, const double* target,
                                const int32_t* order, int64_t n_batches, int64_t B, float lr,
                                int64_t step0, float* loss_out, void* stream) {
  int rc = check_mlp(h);
  if (rc) return rc;
  if (h->width > kFusedMaxWidth)
    return fail(ARGUS_E_UNSUPPORTED, "the epoch entry point covers widths up to 256");
  if (!h->loaded) return fail(ARGUS_E_INVAL, "weights not loaded");
  if (!master || !adam_m || !adam_v || !theta || !target || !order)
    return fail(ARGUS_E_INVAL, "NULL argument");
  if (B < 64 || B % 64 || B > h->max_batch)
    return fail(ARGUS_E_INVAL, "batch must be a multiple of 64 and <= max_batch");
  if (n_batches < 0 || step0 < 0) return fail(ARGUS_E_INVAL, "bad counts");
  hipStream_t st = (hipStream_t)stream;
  for (int64_t b = 0; b < n_batches; ++b)
    if ((rc = train_fused(h, theta, target, order + b * B, B, master, adam_m, adam_v, true, lr,
                          step0 + b + 1, h->g.as<float>(), loss_out ? loss_out + b : nullptr,
                          st)))
      return rc;
  return ARGUS_OK;
}

int argus_da_stage1(const double* theta_prop, const double* lo, const double* hi,
                    const double* lh_cur, const double* lh_prop, const double* logu1, int64_t Q,
                    int32_t d, int32_t* idx, int32_t* count, int32_t* work, void* stream) {
  if (Q < 0 || d < 1) return fail(ARGUS_E_INVAL, "bad sizes");
  if (!count) return fail(ARGUS_E_INVAL, "count is NULL");
  hipStream_t st = (hipStream_t)stream;
  const int nb = (int)blocks(Q, kScanBlock);
  if (Q == 0) {
    hipLaunchKernelGGL(k_da1_none, dim3(1), dim3(1), 0, st, count);
    HIPCHK(hipGetLastError());
    return ARGUS_OK;
  }
  if (!theta_prop || !lo || !hi || !lh_cur || !lh_prop || !logu1 || !idx || !work)
    return fail(ARGUS_E_INVAL, "NULL argument");
  // work = [stage-1 flags (Q) | per-block counts (nb) | (unused, nb)]
  DA1Args a{theta_prop, lo, hi, lh_cur, lh_prop, logu1, Q, d,
            work + Q, idx, count, work};
  hipLaunchKernelGGL(k_da1_count, dim3(nb), dim3(kScanBlock), 0, st, a);
  HIPCHK(hipGetLastError());
  hipLaunchKernelGGL(k_da1_write, dim3(nb), dim3(kScanBlock), 0, st, a, nb);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

int64_t argus_da_work_size(int64_t Q) {
  return Q <= 0 ? 0 : Q + 2 * ((Q + kScanBlock - 1) / kScanBlock);
}

int argus_gather_rows(const double* src, const int32_t* idx, const int32_t* count, int64_t cap,
                      int32_t d, double* dst, void* stream) {
  if (cap < 0 || d < 1) return fail(ARGUS_E_INVAL, "bad sizes");
  if (cap == 0) return ARGUS_OK;
  if (!src || !idx || !count || !dst) return fail(ARGUS_E_INVAL, "NULL argument");
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks(cap * d, 256)), dim3(256), 0,
                     (hipStream_t)stream, src, idx, count, cap, d, dst);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

int argus_da_stage2(const int32_t* idx, const int32_t* count, int64_t cap, const double* ll_prop,
                    const double* lh_prop, const double* logu2, const double* theta_prop,
                    double* theta_cur, double* ll_cur, double* lh_cur, int32_t* acc, int32_t d,
                    void* stream) {
  if (cap < 0 || d < 1) return fail(ARGUS_E_INVAL, "bad sizes");
  if (cap == 0) return ARGUS_OK;
  if (!idx || !count || !ll_prop || !lh_prop || !logu2 || !theta_prop || !theta_cur || !ll_cur ||
      !lh_cur || !acc)
    return fail(ARGUS_E_INVAL, "NULL argument");
  DA2Args a{idx, count, ll_prop, lh_prop, logu2, theta_prop, theta_cur, ll_cur, lh_cur, acc, d};
  hipLaunchKernelGGL(k_da2, dim3(blocks(cap, 256)), dim3(256), 0, (hipStream_t)stream, a);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

}  // extern "C"
