// Internal declarations shared by the host API and the kernel translation
// units of libargus. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace argus {

constexpr int kWave = 64;
constexpr double kPi = 3.14159265358979323846;
constexpr double kLn2 = 0.69314718055994530942;
constexpr double kLn10 = 2.30258509299404568402;
constexpr double kLn2Pi = 1.83787706640934548356;
constexpr double kYear = 31557600.0;
constexpr double kNuRef = 1400.0;  // MHz: reference frequency of the DM delay state

// status words; kPNF marks "a parameter of this filter is not finite" and has
// priority over the innovation flags when a sample's pulsars are combined
constexpr int kNonPD = 1;
constexpr int kNonFinite = 2;
constexpr int kPNF = 4;

// Per-TOA record, 64 B, in stream order (per-pulsar CSR for models 1/2, the
// merged time-ordered stream for model 3). All entries are theta-independent.
struct alignas(64) TOARec {
  double dt;     // t_k - t_{k-1} (t_0 = epoch 0)
  double h2;     // dt^2 / 2
  double h3;     // dt^3 / 3
  double phc;    // exp(-lambda_c dt), common OU decay
  double qcu;    // 1 - phc^2, common OU noise per unit variance
  double y;      // residual
  double s2;     // sigma_k^2
  int32_t psr;   // merged stream (model 3): pulsar of this TOA; per-pulsar
  int32_t pad;   // streams: these 8 bytes hold phc^2 instead (rec_phc2)
};
static_assert(sizeof(TOARec) == 64, "TOA record is one 64-B line");

// The TOA stream is read-only for the whole of every kernel that reads it and
// all lanes of a wave read the same record, so kernels address it through the
// constant address space: the compiler then issues one scalar 64-B load
// (s_load_dwordx16) per record instead of 64 vector loads.
typedef __attribute__((address_space(4))) const TOARec* RecPtr;
typedef __attribute__((address_space(4))) const double* ConstDPtr;

__device__ __forceinline__ TOARec load_rec(RecPtr r, int64_t k) {
  TOARec x;
  x.dt = r[k].dt;
  x.h2 = r[k].h2;
  x.h3 = r[k].h3;
  x.phc = r[k].phc;
  x.qcu = r[k].qcu;
  x.y = r[k].y;
  x.s2 = r[k].s2;
  x.psr = r[k].psr;
  x.pad = 0;
  return x;
}

// A record as one 64-B vector (one scalar load of all 16 words). Handing the
// whole vector to rec_keep at the top of the next step keeps all 16 SGPRs
// live until then: otherwise the compiler may reuse the words the step does
// not read while the load that writes them is still in flight, which forces
// a wait for the load right after it is issued.
typedef double RecVec __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(4))) const RecVec* RecVecPtr;
__device__ __forceinline__ RecVec load_rec_v(RecVecPtr r, int k) { return r[k]; }
__device__ __forceinline__ void rec_keep(const RecVec& v) { asm volatile("" ::"s"(v)); }
__device__ __forceinline__ TOARec rec_fields(const RecVec& v) {
  TOARec x;
  x.dt = v[0];
  x.h2 = v[1];
  x.h3 = v[2];
  x.phc = v[3];
  x.qcu = v[4];
  x.y = v[5];
  x.s2 = v[6];
  x.psr = 0;
  x.pad = 0;
  return x;
}

// One pulsar's TOA records read with vector (buffer) loads into VGPRs, for
// kernels whose SGPRs cannot hold records in flight: the loads are issued
// ahead of use and waited for in order. The descriptor covers the pulsar's
// n records (n * 64 bytes must fit in 31 bits; the host checks); a read
// beyond them returns zeros. Word 3 of the descriptor is the raw-buffer
// format of the gfx9 family.
struct RecBuf {
  __amdgpu_buffer_rsrc_t r;
};
__device__ __forceinline__ RecBuf rec_buffer(const TOARec* first, int n) {
  return RecBuf{__builtin_amdgcn_make_buffer_rsrc(const_cast<TOARec*>(first), (short)0, n * 64,
                                                  0x00020000)};
}
__device__ __forceinline__ TOARec load_rec_vgpr(const RecBuf& b, int k) {
  typedef double D2 __attribute__((ext_vector_type(2)));
  const int o = k * 64;
  const D2 a = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(b.r, o, 0, 0));
  const D2 c = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(b.r, o + 16, 0, 0));
  const D2 d = __builtin_bit_cast(D2, __builtin_amdgcn_raw_buffer_load_b128(b.r, o + 32, 0, 0));
  const double s2 = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b.r, o + 48, 0, 0));
  TOARec x;
  x.dt = a[0];
  x.h2 = a[1];
  x.h3 = c[0];
  x.phc = c[1];
  x.qcu = d[0];
  x.y = d[1];
  x.s2 = s2;
  x.psr = 0;
  x.pad = 0;
  return x;
}

// exp(x) - 1 for the OU decays (x = -rate * dt <= 0 in every use). Range
// reduction x = k ln2 + r, |r| <= ln2/2, with ln 2 split in two parts so that
// k ln2_hi is exact (Cody & Waite 1980; the split of fdlibm); expm1(r) from
// its Taylor series to degree 13, whose truncation error r^13/14! < 1.2e-17
// relative; then expm1(x) = 2^k (expm1(r) + 1) - 1, formed as
// 2^k expm1(r) + (2^k - 1), which is exact-ish because for k != 0 the result
// is at least 0.29 in magnitude. 2^k underflows to 0 for x < -745: -1.
// Taylor coefficients 1/n!, n = 2..13, read from constant memory so that the
// compiler keeps them in SGPRs (a VOP3 FMA takes one SGPR operand) instead of
// copying each into the accumulator of a two-address FMA.
__constant__ double kExpm1Coef[12] = {
    1.0 / 2.0,        1.0 / 6.0,         1.0 / 24.0,        1.0 / 120.0,
    1.0 / 720.0,      1.0 / 5040.0,      1.0 / 40320.0,     1.0 / 362880.0,
    1.0 / 3628800.0,  1.0 / 39916800.0,  1.0 / 479001600.0, 1.0 / 6227020800.0};

// c13 is the top coefficient 1/13!, passed in so that a loop can hold it in
// a VGPR: the first Horner step then reads one SGPR (the next coefficient)
// instead of needing a copy. The clamp keeps the conversion of k to int
// defined; 2^k is 0 below k = -1075 either way. For k = 0 the last fma
// returns p exactly.
__device__ __forceinline__ double expm1_v(double x, double c13) {
  const double kInvLn2 = 1.44269504088896338700;
  const double kLn2Hi = 6.93147180369123816490e-01;
  const double kLn2Lo = 1.90821492927058770002e-10;
  const double kf = __builtin_rint(x * kInvLn2);
  double r = __builtin_fma(-kf, kLn2Hi, x);
  r = __builtin_fma(-kf, kLn2Lo, r);
  // Q(r) = sum_{n=2}^{13} r^(n-2) / n!
  double q = __builtin_fma(c13, r, kExpm1Coef[10]);
#pragma unroll
  for (int i = 9; i >= 0; --i) q = __builtin_fma(q, r, kExpm1Coef[i]);
  const double p = __builtin_fma(r * r, q, r);      // expm1(r)
  const double t = __builtin_ldexp(1.0, (int)__builtin_fmax(kf, -1100.0));
  return __builtin_fma(t, p, t - 1.0);
}
__device__ __forceinline__ double expm1_k(double x) { return expm1_v(x, kExpm1Coef[11]); }

// The same with every coefficient held in VGPRs (for loops short of SGPRs):
// the Horner steps then read no SGPR at all.
struct Expm1Coef {
  double c[12];
};
__device__ __forceinline__ Expm1Coef expm1_coef_vgpr() {
  Expm1Coef k;
#pragma unroll
  for (int i = 0; i < 12; ++i) {
    k.c[i] = kExpm1Coef[i];
    asm volatile("" : "+v"(k.c[i]));
  }
  return k;
}
__device__ __forceinline__ double expm1_c(double x, const Expm1Coef& k) {
  const double kInvLn2 = 1.44269504088896338700;
  const double kLn2Hi = 6.93147180369123816490e-01;
  const double kLn2Lo = 1.90821492927058770002e-10;
  const double kf = __builtin_rint(x * kInvLn2);
  double r = __builtin_fma(-kf, kLn2Hi, x);
  r = __builtin_fma(-kf, kLn2Lo, r);
  double q = __builtin_fma(k.c[11], r, k.c[10]);
#pragma unroll
  for (int i = 9; i >= 0; --i) q = __builtin_fma(q, r, k.c[i]);
  const double p = __builtin_fma(r * r, q, r);
  const double t = __builtin_ldexp(1.0, (int)__builtin_fmax(kf, -1100.0));
  return __builtin_fma(t, p, t - 1.0);
}

// A copy of a wave-uniform value held in a VGPR, so that FP64 operations
// pairing it with a per-TOA SGPR operand need no register copy (a VOP3
// instruction reads at most one SGPR).
__device__ __forceinline__ double in_vgpr(double x) {
  asm volatile("" : "+v"(x));
  return x;
}

// Orders the fetch pipeline of the filter loops: the record whose first
// field is d (fetched one step earlier) is waited for here, and no later
// memory access is moved above this point, so the fetch issued next has a
// whole step to arrive (a scalar-load wait covers every load in flight).
__device__ __forceinline__ void sgpr_ready(double d) {
  asm volatile("" ::"s"(d) : "memory");
}

// 1/S from the hardware reciprocal refined by two Newton steps (error within
// an ulp or so; S > 0 in every use that is not already flagged).
__device__ __forceinline__ double rcp_nr(double S) {
  double r = __builtin_amdgcn_rcp(S);
  double e = __builtin_fma(-S, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-S, r, 1.0);
  return __builtin_fma(r, e, r);
}

// Model constants shared by all kernels.
struct ModelConst {
  double s_r2, s_f2;   // prior variances of r and f
  double ss2;          // sigma_s^2 (models 2, 3)
  double log_fyr;      // ln(1/yr)
  double log_T;        // ln(t_span)
  double lam;          // 2 pi / t_span
};

// Arguments of the batched per-pulsar filter (models 1, 2, 4).
struct FilterArgs {
  const TOARec* rec;     // [N]
  const double* chrom;   // [N] chromatic factor (nu_ref / nu)^2 per TOA (model 4), else null
  const int64_t* off;    // [P+1]
  const double* theta;   // [S*D]
  const int32_t* col;    // [C] theta column of canonical param, or -1
  const double* fixed;   // [C]
  const int32_t* items;  // [n_items*2] (sample tile, pulsar), longest first; or
                         // NULL: item i is (i % tiles, porder[i / tiles])
  const int32_t* porder; // [P] pulsars longest first (used when items is NULL)
  int32_t tiles;         // ceil(S / 64) (used when items is NULL)
  const double* maxdt;   // [P] largest TOA interval of each pulsar (model 2)
  int32_t* redo;         // model 2: [n_items] 1 where the fast form left the
                         // item to the general form, else 0
  // per-SIMD mode: items of SIMD j of block b are [bin_off[4b+j], bin_off[4b+j+1])
  const int32_t* bin_off;
  int32_t* counter;      // work-queue head (zero before launch)
  double* part;          // [P*S] per-pulsar log-likelihood terms
  int32_t* pstat;        // [P*S] per-pulsar status words
  int64_t S;
  int32_t D, P, n_items, dynamic;  // dynamic: 0 static, 1 global queue, 2 per-SIMD queues
  ModelConst mc;
};

struct ReduceArgs {
  const double* part;
  const int32_t* pstat;
  double* logl;
  int32_t* status;
  int32_t* counter;  // reset to 0 for the next launch
  int64_t S;
  int32_t P;
};

// Plain per-sample filter (baseline): reads raw t/y/sigma.
struct PlainArgs {
  const double* t;
  const double* y;
  const double* sig;
  const int64_t* off;
  const double* theta_row;  // [D] one sample
  const int32_t* col;
  const double* fixed;
  double* logl;             // one output
  int32_t* status;          // one output or NULL
  int32_t D, P, model;
  ModelConst mc;
};

// phc^2 of record k of a per-pulsar stream (the record's last 8 bytes)
__device__ __forceinline__ double rec_phc2(RecPtr r, int64_t k) {
  return ((ConstDPtr)r)[8 * k + 7];
}

struct StageArgs {
  const double* t;
  const double* y;
  const double* sig;
  const int64_t* src;   // [N] source TOA index of stream element k
  const int64_t* prev;  // [N] source index of the previous element, -1 first
  const int32_t* psr;   // [N] pulsar of stream element k
  TOARec* rec;
  int64_t N;
  double lam;
  int32_t merged;       // 1: merged stream (model 3) stores the pulsar index;
                        // 0: per-pulsar streams store phc^2 in the last 8 bytes
};

hipError_t launch_stage(const StageArgs& a, hipStream_t st);
hipError_t launch_hd(const double* pos, int P, double* G, hipStream_t st);
// Model 2 launches the fast filter, then (with_redo) the general filter over
// the items the fast one flagged.
hipError_t launch_filter(int model, const FilterArgs& a, int grid, int block,
                         hipStream_t st, bool with_redo = true);
// Time-parallel filter (models 1, 2): one workgroup of nw waves (4, 8 or 16)
// per item, grid workgroups striding over the items.
hipError_t launch_scan(int model, const FilterArgs& a, int grid, int nw, hipStream_t st);
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);
hipError_t launch_plain(const PlainArgs& a, hipStream_t st);

}  // namespace argus
