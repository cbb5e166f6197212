// Joint Kalman filter of P pulsars whose common OU process is coupled by the
// Hellings-Downs correlation (paper: Functionality, "State-space model
// construction": HD correlations enter through the covariance structure that
// couples the processes across pulsars). State: P x [r, f, a, g], n = 4P.
// TOAs of all pulsars form one time-ordered stream; at each TOA all 4P states
// propagate over the interval since the previous TOA and the measurement of
// pulsar p updates the joint state.
//
// Blocked evaluation (same recursion, TOAs taken kB at a time). Given the
// posterior (x0, P0) at the start of a block, the block's measurements are
// jointly Gaussian: y_k = h_k^T (A_k x0 + xi_k) + eps_k with A_k the
// block-diagonal transition from the block start to TOA k and xi_k the
// process noise accumulated since then, whose covariances are closed forms
// of the elapsed time tau (spin: sigma_s^2 [[t^3/3, t^2/2], [t^2/2, t]];
// OU: v (1 - e^{-2 rate t}); common: Gamma v_c (1 - e^{-2 lambda t})) and
// Cov(xi_k, xi_j) = A_{k<-j} Qacc(tau_j) for k >= j. With
//   Sigma_B[k][j] = h_k^T A_k P0 A_j^T h_j + h_k^T A_{k<-j} Qacc_j h_j + R_k d_kj,
//   r_k = y_k - h_k^T A_k x0,
//   G = Cov(x_end, y) = A_end P0 A^T H^T + (A_{end<-j} Qacc_j h_j)_j,
// Gaussian elimination of Sigma_B in TOA order (an L D L^T factorisation)
// reproduces the sequential filter exactly: pivot k is the innovation
// variance S_k and the eliminated residual is the innovation e_k, so the
// block adds -1/2 sum_k (ln 2 pi + ln S_k + e_k^2 / S_k) to log L
// (prediction-error decomposition). Eliminating the rows of G alongside
// gives, column by column, u_k (the cross-covariance of the end state with
// innovation k), and the posterior at the block's last TOA is
//   x_end = A_end x0 + sum_k u_k e_k / S_k,
//   P_end = A_end P0 A_end^T + Qacc_end - sum_k u_k u_k^T / S_k,
// a rank-kB downdate U M^T (M = U S^{-1}, n x kB by kB x n) that runs on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// Mapping on CDNA4: one workgroup (16 waves, 4 per SIMD, so that LDS latency
// overlaps across waves) per parameter sample; P0 (full n x n, FP64) and the
// block's work arrays live in LDS (~145 KB). Per block of kB TOAs, three
// barriers:
//   A  all waves: G (n x kB) and the full Sigma_B from the 4x4 pulsar
//      blocks of P0, and the last column of every elimination row (the
//      negated predicted mean of a state row, the residual of a TOA row),
//      so that the elimination waves load their rows without divergence.
//   C  waves 0-1: the elimination in registers. Lanes 0-15 of each wave hold
//      the rows of Sigma_B with the residual, lanes 16-63 hold 48 rows of G
//      with the predicted mean; pivot, innovation and the
//      pivot column reach every lane by v_readlane, so the whole
//      factorisation runs without LDS round trips or barriers.
//      Waves 5, 9, 13 (beside wave 1): the noise part of the next block's
//      Sigma_B. Waves on the other two SIMDs: P0 <- A_end P0 A_end^T +
//      Qacc_end on the lower triangle (4-row column segments, consecutive
//      lanes on consecutive columns), the log-likelihood ledger of the
//      previous block (pivots and innovations left in LDS by the
//      elimination), the per-TOA constants of the block after next (elapsed
//      times, decays) from records staged in LDS with the global loads of the
//      records of the block after that.
//   D  all waves: P -= U M^T on MFMA tiles (lower tiles, mirrored).
// The final block is padded to kB with identity rows of Sigma_B, zero
// residuals and zero columns of G: their pivots are exactly 1 and their
// innovations exactly 0, so they leave log L, x and P unchanged while every
// loop keeps a fixed trip count.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

constexpr int kWaves = 16;                               // 4 per SIMD
constexpr int kThreads = kWaves * kWave;
constexpr int kMaxP = kJointBlockedMaxPsr;
constexpr int kB = 16;                                   // TOAs per block
constexpr int kNPad = ((4 * kMaxP + 15) / 16) * 16;     // padded state dim
constexpr int kLdP = kNPad + 2;                          // P row: 16-B aligned
constexpr int kLdB = kB + 1;                             // rows of n x kB arrays
constexpr int kPairs = kB * (kB + 1) / 2;               // lower triangle
constexpr int kGRows = kWave - kB;                       // G rows per wave
constexpr int kNBuf = 3;                                 // block-constant buffers
static_assert(2 * kGRows >= kNPad, "two elimination waves cover every row");
static_assert(kGRows % 4 == 0, "a pulsar's four rows stay in one wave");
static_assert(kThreads / 16 * 2 >= kNPad * kB / 16, "phase A covers G in two passes");

// Work of phase C by wave (SIMD = wave % 4): the elimination on waves 0 and
// 1 (SIMDs 0 and 1; waves 4, 8, 12 beside wave 0 stay idle in C so as not to
// take its issue slots, the longer of the two); the noise part of the next
// block's Sigma_B on waves 5, 9, 13 beside wave 1; SIMDs 2 and 3 take the
// rest.
constexpr int kWLedger = 2;      // ledger of the previous block
constexpr int kWToa = 3;         // per-TOA constants two blocks ahead, records
__device__ __forceinline__ int pairs_slot(int w) {      // -1: not a pairs wave
  return w == 5 ? 0 : w == 9 ? 1 : w == 13 ? 2 : -1;
}
constexpr int kTfWaves = 6;      // transform: waves 6, 10, 14 and 7, 11, 15
constexpr int kTfRounds = 3;     // units per lane (2 P (P + 1) <= kTfRounds * 384)
static_assert(2 * kMaxP * (kMaxP + 1) <= kTfRounds * kTfWaves * kWave, "transform units");
__device__ __forceinline__ int transform_slot(int w) {  // -1: not a transform wave
  return w == 6 ? 0 : w == 10 ? 1 : w == 14 ? 2 : w == 7 ? 3 : w == 11 ? 4 : w == 15 ? 5 : -1;
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool finite_d(double v) {
  return __builtin_amdgcn_class(v, 0x1F8);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// value of lane + 1 within each row of 16 lanes (0 for the last lane)
__device__ __forceinline__ double next_lane_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0x101, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x101, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// row k, column j of the pair with lower-triangle index e (row-major)
__device__ __forceinline__ void pair_of(int e, int& k, int& j) {
  k = 0;
  while ((k + 1) * (k + 2) / 2 <= e) ++k;
  j = e - k * (k + 1) / 2;
}

struct JointArgs {
  const TOARec* rec;    // merged stream [N]
  const double* hd;     // [P*P]
  const double* theta;  // [S*D]
  const int32_t* col;
  const double* fixed;
  double* logl;
  int32_t* status;
  int64_t S, N;
  int32_t D, P;
  ModelConst mc;
};

// Per-block constants that depend on the TOA records and the parameters but
// not on the state. The per-TOA part is prepared two blocks ahead, the noise
// of Sigma_B one block ahead.
struct BlockConst {
  double tau[kB];   // time from the block start (previous TOA) to TOA k
  double eg[kB];    // e^{-rate_p tau}
  double ec[kB];    // e^{-lambda tau}
  double ieg[kB], iec[kB];  // their reciprocals
  double qrr[kB], qrf[kB];  // spin noise accumulated over tau
  double qa[kB];    // red noise accumulated over tau
  double sc[kB];    // 1 - e^{-2 lambda tau}
  double R[kB];     // white noise
  double y[kB];
  double nz[4][kB]; // own-pulsar noise of G by state component
  double ecs[kB];   // e^{-lambda (tau_e - tau)} sc: common noise of G per Gamma v_c
  double sn[kB][kB];        // noise + white part of Sigma_B (lower), padded identity
  double eqe[kMaxP], qae[kMaxP];  // per pulsar: red decay / noise over the block
  double end[6];    // tau_e, ec_e, sc_e, qrr_e, qrf_e, qff_e
  int p[kB];
  int nb;
  int pad_;
};
static_assert(sizeof(BlockConst) % sizeof(double) == 0, "zeroed as doubles");

__device__ __forceinline__ double prm(const JointArgs& a, int c, int64_t s) {
  const int j = a.col[c];
  return j >= 0 ? a.theta[s * a.D + j] : a.fixed[c];
}

// e^{-rate (tk - tj)} from the decays of tk and tj; recomputed directly when
// the decay of tj is too small to divide by
__device__ __forceinline__ double decay_ratio(double ek, double iej, double ej, double x) {
  return ej > 1e-280 ? ek * iej : 1.0 + expm1_k(x);
}

__global__ void __launch_bounds__(kThreads) k_joint(JointArgs a) {
  __shared__ double sP[kNPad * kLdP];      // covariance at the block start
  // rows of the elimination: G = Cov(x_end, y_block) (rows 0 .. kNPad - 1,
  // zero past n) and the full symmetric Sigma_B (rows kNPad .. kNPad + kB - 1)
  __shared__ double sG[(kNPad + kB) * kLdB];
  __shared__ double s_slot[kNPad + kB];    // their last column: -predicted mean, residual
  __shared__ double sU[(kNPad + kB) * kLdB];  // eliminated columns u_k
  __shared__ double sM[(kNPad + kB) * kLdB];  // u_k / S_k
  // (rows kNPad.. take the stores of the Sigma_B lanes, which are not read)
  __shared__ double sx[2][kNPad + kB];     // mean, double-buffered by block
  __shared__ double s_rec[kNBuf][kB][8];   // staged TOA records
  __shared__ double s_led[2][kB][2];       // pivots S_k and innovations e_k
  __shared__ BlockConst s_bc[kNBuf];
  __shared__ double s_hd[kMaxP * kMaxP];
  __shared__ double s_vr[kMaxP], s_gr[kMaxP], s_ef2[kMaxP], s_eq2[kMaxP];
  __shared__ double s_vc;
  __shared__ int s_pnf;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int64_t s = blockIdx.x;
  const int P = a.P;
  const int n = 4 * P;
  const int nt = (n + 15) / 16;
  const int ntl = nt * (nt + 1) / 2;
  const int64_t N = a.N;
  const double lam = a.mc.lam, ss2 = a.mc.ss2;
  const double* recd = reinterpret_cast<const double*>(a.rec);

  for (int i = tid; i < kNPad * kLdP; i += kThreads) sP[i] = 0.0;
  for (int i = tid; i < (kNPad + kB) * kLdB; i += kThreads) sG[i] = 0.0;
  for (int i = tid; i < (kNPad + kB) * kLdB; i += kThreads) sU[i] = sM[i] = 0.0;
  for (int i = tid; i < 2 * (kNPad + kB); i += kThreads) (&sx[0][0])[i] = 0.0;
  for (int i = tid; i < P * P; i += kThreads) s_hd[i] = a.hd[i];
  // padded columns of a short block read finite leftovers, never garbage
  for (int i = tid; i < (int)(sizeof(s_bc) / (sizeof(double))); i += kThreads)
    reinterpret_cast<double*>(s_bc)[i] = 0.0;
  for (int i = tid; i < kNBuf * kB * 8; i += kThreads) (&s_rec[0][0][0])[i] = 0.0;
  __syncthreads();
  // records of the first kNBuf blocks
  for (int i = tid; i < kNBuf * kB * 8; i += kThreads)
    if ((i >> 3) < N) (&s_rec[0][0][0])[i] = recd[i];
  if (tid == 0) {
    const double la = prm(a, 4 * P, s), gc = prm(a, 4 * P + 1, s);
    const double gm1 = gc - 1.0;
    s_vc = exp(2.0 * kLn10 * la + (gc - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
           (12.0 * kPi * kPi * gm1);
    s_pnf = (finite_d(la) && finite_d(gc)) ? 0 : 1;
  }
  __syncthreads();
  if (tid < P) {
    const int q = tid;
    const double lsr = prm(a, 4 * q, s), lgr = prm(a, 4 * q + 1, s);
    const double ef = prm(a, 4 * q + 2, s), leq = prm(a, 4 * q + 3, s);
    if (!(finite_d(lsr) && finite_d(lgr) && finite_d(ef) && finite_d(leq)))
      atomicOr(&s_pnf, 1);
    const double gr = exp10(lgr);
    const double sr = exp10(lsr), eq = exp10(leq);
    s_vr[q] = sr * sr / (2.0 * gr);
    s_gr[q] = gr;
    s_ef2[q] = ef * ef;
    s_eq2[q] = eq * eq;
  }
  __syncthreads();
  const double vc = s_vc;
  // prior at the epoch: diag(s_r^2, s_f^2, v_r) per pulsar, G v_c on g-g
  if (tid < P) {
    const int q = tid;
    sP[(4 * q) * kLdP + 4 * q] = a.mc.s_r2;
    sP[(4 * q + 1) * kLdP + 4 * q + 1] = a.mc.s_f2;
    sP[(4 * q + 2) * kLdP + 4 * q + 2] = s_vr[q];
  }
  for (int i = tid; i < P * P; i += kThreads) {
    const int qa = i / P, qb = i - qa * P;
    sP[(4 * qa + 3) * kLdP + 4 * qb + 3] = s_hd[i] * vc;
  }

  // fixed per-thread work assignments
  const int psl = pairs_slot(wave), tsl = transform_slot(wave);
  // transform units of this lane: unit u = the 4 rows of pulsar q in column
  // c <= 4q + 3, packed as q * 256 + c (-1: none)
  int tfu[kTfRounds];
#pragma unroll
  for (int rr = 0; rr < kTfRounds; ++rr) {
    const int u = kWave * (tsl + kTfWaves * rr) + lane;
    int q = (int)((sqrtf(1.0f + 2.0f * (float)u) - 1.0f) * 0.5f);
    q += 2 * (q + 1) * (q + 2) <= u ? 1 : 0;
    q -= 2 * q * (q + 1) > u ? 1 : 0;
    tfu[rr] = (tsl >= 0 && u < 2 * P * (P + 1)) ? q * 256 + (u - 2 * q * (q + 1)) : -1;
  }
  int sk = 0, sj = 0;  // phase A: Sigma_B entry of threads kSig0 .. kSig0 + kPairs
  constexpr int kSig0 = kThreads / 2;
  // phase A: the elimination rows' last column by threads kSlot0 .. (they
  // have no G entry in the second pass)
  constexpr int kSlot0 = 3 * kThreads / 4;
  static_assert(kThreads - kSlot0 >= kNPad + kB && 16 * 3 + 64 >= kNPad, "slot threads");
  if (tid >= kSig0 && tid < kSig0 + kPairs) pair_of(tid - kSig0, sk, sj);
  int pk = 0, pj = 0;  // pairs waves: one noise pair per lane
  const int pe = psl >= 0 ? lane + kWave * psl : kPairs;
  if (pe < kPairs) pair_of(pe, pk, pj);
  int tI[2], tJ[2];    // phase D: 16x16 tiles of this wave (clamped past the end)
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    int J = wave + kWaves * u, I = 0;
    if (J >= ntl) J = 0;
    while (J >= I + 1) {
      J -= I + 1;
      ++I;
    }
    tI[u] = I;
    tJ[u] = J;
  }

  // Per-TOA constants of the block starting at k0 into s_bc[buf] from the
  // records staged in s_rec[buf]; run by one whole wave.
  auto toa_part = [&](int buf, int64_t k0, int lane) {
    BlockConst& bc = s_bc[buf];
    const double(*rec)[8] = s_rec[buf];
    const int64_t rem = N - k0;
    const int nb = rem < kB ? (int)rem : kB;
    const int lr = lane < kB ? lane : 0;
    double dts[kB];
#pragma unroll
    for (int l = 0; l < kB; ++l) dts[l] = rec[l][0];
    const long long pbits = __double_as_longlong(rec[lr][7]);
    const double s2 = rec[lr][6], yv = rec[lr][5];
    // elapsed times (in stream order) and the end of the block
    double tau = 0.0;
#pragma unroll
    for (int l = 0; l < kB; ++l)
      if (l <= lane && l < nb) tau += dts[l];
    const double tau_e = readlane_d(tau, nb - 1);
    // one pass of two exponentials: TOA lanes (red, common decay over tau),
    // pulsar lanes (red decay over the block), the last lane (common decay
    // over the block)
    const bool toa = lane < nb;
    const bool psr = lane >= kB && lane < kB + P;
    const int pq = toa ? (int)(pbits & 0xffffffffll) : (psr ? lane - kB : 0);
    const double gq = s_gr[pq], vq = s_vr[pq], ef2 = s_ef2[pq], eq2 = s_eq2[pq];
    const double x1 = toa ? -gq * tau : (psr ? -gq * tau_e : -lam * tau_e);
    const double x2 = toa ? -lam * tau : 0.0;
    const double em1 = expm1_k(x1), em2 = expm1_k(x2);
    const double eg = 1.0 + em1, ec = 1.0 + em2;
    const double ieg = rcp_nr(eg), iec = rcp_nr(ec);
    const double qrf = ss2 * (tau * tau * 0.5), qrr = ss2 * (tau * tau * tau / 3.0);
    const double qa = vq * (-em1 * (2.0 + em1)), sc = -em2 * (2.0 + em2);
    if (toa) {
      bc.tau[lane] = tau;
      bc.eg[lane] = eg;
      bc.ec[lane] = ec;
      bc.ieg[lane] = ieg;
      bc.iec[lane] = iec;
      bc.qrr[lane] = qrr;
      bc.qrf[lane] = qrf;
      bc.qa[lane] = qa;
      bc.sc[lane] = sc;
      bc.R[lane] = fma(ef2, s2, eq2);
      bc.y[lane] = yv;
      bc.p[lane] = pq;
    } else if (psr) {
      bc.eqe[pq] = eg;
      bc.qae[pq] = qa;
    } else if (lane == kWave - 1) {
      bc.end[0] = tau_e;
      bc.end[1] = eg;
      bc.end[2] = -em1 * (2.0 + em1);
      bc.end[3] = ss2 * (tau_e * tau_e * tau_e / 3.0);
      bc.end[4] = ss2 * (tau_e * tau_e * 0.5);
      bc.end[5] = ss2 * tau_e;
    }
    if (lane == 0) bc.nb = nb;
    wave_sync();
    // noise of G per TOA: decays to the block end from the ratios
    const double eqp = bc.eqe[pq], ec_e = bc.end[1];
    if (toa) {
      const double dte = tau_e - tau;
      const double ege = decay_ratio(eqp, ieg, eg, -gq * dte);
      bc.nz[0][lane] = fma(dte, qrf, qrr);
      bc.nz[1][lane] = qrf;
      bc.nz[2][lane] = ege * qa;
      bc.nz[3][lane] = 0.0;
      bc.ecs[lane] = (ec_e * iec) * sc;
    }
  };

  // Noise part of Sigma_B of the block in s_bc[buf] (per-TOA part ready):
  // common OU (HD-coupled) for every pair, spin and red noise for pairs of
  // one pulsar, R on the diagonal; one pair per lane of the pairs waves.
  auto pairs_part = [&](int buf) {
    BlockConst& bc = s_bc[buf];
    const int nb = bc.nb;
    const int k = pk, j = pj;
    const int p = bc.p[j], pkk = bc.p[k];
    const double tk = bc.tau[k], tj = bc.tau[j];
    const double eck = bc.ec[k], iecj = bc.iec[j], scj = bc.sc[j];
    const double egk = bc.eg[k], iegj = bc.ieg[j], egj = bc.eg[j];
    const double qrfj = bc.qrf[j], qrrj = bc.qrr[j], qaj = bc.qa[j], Rk = bc.R[k];
    const double hv = s_hd[pkk * P + p], gp = s_gr[p];
    if (pe < kPairs) {
      double v = k == j ? 1.0 : 0.0;
      if (k < nb) {
        const double dtk = tk - tj;
        v = (eck * iecj) * (hv * vc) * scj;
        if (pkk == p) v += fma(dtk, qrfj, qrrj) + decay_ratio(egk, iegj, egj, -gp * dtk) * qaj;
        if (k == j) v += Rk;
      }
      bc.sn[k][j] = v;
    }
  };

  // ledger (thread kLedger keeps it): sum e_k^2 / S_k, product of S_k as
  // mantissa and exponent, first failure
  constexpr int kLedger = kWLedger * kWave;
  double quad = 0.0, lm = 1.0;
  int le = 0, st = 0;
  // one block's pivots and innovations folded in by 16 lanes
  auto ledger = [&](int buf, int lane) {
    const int k = lane & 15;
    const double d = s_led[buf][k][0], e = s_led[buf][k][1];
    const int code = !finite_d(d) ? kNonFinite
                     : !(d > 0.0) ? kNonPD
                     : !finite_d(e) ? kNonFinite : 0;
    int first = code ? k : kB;
    double qs = e * rcp_nr(d) * e;
    double mm = __builtin_amdgcn_frexp_mant(d);
    int me = __builtin_amdgcn_frexp_exp(d);
#pragma unroll
    for (int o = 1; o < kB; o <<= 1) {
      const int f2 = __shfl_xor(first, o, kB);
      first = f2 < first ? f2 : first;
      qs += __shfl_xor(qs, o, kB);
      const double pm = mm * __shfl_xor(mm, o, kB);
      me += __shfl_xor(me, o, kB) + __builtin_amdgcn_frexp_exp(pm);
      mm = __builtin_amdgcn_frexp_mant(pm);
    }
    const int fcode = __shfl(code, first < kB ? first : 0, kB);
    if (st == 0 && first < kB) st = fcode;
    quad += qs;
    const double pm = lm * mm;
    lm = __builtin_amdgcn_frexp_mant(pm);
    le += me + __builtin_amdgcn_frexp_exp(pm);
  };

  __syncthreads();
  if (N > 0 && wave == kWToa) toa_part(0, 0, lane);
  if (N > kB && wave == kWToa + 4) toa_part(1, kB, lane);
  __syncthreads();
  if (N > 0 && psl >= 0) pairs_part(0);
  __syncthreads();

  int xb = 0;
  int64_t k0 = 0;
  for (int64_t b = 0; k0 < N; k0 += kB, ++b) {
    // the thread index is re-read opaquely each block so that the per-lane
    // addresses of every phase are recomputed here instead of being hoisted
    // out of the loop and held in registers for its whole length
    int tidv = tid;
    __asm__ volatile("" : "+v"(tidv));
    const int tid = tidv;
    const int lane = tid & (kWave - 1);
    const int cb = (int)(b % kNBuf);
    const BlockConst& bc = s_bc[cb];
    const int nb = bc.nb;
    const double tau_e = bc.end[0], ec_e = bc.end[1];
    // ---- A. G = A_end P0 A^T H^T + noise, and Sigma_B (lower) from P0.
    //         Each row of 16 lanes takes one TOA column j and 16 consecutive
    //         rows; the r row of a pulsar takes its f row from the next lane.
    {
      const int j = (tid >> 4) & 15;
      const bool jv = j < nb;
      const int p = bc.p[j];
      const double t1 = bc.tau[j], g1 = bc.eg[j], c1 = bc.ec[j];
      const double hs = vc * bc.ecs[j];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int i = (tid & 15) + 16 * (tid >> 8) + 64 * t;
        if (i < kNPad) {  // uniform per row of 16 lanes
          const double* r0 = sP + i * kLdP + 4 * p;
          const int q = i >> 2, c = i & 3, qq = q < P ? q : 0;
          const double mA = c == 2 ? bc.eqe[qq] : (c == 3 ? ec_e : 1.0);
          const double hv = s_hd[qq * P + p];
          const double o = bc.nz[c][j];
          const double d0 = r0[0] + t1 * r0[1] + g1 * r0[2] + c1 * r0[3];
          const double d1 = next_lane_d(d0);
          double g = c == 0 ? fma(tau_e, d1, d0) : mA * d0;
          g = fma(c == 3 ? hs : 0.0, hv, g);
          g += q == p ? o : 0.0;
          if (i < n) sG[i * kLdB + j] = jv ? g : 0.0;
        }
      }
    }
    if (tid >= kSig0 && tid < kSig0 + kPairs) {
      const double sn = bc.sn[sk][sj];
      const int pa = bc.p[sk], pb = bc.p[sj];
      const double t1 = bc.tau[sj], g1 = bc.eg[sj], c1 = bc.ec[sj];
      const double t2 = bc.tau[sk], g2 = bc.eg[sk], c2 = bc.ec[sk];
      const double* B = sP + 4 * pa * kLdP + 4 * pb;
      double w[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const double* r = B + c * kLdP;
        w[c] = r[0] + t1 * r[1] + g1 * r[2] + c1 * r[3];
      }
      const double v = w[0] + t2 * w[1] + g2 * w[2] + c2 * w[3];
      const double val = sk < nb ? sn + v : sn;
      sG[(kNPad + sk) * kLdB + sj] = val;
      sG[(kNPad + sj) * kLdB + sk] = val;
    }
    // the last column of every elimination row: the negated predicted mean
    // of the state rows, the residual of the TOA rows
    if (tid >= kSlot0 && tid < kSlot0 + kNPad + kB) {
      const int row = tid - kSlot0;
      const double* x0 = sx[xb];
      double sl = 0.0;
      if (row >= kNPad) {
        const int k = row - kNPad;
        if (k < nb) {
          const double* xp = x0 + 4 * bc.p[k];
          sl = bc.y[k] - (xp[0] + bc.tau[k] * xp[1] + bc.eg[k] * xp[2] + bc.ec[k] * xp[3]);
        }
      } else if (row < n) {
        const int q = row >> 2, c = row & 3;
        const int r1 = c == 0 ? row + 1 : row;
        const double mA = c == 2 ? bc.eqe[q] : (c == 3 ? ec_e : 1.0);
        const double mB = c == 0 ? tau_e : 0.0;
        sl = -fma(mB, x0[r1], mA * x0[row]);
      }
      s_slot[row] = sl;
    }
    __syncthreads();
    // ---- C.
    if (wave < 2) {
      // load a row of Sigma_B (lanes < kB) or of G with its last column
      double v[kB];
      const bool sig = lane < kB;
      const int row = sig ? kNPad + lane : kGRows * wave + lane - kB;
#pragma unroll
      for (int j = 0; j < kB; ++j) v[j] = sG[row * kLdB + j];
      double slot = s_slot[row];
      // elimination in TOA order
      double dk = 1.0, ek = 0.0;
#pragma unroll
      for (int k = 0; k < kB; ++k) {
        const double d = readlane_d(v[k], k);
        const double e = readlane_d(slot, k);
        double colk[kB];
#pragma unroll
        for (int j = k + 1; j < kB; ++j) colk[j] = readlane_d(v[k], j);
        const double inv = rcp_nr(d);
        const double m = v[k] * inv;
#pragma unroll
        for (int j = k + 1; j < kB; ++j) v[j] = fma(-m, colk[j], v[j]);
        slot = fma(-m, e, slot);
        sM[row * kLdB + k] = m;
        dk = lane == k ? d : dk;
        ek = lane == k ? e : ek;
      }
#pragma unroll
      for (int k = 0; k < kB; ++k) sU[row * kLdB + k] = v[k];
      sx[xb ^ 1][row] = -slot;
      if (wave == 0 && sig) {
        s_led[b & 1][lane][0] = dk;
        s_led[b & 1][lane][1] = ek;
      }
    } else if (wave == kWLedger) {
      if (lane < kB && b > 0) ledger((b - 1) & 1, lane);
    } else if (wave == kWToa) {
      // records of block b + 3 (issued first, stored last), per-TOA
      // constants of block b + 2
      const int64_t k3 = k0 + 3 * kB;
      const bool ok = k3 + (lane >> 2) < N;
      double r0 = 0.0, r1 = 0.0;
      if (ok) {
        r0 = recd[k3 * 8 + 2 * lane];
        r1 = recd[k3 * 8 + 2 * lane + 1];
      }
      if (k0 + 2 * kB < N) toa_part((int)((b + 2) % kNBuf), k0 + 2 * kB, lane);
      if (ok) {
        s_rec[cb][lane >> 2][2 * (lane & 3)] = r0;
        s_rec[cb][lane >> 2][2 * (lane & 3) + 1] = r1;
      }
    } else if (psl >= 0) {
      if (k0 + kB < N) pairs_part((int)((b + 1) % kNBuf));
    } else if (tsl >= 0) {
      // P0 <- A_end P0 A_end^T + Qacc_end on the lower triangle of 4x4
      // pulsar blocks (the downdate below rewrites the upper triangle from
      // the lower); consecutive lanes take consecutive columns, the column
      // mix of the r column takes the f column from the next lane
      const double sce = bc.end[2] * vc, e3 = bc.end[3], e4 = bc.end[4], e5 = bc.end[5];
#pragma unroll
      for (int rr = 0; rr < kTfRounds; ++rr) {
        const int tu = tfu[rr];
        // units are a prefix of the lanes: none in lane 0, none in the wave
        if (__builtin_amdgcn_readfirstlane(tu) < 0) continue;
        const bool live = tu >= 0;
        const int q = live ? tu >> 8 : 0, c = live ? tu & 255 : 0, cc = c & 3, qc = c >> 2;
        double x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = sP[(4 * q + i) * kLdP + c];
        const double eq_r = bc.eqe[q], eq_c = bc.eqe[qc], qa_r = bc.qae[q];
        const double hv = s_hd[q * P + qc];
        x[0] = fma(tau_e, x[1], x[0]);
        x[2] *= eq_r;
        x[3] *= ec_e;
        const double mc = cc == 2 ? eq_c : (cc == 3 ? ec_e : 1.0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double nx = next_lane_d(x[i]);
          x[i] = cc == 0 ? fma(tau_e, nx, x[i]) : mc * x[i];
        }
        const bool own = qc == q;
        x[0] += own ? (cc == 0 ? e3 : (cc == 1 ? e4 : 0.0)) : 0.0;
        x[1] += own ? (cc == 0 ? e4 : (cc == 1 ? e5 : 0.0)) : 0.0;
        x[2] += own && cc == 2 ? qa_r : 0.0;
        x[3] = fma(hv * sce, cc == 3 ? 1.0 : 0.0, x[3]);
        if (live) {
#pragma unroll
          for (int i = 0; i < 4; ++i) sP[(4 * q + i) * kLdP + c] = x[i];
        }
      }
    }
    __syncthreads();
    // ---- D. P -= U M^T on the FP64 matrix cores, lower tiles, mirrored
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      if (wave + kWaves * u >= ntl) break;
      const int I = tI[u], J = tJ[u];
      f64x4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc[r] = sP[(16 * I + (lane >> 4) + 4 * r) * kLdP + 16 * J + (lane & 15)];
      const double* pu = sU + (16 * I + (lane & 15)) * kLdB + (lane >> 4);
      const double* pm = sM + (16 * J + (lane & 15)) * kLdB + (lane >> 4);
#pragma unroll
      for (int kc = 0; kc < kB / 4; ++kc)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-pu[4 * kc], pm[4 * kc], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 16 * I + (lane >> 4) + 4 * r, col = 16 * J + (lane & 15);
        if (I > J || row >= col) {
          sP[row * kLdP + col] = acc[r];
          sP[col * kLdP + row] = acc[r];
        }
      }
    }
    __syncthreads();
    xb ^= 1;
  }
  if (wave == kWLedger && lane < kB && k0 > 0) ledger((int)(((k0 / kB) - 1) & 1), lane);
  if (tid == kLedger) {
    if (s_pnf) st = kNonFinite;
    double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
    if (st == 0 && !finite_d(ll)) st = kNonFinite;
    a.logl[s] = st ? -INFINITY : ll;
    if (a.status) a.status[s] = st;
  }
}

// ---------------------------------------------------------------------------
// Sequential joint filter for arrays beyond the blocked kernel's LDS layout
// (P > 22): the same recursion one TOA at a time, one workgroup of NT
// threads per sample. The covariance's lower 4x4 pulsar blocks (a >= b) are
// spread over the threads' registers: blocks t + NT j, j < NR, of the lower
// triangle (row order) belong to thread t, and no thread touches another's
// entries. One block per thread in 1024 threads up to 44 pulsars, two in
// 768 (three waves per SIMD leave 168 registers) up to 54, four in 512 (256
// registers) up to 63; more blocks per thread spill. Per TOA of pulsar q (record: dt, the spin-noise moments, common
// decay and noise fraction, residual, white variance):
//   A  every block: X <- F_a X F_b^T + Q_ab with F_p = [[1, dt, 0, 0],
//      [0, 1, 0, 0], [0, 0, phi_p, 0], [0, 0, 0, phi_c]], Q_aa the pulsar's
//      spin and red noise, and Gamma_ab v_c (1 - phi_c^2) on the g-g entry
//      of every block; the blocks of column q (or row q, transposed) write
//      u = P- h_q to LDS; thread p < P predicts pulsar p's mean (kept in its
//      registers) and pulsar q's thread writes h_q . x-.
//   B  S = h_q . u + R, e = y - h_q . x-, K = u / S; every block takes the
//      Joseph update in the W = P- - K u^T, z = R K - W h, P+ = W + z K^T
//      form, row by row; thread p < P updates its mean and forms pulsar p's
//      decays of the TOA after next; thread 0 adds the log-likelihood terms.
// One barrier per TOA, between A and B: u and h_q . x- alternate between two
// LDS buffers (B of TOA k reads one while A of TOA k + 1 writes the other),
// and the decays, written two TOAs ahead into one of three buffers, are read
// only after the barrier that follows their writing.
__device__ __forceinline__ void lower_block(int e, int& r, int& c) {
  r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
  r += (r + 1) * (r + 2) / 2 <= e ? 1 : 0;
  r -= r * (r + 1) / 2 > e ? 1 : 0;
  c = e - r * (r + 1) / 2;
}

struct SeqTOA {
  double dt, h2, h3, phc, qc;  // interval, spin moments, common decay, common noise
  int q;
};

// phase A on one block (rows of pulsar pa, columns of pulsar pb)
__device__ __forceinline__ void seq_predict(double (&M)[4][4], int pa, int pb, double gam,
                                            const SeqTOA& o, double ss2, const double* s_ph,
                                            const double* s_qa, double* s_u) {
  const double fa = s_ph[pa], fb = s_ph[pb];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    M[0][c] = fma(o.dt, M[1][c], M[0][c]);
    M[2][c] *= fa;
    M[3][c] *= o.phc;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    M[i][0] = fma(o.dt, M[i][1], M[i][0]);
    M[i][2] *= fb;
    M[i][3] *= o.phc;
  }
  if (pa == pb) {
    M[0][0] = fma(ss2, o.h3, M[0][0]);
    M[0][1] = fma(ss2, o.h2, M[0][1]);
    M[1][0] = fma(ss2, o.h2, M[1][0]);
    M[1][1] = fma(ss2, o.dt, M[1][1]);
    M[2][2] += s_qa[pa];
  }
  M[3][3] = fma(gam, o.qc, M[3][3]);
  if (pb == o.q) {
#pragma unroll
    for (int i = 0; i < 4; ++i) s_u[4 * pa + i] = M[i][0] + M[i][2] + M[i][3];
  } else if (pa == o.q) {
#pragma unroll
    for (int c = 0; c < 4; ++c) s_u[4 * pb + c] = M[0][c] + M[2][c] + M[3][c];
  }
}

// phase B on one block, a row at a time (few values live)
__device__ __forceinline__ void seq_update(double (&M)[4][4], int pa, int pb, double inv,
                                           double R, double hu, const double* s_u) {
  double uj[4], Kj[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uj[c] = s_u[4 * pb + c];
    Kj[c] = uj[c] * inv;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double ui = s_u[4 * pa + i], Ki = ui * inv;
    // z = R K - W h with W h = u - K (h . u)
    const double zi = fma(R, Ki, -fma(-Ki, hu, ui));
#pragma unroll
    for (int c = 0; c < 4; ++c) M[i][c] = fma(zi, Kj[c], fma(-Ki, uj[c], M[i][c]));
  }
}

template <int NT, int NR>
__global__ void __launch_bounds__(NT) k_joint_seq(JointArgs a) {
  __shared__ double s_u[2][4 * kJointMaxPsr];
  __shared__ double s_ph[3][kJointMaxPsr], s_qa[3][kJointMaxPsr];  // red decay, noise by TOA
  __shared__ double s_vr[kJointMaxPsr], s_gr[kJointMaxPsr], s_ef2[kJointMaxPsr],
      s_eq2[kJointMaxPsr];
  __shared__ double s_hx[2], s_vc;
  __shared__ int s_pnf;
  const int tid = threadIdx.x;
  const int64_t s = blockIdx.x;
  const int P = a.P;
  const int nb = P * (P + 1) / 2;
  const int64_t N = a.N;
  const double ss2 = a.mc.ss2;
  const RecPtr rec = (RecPtr)a.rec;

  if (tid == 0) {
    const double la = prm(a, 4 * P, s), gc = prm(a, 4 * P + 1, s);
    const double gm1 = gc - 1.0;
    s_vc = exp(2.0 * kLn10 * la + (gc - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
           (12.0 * kPi * kPi * gm1);
    s_pnf = (finite_d(la) && finite_d(gc)) ? 0 : 1;
  }
  __syncthreads();
  if (tid < P) {
    const int q = tid;
    const double lsr = prm(a, 4 * q, s), lgr = prm(a, 4 * q + 1, s);
    const double ef = prm(a, 4 * q + 2, s), leq = prm(a, 4 * q + 3, s);
    if (!(finite_d(lsr) && finite_d(lgr) && finite_d(ef) && finite_d(leq)))
      atomicOr(&s_pnf, 1);
    const double gr = exp10(lgr);
    const double sr = exp10(lsr), eq = exp10(leq);
    s_vr[q] = sr * sr / (2.0 * gr);
    s_gr[q] = gr;
    s_ef2[q] = ef * ef;
    s_eq2[q] = eq * eq;
    // decays of the first two TOAs
    for (int k = 0; k < 2; ++k) {
      const double dtk = k < N ? rec[k].dt : 0.0;
      const double em = expm1_k(-gr * dtk);
      s_ph[k][q] = 1.0 + em;
      s_qa[k][q] = s_vr[q] * (-em * (2.0 + em));
    }
  }
  __syncthreads();
  const double vc = s_vc;

  // this thread's blocks: rows of pulsar ba[j], columns of pulsar bb[j];
  // the prior: diag(s_r^2, s_f^2, v_r) per pulsar, Gamma v_c on g-g
  int ba[NR], bb[NR];
  double gam[NR];
  double X[NR][4][4];
#pragma unroll
  for (int j = 0; j < NR; ++j) {
    const int e = tid + NT * j;
    int r = -1, c = -1;
    if (e < nb) lower_block(e, r, c);
    ba[j] = r;
    bb[j] = c;
    gam[j] = e < nb ? a.hd[r * P + c] : 0.0;
    double (&M)[4][4] = X[j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) M[i][cc] = 0.0;
    if (e < nb) {
      if (r == c) {
        M[0][0] = a.mc.s_r2;
        M[1][1] = a.mc.s_f2;
        M[2][2] = s_vr[r];
      }
      M[3][3] = gam[j] * vc;
    }
  }
  // the mean of pulsar tid (tid < P)
  double xm[4] = {0.0, 0.0, 0.0, 0.0};
  const double gr_own = tid < P ? s_gr[tid] : 0.0, vr_own = tid < P ? s_vr[tid] : 0.0;

  double quad = 0.0, lm = 1.0;
  int le = 0, st = 0;
  for (int64_t k = 0; k < N; ++k) {
    const TOARec r = load_rec(rec, k);
    const SeqTOA o{r.dt, r.h2, r.h3, r.phc, vc * r.qcu, __builtin_amdgcn_readfirstlane(r.psr)};
    const int ub = (int)(k & 1), db = (int)(k % 3);
    double* su = s_u[ub];
    // ---- A. predict every block, u = P- h_q, predicted mean
#pragma unroll
    for (int j = 0; j < NR; ++j)
      if (ba[j] >= 0) seq_predict(X[j], ba[j], bb[j], gam[j], o, ss2, s_ph[db], s_qa[db], su);
    if (tid < P) {
      xm[0] = fma(o.dt, xm[1], xm[0]);
      xm[2] *= s_ph[db][tid];
      xm[3] *= o.phc;
      if (tid == o.q) s_hx[ub] = xm[0] + xm[2] + xm[3];
    }
    __syncthreads();
    // ---- B. innovation, gain, Joseph update of every block
    const int q = o.q;
    const double hu = su[4 * q] + su[4 * q + 2] + su[4 * q + 3];
    const double R = fma(s_ef2[q], r.s2, s_eq2[q]);
    const double S = hu + R;
    const double e = r.y - s_hx[ub];
    const double inv = rcp_nr(S);
#pragma unroll
    for (int j = 0; j < NR; ++j)
      if (ba[j] >= 0) seq_update(X[j], ba[j], bb[j], inv, R, hu, su);
    if (tid < P) {
#pragma unroll
      for (int i = 0; i < 4; ++i) xm[i] = fma(su[4 * tid + i] * inv, e, xm[i]);
    }
    if (tid == 0) {
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && st == 0) st = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
      quad = fma(e * e, inv, quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    }
    // the decays of the TOA after next, into the buffer that TOA k - 1 used:
    // its readers (phase A of k - 1) are behind this TOA's barrier, and the
    // TOA after next reads it after the next TOA's barrier
    if (tid < P && k + 2 < N) {
      const double em = expm1_k(-gr_own * rec[k + 2].dt);
      s_ph[(k + 2) % 3][tid] = 1.0 + em;
      s_qa[(k + 2) % 3][tid] = vr_own * (-em * (2.0 + em));
    }
  }
  if (tid == 0) {
    if (s_pnf) st = kNonFinite;
    double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
    if (st == 0 && !finite_d(ll)) st = kNonFinite;
    a.logl[s] = st ? -INFINITY : ll;
    if (a.status) a.status[s] = st;
  }
}

}  // namespace

int joint_loglike(argus_dataset* ds, const double* theta, int64_t S, double* logl,
                  int32_t* status, hipStream_t st) {
  JointArgs a{};
  a.rec = ds->rec.as<TOARec>();
  a.hd = ds->hd.as<double>();
  a.theta = theta;
  a.col = ds->col.as<int32_t>();
  a.fixed = ds->fixed.as<double>();
  a.logl = logl;
  a.status = status;
  a.S = S;
  a.N = ds->N;
  a.D = ds->D;
  a.P = ds->P;
  a.mc = ds->mc;
  const char* force = std::getenv("ARGUS_JOINT");
  const bool seq = ds->P > kJointBlockedMaxPsr || (force && !std::strcmp(force, "seq"));
  if (!seq) {
    hipLaunchKernelGGL(k_joint, dim3((unsigned)S), dim3(kThreads), 0, st, a);
  } else {
    // threads and blocks per thread
    const int nb = ds->P * (ds->P + 1) / 2;
    const dim3 g((unsigned)S);
    if (nb <= 1024)
      hipLaunchKernelGGL((k_joint_seq<1024, 1>), g, dim3(1024), 0, st, a);
    else if (nb <= 2 * 768)
      hipLaunchKernelGGL((k_joint_seq<768, 2>), g, dim3(768), 0, st, a);
    else
      hipLaunchKernelGGL((k_joint_seq<512, 4>), g, dim3(512), 0, st, a);
  }
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

}  // namespace argus
