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
// Mapping on CDNA4: one workgroup (4 waves) per parameter sample; P0 (full
// n x n, FP64) and the block's work arrays live in LDS (~130 KB). Per block
// of kB TOAs, three barriers:
//   A  all waves: T = P0 A^T H^T (n x kB) and the lower triangle of Sigma_B
//      from the 4x4 pulsar blocks of P0.
//   C  waves 0-1: the elimination in registers. Lanes 0-15 of each wave hold
//      the rows of Sigma_B with the residual, lanes 16-63 hold 48 rows of G
//      (formed from T) with the predicted mean; pivot, innovation and the
//      pivot column reach every lane by v_readlane, so the whole
//      factorisation runs without LDS round trips or barriers.
//      wave 2: P0 <- A_end P0 A_end^T + Qacc_end (one 4x4 pulsar block per
//      lane). wave 3: the next block's per-TOA constants (elapsed times,
//      decays, the noise part of its Sigma_B) from records staged in LDS, and
//      the global loads of the records of the block after it.
//   D  all waves: P -= U M^T on MFMA tiles (lower tiles, mirrored).
// The final block is padded to kB with identity rows of Sigma_B, zero
// residuals and zero columns of G: their pivots are exactly 1 and their
// innovations exactly 0, so they leave log L, x and P unchanged while every
// loop keeps a fixed trip count.
#include <hip/hip_runtime.h>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxP = kJointMaxPsr;
constexpr int kB = 16;                                   // TOAs per block
constexpr int kNPad = ((4 * kMaxP + 15) / 16) * 16;     // padded state dim
constexpr int kLdP = kNPad + 2;                          // P row: 16-B aligned
constexpr int kLdB = kB + 1;                             // rows of n x kB arrays
constexpr int kPairs = kB * (kB + 1) / 2;               // lower triangle
constexpr int kGRows = kWave - kB;                       // G rows per wave
static_assert(2 * kGRows >= kNPad, "two elimination waves cover every row");
static_assert(kGRows % 4 == 0, "a pulsar's four rows stay in one wave");

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
// not on the state; prepared one block ahead.
struct BlockConst {
  double tau[kB];   // time from the block start (previous TOA) to TOA k
  double eg[kB];    // e^{-rate_p tau}
  double ec[kB];    // e^{-lambda tau}
  double qrr[kB], qrf[kB];  // spin noise accumulated over tau
  double qa[kB];    // red noise accumulated over tau
  double sc[kB];    // 1 - e^{-2 lambda tau}
  double y[kB];
  double ege[kB], ece[kB];  // decays from TOA k to the block end
  double nz[4][kB];         // own-pulsar noise of G by state component
  double ecs[kB];           // ece * sc: common noise of G per unit Gamma v_c
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

__global__ void __launch_bounds__(kThreads) k_joint(JointArgs a) {
  __shared__ double sP[kNPad * kLdP];      // covariance at the block start
  __shared__ double sT[kNPad * kLdB];      // P0 A^T H^T
  __shared__ double sU[(kNPad + kB) * kLdB];  // eliminated columns u_k
  __shared__ double sM[(kNPad + kB) * kLdB];  // u_k / S_k
  // (rows kNPad.. take the stores of the Sigma_B lanes, which are not read)
  __shared__ double sS[kB * kLdB];         // Sigma_B, lower triangle
  __shared__ double sx[2][kNPad + kB];     // mean, double-buffered by block
  __shared__ double s_rec[2][kB][8];       // staged TOA records
  __shared__ BlockConst s_bc[2];
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
  const int nblk = P * (P + 1) / 2;
  const int64_t N = a.N;
  const double lam = a.mc.lam, ss2 = a.mc.ss2;
  const double* recd = reinterpret_cast<const double*>(a.rec);

  for (int i = tid; i < kNPad * kLdP; i += kThreads) sP[i] = 0.0;
  for (int i = tid; i < kNPad * kLdB; i += kThreads) sT[i] = 0.0;
  for (int i = tid; i < (kNPad + kB) * kLdB; i += kThreads) sU[i] = sM[i] = 0.0;
  for (int i = tid; i < 2 * (kNPad + kB); i += kThreads) (&sx[0][0])[i] = 0.0;
  for (int i = tid; i < P * P; i += kThreads) s_hd[i] = a.hd[i];
  // padded columns of a short block read finite leftovers, never garbage
  for (int i = tid; i < (int)(sizeof(s_bc) / sizeof(double)); i += kThreads)
    reinterpret_cast<double*>(s_bc)[i] = 0.0;
  for (int i = tid; i < 2 * kB * 8; i += kThreads) (&s_rec[0][0][0])[i] = 0.0;
  __syncthreads();
  // records of the first two blocks
  for (int i = tid; i < 2 * kB * 8; i += kThreads)
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
  int sk = 0, sj = 0;  // phase A: Sigma_B entry of threads < kPairs
  if (tid < kPairs) pair_of(tid, sk, sj);
  int pk3[3], pj3[3];  // wave 3: noise pairs of its lanes
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    pk3[u] = pj3[u] = 0;
    if (lane + kWave * u < kPairs) pair_of(lane + kWave * u, pk3[u], pj3[u]);
  }
  int tba[4], tbb[4];  // wave 2: 4x4 pulsar blocks of its lanes
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    int bb = lane + kWave * u, ba = 0;
    while (bb >= ba + 1) {
      bb -= ba + 1;
      ++ba;
    }
    tba[u] = ba;
    tbb[u] = bb;
  }

  // Per-block constants of block b (first TOA k0) into s_bc[b & 1] from the
  // records staged in s_rec[b & 1]; run by one whole wave.
  auto prep = [&](int buf, int64_t k0) {
    BlockConst& bc = s_bc[buf];
    const double(*rec)[8] = s_rec[buf];
    const int64_t rem = N - k0;
    const int nb = rem < kB ? (int)rem : kB;
    if (lane < kB) {
      double tau = 0.0;
#pragma unroll
      for (int l = 0; l < kB; ++l) {
        const double dt = rec[l][0];
        if (l <= lane && l < nb) tau += dt;
      }
      if (lane < nb) {
        const int p = (int)(__double_as_longlong(rec[lane][7]) & 0xffffffffll);
        const double em = expm1_k(-s_gr[p] * tau);
        const double emc = expm1_k(-lam * tau);
        bc.tau[lane] = tau;
        bc.eg[lane] = 1.0 + em;
        bc.ec[lane] = 1.0 + emc;
        bc.qrr[lane] = ss2 * (tau * tau * tau / 3.0);
        bc.qrf[lane] = ss2 * (tau * tau * 0.5);
        bc.qa[lane] = s_vr[p] * (-em * (2.0 + em));
        bc.sc[lane] = -emc * (2.0 + emc);
        bc.y[lane] = rec[lane][5];
        bc.sn[lane][lane] = fma(s_ef2[p], rec[lane][6], s_eq2[p]);  // R_k for now
        bc.p[lane] = p;
        if (lane == nb - 1) bc.end[0] = tau;
      }
    }
    if (lane == 0) bc.nb = nb;
    wave_sync();
    const double tau_e = bc.end[0];
    if (lane < nb) {
      const double dte = tau_e - bc.tau[lane];
      const double ege = 1.0 + expm1_k(-s_gr[bc.p[lane]] * dte);
      const double ece = 1.0 + expm1_k(-lam * dte);
      bc.ege[lane] = ege;
      bc.ece[lane] = ece;
      bc.nz[0][lane] = fma(dte, bc.qrf[lane], bc.qrr[lane]);
      bc.nz[1][lane] = bc.qrf[lane];
      bc.nz[2][lane] = ege * bc.qa[lane];
      bc.nz[3][lane] = 0.0;
      bc.ecs[lane] = ece * bc.sc[lane];
    } else if (lane >= kB && lane < kB + P) {
      const int q = lane - kB;
      const double em = expm1_k(-s_gr[q] * tau_e);
      bc.eqe[q] = 1.0 + em;
      bc.qae[q] = s_vr[q] * (-em * (2.0 + em));
    } else if (lane == kWave - 1) {
      const double emc = expm1_k(-lam * tau_e);
      bc.end[1] = 1.0 + emc;
      bc.end[2] = -emc * (2.0 + emc);
      bc.end[3] = ss2 * (tau_e * tau_e * tau_e / 3.0);
      bc.end[4] = ss2 * (tau_e * tau_e * 0.5);
      bc.end[5] = ss2 * tau_e;
    }
    // noise part of Sigma_B: common OU (HD-coupled) for every pair, spin and
    // red noise for pairs of one pulsar, R on the diagonal
    double sv[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const int k = pk3[u], j = pj3[u];
      sv[u] = k == j ? 1.0 : 0.0;
      if (lane + kWave * u < kPairs && k < nb) {
        const int p = bc.p[j], pk = bc.p[k];
        const double dtk = bc.tau[k] - bc.tau[j];
        double v = (1.0 + expm1_k(-lam * dtk)) * (s_hd[pk * P + p] * vc) * bc.sc[j];
        if (pk == p)
          v += fma(dtk, bc.qrf[j], bc.qrr[j]) + (1.0 + expm1_k(-s_gr[p] * dtk)) * bc.qa[j];
        if (k == j) v += bc.sn[k][k];
        sv[u] = v;
      }
    }
    wave_sync();  // R_k read above before the diagonal is overwritten
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (lane + kWave * u < kPairs) bc.sn[pk3[u]][pj3[u]] = sv[u];
  };

  // ledger (thread 0 keeps it): sum e_k^2 / S_k, product of S_k as mantissa
  // and exponent, first failure
  double quad = 0.0, lm = 1.0;
  int le = 0, st = 0;
  __syncthreads();
  if (wave == 3 && N > 0) prep(0, 0);
  __syncthreads();

  int xb = 0;
  for (int64_t k0 = 0, b = 0; k0 < N; k0 += kB, ++b) {
    const int cb = (int)(b & 1);
    const BlockConst& bc = s_bc[cb];
    const int nb = bc.nb;
    // ---- A. T = P0 A^T H^T and Sigma_B (lower) from P0
#pragma unroll
    for (int t = 0; t < (kNPad * kB + kThreads - 1) / kThreads; ++t) {
      const int e = tid + kThreads * t;
      const int i = e >> 4, j = e & (kB - 1);
      if (i < n) {
        double v = 0.0;
        if (j < nb) {
          const double* r = sP + i * kLdP + 4 * bc.p[j];
          v = r[0] + bc.tau[j] * r[1] + bc.eg[j] * r[2] + bc.ec[j] * r[3];
        }
        sT[i * kLdB + j] = v;
      }
    }
    if (tid < kPairs) {
      double v = bc.sn[sk][sj];
      if (sk < nb) {
        const double* B = sP + 4 * bc.p[sk] * kLdP + 4 * bc.p[sj];
        const double t1 = bc.tau[sj], g1 = bc.eg[sj], c1 = bc.ec[sj];
        double w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double* r = B + c * kLdP;
          w[c] = r[0] + t1 * r[1] + g1 * r[2] + c1 * r[3];
        }
        v += w[0] + bc.tau[sk] * w[1] + bc.eg[sk] * w[2] + bc.ec[sk] * w[3];
      }
      sS[sk * kLdB + sj] = v;
    }
    __syncthreads();
    // ---- C.
    const double* x0 = sx[xb];
    const double tau_e = bc.end[0], ec_e = bc.end[1];
    if (wave < 2) {
      // load: Sigma_B row + residual (lanes < kB) or a row of G + predicted
      // mean, stored negated so that both kinds of row eliminate alike
      double v[kB], slot;
      const bool sig = lane < kB;
      const int row = sig ? kNPad + lane : kGRows * wave + lane - kB;
      if (sig) {
        const int k = lane;
#pragma unroll
        for (int j = 0; j < kB; ++j) v[j] = sS[(j <= k ? k * kLdB + j : j * kLdB + k)];
        const int pk = bc.p[k < nb ? k : 0];
        const double* xp = x0 + 4 * pk;
        const double r = bc.y[k] - (xp[0] + bc.tau[k] * xp[1] + bc.eg[k] * xp[2] + bc.ec[k] * xp[3]);
        slot = k < nb ? r : 0.0;
      } else {
        // G row = (A_end row) T + own-pulsar noise + HD-coupled common noise
        const bool live = row < n;
        const int q = live ? row >> 2 : 0, c = row & 3;
        const int r1 = c == 0 ? row + 1 : row;
        const double mA = !live ? 0.0 : c == 2 ? bc.eqe[q] : (c == 3 ? ec_e : 1.0);
        const double mB = live && c == 0 ? tau_e : 0.0;
        const double f3 = live && c == 3 ? vc : 0.0;
        const int own = live ? q : -1;
        const double* hq = s_hd + q * P;
#pragma unroll
        for (int j = 0; j < kB; ++j) {
          const int p = bc.p[j];
          double g = fma(mB, sT[r1 * kLdB + j], mA * sT[row * kLdB + j]);
          g = fma(f3 * bc.ecs[j], hq[p], g);
          const double o = bc.nz[c][j];
          g += own == p ? o : 0.0;
          v[j] = j < nb ? g : 0.0;
        }
        slot = -fma(mB, x0[r1], mA * x0[row]);
      }
      // elimination in TOA order
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
        // first failure: non-finite S, then S <= 0, then non-finite e
        const int nf_d = !finite_d(d), np_d = !(d > 0.0), nf_e = !finite_d(e);
        const int code = (nf_d * kNonFinite) | ((nf_d ^ 1) & np_d) * kNonPD |
                         ((nf_d | np_d) ^ 1) * nf_e * kNonFinite;
        st = st | ((st == 0) * code);
        quad = fma(e * inv, e, quad);
        const double pm = lm * d;
        lm = __builtin_amdgcn_frexp_mant(pm);
        le += __builtin_amdgcn_frexp_exp(pm);
      }
#pragma unroll
      for (int k = 0; k < kB; ++k) sU[row * kLdB + k] = v[k];
      sx[xb ^ 1][row] = -slot;
    } else if (wave == 2) {
      // P0 <- A_end P0 A_end^T + Qacc_end, one 4x4 pulsar block per lane
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (lane + kWave * u >= nblk) break;
        const int ba = tba[u], bb = tbb[u];
        double B[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) B[i][j] = sP[(4 * ba + i) * kLdP + 4 * bb + j];
        const double pa = bc.eqe[ba], pb = bc.eqe[bb];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          B[0][j] = fma(tau_e, B[1][j], B[0][j]);
          B[2][j] *= pa;
          B[3][j] *= ec_e;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          B[i][0] = fma(tau_e, B[i][1], B[i][0]);
          B[i][2] *= pb;
          B[i][3] *= ec_e;
        }
        B[3][3] = fma(s_hd[ba * P + bb] * vc, bc.end[2], B[3][3]);
        if (ba == bb) {
          B[0][0] += bc.end[3];
          B[0][1] += bc.end[4];
          B[1][0] += bc.end[4];
          B[1][1] += bc.end[5];
          B[2][2] += bc.qae[ba];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            sP[(4 * ba + i) * kLdP + 4 * bb + j] = B[i][j];
            sP[(4 * bb + j) * kLdP + 4 * ba + i] = B[i][j];
          }
      }
    } else {
      // records of block b + 2 (issued first, stored last), constants of b + 1
      const int64_t k2 = k0 + 2 * kB;
      const bool ok = k2 + (lane >> 2) < N;
      double r0 = 0.0, r1 = 0.0;
      if (ok) {
        r0 = recd[k2 * 8 + 2 * lane];
        r1 = recd[k2 * 8 + 2 * lane + 1];
      }
      if (k0 + kB < N) prep(cb ^ 1, k0 + kB);
      if (ok) {
        s_rec[cb][lane >> 2][2 * (lane & 3)] = r0;
        s_rec[cb][lane >> 2][2 * (lane & 3) + 1] = r1;
      }
    }
    __syncthreads();
    // ---- D. P -= U M^T on the FP64 matrix cores, lower tiles, mirrored
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int t = wave + 4 * u;
      if (t >= nt * (nt + 1) / 2) break;
      int I = 0, J = t;
      while (J >= I + 1) {
        J -= I + 1;
        ++I;
      }
      f64x4 acc;
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc[r] = sP[(16 * I + (lane >> 4) + 4 * r) * kLdP + 16 * J + (lane & 15)];
      const double* ua = sU + (16 * I + (lane & 15)) * kLdB + (lane >> 4);
      const double* mb = sM + (16 * J + (lane & 15)) * kLdB + (lane >> 4);
#pragma unroll
      for (int kc = 0; kc < kB / 4; ++kc)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-ua[4 * kc], mb[4 * kc], acc, 0, 0, 0);
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
  hipLaunchKernelGGL(k_joint, dim3((unsigned)S), dim3(kThreads), 0, st, a);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

}  // namespace argus
