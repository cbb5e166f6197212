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
//   r_k = y_k - h_k^T A_k x0,  L L^T = Sigma_B,  a = L^{-1} r,
// the Cholesky pivots are exactly the sequential filter's innovation
// variances S_k = L_kk^2 and a_k = e_k / sqrt(S_k), so the block adds
// -1/2 sum_k (ln 2 pi + ln S_k + a_k^2) to log L (prediction-error
// decomposition). The posterior at the block's last TOA is
//   G = Cov(x_end, y) = A_end P0 A^T H^T + (A_{end<-j} Qacc_j h_j)_j,
//   V = G L^{-T},  x_end = A_end x0 + V a,
//   P_end = A_end P0 A_end^T + Qacc_end - V V^T,
// and the rank-kB downdate V V^T (an n x kB by kB x n product) runs on the
// FP64 matrix cores (v_mfma_f64_16x16x4f64).
//
// Mapping on CDNA4: one workgroup (256 threads) per parameter sample; P0
// (full n x n, FP64) and the block's work arrays live in LDS (~110 KB).
// Per block: per-TOA constants (threads j < kB) | T = P0 A^T H^T | Sigma_B and
// G | Cholesky with the residual as an extra column (wave 0) | V and the
// mean (row threads) | structured transition + accumulated noise of P0 (one
// 4x4 block per thread) | P -= V V^T on MFMA tiles. Seven barriers per kB
// TOAs instead of one per TOA.
#include <hip/hip_runtime.h>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxP = kJointMaxPsr;
constexpr int kB = 16;                                   // TOAs per block
constexpr int kNPad = ((4 * kMaxP + 15) / 16) * 16;     // padded state dim

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool finite_d(double v) {
  return __builtin_amdgcn_class(v, 0x1F8);
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

__device__ __forceinline__ double prm(const JointArgs& a, int c, int64_t s) {
  const int j = a.col[c];
  return j >= 0 ? a.theta[s * a.D + j] : a.fixed[c];
}

__global__ void __launch_bounds__(kThreads) k_joint(JointArgs a) {
  __shared__ double sP[kNPad * kNPad];    // covariance at the block start
  __shared__ double sT[kNPad][kB];        // P0 A^T H^T
  __shared__ double sG[kNPad][kB];        // G, then V
  __shared__ double sS[kB][kB + 1];       // Sigma_B | r  ->  L | a
  __shared__ double sx[2][kNPad];         // mean, double-buffered by block
  __shared__ double s_hd[kMaxP * kMaxP];
  __shared__ double s_vr[kMaxP], s_gr[kMaxP], s_ef2[kMaxP], s_eq2[kMaxP];
  __shared__ double s_eqe[kMaxP], s_qae[kMaxP];  // red decay / noise to the block end
  __shared__ double s_tau[kB], s_eg[kB], s_ec[kB], s_qrr[kB], s_qrf[kB], s_qa[kB];
  __shared__ double s_sc[kB], s_R[kB], s_ege[kB], s_ece[kB];
  __shared__ int s_p[kB];
  __shared__ double s_end[6];  // tau_end, ec_end, sc_end, qrr_end, qrf_end, qff_end
  __shared__ double s_vc;
  __shared__ int s_pnf;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  const int64_t s = blockIdx.x;
  const int P = a.P;
  const int n = 4 * P;
  const int np = ((n + 15) / 16) * 16;
  const double lam = a.mc.lam, ss2 = a.mc.ss2;

  for (int i = tid; i < np * np; i += kThreads) sP[i] = 0.0;
  for (int i = tid; i < 2 * kNPad; i += kThreads) (&sx[0][0])[i] = 0.0;
  for (int i = tid; i < P * P; i += kThreads) s_hd[i] = a.hd[i];
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
    sP[(4 * q) * np + 4 * q] = a.mc.s_r2;
    sP[(4 * q + 1) * np + 4 * q + 1] = a.mc.s_f2;
    sP[(4 * q + 2) * np + 4 * q + 2] = s_vr[q];
  }
  for (int i = tid; i < P * P; i += kThreads) {
    const int qa = i / P, qb = i - qa * P;
    sP[(4 * qa + 3) * np + 4 * qb + 3] = s_hd[i] * vc;
  }
  // block ownership for the structured transition: 4x4 block (ba, bb), ba >= bb
  int ba = 0, bb = 0;
  {
    int t = tid, r = 0;
    while (t >= r + 1) {
      t -= r + 1;
      ++r;
    }
    ba = r;
    bb = t;
  }
  const bool owner = tid < P * (P + 1) / 2;
  // ledger (thread 0): sum a_k^2, product of S_k as mantissa and exponent,
  // first failure
  double quad = 0.0, lm = 1.0;
  int le = 0, st = 0;
  int xb = 0;
  __syncthreads();

  for (int64_t k0 = 0; k0 < a.N; k0 += kB) {
    const int nb = (int)(a.N - k0 < kB ? a.N - k0 : kB);
    // ---- 1. per-TOA constants of the block: elapsed tau, decays, noise
    if (tid < nb) {
      const int j = tid;
      double tau = 0.0;
      for (int l = 0; l <= j; ++l) tau += a.rec[k0 + l].dt;
      const TOARec r = a.rec[k0 + j];
      const int p = r.psr;
      const double em = expm1_k(-s_gr[p] * tau);
      const double emc = expm1_k(-lam * tau);
      s_tau[j] = tau;
      s_eg[j] = 1.0 + em;
      s_ec[j] = 1.0 + emc;
      s_qrr[j] = ss2 * (tau * tau * tau / 3.0);
      s_qrf[j] = ss2 * (tau * tau * 0.5);
      s_qa[j] = s_vr[p] * (-em * (2.0 + em));
      s_sc[j] = -emc * (2.0 + emc);
      s_R[j] = fma(s_ef2[p], r.s2, s_eq2[p]);
      s_p[j] = p;
      sS[j][kB] = r.y;  // residual formed in phase 2
      if (j == nb - 1) s_end[0] = tau;
    }
    __syncthreads();
    // ---- 2. residuals, decays to the block end, T = P0 A^T H^T
    const double tau_e = s_end[0];
    const double* x0 = sx[xb];
    if (tid < nb) {
      const int j = tid, p = s_p[j];
      const double dte = tau_e - s_tau[j];
      s_ege[j] = 1.0 + expm1_k(-s_gr[p] * dte);
      s_ece[j] = 1.0 + expm1_k(-lam * dte);
      sS[j][kB] -= x0[4 * p] + s_tau[j] * x0[4 * p + 1] + s_eg[j] * x0[4 * p + 2] +
                   s_ec[j] * x0[4 * p + 3];
    } else if (tid >= kWave && tid < kWave + P) {
      const int q = tid - kWave;
      const double em = expm1_k(-s_gr[q] * tau_e);
      s_eqe[q] = 1.0 + em;
      s_qae[q] = s_vr[q] * (-em * (2.0 + em));
    } else if (tid == 2 * kWave) {
      const double emc = expm1_k(-lam * tau_e);
      s_end[1] = 1.0 + emc;
      s_end[2] = -emc * (2.0 + emc);
      s_end[3] = ss2 * (tau_e * tau_e * tau_e / 3.0);
      s_end[4] = ss2 * (tau_e * tau_e * 0.5);
      s_end[5] = ss2 * tau_e;
    }
    for (int idx = tid; idx < n * nb; idx += kThreads) {
      const int i = idx / nb, j = idx - i * nb;
      const double* row = sP + i * np + 4 * s_p[j];
      sT[i][j] = row[0] + s_tau[j] * row[1] + s_eg[j] * row[2] + s_ec[j] * row[3];
    }
    __syncthreads();
    // ---- 3. Sigma_B (lower triangle) and G
    const double ec_e = s_end[1];
    for (int idx = tid; idx < nb * nb; idx += kThreads) {
      const int k = idx / nb, j = idx - k * nb;
      if (j > k) continue;
      const int p = s_p[j], pk = s_p[k];
      const double base = sT[4 * pk][j] + s_tau[k] * sT[4 * pk + 1][j] +
                          s_eg[k] * sT[4 * pk + 2][j] + s_ec[k] * sT[4 * pk + 3][j];
      const double dtk = s_tau[k] - s_tau[j];
      double noise = (1.0 + expm1_k(-lam * dtk)) * (s_hd[pk * P + p] * vc) * s_sc[j];
      if (pk == p)
        noise += fma(dtk, s_qrf[j], s_qrr[j]) + (1.0 + expm1_k(-s_gr[p] * dtk)) * s_qa[j];
      sS[k][j] = base + noise + (k == j ? s_R[k] : 0.0);
    }
    for (int idx = tid; idx < n * nb; idx += kThreads) {
      const int i = idx / nb, j = idx - i * nb;
      const int q = i >> 2, c = i & 3, p = s_p[j];
      double g;
      if (c == 0)
        g = fma(tau_e, sT[i + 1][j], sT[i][j]);
      else if (c == 1)
        g = sT[i][j];
      else if (c == 2)
        g = s_eqe[q] * sT[i][j];
      else
        g = ec_e * sT[i][j] + s_ece[j] * (s_hd[q * P + p] * vc) * s_sc[j];
      if (q == p) {
        if (c == 0) g += fma(tau_e - s_tau[j], s_qrf[j], s_qrr[j]);
        else if (c == 1) g += s_qrf[j];
        else if (c == 2) g += s_ege[j] * s_qa[j];
      }
      sG[i][j] = g;
    }
    __syncthreads();
    // ---- 4. Cholesky of Sigma_B with the residual column (wave 0)
    if (wave == 0) {
      for (int k = 0; k < nb; ++k) {
        const double d = sS[k][k];
        const double lk = sqrt(d);
        const double il = 1.0 / lk;
        const double ak = sS[k][kB] * il;
        if (lane == 0) {
          if (st == 0) {
            if (!finite_d(d)) st = kNonFinite;
            else if (!(d > 0.0)) st = kNonPD;
            else if (!finite_d(ak)) st = kNonFinite;
          }
          quad = fma(ak, ak, quad);
          const double pm = lm * d;
          lm = __builtin_amdgcn_frexp_mant(pm);
          le += __builtin_amdgcn_frexp_exp(pm);
        }
        const int i1 = k + 1 + lane;
        if (i1 < nb) sS[i1][k] *= il;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int m = nb - k - 1;
        for (int f = lane; f < m * m; f += kWave) {
          const int i = k + 1 + f / m, j = k + 1 + f % m;
          if (j <= i) sS[i][j] = fma(-sS[i][k], sS[j][k], sS[i][j]);
        }
        if (lane < m) sS[k + 1 + lane][kB] = fma(-sS[k + 1 + lane][k], ak, sS[k + 1 + lane][kB]);
        if (lane == 0) {
          sS[k][k] = lk;
          sS[k][kB] = ak;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
    }
    __syncthreads();
    // ---- 5. V = G L^{-T} and the mean at the block end (row threads)
    if (tid < n) {
      const int i = tid, q = i >> 2, c = i & 3;
      double g[kB];
#pragma unroll
      for (int k = 0; k < kB; ++k) g[k] = k < nb ? sG[i][k] : 0.0;
      double xv = 0.0;
#pragma unroll
      for (int k = 0; k < kB; ++k) {
        if (k < nb) {
          const double v = g[k] * rcp_nr(sS[k][k]);
          g[k] = v;
          xv = fma(v, sS[k][kB], xv);
#pragma unroll
          for (int k2 = k + 1; k2 < kB; ++k2)
            if (k2 < nb) g[k2] = fma(-v, sS[k2][k], g[k2]);
        }
      }
#pragma unroll
      for (int k = 0; k < kB; ++k)
        if (k < nb) sG[i][k] = g[k];
      double xa;
      if (c == 0) xa = fma(tau_e, x0[i + 1], x0[i]);
      else if (c == 1) xa = x0[i];
      else if (c == 2) xa = s_eqe[q] * x0[i];
      else xa = ec_e * x0[i];
      sx[xb ^ 1][i] = xa + xv;
    }
    // ---- 6a. P0 <- A_end P0 A_end^T + Qacc_end (one 4x4 block per thread)
    if (owner) {
      double B[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) B[i][j] = sP[(4 * ba + i) * np + 4 * bb + j];
      const double pa = s_eqe[ba], pb = s_eqe[bb];
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
      B[3][3] = fma(s_hd[ba * P + bb] * vc, s_end[2], B[3][3]);
      if (ba == bb) {
        B[0][0] += s_end[3];
        B[0][1] += s_end[4];
        B[1][0] += s_end[4];
        B[1][1] += s_end[5];
        B[2][2] += s_qae[ba];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          sP[(4 * ba + i) * np + 4 * bb + j] = B[i][j];
          sP[(4 * bb + j) * np + 4 * ba + i] = B[i][j];
        }
    }
    __syncthreads();
    // ---- 6b. P0 -= V V^T on the FP64 matrix cores, lower tiles, mirrored
    {
      const int nt = np / 16;
      const int ntiles = nt * (nt + 1) / 2;
      for (int t = wave; t < ntiles; t += kThreads / kWave) {
        int I = 0, tt = t;
        while (tt >= I + 1) {
          tt -= I + 1;
          ++I;
        }
        const int J = tt;
        f64x4 acc;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[r] = sP[(16 * I + (lane >> 4) + 4 * r) * np + 16 * J + (lane & 15)];
        const int ra = 16 * I + (lane & 15), rb = 16 * J + (lane & 15);
#pragma unroll
        for (int kc = 0; kc < kB / 4; ++kc) {
          const int k = 4 * kc + (lane >> 4);
          const double va = (ra < n && k < nb) ? -sG[ra][k] : 0.0;
          const double vb = (rb < n && k < nb) ? sG[rb][k] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(va, vb, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = 16 * I + (lane >> 4) + 4 * r, col = 16 * J + (lane & 15);
          if (I > J || row >= col) {
            sP[row * np + col] = acc[r];
            sP[col * np + row] = acc[r];
          }
        }
      }
    }
    __syncthreads();
    xb ^= 1;
  }
  if (tid == 0) {
    if (s_pnf) st = kNonFinite;
    double ll = -0.5 * ((double)a.N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
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
