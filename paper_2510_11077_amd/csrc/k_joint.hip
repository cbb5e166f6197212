// Joint Kalman filter of P pulsars whose common OU process is coupled by the
// Hellings-Downs correlation (paper: Functionality, "State-space model
// construction": HD correlations enter through the covariance structure that
// couples the processes across pulsars). State: P x [r, f, a, g], n = 4P.
// TOAs of all pulsars form one time-ordered stream; at each TOA all 4P states
// propagate over the interval since the previous TOA and the measurement of
// pulsar p updates the joint state.
//
// Mapping on CDNA4: one workgroup (256 threads) per parameter sample. The
// symmetric covariance is cut into 4x4 blocks (a, b), a >= b; each thread
// holds one block in VGPRs (P(P+1)/2 <= 256). Per TOA:
//   phase A  every thread predicts its block, F_a P_ab F_b^T + Q_ab (F is
//            block-diagonal and sparse, Q is block-diagonal plus the HD
//            term G_ab v_c (1 - phi_c^2) on the (g, g) entry); the threads of
//            block row/column p write u = P H^T for their pulsar to LDS; the
//            diagonal owner of p forms the innovation; P threads precompute
//            the red-OU decay of every pulsar for the next TOA.
//   barrier
//   phase B  every thread applies the Joseph rank-2 update
//            P_ab - K_a u_b^T - u_a K_b^T + S K_a K_b^T to its block.
// LDS buffers alternate between TOAs, so one barrier per TOA suffices.
#include <hip/hip_runtime.h>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxP = kJointMaxPsr;
constexpr int kChunk = 64;  // TOAs per decay table / ledger fold

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
  // red-OU decay and noise of every pulsar for the next kChunk TOAs
  __shared__ double s_ph[kChunk][kMaxP], s_q[kChunk][kMaxP];
  // (S, e) of each TOA of the chunk, folded into the likelihood by wave 0
  __shared__ double s_led[kChunk][2];
  __shared__ double s_rec[kChunk][8];
  __shared__ double s_u[2][4 * kMaxP];
  __shared__ double s_e[2];
  __shared__ double s_vr[kMaxP], s_gr[kMaxP], s_ef2[kMaxP], s_eq2[kMaxP];
  __shared__ double s_vc;
  __shared__ int s_pnf;

  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int64_t s = blockIdx.x;
  const int P = a.P;
  const int nb = P * (P + 1) / 2;
  // block owned by this thread: (ba, bb), ba >= bb
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
  const bool owner = tid < nb;
  const bool diag = owner && ba == bb;

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
  const double gvc = owner ? a.hd[ba * P + bb] * vc : 0.0;  // G_ab v_c
  // covariance block B[i][j] = Cov(state i of pulsar ba, state j of pulsar bb)
  double B[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) B[i][j] = 0.0;
  if (diag) {
    B[0][0] = a.mc.s_r2;
    B[1][1] = a.mc.s_f2;
    B[2][2] = s_vr[ba];
  }
  B[3][3] = gvc;
  double x[4] = {0.0, 0.0, 0.0, 0.0};  // mean of pulsar ba (diagonal owners)
  const double ss2 = a.mc.ss2;
  // per-lane ledger of wave 0: lane l folds TOAs k = l mod kChunk
  double quad = 0.0, lm = 1.0;
  int le = 0, fail_code = 0;
  int64_t fail_k = INT64_MAX;

  for (int64_t k0 = 0; k0 < a.N; k0 += kChunk) {
    const int n = (int)(a.N - k0 < kChunk ? a.N - k0 : kChunk);
    // stage the chunk's TOA records in LDS (8 doubles each; the last slot
    // carries the pulsar index) and build its decay table, (TOA j, pulsar q)
    // spread over all threads
    for (int idx = tid; idx < n * 8; idx += kThreads)
      s_rec[idx >> 3][idx & 7] = reinterpret_cast<const double*>(a.rec + k0)[idx];
    for (int idx = tid; idx < n * P; idx += kThreads) {
      const int q = idx / n, j = idx - q * n;
      const double em = expm1_k(-s_gr[q] * a.rec[k0 + j].dt);
      s_ph[j][q] = 1.0 + em;
      s_q[j][q] = s_vr[q] * (-em * (2.0 + em));
    }
    __syncthreads();
    // values of TOA j used before the barrier; those of j + 1 are read from
    // LDS during the update phase of j, off the critical path
    double r_dt = s_rec[0][0], r_h2 = s_rec[0][1], r_h3 = s_rec[0][2];
    double r_phc = s_rec[0][3], r_qcu = s_rec[0][4], r_y = s_rec[0][5];
    double r_s2 = s_rec[0][6];
    int r_p = __double_as_longlong(s_rec[0][7]) & 0xffffffff;
    double pa = s_ph[0][ba], pb = s_ph[0][bb], qa = s_q[0][ba];
    for (int j = 0; j < n; ++j) {
      const int64_t k = k0 + j;
      const int buf = (int)(k & 1);
      const int p = __builtin_amdgcn_readfirstlane(r_p);
      const double dt = r_dt, phc = r_phc;
      if (owner) {
        // rows: F_a B
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          B[0][c] = fma(dt, B[1][c], B[0][c]);
          B[2][c] *= pa;
          B[3][c] *= phc;
        }
        // columns: (F_a B) F_b^T
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          B[i][0] = fma(dt, B[i][1], B[i][0]);
          B[i][2] *= pb;
          B[i][3] *= phc;
        }
        B[3][3] = fma(gvc, r_qcu, B[3][3]);
        if (diag) {
          B[0][0] += ss2 * r_h3;
          B[0][1] += ss2 * r_h2;
          B[1][0] += ss2 * r_h2;
          B[1][1] += ss2 * dt;
          B[2][2] += qa;
          x[0] = fma(dt, x[1], x[0]);
          x[2] *= pa;
          x[3] *= phc;
          if (ba == p) s_e[buf] = r_y - (x[0] + x[2] + x[3]);
        }
        // u = P H^T for the pulsar paired with p in this block
        if (bb == p) {
#pragma unroll
          for (int i = 0; i < 4; ++i) s_u[buf][4 * ba + i] = B[i][0] + B[i][2] + B[i][3];
        } else if (ba == p) {
#pragma unroll
          for (int c = 0; c < 4; ++c) s_u[buf][4 * bb + c] = B[0][c] + B[2][c] + B[3][c];
        }
      }
      __syncthreads();
      const double s2 = r_s2;
      if (j + 1 < n) {
        r_dt = s_rec[j + 1][0];
        r_h2 = s_rec[j + 1][1];
        r_h3 = s_rec[j + 1][2];
        r_phc = s_rec[j + 1][3];
        r_qcu = s_rec[j + 1][4];
        r_y = s_rec[j + 1][5];
        r_s2 = s_rec[j + 1][6];
        r_p = __double_as_longlong(s_rec[j + 1][7]) & 0xffffffff;
        pa = s_ph[j + 1][ba];
        pb = s_ph[j + 1][bb];
        qa = s_q[j + 1][ba];
      }
      const double* u = s_u[buf];
      const double S =
          (u[4 * p] + u[4 * p + 2] + u[4 * p + 3]) + fma(s_ef2[p], s2, s_eq2[p]);
      const double inv = rcp_nr(S);
      if (owner) {
        double ua[4], ub[4], ka[4], kb[4], da[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          ua[i] = u[4 * ba + i];
          ub[i] = u[4 * bb + i];
          ka[i] = ua[i] * inv;
          kb[i] = ub[i] * inv;
          da[i] = fma(S, ka[i], -ua[i]);
        }
        // Joseph form P - K u^T - u K^T + S K K^T = P - K u^T + (S K - u) K^T
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int c = 0; c < 4; ++c) B[i][c] = fma(da[i], kb[c], fma(-ka[i], ub[c], B[i][c]));
        if (diag) {
          const double e = s_e[buf];
#pragma unroll
          for (int i = 0; i < 4; ++i) x[i] = fma(ka[i], e, x[i]);
        }
      }
      if (tid == 0) {
        s_led[j][0] = S;
        s_led[j][1] = s_e[buf];
      }
    }
    // wave 0 folds the chunk's innovations into its per-lane ledger
    if (tid < kWave && lane < n) {
      const double S = s_led[lane][0], e = s_led[lane][1];
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && fail_code == 0) {
        fail_code = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
        fail_k = k0 + lane;
      }
      quad = fma(e * e, rcp_nr(S), quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    }
  }
  // wave 0: combine the lanes in lane order; first failure = smallest TOA
  if (tid < kWave) {
    __shared__ double s_fold[kWave][2];
    __shared__ int64_t s_fk[kWave];
    __shared__ int s_fc[kWave];
    s_fold[lane][0] = quad;
    s_fold[lane][1] = log(lm) + (double)le * kLn2;
    s_fk[lane] = fail_k;
    s_fc[lane] = fail_code;
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
      double qs = 0.0, ls = 0.0;
      int64_t fk = INT64_MAX;
      int st = 0;
      for (int l = 0; l < kWave; ++l) {
        qs += s_fold[l][0];
        ls += s_fold[l][1];
        if (s_fk[l] < fk) {
          fk = s_fk[l];
          st = s_fc[l];
        }
      }
      if (s_pnf) st = kNonFinite;
      double ll = -0.5 * ((double)a.N * kLn2Pi + ls + qs);
      if (st == 0 && !finite_d(ll)) st = kNonFinite;
      a.logl[s] = st ? -INFINITY : ll;
      if (a.status) a.status[s] = st;
    }
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
