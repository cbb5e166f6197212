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
  __shared__ double s_phr[2][kMaxP], s_qr[2][kMaxP];
  __shared__ double s_u[2][4 * kMaxP];
  __shared__ double s_e[2];
  __shared__ double s_vr[kMaxP], s_gr[kMaxP], s_ef2[kMaxP], s_eq2[kMaxP];
  __shared__ double s_vc;
  __shared__ int s_pnf;

  const int tid = threadIdx.x;
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
  // threads that evaluate per-pulsar red-OU decays: the last P threads
  const int q_phi = tid - (kThreads - P);
  const bool phi_thr = q_phi >= 0;

  if (tid == 0) {
    const double la = prm(a, 4 * P, s), gc = prm(a, 4 * P + 1, s);
    const double gm1 = gc - 1.0;
    s_vc = exp(2.0 * kLn10 * la + (gc - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
           (12.0 * kPi * kPi * gm1);
    s_pnf = (finite_d(la) && finite_d(gc)) ? 0 : 1;
  }
  __syncthreads();
  double gr_q = 0.0, vr_q = 0.0;
  if (phi_thr) {
    const int q = q_phi;
    const double lsr = prm(a, 4 * q, s), lgr = prm(a, 4 * q + 1, s);
    const double ef = prm(a, 4 * q + 2, s), leq = prm(a, 4 * q + 3, s);
    if (!(finite_d(lsr) && finite_d(lgr) && finite_d(ef) && finite_d(leq)))
      atomicOr(&s_pnf, 1);
    gr_q = exp10(lgr);
    const double sr = exp10(lsr), eq = exp10(leq);
    vr_q = sr * sr / (2.0 * gr_q);
    s_vr[q] = vr_q;
    s_gr[q] = gr_q;
    s_ef2[q] = ef * ef;
    s_eq2[q] = eq * eq;
    if (a.N > 0) {
      const double em = expm1(-gr_q * a.rec[0].dt);
      s_phr[0][q] = 1.0 + em;
      s_qr[0][q] = vr_q * (-em * (2.0 + em));
    }
  }
  __syncthreads();
  const double vc = s_vc;
  const double gvc = owner ? a.hd[ba * P + bb] * vc : 0.0;  // G_ab v_c
  // covariance block P[i][j] = Cov(state i of pulsar ba, state j of pulsar bb)
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
  double quad = 0.0, lm = 1.0;
  int le = 0, st = s_pnf ? kPNF : 0;

  const RecPtr rec = (RecPtr)a.rec;
  for (int64_t k = 0; k < a.N; ++k) {
    const int buf = (int)(k & 1);
    const TOARec r = load_rec(rec, k);
    const int p = r.psr;
    const double dt = r.dt, phc = r.phc;
    if (owner) {
      const double pa = s_phr[buf][ba], pb = s_phr[buf][bb];
      // rows: F_a B
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        B[0][j] = fma(dt, B[1][j], B[0][j]);
        B[2][j] *= pa;
        B[3][j] *= phc;
      }
      // columns: (F_a B) F_b^T
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        B[i][0] = fma(dt, B[i][1], B[i][0]);
        B[i][2] *= pb;
        B[i][3] *= phc;
      }
      B[3][3] = fma(gvc, r.qcu, B[3][3]);
      if (diag) {
        B[0][0] += ss2 * r.h3;
        B[0][1] += ss2 * r.h2;
        B[1][0] += ss2 * r.h2;
        B[1][1] += ss2 * dt;
        B[2][2] += s_qr[buf][ba];
        x[0] = fma(dt, x[1], x[0]);
        x[2] *= pa;
        x[3] *= phc;
        if (ba == p) s_e[buf] = r.y - (x[0] + x[2] + x[3]);
      }
      // u = P H^T for the pulsar paired with p in this block
      if (bb == p) {
#pragma unroll
        for (int i = 0; i < 4; ++i) s_u[buf][4 * ba + i] = B[i][0] + B[i][2] + B[i][3];
      } else if (ba == p) {
#pragma unroll
        for (int j = 0; j < 4; ++j) s_u[buf][4 * bb + j] = B[0][j] + B[2][j] + B[3][j];
      }
    }
    if (phi_thr && k + 1 < a.N) {
      const double em = expm1(-gr_q * rec[k + 1].dt);
      s_phr[buf ^ 1][q_phi] = 1.0 + em;
      s_qr[buf ^ 1][q_phi] = vr_q * (-em * (2.0 + em));
    }
    __syncthreads();
    const double* u = s_u[buf];
    const double S =
        (u[4 * p] + u[4 * p + 2] + u[4 * p + 3]) + fma(s_ef2[p], r.s2, s_eq2[p]);
    const double inv = rcp_nr(S);
    const double e = s_e[buf];
    if (owner) {
      double ua[4], ub[4], ka[4], kb[4], wa[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ua[i] = u[4 * ba + i];
        ub[i] = u[4 * bb + i];
        ka[i] = ua[i] * inv;
        kb[i] = ub[i] * inv;
        wa[i] = S * ka[i];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
          B[i][j] = fma(wa[i], kb[j], fma(-ua[i], kb[j], fma(-ka[i], ub[j], B[i][j])));
      if (diag) {
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = fma(ka[i], e, x[i]);
      }
    }
    if (tid == 0) {
      if (st == 0) {
        if (!finite_d(S) || !finite_d(e))
          st = kNonFinite;
        else if (!(S > 0.0))
          st = kNonPD;
      }
      quad = fma(e * e, inv, quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    }
  }
  if (tid == 0) {
    if (st & kPNF) st = kNonFinite;
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
