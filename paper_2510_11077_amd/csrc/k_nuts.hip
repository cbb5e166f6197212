// No-U-Turn Sampler transitions of S independent chains on the gradient
// path (paper: Functionality, "Sampler Integration"; its posteriors come
// from NUTS, Hoffman & Gelman 2014): multinomial trajectory sampling and the
// generalised no-U-turn criterion (Betancourt 2017).
//
// Definition (per chain; H = -logL + p^T M^-1 p / 2, M^-1 = diag(m_inv)):
// the trajectory starts as the current point; doubling j draws a direction
// v = dirs[j] and grows a subtree of 2^j leapfrog leaves from the trajectory
// end on that side. A leaf has log weight -H and diverges when
// H - H0 > 1000, H is not a number, its position leaves the prior box or its
// likelihood fails. Inside a subtree, two halves A, B (build order) merge to
// W = logaddexp(W_A, W_B), take B's proposal when u < exp(W_B - W) (u the
// merge's uniform, merges numbered in post-order within the subtree), sum
// their momenta to rho, and make a U-turn unless (m_inv p_first) . rho > 0
// and (m_inv p_last) . rho > 0; a U-turn or divergence ends the transition
// with the subtree discarded. A valid subtree's proposal replaces the
// trajectory's when u_top[j] < exp(W_sub - W_traj); the trajectory then
// ends on a U-turn between its two ends or after max_depth doublings.
//
// GPU form: the recursion is unrolled into a lockstep loop over leaves. All
// chains take their leapfrog step together (one batched gradient evaluation
// per leaf); a chain that has stopped keeps its position and its gradient
// result is ignored. Within a subtree the halves are merged as in a binary
// counter: after leaf i the stack holds popcount(i + 1) complete subtrees,
// and every trailing one bit of i + 1 is one merge, which is exactly the
// post-order of the recursive build. Each stack entry keeps its log weight,
// momentum sum, first-leaf momentum and proposal (position, gradient,
// logL). Kernels run one wave per chain, lanes over parameters; the host
// reads back the number of chains still building after every 8th leaf of a
// subtree and at its end, and stops the subtree once none is left.
#include <cmath>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

constexpr double kDivergence = 1000.0;

struct NutsArgs {
  int64_t S;
  int32_t D, MD, USZ;
  const double* eps;     // [S]
  const double* m_inv;   // [D]
  const double* lo;      // [D]
  const double* hi;      // [D]
  const double* z;       // [S*D]
  const int32_t* dirs;   // [S*MD]
  const double* u_top;   // [S*MD]
  const double* u_sub;   // [S*MD*USZ]
  double* theta;         // [S*D] in/out
  double* logl;          // [S]
  double* grad;          // [S*D]
  int32_t* depth;        // [S] out
  int32_t* nlf;          // [S] out
  int32_t* divergent;    // [S] out
  double* accept_stat;   // [S] out or null
  // workspace
  double *tl_x, *tl_p, *tl_g, *tr_x, *tr_p, *tr_g;  // trajectory ends [S*D]
  double *pr_x, *pr_g, *pr_l;                        // trajectory proposal
  double *t_rho, *t_w, *h0, *acc;                    // [S*D], [S], [S], [S]
  double *cx, *cp, *cg, *cl;                         // cursor leaf [S*D] x3, [S]
  double *s_w, *s_rho, *s_pf, *s_px, *s_pg, *s_pl;   // stack [S*MD(*D)]
  int32_t *done, *sub_ok, *sub_div, *inbox, *active;  // [S] flags; active: counter
  int32_t j, i;                                      // doubling, leaf index
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ bool finite_d(double v) {
  return __builtin_amdgcn_class(v, 0x1F8);
}

__device__ __forceinline__ double logaddexp(double a, double b) {
  const double m = a > b ? a : b;
  if (m == -INFINITY) return -INFINITY;
  return m + log1p(exp(-fabs(a - b)));
}

#define CHAIN_PROLOGUE                                                           \
  const int lane = threadIdx.x & (kWave - 1);                                    \
  const int64_t s = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; \
  if (s >= a.S) return;                                                          \
  const int64_t b = s * a.D;

__global__ void __launch_bounds__(256) k_nuts_begin(NutsArgs a) {
  CHAIN_PROLOGUE
  double kin = 0.0;
  for (int j = lane; j < a.D; j += kWave) {
    const double mi = a.m_inv[j];
    const double p = a.z[b + j] / sqrt(mi);
    kin = fma(mi * p, p, kin);
    const double x = a.theta[b + j], g = a.grad[b + j];
    a.tl_x[b + j] = a.tr_x[b + j] = a.pr_x[b + j] = a.cx[b + j] = x;
    a.tl_p[b + j] = a.tr_p[b + j] = a.t_rho[b + j] = p;
    a.tl_g[b + j] = a.tr_g[b + j] = a.pr_g[b + j] = g;
  }
  kin = wave_sum(kin);
  if (lane == 0) {
    const double h0 = 0.5 * kin - a.logl[s];
    a.h0[s] = h0;
    a.t_w[s] = -h0;
    a.pr_l[s] = a.logl[s];
    a.acc[s] = 0.0;
    a.done[s] = 0;
    a.depth[s] = 0;
    a.nlf[s] = 0;
    a.divergent[s] = 0;
  }
}

// start of doubling j: the cursor takes the trajectory end on side v
__global__ void __launch_bounds__(256) k_nuts_sub_begin(NutsArgs a) {
  CHAIN_PROLOGUE
  if (a.done[s]) return;
  const bool right = a.dirs[s * a.MD + a.j] > 0;
  const double* ex = right ? a.tr_x : a.tl_x;
  const double* ep = right ? a.tr_p : a.tl_p;
  const double* eg = right ? a.tr_g : a.tl_g;
  for (int j = lane; j < a.D; j += kWave) {
    a.cx[b + j] = ex[b + j];
    a.cp[b + j] = ep[b + j];
    a.cg[b + j] = eg[b + j];
  }
  if (lane == 0) {
    a.sub_ok[s] = 1;
    a.sub_div[s] = 0;
  }
}

// first half kick and drift of the next leaf
__global__ void __launch_bounds__(256) k_nuts_drift(NutsArgs a) {
  CHAIN_PROLOGUE
  if (a.done[s] || !a.sub_ok[s]) return;
  const double e = a.eps[s] * (double)a.dirs[s * a.MD + a.j];
  bool in = true;
  for (int j = lane; j < a.D; j += kWave) {
    const double p = fma(0.5 * e, a.cg[b + j], a.cp[b + j]);
    const double x = fma(e * a.m_inv[j], p, a.cx[b + j]);
    in = in && x >= a.lo[j] && x <= a.hi[j];
    a.cp[b + j] = p;
    a.cx[b + j] = x;
  }
  const bool all_in = __all(in);
  if (lane == 0) a.inbox[s] = all_in ? 1 : 0;
}

// second half kick, the leaf's energy, push and merges; counts the chains
// still building this subtree
__global__ void __launch_bounds__(256) k_nuts_leaf(NutsArgs a) {
  CHAIN_PROLOGUE
  if (a.done[s] || !a.sub_ok[s]) return;
  const double e = a.eps[s] * (double)a.dirs[s * a.MD + a.j];
  double kin = 0.0;
  for (int j = lane; j < a.D; j += kWave) {
    const double p = fma(0.5 * e, a.cg[b + j], a.cp[b + j]);
    a.cp[b + j] = p;
    kin = fma(a.m_inv[j] * p, p, kin);
  }
  kin = wave_sum(kin);
  const double l = a.cl[s];
  const bool ok = a.inbox[s] != 0 && finite_d(l);
  const double h = ok ? 0.5 * kin - l : INFINITY;
  const double h0 = a.h0[s];
  const bool div = !(h - h0 <= kDivergence);
  if (lane == 0) {
    a.nlf[s] += 1;
    a.acc[s] += finite_d(h) ? fmin(1.0, exp(h0 - h)) : 0.0;
  }
  if (div) {
    if (lane == 0) {
      a.sub_ok[s] = 0;
      a.sub_div[s] = 1;
    }
    return;
  }
  // push the leaf at position popcount(i)
  const int i = a.i;
  int pos = __builtin_popcount((unsigned)i);
  const int64_t base = s * a.MD;
  {
    const int64_t o = (base + pos) * a.D;
    for (int j = lane; j < a.D; j += kWave) {
      const double p = a.cp[b + j];
      a.s_rho[o + j] = p;
      a.s_pf[o + j] = p;
      a.s_px[o + j] = a.cx[b + j];
      a.s_pg[o + j] = a.cg[b + j];
    }
    if (lane == 0) {
      a.s_w[base + pos] = -h;
      a.s_pl[base + pos] = l;
    }
  }
  // carries of i + 1: merge the top two entries, post-order index m. The
  // newer entry's weight and proposal logL stay in registers (every lane
  // holds them), so no lane reads a scalar another lane has just stored.
  int m = i - __builtin_popcount((unsigned)i);
  bool valid = true;
  double wb = -h, lb = l;
  for (unsigned c = (unsigned)i + 1; (c & 1u) == 0 && valid; c >>= 1, ++m, --pos) {
    const int64_t oa = (base + pos - 1) * a.D, ob = (base + pos) * a.D;
    const double wa = a.s_w[base + pos - 1];
    const double w = logaddexp(wa, wb);
    const double u = a.u_sub[((int64_t)s * a.MD + a.j) * a.USZ + m];
    const bool take_b = u < exp(wb - w);
    const double lm = take_b ? lb : a.s_pl[base + pos - 1];
    double d1 = 0.0, d2 = 0.0;
    for (int j = lane; j < a.D; j += kWave) {
      const double rho = a.s_rho[oa + j] + a.s_rho[ob + j];
      a.s_rho[oa + j] = rho;
      if (take_b) {
        a.s_px[oa + j] = a.s_px[ob + j];
        a.s_pg[oa + j] = a.s_pg[ob + j];
      }
      const double mi = a.m_inv[j];
      d1 = fma(mi * a.s_pf[oa + j], rho, d1);
      d2 = fma(mi * a.cp[b + j], rho, d2);
    }
    d1 = wave_sum(d1);
    d2 = wave_sum(d2);
    if (lane == 0) {
      a.s_w[base + pos - 1] = w;
      a.s_pl[base + pos - 1] = lm;
    }
    wb = w;
    lb = lm;
    valid = d1 > 0.0 && d2 > 0.0;
  }
  if (lane == 0) {
    if (!valid)
      a.sub_ok[s] = 0;
    else
      atomicAdd(a.active, 1);
  }
}

// end of doubling j: accept the subtree into the trajectory or stop
__global__ void __launch_bounds__(256) k_nuts_top(NutsArgs a) {
  CHAIN_PROLOGUE
  if (a.done[s]) return;
  if (!a.sub_ok[s]) {
    if (lane == 0) {
      a.done[s] = 1;
      a.divergent[s] = a.sub_div[s];
    }
    return;
  }
  const int64_t o = (s * a.MD) * a.D;  // the whole subtree is stack entry 0
  const double ws = a.s_w[s * a.MD], wt = a.t_w[s];
  const bool take = a.u_top[s * a.MD + a.j] < exp(ws - wt);
  const bool right = a.dirs[s * a.MD + a.j] > 0;
  double* ex = right ? a.tr_x : a.tl_x;
  double* ep = right ? a.tr_p : a.tl_p;
  double* eg = right ? a.tr_g : a.tl_g;
  double d1 = 0.0, d2 = 0.0;
  for (int j = lane; j < a.D; j += kWave) {
    if (take) {
      a.pr_x[b + j] = a.s_px[o + j];
      a.pr_g[b + j] = a.s_pg[o + j];
    }
    const double rho = a.t_rho[b + j] + a.s_rho[o + j];
    a.t_rho[b + j] = rho;
    ex[b + j] = a.cx[b + j];
    ep[b + j] = a.cp[b + j];
    eg[b + j] = a.cg[b + j];
    const double mi = a.m_inv[j];
    d1 = fma(mi * a.tl_p[b + j], rho, d1);
    d2 = fma(mi * a.tr_p[b + j], rho, d2);
  }
  d1 = wave_sum(d1);
  d2 = wave_sum(d2);
  if (lane == 0) {
    if (take) a.pr_l[s] = a.s_pl[s * a.MD];
    a.t_w[s] = logaddexp(wt, ws);
    a.depth[s] = a.j + 1;
    const bool stop = !(d1 > 0.0 && d2 > 0.0) || a.j + 1 >= a.MD;
    if (stop)
      a.done[s] = 1;
    else
      atomicAdd(a.active, 1);
  }
}

__global__ void __launch_bounds__(256) k_nuts_end(NutsArgs a) {
  CHAIN_PROLOGUE
  for (int j = lane; j < a.D; j += kWave) {
    a.theta[b + j] = a.pr_x[b + j];
    a.grad[b + j] = a.pr_g[b + j];
  }
  if (lane == 0) {
    a.logl[s] = a.pr_l[s];
    if (a.accept_stat) a.accept_stat[s] = a.acc[s] / (double)(a.nlf[s] > 0 ? a.nlf[s] : 1);
  }
}

__global__ void k_zero_int(int32_t* p) { *p = 0; }

}  // namespace

int nuts_step(argus_dataset* ds, int64_t S, int32_t max_depth, const double* eps,
              const double* m_inv, const double* lo, const double* hi, const double* z,
              const int32_t* dirs, const double* u_top, const double* u_sub, double* theta,
              double* logl, double* grad, int32_t* depth, int32_t* n_leapfrog,
              int32_t* divergent, double* accept_stat, hipStream_t st) {
  int rc = ARGUS_OK;
  Workspace* w = get_workspace(ds, S, &rc);
  if (!w) return rc;
  const int64_t D = ds->D, MD = max_depth;
  const int64_t sd = S * D;
  // doubles: 6 trajectory ends + 2 proposal + rho + 3 cursor vectors, 4
  // stack vectors per level; scalars: pr_l, t_w, h0, acc, cl, s_w, s_pl
  const size_t nd = (size_t)(12 * sd + 4 * sd * MD + 5 * S + 2 * S * MD);
  const size_t ni = (size_t)(5 * S + 64);
  if (w->nuts_md < max_depth) {
    if ((rc = w->nuts_f.alloc(nd * sizeof(double))) || (rc = w->nuts_i.alloc(ni * sizeof(int32_t))))
      return rc;
    w->nuts_md = max_depth;
  }
  NutsArgs a{};
  a.S = S;
  a.D = (int32_t)D;
  a.MD = max_depth;
  a.USZ = max_depth > 1 ? 1 << (max_depth - 1) : 1;
  a.eps = eps;
  a.m_inv = m_inv;
  a.lo = lo;
  a.hi = hi;
  a.z = z;
  a.dirs = dirs;
  a.u_top = u_top;
  a.u_sub = u_sub;
  a.theta = theta;
  a.logl = logl;
  a.grad = grad;
  a.depth = depth;
  a.nlf = n_leapfrog;
  a.divergent = divergent;
  a.accept_stat = accept_stat;
  double* f = w->nuts_f.as<double>();
  auto take = [&](int64_t n) {
    double* p = f;
    f += n;
    return p;
  };
  a.tl_x = take(sd);
  a.tl_p = take(sd);
  a.tl_g = take(sd);
  a.tr_x = take(sd);
  a.tr_p = take(sd);
  a.tr_g = take(sd);
  a.pr_x = take(sd);
  a.pr_g = take(sd);
  a.t_rho = take(sd);
  a.cx = take(sd);
  a.cp = take(sd);
  a.cg = take(sd);
  a.s_rho = take(sd * MD);
  a.s_pf = take(sd * MD);
  a.s_px = take(sd * MD);
  a.s_pg = take(sd * MD);
  a.pr_l = take(S);
  a.t_w = take(S);
  a.h0 = take(S);
  a.acc = take(S);
  a.cl = take(S);
  a.s_w = take(S * MD);
  a.s_pl = take(S * MD);
  int32_t* ip = w->nuts_i.as<int32_t>();
  a.done = ip;
  a.sub_ok = ip + S;
  a.sub_div = ip + 2 * S;
  a.inbox = ip + 3 * S;
  a.active = ip + 4 * S;
  const dim3 grid((unsigned)((S + 3) / 4)), block(256);
  hipLaunchKernelGGL(k_nuts_begin, grid, block, 0, st, a);
  HIPCHK(hipGetLastError());
  int32_t n_active = 0;
  for (int32_t j = 0; j < max_depth; ++j) {
    a.j = j;
    hipLaunchKernelGGL(k_nuts_sub_begin, grid, block, 0, st, a);
    HIPCHK(hipGetLastError());
    const int64_t leaves = (int64_t)1 << j;
    for (int64_t i = 0; i < leaves; ++i) {
      a.i = (int32_t)i;
      hipLaunchKernelGGL(k_nuts_drift, grid, block, 0, st, a);
      HIPCHK(hipGetLastError());
      if ((rc = grad_loglike(ds, a.cx, S, a.cl, a.cg, nullptr, st))) return rc;
      hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, a.active);
      hipLaunchKernelGGL(k_nuts_leaf, grid, block, 0, st, a);
      HIPCHK(hipGetLastError());
      // the count is read back after every 8th leaf and at the subtree's
      // end only: a read-back stalls the host until the stream drains, and
      // the leaves a stopped chain is carried through change nothing for it
      if (i == leaves - 1 || ((i + 1) & 7) == 0) {
        HIPCHK(hipMemcpyAsync(&n_active, a.active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (n_active == 0) break;
      }
    }
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(1), 0, st, a.active);
    hipLaunchKernelGGL(k_nuts_top, grid, block, 0, st, a);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(&n_active, a.active, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (n_active == 0) break;
  }
  hipLaunchKernelGGL(k_nuts_end, grid, block, 0, st, a);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

}  // namespace argus
