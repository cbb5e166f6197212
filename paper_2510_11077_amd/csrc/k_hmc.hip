// Hamiltonian Monte Carlo transitions of S independent chains on the
// gradient path (paper: Functionality, "Sampler Integration": the
// likelihood and its gradient feed gradient-based samplers such as HMC).
// Per chain (Duane et al. 1987; Neal 2011), with the momentum drawn from
// N(0, M), M = diag(1 / m_inv), from standard normal draws z:
//   p = z / sqrt(m_inv),  H0 = -logL(theta) + 1/2 sum m_inv p^2,
//   n_leapfrog times: p += eps/2 g; x += eps m_inv p; (logL, g) at x;
//                     p += eps/2 g,
//   H1 = -logL(x) + 1/2 sum m_inv p^2, accepted when log u < H0 - H1.
// The prior is uniform on the box [lo, hi]: a trajectory that leaves it, or
// whose likelihood fails, at any leapfrog position is rejected. The
// gradient evaluations are the library's batched gradient sweep; the
// kernels here are the elementwise leapfrog updates, one wave per chain
// (lanes over parameters, energies reduced across the wave).
#include <cmath>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

struct HmcArgs {
  int64_t S;
  int32_t D;
  const double* eps;    // [S]
  const double* m_inv;  // [D]
  const double* lo;     // [D]
  const double* hi;     // [D]
  const double* z;      // [S*D]
  const double* logu;   // [S]
  double* theta;        // [S*D] current positions (in/out)
  double* logl;         // [S]   logL at theta (in/out)
  double* grad;         // [S*D] gradient at theta (in/out)
  int32_t* accepted;    // [S]   incremented on acceptance
  double* dh;           // [S]   H1 - H0, or null
  double* x;            // [S*D] proposal position
  double* p;            // [S*D] momentum
  double* g;            // [S*D] gradient at x
  const double* l;      // [S]   logL at x
  double* h0;           // [S]
  int32_t* ok;          // [S]   inside the box with a finite logL so far
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ bool finite_d(double v) {
  return __builtin_amdgcn_class(v, 0x1F8);
}

// momentum from z, H0, the first half kick and drift
__global__ void __launch_bounds__(256) k_hmc_begin(HmcArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t s = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (s >= a.S) return;
  const double e = a.eps[s];
  double kin = 0.0;
  bool in = true;
  for (int j = lane; j < a.D; j += kWave) {
    const int64_t i = s * a.D + j;
    const double mi = a.m_inv[j];
    double p = a.z[i] / sqrt(mi);
    kin = fma(mi * p, p, kin);
    p = fma(0.5 * e, a.grad[i], p);
    const double x = fma(e * mi, p, a.theta[i]);
    in = in && x >= a.lo[j] && x <= a.hi[j];
    a.p[i] = p;
    a.x[i] = x;
  }
  kin = wave_sum(kin);
  const bool all_in = __all(in);
  if (lane == 0) {
    a.h0[s] = 0.5 * kin - a.logl[s];
    a.ok[s] = all_in ? 1 : 0;
  }
}

// after the gradient at x: the closing half kick, and for a middle step the
// next half kick and drift
__global__ void __launch_bounds__(256) k_hmc_mid(HmcArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t s = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (s >= a.S) return;
  const double e = a.eps[s];
  bool in = true;
  for (int j = lane; j < a.D; j += kWave) {
    const int64_t i = s * a.D + j;
    const double gi = a.g[i];
    double p = fma(0.5 * e, gi, a.p[i]);
    p = fma(0.5 * e, gi, p);
    const double x = fma(e * a.m_inv[j], p, a.x[i]);
    in = in && x >= a.lo[j] && x <= a.hi[j];
    a.p[i] = p;
    a.x[i] = x;
  }
  const bool all_in = __all(in);
  if (lane == 0 && !(all_in && finite_d(a.l[s]))) a.ok[s] = 0;
}

// closing half kick, H1, the accept test and the copy of accepted states
__global__ void __launch_bounds__(256) k_hmc_end(HmcArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int64_t s = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  if (s >= a.S) return;
  const double e = a.eps[s];
  double kin = 0.0;
  for (int j = lane; j < a.D; j += kWave) {
    const int64_t i = s * a.D + j;
    const double p = fma(0.5 * e, a.g[i], a.p[i]);
    kin = fma(a.m_inv[j] * p, p, kin);
  }
  kin = wave_sum(kin);
  const double l1 = a.l[s];
  const bool ok = a.ok[s] != 0 && finite_d(l1);
  const double h1 = ok ? 0.5 * kin - l1 : INFINITY;
  const double dh = h1 - a.h0[s];
  const bool acc = a.logu[s] < -dh;  // a NaN dH rejects
  if (acc) {
    for (int j = lane; j < a.D; j += kWave) {
      const int64_t i = s * a.D + j;
      a.theta[i] = a.x[i];
      a.grad[i] = a.g[i];
    }
  }
  if (lane == 0) {
    if (acc) {
      a.logl[s] = l1;
      a.accepted[s] += 1;
    }
    if (a.dh) a.dh[s] = dh;
  }
}

}  // namespace

int hmc_step(argus_dataset* ds, int64_t S, int32_t n_leapfrog, const double* eps,
             const double* m_inv, const double* lo, const double* hi, const double* z,
             const double* logu, double* theta, double* logl, double* grad,
             int32_t* accepted, double* dh, hipStream_t st) {
  int rc = ARGUS_OK;
  Workspace* w = get_workspace(ds, S, &rc);
  if (!w) return rc;
  const size_t sd = (size_t)S * ds->D;
  if (w->hmc_x.p == nullptr) {
    if ((rc = w->hmc_x.alloc(sd * sizeof(double))) || (rc = w->hmc_p.alloc(sd * sizeof(double))) ||
        (rc = w->hmc_g.alloc(sd * sizeof(double))) ||
        (rc = w->hmc_l.alloc((size_t)S * sizeof(double))) ||
        (rc = w->hmc_h0.alloc((size_t)S * sizeof(double))) ||
        (rc = w->hmc_ok.alloc((size_t)S * sizeof(int32_t))))
      return rc;
  }
  HmcArgs a{};
  a.S = S;
  a.D = ds->D;
  a.eps = eps;
  a.m_inv = m_inv;
  a.lo = lo;
  a.hi = hi;
  a.z = z;
  a.logu = logu;
  a.theta = theta;
  a.logl = logl;
  a.grad = grad;
  a.accepted = accepted;
  a.dh = dh;
  a.x = w->hmc_x.as<double>();
  a.p = w->hmc_p.as<double>();
  a.g = w->hmc_g.as<double>();
  a.l = w->hmc_l.as<double>();
  a.h0 = w->hmc_h0.as<double>();
  a.ok = w->hmc_ok.as<int32_t>();
  const dim3 grid((unsigned)((S + 3) / 4)), block(256);
  hipLaunchKernelGGL(k_hmc_begin, grid, block, 0, st, a);
  HIPCHK(hipGetLastError());
  for (int32_t k = 0; k < n_leapfrog; ++k) {
    if ((rc = grad_loglike(ds, a.x, S, w->hmc_l.as<double>(), a.g, nullptr, st))) return rc;
    if (k + 1 < n_leapfrog)
      hipLaunchKernelGGL(k_hmc_mid, grid, block, 0, st, a);
    else
      hipLaunchKernelGGL(k_hmc_end, grid, block, 0, st, a);
    HIPCHK(hipGetLastError());
  }
  return ARGUS_OK;
}

}  // namespace argus
