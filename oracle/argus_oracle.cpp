// Reference CPU implementation of the state-space PTA log-likelihood.
//
// TEST INFRASTRUCTURE ONLY. This file is the oracle that the GPU library is
// checked against. Only tests, the smoke check and the CPU-baseline leg of the
// benchmark may load it; the product path never does. It shares no code,
// header or table with the HIP library.
//
// What it computes (paper: Summary; Statement of Need; Functionality, items
// "State-space model construction" and "Kalman filter likelihood evaluation"):
// each noise process is a linear SDE; the processes are stacked into one
// linear-Gaussian state-space model; the Kalman filter (Kalman 1960) evaluates
// the likelihood of the timing residuals by the prediction-error decomposition
//     log L = sum_k -1/2 (ln 2 pi + ln S_k + e_k^2 / S_k).
// The paper prints no equations, so the concrete model is the reading written
// out in the design notes (spin random walk, OU red noise, OU common process
// with Hellings-Downs coupling, EFAC/EQUAD white noise). The code follows the
// textbook recursion literally: dense F, Q, H; the covariance update in Joseph
// form with the matrix (I - K H) formed explicitly; symmetrisation afterwards.
// No structure is exploited, by design. The latent-state posteriors (the
// filter tracking the realised noise; paper: Summary, Statement of Need) come
// from the textbook Rauch-Tung-Striebel recursion on the filtered and
// predicted moments.
//
// Everything is templated on the scalar type so that the same recursion runs
// in complex arithmetic for complex-step derivatives (Squire & Trapp 1998).
//
// Parity unpinned: whether these model readings are the ones the paper's
// software uses (the paper states no equations). All arithmetic below is
// pinned by tests against the dense Gaussian likelihood, closed-form
// discretisations, Hellings-Downs quadrature and filter invariants; the
// smoother against Gaussian conditioning on the dense covariance (40-digit
// and fp64) and the white-noise posterior identity.

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

using cd = std::complex<double>;

constexpr double kPi = 3.14159265358979323846;
constexpr double kLn10 = 2.30258509299404568402;
constexpr double kYear = 31557600.0;  // Julian year, seconds

enum { M_SPIN = 1, M_PSR4 = 2, M_JOINT = 3, M_DM = 4 };
constexpr double kNuRef = 1400.0;  // MHz: the DM state is the delay at this frequency
enum { S_NONPD = 1, S_NONFINITE = 2 };

// ---------------------------------------------------------------- scalars
inline double re(double x) { return x; }
inline double re(const cd& z) { return z.real(); }

// 10^x, written so that the complex version is analytic and its real part is
// the double version.
inline double p10(double x) { return std::pow(10.0, x); }
inline cd p10(const cd& z) {
  double r = std::pow(10.0, z.real());
  double a = z.imag() * kLn10;
  return cd(r * std::cos(a), r * std::sin(a));
}
inline double xexp(double x) { return std::exp(x); }
inline cd xexp(const cd& z) { return std::exp(z); }
inline double xlog(double x) { return std::log(x); }
inline cd xlog(const cd& z) { return std::log(z); }
// exp(z) - 1 without cancellation; complex version from
// exp(x+iy) - 1 = (expm1(x) cos y - 2 sin^2(y/2)) + i exp(x) sin y.
inline double xexpm1(double x) { return std::expm1(x); }
inline cd xexpm1(const cd& z) {
  double x = z.real(), y = z.imag();
  double s = std::sin(0.5 * y);
  return cd(std::expm1(x) * std::cos(y) - 2.0 * s * s, std::exp(x) * std::sin(y));
}

// ------------------------------------------------------------ dataset view
struct DS {
  int model = 0;
  int P = 0;
  const int64_t* off = nullptr;
  const double* t = nullptr;
  const double* y = nullptr;
  const double* sig = nullptr;
  const double* pos = nullptr;
  const double* freq = nullptr;  // MHz per TOA (model 4)
  double t_span = 0, s_r = 0, s_f = 0, sigma_s = 0;
  // merged, time-ordered stream (joint model only)
  std::vector<int64_t> m_idx;  // global TOA index
  std::vector<int> m_psr;      // pulsar of each merged TOA
  std::vector<double> hd;      // P x P Hellings-Downs matrix
};

// canonical parameters per pulsar, and the state dimension of one filter
int per_psr(const DS& d) { return d.model == M_DM ? 6 : 4; }
int n_canon(const DS& d) { return d.model == M_SPIN ? 2 : per_psr(d) * d.P + 2; }
int state_dim(const DS& d) {
  switch (d.model) {
    case M_SPIN: return 2;
    case M_PSR4: return 4;
    case M_DM: return 5;
    default: return 4 * d.P;
  }
}

// Hellings & Downs (1983) overlap reduction, earth term plus the pulsar term
// on the diagonal: G_ab = 3/2 x ln x - x/4 + 1/2 + delta_ab/2,
// x = (1 - cos zeta_ab)/2, with x ln x = 0 at x = 0.
void hd_matrix(const double* pos, int P, double* G) {
  for (int a = 0; a < P; ++a)
    for (int b = 0; b < P; ++b) {
      double c = pos[3 * a] * pos[3 * b] + pos[3 * a + 1] * pos[3 * b + 1] +
                 pos[3 * a + 2] * pos[3 * b + 2];
      // a pulsar's separation from itself is exactly zero
      double x = a == b ? 0.0 : 0.5 * (1.0 - c);
      if (x < 0) x = 0;
      double xl = x > 0 ? x * std::log(x) : 0.0;
      G[a * P + b] = 1.5 * xl - 0.25 * x + 0.5 + (a == b ? 0.5 : 0.0);
    }
}

// Stationary variance of a one-state OU common process whose variance equals
// that of the power-law residual spectrum
//   PSD(f) = A^2 / (12 pi^2) f_yr^(gamma-3) f^(-gamma)
// integrated from f_low = 1/T_span to infinity.
template <class T>
T common_variance(const T& log10A, const T& gam, double t_span) {
  const double fyr = 1.0 / kYear;
  T A = p10(log10A);
  return A * A * xexp((gam - 3.0) * std::log(fyr)) *
         xexp((gam - 1.0) * std::log(t_span)) /
         (12.0 * kPi * kPi * (gam - 1.0));
}

// --------------------------------------------------------- model parameters
template <class T>
struct Psr {
  T vr, gr, efac2, equad2;
  T vd, gd;  // DM OU variance and rate (model 4)
};
template <class T>
struct Par {
  T ss2;  // spin random-walk diffusion, sigma_s^2
  T vc;   // common OU stationary variance
  double lam;  // common OU rate 2 pi / T_span
  std::vector<Psr<T>> psr;
};

template <class T>
Par<T> make_par(const DS& d, const T* c) {
  Par<T> p;
  p.lam = 2.0 * kPi / d.t_span;
  if (d.model == M_SPIN) {
    T ss = p10(c[0]);
    p.ss2 = ss * ss;
    p.vc = T(0.0);
    p.psr.resize(1);
    p.psr[0] = {T(0.0), T(1.0), c[1] * c[1], T(0.0), T(0.0), T(1.0)};
    return p;
  }
  const int k = per_psr(d);
  p.ss2 = T(d.sigma_s * d.sigma_s);
  p.vc = common_variance(c[k * d.P], c[k * d.P + 1], d.t_span);
  p.psr.resize(d.P);
  for (int q = 0; q < d.P; ++q) {
    const T* cq = c + k * q;
    T sr = p10(cq[0]);
    T gr = p10(cq[1]);
    T eq = p10(cq[3]);
    p.psr[q] = {sr * sr / (2.0 * gr), gr, cq[2] * cq[2], eq * eq, T(0.0), T(1.0)};
    if (d.model == M_DM) {
      T sd = p10(cq[4]);
      T gd = p10(cq[5]);
      p.psr[q].vd = sd * sd / (2.0 * gd);
      p.psr[q].gd = gd;
    }
  }
  return p;
}

// ------------------------------------------------------------ dense algebra
template <class T>
void mm(int n, const T* A, const T* B, T* C) {  // C = A B
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T s = T(0.0);
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[k * n + j];
      C[i * n + j] = s;
    }
}
template <class T>
void mmt(int n, const T* A, const T* B, T* C) {  // C = A B^T
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      T s = T(0.0);
      for (int k = 0; k < n; ++k) s += A[i * n + k] * B[j * n + k];
      C[i * n + j] = s;
    }
}

// Transition and process noise of one pulsar's 4-block [r, f, a, g] (or the
// 2-block [r, f] of the spin-only model) over an interval dt, written into the
// n x n matrices F, Q at offset o. Closed forms of Van Loan (1978):
//   spin (dr = f dt, df = sigma_s dW): F = [[1,dt],[0,1]],
//        Q = sigma_s^2 [[dt^3/3, dt^2/2],[dt^2/2, dt]];
//   OU (dz = -g z dt + s dW, v = s^2/2g): F = e^{-g dt}, Q = v (1 - e^{-2 g dt}).
template <class T>
void block_fq(const DS& d, const Par<T>& p, int q, double dt, int n, int o,
              T* F, T* Q) {
  F[o * n + o] = T(1.0);
  F[o * n + o + 1] = T(dt);
  F[(o + 1) * n + o + 1] = T(1.0);
  Q[o * n + o] = p.ss2 * (dt * dt * dt / 3.0);
  Q[o * n + o + 1] = p.ss2 * (dt * dt / 2.0);
  Q[(o + 1) * n + o] = p.ss2 * (dt * dt / 2.0);
  Q[(o + 1) * n + o + 1] = p.ss2 * dt;
  if (d.model == M_SPIN) return;
  const Psr<T>& s = p.psr[q];
  F[(o + 2) * n + o + 2] = xexp(-s.gr * dt);
  Q[(o + 2) * n + o + 2] = s.vr * (-xexpm1(-2.0 * s.gr * dt));
  F[(o + 3) * n + o + 3] = T(std::exp(-p.lam * dt));
  if (d.model != M_JOINT)
    Q[(o + 3) * n + o + 3] = p.vc * (-std::expm1(-2.0 * p.lam * dt));
  if (d.model == M_DM) {  // DM delay at the reference frequency: OU
    F[(o + 4) * n + o + 4] = xexp(-s.gd * dt);
    Q[(o + 4) * n + o + 4] = s.vd * (-xexpm1(-2.0 * s.gd * dt));
  }
}

// Full F, Q of the filter that processes pulsar q (per-pulsar models) or the
// joint state (joint model).
template <class T>
void model_fq(const DS& d, const Par<T>& p, int q, double dt, int n, T* F,
              T* Q) {
  std::fill(F, F + n * n, T(0.0));
  std::fill(Q, Q + n * n, T(0.0));
  if (d.model != M_JOINT) {
    block_fq(d, p, q, dt, n, 0, F, Q);
    return;
  }
  for (int a = 0; a < d.P; ++a) block_fq(d, p, a, dt, n, 4 * a, F, Q);
  // common process: process-noise cross-covariance G_ab * q_c(dt)
  double qc_unit = -std::expm1(-2.0 * p.lam * dt);
  for (int a = 0; a < d.P; ++a)
    for (int b = 0; b < d.P; ++b)
      Q[(4 * a + 3) * n + 4 * b + 3] = p.vc * (d.hd[a * d.P + b] * qc_unit);
}

template <class T>
void model_p0(const DS& d, const Par<T>& p, int q, int n, T* P0) {
  std::fill(P0, P0 + n * n, T(0.0));
  auto blk = [&](int a, int o) {
    P0[o * n + o] = T(d.s_r * d.s_r);
    P0[(o + 1) * n + o + 1] = T(d.s_f * d.s_f);
    if (d.model == M_SPIN) return;
    P0[(o + 2) * n + o + 2] = p.psr[a].vr;
    if (d.model != M_JOINT) P0[(o + 3) * n + o + 3] = p.vc;
    if (d.model == M_DM) P0[(o + 4) * n + o + 4] = p.psr[a].vd;
  };
  if (d.model != M_JOINT) {
    blk(q, 0);
    return;
  }
  for (int a = 0; a < d.P; ++a) blk(a, 4 * a);
  for (int a = 0; a < d.P; ++a)
    for (int b = 0; b < d.P; ++b)
      P0[(4 * a + 3) * n + 4 * b + 3] = p.vc * d.hd[a * d.P + b];
}

// Optional per-step record (double runs only): predicted x, P, innovation,
// its variance and the filtered x, P after each TOA.
struct Trace {
  double* e = nullptr;      // [N]
  double* S = nullptr;      // [N]
  double* x = nullptr;      // [N*n] filtered
  double* Pf = nullptr;     // [N*n*n] filtered
  double* Pp = nullptr;     // [N*n*n] predicted
  double* xp = nullptr;     // [N*n] predicted (optional)
};

template <class T>
void put(double* dst, const T* src, int m) {
  for (int i = 0; i < m; ++i) dst[i] = re(src[i]);
}

// The Kalman recursion over one time-ordered stream. Returns the
// log-likelihood; on failure returns -inf and sets *status.
// psr_of(k) gives the pulsar of stream element k, idx(k) the TOA index.
template <class T, class IdxF, class PsrF>
T kalman(const DS& d, const Par<T>& p, int q_fixed, int64_t N, IdxF idx,
         PsrF psr_of, int32_t* status, Trace* tr) {
  const int n = state_dim(d);
  std::vector<T> x(n, T(0.0)), xp(n), P(n * n), Pp(n * n), F(n * n), Q(n * n),
      tmp(n * n), A(n * n), H(n), u(n), K(n);
  model_p0(d, p, q_fixed, n, P.data());
  T ll = T(0.0);
  double t_prev = 0.0;  // the prior holds at the dataset epoch t0 = 0
  const double ln2pi = std::log(2.0 * kPi);
  for (int64_t k = 0; k < N; ++k) {
    const int64_t j = idx(k);
    const int q = psr_of(k);
    const double dt = d.t[j] - t_prev;
    t_prev = d.t[j];
    // 1. discretise
    model_fq(d, p, q_fixed, dt, n, F.data(), Q.data());
    // 2. x- = F x
    for (int i = 0; i < n; ++i) {
      T s = T(0.0);
      for (int m = 0; m < n; ++m) s += F[i * n + m] * x[m];
      xp[i] = s;
    }
    // 3. P- = F P F^T + Q
    mm(n, F.data(), P.data(), tmp.data());
    mmt(n, tmp.data(), F.data(), Pp.data());
    for (int i = 0; i < n * n; ++i) Pp[i] += Q[i];
    // measurement row: residual = r + a + g (+ (nu_ref / nu)^2 m) of pulsar q
    std::fill(H.begin(), H.end(), T(0.0));
    const int o = d.model == M_JOINT ? 4 * q : 0;
    H[o] = T(1.0);
    if (d.model != M_SPIN) {
      H[o + 2] = T(1.0);
      H[o + 3] = T(1.0);
    }
    if (d.model == M_DM) {
      const double ck = kNuRef / d.freq[j];
      H[o + 4] = T(ck * ck);
    }
    const Psr<T>& ps = p.psr[d.model == M_JOINT ? q : q_fixed];
    const double sk = d.sig[j];
    T R = ps.efac2 * (sk * sk) + ps.equad2;
    // 4. innovation e = y - H x-
    T hx = T(0.0);
    for (int i = 0; i < n; ++i) hx += H[i] * xp[i];
    T e = d.y[j] - hx;
    // 5. u = P- H^T
    for (int i = 0; i < n; ++i) {
      T s = T(0.0);
      for (int m = 0; m < n; ++m) s += Pp[i * n + m] * H[m];
      u[i] = s;
    }
    // 6. S = H u + R
    T S = R;
    for (int i = 0; i < n; ++i) S += H[i] * u[i];
    if (!std::isfinite(re(S)) || !std::isfinite(re(e))) {
      *status = S_NONFINITE;
      return T(-std::numeric_limits<double>::infinity());
    }
    if (!(re(S) > 0.0)) {
      *status = S_NONPD;
      return T(-std::numeric_limits<double>::infinity());
    }
    // 7. K = u / S ; 8. x = x- + K e
    for (int i = 0; i < n; ++i) {
      K[i] = u[i] / S;
      x[i] = xp[i] + K[i] * e;
    }
    // 9. Joseph form: P = (I - K H) P- (I - K H)^T + K R K^T
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m)
        A[i * n + m] = (i == m ? T(1.0) : T(0.0)) - K[i] * H[m];
    mm(n, A.data(), Pp.data(), tmp.data());
    mmt(n, tmp.data(), A.data(), P.data());
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m) P[i * n + m] += K[i] * R * K[m];
    // 10. symmetrise
    for (int i = 0; i < n; ++i)
      for (int m = i + 1; m < n; ++m) {
        T s = 0.5 * (P[i * n + m] + P[m * n + i]);
        P[i * n + m] = s;
        P[m * n + i] = s;
      }
    // 11. accumulate the prediction-error decomposition
    ll += -0.5 * (ln2pi + xlog(S) + e * e / S);
    if (tr) {
      tr->e[k] = re(e);
      tr->S[k] = re(S);
      put(tr->x + k * n, x.data(), n);
      put(tr->Pf + k * n * n, P.data(), n * n);
      put(tr->Pp + k * n * n, Pp.data(), n * n);
      if (tr->xp) put(tr->xp + k * n, xp.data(), n);
    }
  }
  if (!std::isfinite(re(ll))) {
    *status = S_NONFINITE;
    return T(-std::numeric_limits<double>::infinity());
  }
  return ll;
}

template <class T>
bool finite_params(const T* c, int C) {
  for (int i = 0; i < C; ++i)
    if (!std::isfinite(re(c[i]))) return false;
  return true;
}

// log-likelihood of one pulsar (per-pulsar models)
template <class T>
T psr_loglike(const DS& d, const Par<T>& p, int q, int32_t* st, Trace* tr) {
  const int64_t b = d.off[q], N = d.off[q + 1] - d.off[q];
  return kalman<T>(d, p, q, N, [b](int64_t k) { return b + k; },
                   [q](int64_t) { return q; }, st, tr);
}

template <class T>
T joint_loglike(const DS& d, const Par<T>& p, int32_t* st, Trace* tr) {
  const int64_t N = (int64_t)d.m_idx.size();
  return kalman<T>(d, p, 0, N, [&d](int64_t k) { return d.m_idx[k]; },
                   [&d](int64_t k) { return d.m_psr[k]; }, st, tr);
}

// total log-likelihood of one sample (canonical parameter vector c)
template <class T>
T sample_loglike(const DS& d, const T* c, int32_t* st, T* per_psr) {
  *st = 0;
  if (!finite_params(c, n_canon(d))) {
    *st = S_NONFINITE;
    return T(-std::numeric_limits<double>::infinity());
  }
  Par<T> p = make_par<T>(d, c);
  if (d.model == M_JOINT) return joint_loglike<T>(d, p, st, nullptr);
  T tot = T(0.0);
  for (int q = 0; q < d.P; ++q) {
    int32_t s = 0;
    T l = psr_loglike<T>(d, p, q, &s, nullptr);
    if (per_psr) per_psr[q] = l;
    if (s && !*st) *st = s;
    tot += l;
  }
  if (*st) return T(-std::numeric_limits<double>::infinity());
  return tot;
}

// ------------------------------------------------------------ smoothing
// Solves A X = B in place (A m x m, B m x r, row-major; X returned in B) by
// Gaussian elimination with partial pivoting. Returns false when a pivot is
// exactly zero.
bool gauss_solve(int m, int r, double* A, double* B) {
  for (int c = 0; c < m; ++c) {
    int piv = c;
    for (int i = c + 1; i < m; ++i)
      if (std::fabs(A[i * m + c]) > std::fabs(A[piv * m + c])) piv = i;
    if (A[piv * m + c] == 0.0) return false;
    if (piv != c) {
      for (int j = 0; j < m; ++j) std::swap(A[c * m + j], A[piv * m + j]);
      for (int j = 0; j < r; ++j) std::swap(B[c * r + j], B[piv * r + j]);
    }
    for (int i = c + 1; i < m; ++i) {
      const double f = A[i * m + c] / A[c * m + c];
      if (f == 0.0) continue;
      for (int j = c; j < m; ++j) A[i * m + j] -= f * A[c * m + j];
      for (int j = 0; j < r; ++j) B[i * r + j] -= f * B[c * r + j];
    }
  }
  for (int c = m - 1; c >= 0; --c)
    for (int j = 0; j < r; ++j) {
      double s = B[c * r + j];
      for (int i = c + 1; i < m; ++i) s -= A[c * m + i] * B[i * r + j];
      B[c * r + j] = s / A[c * m + c];
    }
  return true;
}

// Rauch-Tung-Striebel fixed-interval smoother (Rauch, Tung & Striebel 1965)
// over one filter's stream, from the filtered moments (x_k, P_k) and the
// predicted moments (x-_k, P-_k) of every step:
//   G_k  = P_k F_{k+1}^T (P-_{k+1})^{-1},   F_{k+1} = F(t_{k+1} - t_k),
//   xs_k = x_k + G_k (xs_{k+1} - x-_{k+1}),
//   Ps_k = P_k + G_k (Ps_{k+1} - P-_{k+1}) G_k^T,
// starting from the last step's filtered moments. The gain comes from the
// linear system P-_{k+1} G_k^T = F_{k+1} P_k, with P-_{k+1} scaled to unit
// diagonal first (its entries span tens of decades). A component whose
// predicted variance is exactly zero is deterministic given the past; it is
// left out of the system and gets a zero gain column (the minimum-norm
// solution on that null space).
template <class IdxF>
bool rts(const DS& d, const Par<double>& p, int q_fixed, int64_t N, IdxF idx, int n,
         const Trace& tr, double* xs, double* Ps) {
  if (N == 0) return true;
  std::copy(tr.x + (N - 1) * n, tr.x + N * n, xs + (N - 1) * n);
  std::copy(tr.Pf + (N - 1) * n * n, tr.Pf + N * n * n, Ps + (N - 1) * n * n);
  std::vector<double> F(n * n), Q(n * n), FP(n * n), A, B, Gt(n * n), D(n * n),
      T1(n * n), dx(n);
  std::vector<int> J;
  for (int64_t k = N - 2; k >= 0; --k) {
    const double dt = d.t[idx(k + 1)] - d.t[idx(k)];
    model_fq(d, p, q_fixed, dt, n, F.data(), Q.data());
    const double* Pk = tr.Pf + k * n * n;
    const double* Pm = tr.Pp + (k + 1) * n * n;
    mm(n, F.data(), Pk, FP.data());  // F P_k = (P_k F^T)^T
    J.clear();
    for (int i = 0; i < n; ++i)
      if (Pm[i * n + i] > 0.0) J.push_back(i);
    const int m = (int)J.size();
    A.assign((size_t)m * m, 0.0);
    B.assign((size_t)m * n, 0.0);
    for (int a = 0; a < m; ++a) {
      const double da = 1.0 / std::sqrt(Pm[J[a] * n + J[a]]);
      for (int b = 0; b < m; ++b)
        A[a * m + b] = da * Pm[J[a] * n + J[b]] / std::sqrt(Pm[J[b] * n + J[b]]);
      for (int j = 0; j < n; ++j) B[a * n + j] = da * FP[J[a] * n + j];
    }
    if (m > 0 && !gauss_solve(m, n, A.data(), B.data())) return false;
    std::fill(Gt.begin(), Gt.end(), 0.0);  // Gt = G_k^T
    for (int a = 0; a < m; ++a) {
      const double da = 1.0 / std::sqrt(Pm[J[a] * n + J[a]]);
      for (int j = 0; j < n; ++j) Gt[J[a] * n + j] = da * B[a * n + j];
    }
    // xs_k = x_k + G (xs_{k+1} - x-_{k+1})
    for (int i = 0; i < n; ++i) dx[i] = xs[(k + 1) * n + i] - tr.xp[(k + 1) * n + i];
    for (int i = 0; i < n; ++i) {
      double s = tr.x[k * n + i];
      for (int j = 0; j < n; ++j) s += Gt[j * n + i] * dx[j];
      xs[k * n + i] = s;
    }
    // Ps_k = P_k + G (Ps_{k+1} - P-_{k+1}) G^T
    for (int i = 0; i < n * n; ++i) D[i] = Ps[(k + 1) * n * n + i] - Pm[i];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {  // T1 = D G^T
        double s = 0.0;
        for (int l = 0; l < n; ++l) s += D[i * n + l] * Gt[l * n + j];
        T1[i * n + j] = s;
      }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = Pk[i * n + j];
        for (int l = 0; l < n; ++l) s += Gt[l * n + i] * T1[l * n + j];
        Ps[k * n * n + i * n + j] = s;
      }
  }
  return true;
}

// Filter then smooth one stream: pulsar q (per-pulsar models) or the joint
// stream (q ignored). xs [N*n], Ps [N*n*n]; NaN everywhere when the filter
// fails (status set).
double smooth_stream(const DS& d, const Par<double>& p, int q, double* xs, double* Ps,
                     int32_t* st) {
  const int n = state_dim(d);
  const int64_t N = d.model == M_JOINT ? (int64_t)d.m_idx.size() : d.off[q + 1] - d.off[q];
  std::vector<double> e(N), S(N), x(N * n), Pf(N * n * n), Pp(N * n * n), xp(N * n);
  Trace tr{e.data(), S.data(), x.data(), Pf.data(), Pp.data(), xp.data()};
  *st = 0;
  double ll;
  bool ok;
  if (d.model == M_JOINT) {
    ll = joint_loglike<double>(d, p, st, &tr);
    ok = !*st && rts(d, p, 0, N, [&d](int64_t k) { return d.m_idx[k]; }, n, tr, xs, Ps);
  } else {
    ll = psr_loglike<double>(d, p, q, st, &tr);
    const int64_t b = d.off[q];
    ok = !*st && rts(d, p, q, N, [b](int64_t k) { return b + k; }, n, tr, xs, Ps);
  }
  if (!ok) {
    if (!*st) *st = S_NONPD;
    std::fill(xs, xs + N * n, std::numeric_limits<double>::quiet_NaN());
    std::fill(Ps, Ps + N * n * n, std::numeric_limits<double>::quiet_NaN());
  }
  return ll;
}

void build_merged(DS& d) {
  if (d.model != M_JOINT) return;
  const int64_t N = d.off[d.P];
  d.m_idx.resize(N);
  d.m_psr.resize(N);
  std::vector<std::pair<int64_t, int>> v;
  v.reserve(N);
  for (int q = 0; q < d.P; ++q)
    for (int64_t j = d.off[q]; j < d.off[q + 1]; ++j) v.push_back({j, q});
  std::stable_sort(v.begin(), v.end(), [&d](const auto& a, const auto& b) {
    if (d.t[a.first] != d.t[b.first]) return d.t[a.first] < d.t[b.first];
    return a.second < b.second;
  });
  for (int64_t k = 0; k < N; ++k) {
    d.m_idx[k] = v[k].first;
    d.m_psr[k] = v[k].second;
  }
  d.hd.resize((size_t)d.P * d.P);
  hd_matrix(d.pos, d.P, d.hd.data());
}

template <class F>
void parallel_for(int64_t S, int nthreads, F f) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > S) nthreads = (int)std::max<int64_t>(S, 1);
  std::vector<std::thread> th;
  for (int w = 0; w < nthreads; ++w)
    th.emplace_back([=]() {
      for (int64_t s = w; s < S; s += nthreads) f(s);
    });
  for (auto& x : th) x.join();
}

// ------------------------------------------------------ parallel-in-time
// The filter as an associative scan (Sarkka & Garcia-Fernandez 2021). Step k
// is summarised by an element (A, b, C, eta, J): given the filtered state
// x_{k-1}, x_k ~ N(A x_{k-1} + b, C) after y_k, and y_k's likelihood as a
// function of x_{k-1} is proportional to exp(eta^T x - x^T J x / 2). With
// S = h Q h^T + R, K = Q h^T / S:
//   A = (I - K h) F,  b = K y,  C = (I - K h) Q,
//   eta = F^T h^T y / S,  J = F^T h^T h F / S;
// the first step folds in the prior: A = 0, b and C its filtered mean and
// covariance, eta = 0, J = 0. Two elements compose as (i then j)
//   A  = A_j T A_i,              T = (I + C_i J_j)^-1,
//   b  = A_j T (b_i + C_i eta_j) + b_j,
//   C  = A_j T C_i A_j^T + C_j,
//   eta = A_i^T U (eta_j - J_j b_i) + eta_i,   U = (I + J_j C_i)^-1,
//   J  = A_i^T U J_j A_i + J_i,
// and the inclusive prefix up to k has A = 0, b = x_k, C = P_k.
struct Elem {
  std::vector<double> A, b, C, eta, J;
};

Elem elem_zero(int n) {
  Elem e;
  e.A.assign(n * n, 0.0);
  e.b.assign(n, 0.0);
  e.C.assign(n * n, 0.0);
  e.eta.assign(n, 0.0);
  e.J.assign(n * n, 0.0);
  return e;
}

// X = (I + P Q)^-1 Y for n x n P, Q and n x r Y
void solve_ipq(int n, int r, const double* P, const double* Q, const double* Y, double* X) {
  std::vector<double> M(n * n), B(Y, Y + n * r);
  mm(n, P, Q, M.data());
  for (int i = 0; i < n; ++i) M[i * n + i] += 1.0;
  gauss_solve(n, r, M.data(), B.data());
  std::copy(B.begin(), B.end(), X);
}

Elem combine(const Elem& ei, const Elem& ej, int n) {
  Elem o = elem_zero(n);
  std::vector<double> T1(n * n), T2(n * n), TA(n * n), v(n), w(n);
  // T A_i, T C_i and T (b_i + C_i eta_j): one solve with 2n + 1 columns
  std::vector<double> Y(n * (2 * n + 1)), X(n * (2 * n + 1));
  for (int r = 0; r < n; ++r) {
    double s = ei.b[r];
    for (int m = 0; m < n; ++m) s += ei.C[r * n + m] * ej.eta[m];
    for (int c = 0; c < n; ++c) {
      Y[r * (2 * n + 1) + c] = ei.A[r * n + c];
      Y[r * (2 * n + 1) + n + c] = ei.C[r * n + c];
    }
    Y[r * (2 * n + 1) + 2 * n] = s;
  }
  solve_ipq(n, 2 * n + 1, ei.C.data(), ej.J.data(), Y.data(), X.data());
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      double sa = 0.0, sc = 0.0;
      for (int m = 0; m < n; ++m) {
        sa += ej.A[r * n + m] * X[m * (2 * n + 1) + c];
        sc += ej.A[r * n + m] * X[m * (2 * n + 1) + n + c];
      }
      o.A[r * n + c] = sa;
      T1[r * n + c] = sc;  // A_j T C_i
    }
  for (int r = 0; r < n; ++r) {
    double sb = ej.b[r];
    for (int m = 0; m < n; ++m) sb += ej.A[r * n + m] * X[m * (2 * n + 1) + 2 * n];
    o.b[r] = sb;
    for (int c = 0; c < n; ++c) {
      double sc = ej.C[r * n + c];
      for (int m = 0; m < n; ++m) sc += T1[r * n + m] * ej.A[c * n + m];
      o.C[r * n + c] = sc;
    }
  }
  // U J_j A_i and U (eta_j - J_j b_i): one solve with n + 1 columns
  std::vector<double> Y2(n * (n + 1)), X2(n * (n + 1));
  for (int r = 0; r < n; ++r) {
    double s = ej.eta[r];
    for (int m = 0; m < n; ++m) s -= ej.J[r * n + m] * ei.b[m];
    for (int c = 0; c < n; ++c) {
      double t = 0.0;
      for (int m = 0; m < n; ++m) t += ej.J[r * n + m] * ei.A[m * n + c];
      Y2[r * (n + 1) + c] = t;
    }
    Y2[r * (n + 1) + n] = s;
  }
  solve_ipq(n, n + 1, ej.J.data(), ei.C.data(), Y2.data(), X2.data());
  for (int r = 0; r < n; ++r) {
    double se = ei.eta[r];
    for (int m = 0; m < n; ++m) se += ei.A[m * n + r] * X2[m * (n + 1) + n];
    o.eta[r] = se;
    for (int c = 0; c < n; ++c) {
      double sj = ei.J[r * n + c];
      for (int m = 0; m < n; ++m) sj += ei.A[m * n + r] * X2[m * (n + 1) + c];
      o.J[r * n + c] = sj;
    }
  }
  return o;
}

// Elements of every step of pulsar q's stream (per-pulsar models).
std::vector<Elem> scan_elements(const DS& d, const Par<double>& p, int q) {
  const int n = d.model == M_SPIN ? 2 : 4;
  const int64_t b0 = d.off[q], N = d.off[q + 1] - b0;
  std::vector<Elem> el(N, elem_zero(n));
  std::vector<double> F(n * n), Q(n * n), P0(n * n), H(n, 0.0), u(n), K(n), hF(n), IKH(n * n),
      tmp(n * n);
  H[0] = 1.0;
  if (n == 4) H[2] = H[3] = 1.0;
  model_p0(d, p, q, n, P0.data());
  double t_prev = 0.0;
  for (int64_t k = 0; k < N; ++k) {
    const int64_t j = b0 + k;
    model_fq(d, p, q, d.t[j] - t_prev, n, F.data(), Q.data());
    t_prev = d.t[j];
    const double sk = d.sig[j];
    const double R = p.psr[q].efac2 * sk * sk + p.psr[q].equad2;
    Elem& e = el[k];
    // the covariance entering the update: F P0 F^T + Q at the first step, Q after
    std::vector<double> Pp(Q);
    if (k == 0) {
      mm(n, F.data(), P0.data(), tmp.data());
      mmt(n, tmp.data(), F.data(), Pp.data());
      for (int i = 0; i < n * n; ++i) Pp[i] += Q[i];
    }
    double S = R;
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int m = 0; m < n; ++m) s += Pp[i * n + m] * H[m];
      u[i] = s;
      S += H[i] * s;
    }
    for (int i = 0; i < n; ++i) K[i] = u[i] / S;
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m) IKH[i * n + m] = (i == m ? 1.0 : 0.0) - K[i] * H[m];
    // C = (I - K h) Pp (I - K h)^T + K R K^T (Joseph form of (I - K h) Pp)
    mm(n, IKH.data(), Pp.data(), tmp.data());
    mmt(n, tmp.data(), IKH.data(), e.C.data());
    for (int i = 0; i < n; ++i)
      for (int m = 0; m < n; ++m) e.C[i * n + m] += K[i] * R * K[m];
    if (k == 0) {  // prior folded in: A = 0, b = filtered mean (prior mean 0)
      for (int i = 0; i < n; ++i) e.b[i] = K[i] * d.y[j];
      continue;
    }
    mm(n, IKH.data(), F.data(), e.A.data());
    for (int i = 0; i < n; ++i) e.b[i] = K[i] * d.y[j];
    for (int c = 0; c < n; ++c) {
      double s = 0.0;
      for (int m = 0; m < n; ++m) s += H[m] * F[m * n + c];
      hF[c] = s;
    }
    for (int r = 0; r < n; ++r) {
      e.eta[r] = hF[r] * d.y[j] / S;
      for (int c = 0; c < n; ++c) e.J[r * n + c] = hF[r] * hF[c] / S;
    }
  }
  return el;
}

// Inclusive prefix of the elements in one of three evaluation orders:
// 0 left fold; 1 recursive doubling (prefix k combines the prefixes ending
// at k - 2^l and k at level l); 2 chunked (nchunk chunks folded internally,
// the chunk totals folded, then each chunk's prefixes from the total of the
// chunks before it).
std::vector<Elem> scan_prefix(const std::vector<Elem>& el, int n, int order, int nchunk) {
  const int64_t N = (int64_t)el.size();
  std::vector<Elem> pre(el);
  if (N == 0) return pre;
  if (order == 0) {
    for (int64_t k = 1; k < N; ++k) pre[k] = combine(pre[k - 1], el[k], n);
  } else if (order == 1) {
    for (int64_t dd = 1; dd < N; dd *= 2) {
      std::vector<Elem> nxt(pre);
      for (int64_t k = dd; k < N; ++k) nxt[k] = combine(pre[k - dd], pre[k], n);
      pre.swap(nxt);
    }
  } else {
    const int64_t C = std::max<int64_t>(1, std::min<int64_t>(nchunk, N));
    std::vector<int64_t> edge(C + 1);
    for (int64_t c = 0; c <= C; ++c) edge[c] = c * N / C;
    std::vector<Elem> tot(C);
    for (int64_t c = 0; c < C; ++c) {
      Elem a = el[edge[c]];
      for (int64_t k = edge[c] + 1; k < edge[c + 1]; ++k) a = combine(a, el[k], n);
      tot[c] = a;
    }
    for (int64_t c = 1; c < C; ++c) tot[c] = combine(tot[c - 1], tot[c], n);
    for (int64_t c = 0; c < C; ++c) {
      Elem a = c == 0 ? el[edge[0]] : combine(tot[c - 1], el[edge[c]], n);
      pre[edge[c]] = a;
      for (int64_t k = edge[c] + 1; k < edge[c + 1]; ++k) {
        a = combine(a, el[k], n);
        pre[k] = a;
      }
    }
  }
  return pre;
}

}  // namespace

// ====================================================================== C API
extern "C" {

// Dataset description. t, y, sigma hold each pulsar's TOAs contiguously
// (CSR offsets off[P+1]) in ascending time; seconds since the epoch t0 = 0.
typedef struct {
  int32_t model;  // 1 spin-only [r,f]; 2 per-pulsar [r,f,a,g]; 3 joint HD
  int32_t n_psr;
  const int64_t* off;
  const double* t;
  const double* y;
  const double* sigma;
  const double* pos;  // [n_psr*3] unit vectors (joint model), may be NULL
  double t_span;      // seconds
  double s_r, s_f;    // prior std of the spin offset r (s) and f
  double sigma_s;     // spin random-walk amplitude (per-pulsar models 2/3)
  const double* freq; // [N] radio frequency per TOA, MHz (model 4), may be NULL
} oracle_ds;

static DS make_ds(const oracle_ds* o) {
  DS d;
  d.model = o->model;
  d.P = o->n_psr;
  d.off = o->off;
  d.t = o->t;
  d.y = o->y;
  d.sig = o->sigma;
  d.pos = o->pos;
  d.t_span = o->t_span;
  d.s_r = o->s_r;
  d.s_f = o->s_f;
  d.sigma_s = o->sigma_s;
  d.freq = o->freq;
  build_merged(d);
  return d;
}

int oracle_n_canon(const oracle_ds* o) {
  return o->model == M_SPIN ? 2 : (o->model == M_DM ? 6 : 4) * o->n_psr + 2;
}

// logL for S samples of canonical parameters c [S x C]. per_psr (nullable)
// receives [S x P] per-pulsar terms for the per-pulsar models.
int oracle_loglike(const oracle_ds* o, const double* c, int64_t S, double* out,
                   int32_t* status, double* per_psr, int nthreads) {
  DS d = make_ds(o);
  const int C = n_canon(d);
  parallel_for(S, nthreads, [&](int64_t s) {
    int32_t st = 0;
    out[s] = sample_loglike<double>(d, c + s * C, &st,
                                    per_psr ? per_psr + s * d.P : nullptr);
    if (status) status[s] = st;
  });
  return 0;
}

// Complex-step derivatives d logL / d c_j for the canonical indices which[nw],
// step h: Im logL(c + i h e_j) / h. Parameters of one pulsar enter only that
// pulsar's term in the per-pulsar models, so only that term is run.
int oracle_grad_cs(const oracle_ds* o, const double* c, int64_t S,
                   const int32_t* which, int nw, double h, double* grad,
                   int nthreads) {
  DS d = make_ds(o);
  const int C = n_canon(d);
  parallel_for(S, nthreads, [&](int64_t s) {
    std::vector<cd> cc(C);
    for (int j = 0; j < nw; ++j) {
      for (int i = 0; i < C; ++i) cc[i] = cd(c[s * C + i], 0.0);
      const int w = which[j];
      cc[w] += cd(0.0, h);
      int32_t st = 0;
      cd l;
      const int k = per_psr(d);
      if ((d.model == M_PSR4 || d.model == M_DM) && w < k * d.P) {
        Par<cd> p = make_par<cd>(d, cc.data());
        l = psr_loglike<cd>(d, p, w / k, &st, nullptr);
      } else {
        l = sample_loglike<cd>(d, cc.data(), &st, nullptr);
      }
      grad[s * nw + j] = st ? 0.0 : l.imag() / h;
    }
  });
  return 0;
}

// Per-step trace of one filter (pulsar q, or the joint stream when q < 0)
// for one canonical vector. Arrays sized by the stream length N and the
// state dimension n of that filter.
int oracle_trace(const oracle_ds* o, const double* c, int q, double* e,
                 double* S, double* x, double* Pf, double* Pp, double* ll,
                 int32_t* status) {
  DS d = make_ds(o);
  Par<double> p = make_par<double>(d, c);
  Trace tr{e, S, x, Pf, Pp};
  int32_t st = 0;
  if (d.model == M_JOINT)
    *ll = joint_loglike<double>(d, p, &st, &tr);
  else
    *ll = psr_loglike<double>(d, p, q, &st, &tr);
  *status = st;
  return 0;
}

// Smoothed moments of one stream (pulsar q, or the joint stream when the
// model is joint) for one canonical vector: xs [N*n], Ps [N*n*n] in stream
// order, n the filter's state dimension.
int oracle_smooth_stream(const oracle_ds* o, const double* c, int q, double* xs, double* Ps,
                         double* ll, int32_t* status) {
  DS d = make_ds(o);
  int32_t st = 0;
  if (!finite_params(c, n_canon(d))) {
    st = S_NONFINITE;
    *ll = -std::numeric_limits<double>::infinity();
  } else {
    Par<double> p = make_par<double>(d, c);
    *ll = smooth_stream(d, p, q, xs, Ps, &st);
  }
  *status = st;
  if (st) {
    const int n = state_dim(d);
    const int64_t N = d.model == M_JOINT ? (int64_t)d.m_idx.size() : d.off[q + 1] - d.off[q];
    std::fill(xs, xs + N * n, std::numeric_limits<double>::quiet_NaN());
    std::fill(Ps, Ps + N * n * n, std::numeric_limits<double>::quiet_NaN());
  }
  return 0;
}

// Smoothed mean and variance of the emitting pulsar's own state components
// at every TOA, for S canonical vectors c [S x C]: mean, var [S x N x nc]
// in dataset TOA order, nc = 2 (model 1) or 4. The entries of a filter that
// fails are NaN: per pulsar in the per-pulsar models (its innovation
// variance not positive, or a non-finite parameter among its own four and
// the two common ones), all of them in the joint model. status [S] as for
// the likelihood: NONFINITE for a non-finite parameter anywhere in the row,
// else the first failure in pulsar order.
int oracle_smooth(const oracle_ds* o, const double* c, int64_t S, double* mean, double* var,
                  int32_t* status, int nthreads) {
  DS d = make_ds(o);
  const int C = n_canon(d);
  const int nc = d.model == M_JOINT ? 4 : state_dim(d);
  const int kp = per_psr(d);
  const int64_t Nt = d.off[d.P];
  parallel_for(S, nthreads, [&](int64_t s) {
    double* ms = mean + s * Nt * nc;
    double* vs = var + s * Nt * nc;
    const double* cs = c + s * C;
    int32_t sst = 0;
    const double nan = std::numeric_limits<double>::quiet_NaN();
    const bool row_finite = finite_params(cs, C);
    if (!row_finite && d.model != M_PSR4 && d.model != M_DM) {
      std::fill(ms, ms + Nt * nc, nan);
      std::fill(vs, vs + Nt * nc, nan);
      status[s] = S_NONFINITE;
      return;
    }
    // non-finite entries only reach the pulsars that read them
    std::vector<double> cf(cs, cs + C);
    for (double& v : cf)
      if (!std::isfinite(v)) v = 0.0;
    Par<double> p = make_par<double>(d, cf.data());
    if (d.model == M_JOINT) {
      const int n = 4 * d.P;
      const int64_t N = (int64_t)d.m_idx.size();
      std::vector<double> xs(N * n), Ps(N * n * n);
      smooth_stream(d, p, 0, xs.data(), Ps.data(), &sst);
      for (int64_t k = 0; k < N; ++k) {
        const int64_t j = d.m_idx[k];
        const int o4 = 4 * d.m_psr[k];
        for (int a = 0; a < 4; ++a) {
          ms[j * 4 + a] = xs[k * n + o4 + a];
          vs[j * 4 + a] = Ps[k * n * n + (o4 + a) * n + o4 + a];
        }
      }
    } else {
      for (int q = 0; q < d.P; ++q) {
        const int64_t b = d.off[q], N = d.off[q + 1] - b;
        std::vector<double> xs(N * nc, nan), Ps(N * nc * nc, nan);
        int32_t qs = 0;
        if ((d.model == M_PSR4 || d.model == M_DM) &&
            !(finite_params(cs + kp * q, kp) && finite_params(cs + kp * d.P, 2)))
          qs = S_NONFINITE;
        else
          smooth_stream(d, p, q, xs.data(), Ps.data(), &qs);
        if (qs && !sst) sst = qs;
        for (int64_t k = 0; k < N; ++k)
          for (int a = 0; a < nc; ++a) {
            ms[(b + k) * nc + a] = xs[k * nc + a];
            vs[(b + k) * nc + a] = Ps[k * nc * nc + a * nc + a];
          }
      }
    }
    status[s] = row_finite ? sst : S_NONFINITE;
  });
  return 0;
}

// Filtered moments of pulsar q (per-pulsar models) by the associative scan
// in evaluation order `order` (see scan_prefix), and the log-likelihood from
// them: the predicted moments of step k come from the prefix ending at k - 1
// (the prior before the first step). xs [N*n], Ps [N*n*n].
int oracle_scan_filter(const oracle_ds* o, const double* c, int q, int order, int nchunk,
                       double* xs, double* Ps, double* ll) {
  DS d = make_ds(o);
  if (d.model == M_JOINT || d.model == M_DM) return -1;
  Par<double> p = make_par<double>(d, c);
  const int n = d.model == M_SPIN ? 2 : 4;
  std::vector<Elem> el = scan_elements(d, p, q);
  std::vector<Elem> pre = scan_prefix(el, n, order, nchunk);
  const int64_t b0 = d.off[q], N = d.off[q + 1] - b0;
  std::vector<double> F(n * n), Q(n * n), P(n * n), x(n, 0.0), Pp(n * n), tmp(n * n);
  model_p0(d, p, q, n, P.data());
  double acc = 0.0, t_prev = 0.0;
  for (int64_t k = 0; k < N; ++k) {
    const int64_t j = b0 + k;
    model_fq(d, p, q, d.t[j] - t_prev, n, F.data(), Q.data());
    t_prev = d.t[j];
    mm(n, F.data(), P.data(), tmp.data());
    mmt(n, tmp.data(), F.data(), Pp.data());
    double hx = 0.0, S = p.psr[q].efac2 * d.sig[j] * d.sig[j] + p.psr[q].equad2;
    const int hidx[3] = {0, 2, 3};
    for (int a = 0; a < (n == 2 ? 1 : 3); ++a) {
      const int i = hidx[a];
      double fx = 0.0;
      for (int m = 0; m < n; ++m) fx += F[i * n + m] * x[m];
      hx += fx;
      for (int b = 0; b < (n == 2 ? 1 : 3); ++b) S += Pp[i * n + hidx[b]] + Q[i * n + hidx[b]];
    }
    const double e = d.y[j] - hx;
    acc += -0.5 * (std::log(2.0 * kPi) + std::log(S) + e * e / S);
    x = pre[k].b;
    P = pre[k].C;
    std::copy(x.begin(), x.end(), xs + k * n);
    std::copy(P.begin(), P.end(), Ps + k * n * n);
  }
  *ll = acc;
  return 0;
}

// Merged stream order of the joint model: global TOA index and pulsar.
int oracle_merged(const oracle_ds* o, int64_t* idx, int32_t* psr) {
  DS d = make_ds(o);
  for (size_t k = 0; k < d.m_idx.size(); ++k) {
    idx[k] = d.m_idx[k];
    psr[k] = d.m_psr[k];
  }
  return 0;
}

// F(dt), Q(dt) and the prior P0 of the filter for pulsar q (or joint).
int oracle_model_mats(const oracle_ds* o, const double* c, int q, double dt,
                      double* F, double* Q, double* P0) {
  DS d = make_ds(o);
  Par<double> p = make_par<double>(d, c);
  const int n = state_dim(d);
  model_fq(d, p, q, dt, n, F, Q);
  model_p0(d, p, q, n, P0);
  return n;
}

void oracle_hd(const double* pos, int P, double* G) { hd_matrix(pos, P, G); }

double oracle_common_variance(double log10A, double gam, double t_span) {
  return common_variance<double>(log10A, gam, t_span);
}

}  // extern "C"
