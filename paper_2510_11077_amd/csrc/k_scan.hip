// Time-parallel Kalman filter for the per-pulsar models (1, 2): the
// recursion split over the waves of a workgroup by chunks of the TOA stream,
// for calls whose batch is too small to fill the GPU, where the sequential
// filter is bound by one wave's serial chain over the whole stream.
//
// The filter is an associative scan (Sarkka & Garcia-Fernandez 2021): a run
// of TOAs is summarised, as a function of the filtered state x_s before it,
// by x_end | x_s ~ N(A x_s + b, C) after the run's data, and by the run's
// likelihood as a function of x_s, proportional to
// exp(eta^T x_s - x_s^T J x_s / 2). Per TOA (F, Q, h, R, y), from the run
// so far:
//   A <- F A, b <- F b, C <- F C F^T + Q;   g = h A, u = C h^T,
//   S = h u + R, r = y - h b;
//   J += g^T g / S, eta += g^T r / S;   K = u / S;
//   A <- A - K g, b <- b + K r, C <- Joseph update of C with gain K,
// and a filtered state (m, P) before the run becomes, after it,
//   Cs = (P^-1 + J)^-1, mu = m + Cs (eta - J m),
//   m' = A mu + b,  P' = A Cs A^T + C.
// Cs is formed without inverting P or J: with P = G G^T (G from the LDL^T
// factors of P, so a zero-variance state is allowed), Cs = G M^-1 G^T with
// M = I + G^T J G >= I, whose Cholesky factor is well conditioned.
//
// Mapping: one workgroup of NW waves per (64-sample tile, pulsar) item,
// lane = sample, wave w = chunk w of the pulsar's stream.
//   1. wave 0 filters chunk 0 from the prior; waves w >= 1 build their
//      chunk's summary (A, b, C, eta, J) in registers;
//   2. in wave order, wave w turns the filtered state at the end of chunk
//      w - 1 (LDS) into the one at the end of chunk w (NW - 2 steps,
//      separated by barriers);
//   3. waves w >= 1 filter their chunk from that state, accumulating the
//      log-likelihood terms, which wave 0 adds up in chunk order.
// Each TOA is visited twice (phases 1 and 3) and phase 2 is short, so the
// serial chain is about (N / NW) (1 + 2.5) steps + NW combines instead of N
// steps. Covariance updates use the Joseph form evaluated as
// W = P - K u^T, z = R K - W h^T, P' = W + z K^T.
#include "argus_internal.h"

namespace argus {

namespace {

__device__ __forceinline__ bool finite_d(double v) {
  return __builtin_amdgcn_class(v, 0x1F8);
}

// index of entry (i, j) of a symmetric matrix stored as its lower triangle
__host__ __device__ constexpr int si(int i, int j) {
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

template <int NS>
struct Lane {
  double gr, vr, vc, efac2, equad2, ss2;
};

// Transition of one TOA for this lane.
struct Step {
  double dt, q00, q01, q11;  // spin block: dt and sigma_s^2 (dt^3/3, dt^2/2, dt)
  double ph, phc, qr, qc;    // red and common OU decays and noises
  double R, y;
};

template <int NS>
__device__ __forceinline__ Step make_step(const TOARec& r, const Lane<NS>& L, double em) {
  Step t;
  t.dt = r.dt;
  t.q00 = L.ss2 * r.h3;
  t.q01 = L.ss2 * r.h2;
  t.q11 = L.ss2 * r.dt;
  t.ph = 1.0 + em;
  t.phc = r.phc;
  t.qr = L.vr * (-em * (2.0 + em));
  t.qc = L.vc * r.qcu;
  t.R = fma(L.efac2, r.s2, L.equad2);
  t.y = r.y;
  return t;
}

// observation row h: [1, 0] or [1, 0, 1, 1]
template <int NS>
__device__ __forceinline__ constexpr bool hm(int i) {
  return NS == 2 ? i == 0 : i != 1;
}

// P <- F P F^T + Q on the lower triangle
template <int NS>
__device__ __forceinline__ void predict_cov(double* P, const Step& t) {
  const double dt = t.dt;
  const double prf1 = fma(dt, P[si(1, 1)], P[si(1, 0)]);
  P[si(0, 0)] = fma(dt, P[si(1, 0)] + prf1, P[si(0, 0)]) + t.q00;
  P[si(1, 0)] = prf1 + t.q01;
  P[si(1, 1)] = P[si(1, 1)] + t.q11;
  if constexpr (NS == 4) {
    const double ph = t.ph, phc = t.phc;
    P[si(2, 0)] = ph * fma(dt, P[si(2, 1)], P[si(2, 0)]);
    P[si(2, 1)] = ph * P[si(2, 1)];
    P[si(2, 2)] = fma(ph * ph, P[si(2, 2)], t.qr);
    P[si(3, 0)] = phc * fma(dt, P[si(3, 1)], P[si(3, 0)]);
    P[si(3, 1)] = phc * P[si(3, 1)];
    P[si(3, 2)] = (ph * phc) * P[si(3, 2)];
    P[si(3, 3)] = fma(phc * phc, P[si(3, 3)], t.qc);
  }
}

// F v
template <int NS>
__device__ __forceinline__ void predict_vec(double* v, const Step& t) {
  v[0] = fma(t.dt, v[1], v[0]);
  if constexpr (NS == 4) {
    v[2] *= t.ph;
    v[3] *= t.phc;
  }
}

// Joseph update of the symmetric P (lower triangle) with gain K = u / S.
template <int NS>
__device__ __forceinline__ void joseph(double* P, const double* K, const double* u, double R) {
  double z[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double wh = 0.0;
#pragma unroll
    for (int l = 0; l < NS; ++l)
      if (hm<NS>(l)) wh += fma(-K[i], u[l], P[si(i, l)]);
    z[i] = fma(R, K[i], -wh);
  }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = i; j < NS; ++j) P[si(i, j)] = fma(z[i], K[j], fma(-K[i], u[j], P[si(i, j)]));
}

struct LogAcc {
  double m;
  int e;
};

template <int NS>
struct Filt {
  double x[NS];
  double P[NS * (NS + 1) / 2];
  double quad;
  LogAcc L;
  int st;
};

// one filter step with log-likelihood accumulation
template <int NS>
__device__ __forceinline__ void filt_step(Filt<NS>& f, const Step& t) {
  predict_vec<NS>(f.x, t);
  predict_cov<NS>(f.P, t);
  double u[NS], hx = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = 0.0;
#pragma unroll
    for (int l = 0; l < NS; ++l)
      if (hm<NS>(l)) s += f.P[si(i, l)];
    u[i] = s;
    if (hm<NS>(i)) hx += f.x[i];
  }
  double hu = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i)
    if (hm<NS>(i)) hu += u[i];
  const double S = hu + t.R;
  const double e = t.y - hx;
  const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
  if (!good && f.st == 0) f.st = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
  const double inv = rcp_nr(S);
  double K[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    K[i] = u[i] * inv;
    f.x[i] = fma(K[i], e, f.x[i]);
  }
  joseph<NS>(f.P, K, u, t.R);
  f.quad = fma(e * e, inv, f.quad);
  const double pm = f.L.m * S;
  f.L.m = __builtin_amdgcn_frexp_mant(pm);
  f.L.e += __builtin_amdgcn_frexp_exp(pm);
}

// Summary of a run of TOAs (see the header): A full, C and J symmetric.
template <int NS>
struct Elem {
  double A[NS][NS];
  double b[NS];
  double C[NS * (NS + 1) / 2];
  double eta[NS];
  double J[NS * (NS + 1) / 2];
};

template <int NS>
__device__ __forceinline__ void elem_identity(Elem<NS>& E) {
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int j = 0; j < NS; ++j) E.A[i][j] = i == j ? 1.0 : 0.0;
    E.b[i] = 0.0;
    E.eta[i] = 0.0;
  }
#pragma unroll
  for (int i = 0; i < NS * (NS + 1) / 2; ++i) E.C[i] = E.J[i] = 0.0;
}

template <int NS>
__device__ __forceinline__ void elem_step(Elem<NS>& E, const Step& t) {
  // predict: A <- F A, b <- F b, C <- F C F^T + Q
#pragma unroll
  for (int c = 0; c < NS; ++c) {
    E.A[0][c] = fma(t.dt, E.A[1][c], E.A[0][c]);
    if constexpr (NS == 4) {
      E.A[2][c] *= t.ph;
      E.A[3][c] *= t.phc;
    }
  }
  predict_vec<NS>(E.b, t);
  predict_cov<NS>(E.C, t);
  // the measurement as a function of the state before the run
  double g[NS], u[NS], hb = 0.0, hu = 0.0;
#pragma unroll
  for (int c = 0; c < NS; ++c) {
    double s = 0.0, v = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i)
      if (hm<NS>(i)) {
        s += E.A[i][c];
        v += E.C[si(c, i)];
      }
    g[c] = s;
    u[c] = v;
    if (hm<NS>(c)) {
      hb += E.b[c];
      hu += v;
    }
  }
  const double S = hu + t.R;
  const double r = t.y - hb;
  const double inv = rcp_nr(S);
  double gi[NS], K[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    gi[i] = g[i] * inv;
    K[i] = u[i] * inv;
    E.eta[i] = fma(gi[i], r, E.eta[i]);
  }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) E.J[si(i, j)] = fma(gi[i], g[j], E.J[si(i, j)]);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
#pragma unroll
    for (int c = 0; c < NS; ++c) E.A[i][c] = fma(-K[i], g[c], E.A[i][c]);
    E.b[i] = fma(K[i], r, E.b[i]);
  }
  joseph<NS>(E.C, K, u, t.R);
}

// (m, P) <- the filtered state after the run summarised by E, given (m, P)
// before it.
template <int NS>
__device__ __forceinline__ void apply_elem(double* m, double* P, const Elem<NS>& E) {
  // P = L D L^T (unit lower L); G = L sqrt(D); zero or negative-rounded
  // pivots give zero columns
  double Lf[NS][NS], D[NS], G[NS][NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    double d = P[si(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma(-Lf[j][k] * Lf[j][k], D[k], d);
    D[j] = d > 0.0 ? d : 0.0;
    const double id = d > 0.0 ? 1.0 / d : 0.0;
#pragma unroll
    for (int i = j + 1; i < NS; ++i) {
      double s = P[si(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) s = fma(-Lf[i][k] * Lf[j][k], D[k], s);
      Lf[i][j] = s * id;
    }
  }
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const double sq = __builtin_sqrt(D[j]);
#pragma unroll
    for (int i = 0; i < NS; ++i) G[i][j] = i < j ? 0.0 : (i == j ? sq : Lf[i][j] * sq);
  }
  // M = I + G^T J G
  double T[NS][NS], M[NS * (NS + 1) / 2];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j < NS; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < NS; ++k) s = fma(E.J[si(i, k)], G[k][j], s);
      T[i][j] = s;
    }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double s = i == j ? 1.0 : 0.0;
#pragma unroll
      for (int k = i; k < NS; ++k) s = fma(G[k][i], T[k][j], s);
      M[si(i, j)] = s;
    }
  // M = Lm Lm^T (pivots >= 1)
  double Lm[NS][NS], il[NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    double d = M[si(j, j)];
#pragma unroll
    for (int k = 0; k < j; ++k) d = fma(-Lm[j][k], Lm[j][k], d);
    const double l = __builtin_sqrt(d);
    il[j] = 1.0 / l;
#pragma unroll
    for (int i = j + 1; i < NS; ++i) {
      double s = M[si(i, j)];
#pragma unroll
      for (int k = 0; k < j; ++k) s = fma(-Lm[i][k], Lm[j][k], s);
      Lm[i][j] = s * il[j];
    }
  }
  // W = Lm^-1 G^T, Cs = W^T W
  double W[NS][NS], Cs[NS * (NS + 1) / 2];
#pragma unroll
  for (int c = 0; c < NS; ++c)
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      double s = G[c][r];
#pragma unroll
      for (int k = 0; k < r; ++k) s = fma(-Lm[r][k], W[k][c], s);
      W[r][c] = s * il[r];
    }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < NS; ++r) s = fma(W[r][i], W[r][j], s);
      Cs[si(i, j)] = s;
    }
  // mu = m + Cs (eta - J m)
  double v[NS], mu[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = E.eta[i];
#pragma unroll
    for (int k = 0; k < NS; ++k) s = fma(-E.J[si(i, k)], m[k], s);
    v[i] = s;
  }
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = m[i];
#pragma unroll
    for (int k = 0; k < NS; ++k) s = fma(Cs[si(i, k)], v[k], s);
    mu[i] = s;
  }
  // m' = A mu + b, P' = A Cs A^T + C
  double AC[NS][NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double s = E.b[i];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      s = fma(E.A[i][k], mu[k], s);
      double t = 0.0;
#pragma unroll
      for (int l = 0; l < NS; ++l) t = fma(E.A[i][l], Cs[si(l, k)], t);
      AC[i][k] = t;
    }
    m[i] = s;
  }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double s = E.C[si(i, j)];
#pragma unroll
      for (int k = 0; k < NS; ++k) s = fma(AC[i][k], E.A[j][k], s);
      P[si(i, j)] = s;
    }
}

__device__ __forceinline__ double load_param(const FilterArgs& a, int c, int64_t s) {
  const int j = a.col[c];
  return j >= 0 ? a.theta[s * a.D + j] : a.fixed[c];
}

template <int MODEL, int NW>
__global__ void __launch_bounds__(NW * 64) k_scan(FilterArgs a) {
  constexpr int NS = MODEL == 1 ? 2 : 4;
  constexpr int NP = NS * (NS + 1) / 2;
  constexpr int NF = NS + NP;  // fields of a filtered state
  __shared__ double s_state[NW > 1 ? NW - 1 : 1][NF][kWave];
  __shared__ double s_ll[NW][kWave];
  __shared__ int s_st[NW][kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const RecPtr rec = (RecPtr)a.rec;
  for (int it = blockIdx.x; it < a.n_items; it += gridDim.x) {
    const int tile = a.items[2 * it];
    const int p = a.items[2 * it + 1];
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    const int64_t kb = a.off[p], N = a.off[p + 1] - kb;
    const int64_t c0 = kb + N * w / NW, c1 = kb + N * (w + 1) / NW;

    // this lane's parameters
    Lane<NS> L;
    bool pnf;
    if (MODEL == 1) {
      const double lss = load_param(a, 0, s), efac = load_param(a, 1, s);
      pnf = !(finite_d(lss) && finite_d(efac));
      const double ss = exp10(lss);
      L = Lane<NS>{1.0, 0.0, 0.0, efac * efac, 0.0, ss * ss};
    } else {
      const int q0 = 4 * p, qc = 4 * a.P;
      const double lsr = load_param(a, q0, s), lgr = load_param(a, q0 + 1, s);
      const double efac = load_param(a, q0 + 2, s), leq = load_param(a, q0 + 3, s);
      const double la = load_param(a, qc, s), gc = load_param(a, qc + 1, s);
      pnf = !(finite_d(lsr) && finite_d(lgr) && finite_d(efac) && finite_d(leq) &&
              finite_d(la) && finite_d(gc));
      const double gr = exp10(lgr), sr = exp10(lsr), eq = exp10(leq);
      const double gm1 = gc - 1.0;
      const double vc = exp(2.0 * kLn10 * la + (gc - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
                        (12.0 * kPi * kPi * gm1);
      L = Lane<NS>{gr, sr * sr / (2.0 * gr), vc, efac * efac, eq * eq, a.mc.ss2};
    }
    // the chunk's steps, each record fetched one step ahead (the index is
    // clamped, so the last iteration repeats a harmless load)
    auto run = [&](auto&& body) {
      if (c1 <= c0) return;
      TOARec rn = load_rec(rec, c0);
      for (int64_t k = c0; k < c1; ++k) {
        const TOARec r = rn;
        rn = load_rec(rec, k + 1 < c1 ? k + 1 : k);
        body(make_step<NS>(r, L, NS == 4 ? expm1_k(-L.gr * r.dt) : 0.0));
      }
    };

    // ---- phase 1: chunk 0 filtered from the prior; the others summarised
    Elem<NS> E;
    if (w == 0) {
      Filt<NS> f;
#pragma unroll
      for (int i = 0; i < NS; ++i) f.x[i] = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) f.P[i] = 0.0;
      f.P[si(0, 0)] = a.mc.s_r2;
      f.P[si(1, 1)] = a.mc.s_f2;
      if constexpr (NS == 4) {
        f.P[si(2, 2)] = L.vr;
        f.P[si(3, 3)] = L.vc;
      }
      f.quad = 0.0;
      f.L = {1.0, 0};
      f.st = pnf ? kPNF : 0;
      run([&](const Step& t) { filt_step<NS>(f, t); });
      if (NW > 1) {
#pragma unroll
        for (int i = 0; i < NS; ++i) s_state[0][i][lane] = f.x[i];
#pragma unroll
        for (int i = 0; i < NP; ++i) s_state[0][NS + i][lane] = f.P[i];
      }
      s_ll[0][lane] = -0.5 * ((double)(c1 - c0) * kLn2Pi +
                              (log(f.L.m) + (double)f.L.e * kLn2) + f.quad);
      s_st[0][lane] = f.st;
    } else {
      elem_identity<NS>(E);
      run([&](const Step& t) { elem_step<NS>(E, t); });
    }

    // ---- phase 2: filtered state at the end of chunk w, in chunk order
#pragma unroll 1
    for (int i = 1; i < NW - 1; ++i) {
      __syncthreads();
      if (w == i) {
        double m[NS], P[NP];
#pragma unroll
        for (int j = 0; j < NS; ++j) m[j] = s_state[i - 1][j][lane];
#pragma unroll
        for (int j = 0; j < NP; ++j) P[j] = s_state[i - 1][NS + j][lane];
        if (c1 > c0) apply_elem<NS>(m, P, E);
#pragma unroll
        for (int j = 0; j < NS; ++j) s_state[i][j][lane] = m[j];
#pragma unroll
        for (int j = 0; j < NP; ++j) s_state[i][NS + j][lane] = P[j];
      }
    }
    __syncthreads();

    // ---- phase 3: chunks 1.. filtered from their start states
    if (w > 0) {
      Filt<NS> f;
#pragma unroll
      for (int j = 0; j < NS; ++j) f.x[j] = s_state[w - 1][j][lane];
#pragma unroll
      for (int j = 0; j < NP; ++j) f.P[j] = s_state[w - 1][NS + j][lane];
      f.quad = 0.0;
      f.L = {1.0, 0};
      f.st = 0;
      run([&](const Step& t) { filt_step<NS>(f, t); });
      s_ll[w][lane] = -0.5 * ((double)(c1 - c0) * kLn2Pi +
                              (log(f.L.m) + (double)f.L.e * kLn2) + f.quad);
      s_st[w][lane] = f.st;
    }
    __syncthreads();
    if (w == 0) {
      double ll = 0.0;
      int st = 0;
#pragma unroll
      for (int j = 0; j < NW; ++j) {
        ll += s_ll[j][lane];
        if (st == 0) st = s_st[j][lane];
      }
      if (st == 0 && !finite_d(ll)) st = kNonFinite;
      if (valid) {
        a.part[(int64_t)p * a.S + s] = st ? -INFINITY : ll;
        a.pstat[(int64_t)p * a.S + s] = st;
      }
    }
    // the state and partial buffers are rewritten by the next item
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_scan(int model, const FilterArgs& a, int grid, int nw, hipStream_t st) {
  const dim3 g((unsigned)grid), b((unsigned)(nw * kWave));
  if (model == 1) {
    if (nw == 4)
      hipLaunchKernelGGL((k_scan<1, 4>), g, b, 0, st, a);
    else if (nw == 8)
      hipLaunchKernelGGL((k_scan<1, 8>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_scan<1, 16>), g, b, 0, st, a);
  } else {
    if (nw == 4)
      hipLaunchKernelGGL((k_scan<2, 4>), g, b, 0, st, a);
    else if (nw == 8)
      hipLaunchKernelGGL((k_scan<2, 8>), g, b, 0, st, a);
    else
      hipLaunchKernelGGL((k_scan<2, 16>), g, b, 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace argus
