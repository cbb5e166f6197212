// Gradient of the batched per-pulsar log-likelihood by a hand-written
// adjoint (reverse-mode) Kalman sweep. The paper's samplers consume the
// likelihood and its gradient (Functionality, "Sampler Integration"); here
// the gradient is the exact derivative of the same recursion. The same
// checkpointed pass, carrying the information pair of the modified
// Bryson-Frazier recursion backwards instead of the adjoints, is the
// fixed-interval smoother of the latent noise (the filter tracking the
// realised noise: Summary, Statement of Need).
//
// Per TOA the forward map is (x, P) -> (x+, P+) with
//   x- = F x, P- = F P F^T + Q, e = y - h.x-, u = P- h, S = h.u + R,
//   x+ = x- + u e / S,  P+ = P- - u u^T / S   (the Joseph form evaluated at the
//   optimal gain; its derivative in K vanishes there, so this is also the
//   derivative of the Joseph update the forward pass computes),
//   l += -1/2 (ln S + e^2 / S).
// With adjoints xb = dL/dx+ and the symmetric Mb = dL/dP+ (Frobenius pairing),
//   a = xb.u, w = Mb u, b = u.w,
//   g_e = (a - e)/S, g_S = (b - a e - S/2 + e^2/2)/S^2,
//   g_u = (e/S) xb - (2/S) w,
//   xb- = xb - g_e h,  Mb- = Mb + sym(g_u h^T) + g_S h h^T,  Rb = g_S,
//   Qb = Mb-,  Fb = xb- x^T + 2 Mb- F P,  xb <- F^T xb-,  Mb <- F^T Mb- F,
// and the parameters enter through F (red-OU decay), Q (red and common OU
// noise, spin noise), R (EFAC, EQUAD) and the prior P0.
//
// Memory: level-1 checkpoints of (x, P) every c1 = ceil(sqrt(N_p)) TOAs
// (rounded up to a multiple of 4) in HBM; in the reverse sweep each segment
// is recomputed once to level-2 checkpoints every 4 TOAs (a per-wave scratch
// area that stays cache-resident), and each 4-TOA piece is reversed from its
// checkpoint with the state before each TOA recomputed in registers. Work: about 5 forward passes, no per-TOA HBM
// traffic. Mapping as the forward filter: one wavefront per (64-sample tile,
// pulsar), lane = sample, TOA records read with scalar loads.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "argus_host.h"
#include "argus_internal.h"

namespace argus {

namespace {

__device__ __forceinline__ bool finite_d(double v) {
  return __builtin_amdgcn_class(v, 0x1F8);
}

struct Cov4 {
  double rr, rf, ff, ra, fa, aa, rg, fg, ag, gg;
};
struct State {
  double xr, xf, xa, xg;
  Cov4 P;
};
struct LaneP {
  double gr, vr, vc, efac2, equad2, ss2;
};
struct Grad {
  double gam, v, vc, ef2, eq2, ss2;
};

constexpr int kFields = 14;  // x (4) + P (10)

struct AdjArgs {
  const TOARec* rec;
  const double* chrom;      // [N] chromatic factor per TOA (model 4)
  const int64_t* off;
  const double* theta;
  const int32_t* col;
  const double* fixed;
  const int32_t* items;
  int32_t* counter;
  const int32_t* c1;        // [P] level-1 stride per pulsar (multiple of 4)
  const int64_t* seg_base;  // [P] first segment index of each pulsar
  double* ckpt;             // [tiles * tot_seg * 14 * 64]
  double* scratch;          // [nwaves * max_sub * 14 * 64]
  double* part;             // [P*S] log-likelihood terms
  int32_t* pstat;           // [P*S]
  double* gpart;            // [P * 6 * S] per-pulsar parameter gradients
  const int32_t* tp_item;   // time-parallel smoother: per item its chunk count and first slot
  const int32_t* tp_units;  // (item, chunk) units, longest chunk first
  double* tpsum;            // [slots * 30 * 64] chunk summaries
  double* tpadj;            // [slots * 14 * 64] adjoints after each chunk / the final state
  double* smean;            // smoothing: [N * nc * S] posterior means
  double* svar;             // smoothing: [N * nc * S] posterior variances, or null
  int64_t S, tot_seg;
  int32_t D, P, n_items, max_sub, model, nc, n_units;
  ModelConst mc;
};

__device__ __forceinline__ void put_state(double* base, int lane, const State& s) {
  const double v[kFields] = {s.xr,   s.xf,   s.xa,   s.xg,   s.P.rr, s.P.rf, s.P.ff,
                             s.P.ra, s.P.fa, s.P.aa, s.P.rg, s.P.fg, s.P.ag, s.P.gg};
#pragma unroll
  for (int f = 0; f < kFields; ++f) base[f * kWave + lane] = v[f];
}
__device__ __forceinline__ State get_state(const double* base, int lane) {
  double v[kFields];
#pragma unroll
  for (int f = 0; f < kFields; ++f) v[f] = base[f * kWave + lane];
  return State{v[0], v[1], v[2], v[3],
               Cov4{v[4], v[5], v[6], v[7], v[8], v[9], v[10], v[11], v[12], v[13]}};
}

// Predicted state and covariance over one interval (F P F^T + Q).
struct Pred {
  double xr, xf, xa, xg;
  Cov4 P;
  double em, ph;
};
__device__ __forceinline__ Pred predict(const State& s, const TOARec& r, const LaneP& L) {
  Pred o;
  const double dt = r.dt;
  o.em = expm1_k(-L.gr * dt);
  o.ph = 1.0 + o.em;
  const double qr = L.vr * (-o.em * (2.0 + o.em));
  const double phc = r.phc, qc = L.vc * r.qcu;
  o.xr = fma(dt, s.xf, s.xr);
  o.xf = s.xf;
  o.xa = o.ph * s.xa;
  o.xg = phc * s.xg;
  const double prf1 = fma(dt, s.P.ff, s.P.rf);
  o.P.rr = fma(dt, s.P.rf + prf1, s.P.rr) + L.ss2 * r.h3;
  o.P.rf = prf1 + L.ss2 * r.h2;
  o.P.ff = s.P.ff + L.ss2 * dt;
  o.P.ra = o.ph * fma(dt, s.P.fa, s.P.ra);
  o.P.fa = o.ph * s.P.fa;
  o.P.aa = fma(o.ph * o.ph, s.P.aa, qr);
  o.P.rg = phc * fma(dt, s.P.fg, s.P.rg);
  o.P.fg = phc * s.P.fg;
  o.P.ag = (o.ph * phc) * s.P.ag;
  o.P.gg = fma(phc * phc, s.P.gg, qc);
  return o;
}

#define JOSEPH(pij, ki, uj, di, kj) pij = fma(di, kj, fma(-(ki), uj, pij))

// One forward step in place; returns S, e, 1/S, the gain k and the red decay.
__device__ __forceinline__ void fwd_step(State& s, const TOARec& r, const LaneP& L, double& S,
                                         double& e, double& inv, double kk[4], double& phr) {
  const Pred p = predict(s, r, L);
  phr = p.ph;
  e = r.y - (p.xr + p.xa + p.xg);
  const double ur = p.P.rr + p.P.ra + p.P.rg;
  const double uf = p.P.rf + p.P.fa + p.P.fg;
  const double ua = p.P.ra + p.P.aa + p.P.ag;
  const double ug = p.P.rg + p.P.ag + p.P.gg;
  const double R = fma(L.efac2, r.s2, L.equad2);
  S = (ur + ua + ug) + R;
  inv = rcp_nr(S);
  const double kr = ur * inv, kf = uf * inv, ka = ua * inv, kg = ug * inv;
  kk[0] = kr;
  kk[1] = kf;
  kk[2] = ka;
  kk[3] = kg;
  s.xr = fma(kr, e, p.xr);
  s.xf = fma(kf, e, p.xf);
  s.xa = fma(ka, e, p.xa);
  s.xg = fma(kg, e, p.xg);
  // Joseph form (I - k h^T) P- (I - k h^T)^T + R k k^T, evaluated as
  // W = P- - k u^T, z = R k - W h, P+ = W + z k^T. Regrouping it to
  // P- - k u^T + (S k - u) k^T (exact at the computed k) would lose the
  // low digits of R inside the rounded S = h.u + R: after a long gap, when
  // h.u >> R, the observed variance then carries a relative error of
  // eps h.u / R. Here the rounding of W enters W h as well and is damped by
  // the factor R / S.
  const double wrr = fma(-kr, ur, p.P.rr), wra = fma(-kr, ua, p.P.ra), wrg = fma(-kr, ug, p.P.rg);
  const double wfr = fma(-kf, ur, p.P.rf), wfa = fma(-kf, ua, p.P.fa), wfg = fma(-kf, ug, p.P.fg);
  const double war = fma(-ka, ur, p.P.ra), waa = fma(-ka, ua, p.P.aa), wag = fma(-ka, ug, p.P.ag);
  const double wgr = fma(-kg, ur, p.P.rg), wga = fma(-kg, ua, p.P.ag), wgg = fma(-kg, ug, p.P.gg);
  const double wrf = fma(-kr, uf, p.P.rf), wff = fma(-kf, uf, p.P.ff);
  const double zr = fma(R, kr, -((wrr + wra) + wrg));
  const double zf = fma(R, kf, -((wfr + wfa) + wfg));
  const double za = fma(R, ka, -((war + waa) + wag));
  const double zg = fma(R, kg, -((wgr + wga) + wgg));
  s.P.rr = fma(zr, kr, wrr);
  s.P.rf = fma(zr, kf, wrf);
  s.P.ff = fma(zf, kf, wff);
  s.P.ra = fma(zr, ka, wra);
  s.P.fa = fma(zf, ka, wfa);
  s.P.aa = fma(za, ka, waa);
  s.P.rg = fma(zr, kg, wrg);
  s.P.fg = fma(zf, kg, wfg);
  s.P.ag = fma(za, kg, wag);
  s.P.gg = fma(zg, kg, wgg);
}

__device__ __forceinline__ void fwd_step(State& s, const TOARec& r, const LaneP& L, double& S,
                                         double& e, double& inv) {
  double kk[4], ph;
  fwd_step(s, r, L, S, e, inv, kk, ph);
}

__device__ __forceinline__ void fwd_only(State& s, const TOARec& r, const LaneP& L) {
  double S, e, inv;
  fwd_step(s, r, L, S, e, inv);
}

// Reverse of one step. sp = posterior before the step; (xb, Mb) adjoints of
// the posterior after it, replaced by the adjoints of sp.
__device__ __forceinline__ void rev_step(const State& sp, const TOARec& r, const LaneP& L,
                                         double xb[4], Cov4& M, Grad& G) {
  const Pred p = predict(sp, r, L);
  const double dt = r.dt, phc = r.phc;
  const double e = r.y - (p.xr + p.xa + p.xg);
  const double u[4] = {p.P.rr + p.P.ra + p.P.rg, p.P.rf + p.P.fa + p.P.fg,
                       p.P.ra + p.P.aa + p.P.ag, p.P.rg + p.P.ag + p.P.gg};
  const double S = (u[0] + u[2] + u[3]) + fma(L.efac2, r.s2, L.equad2);
  const double inv = rcp_nr(S);
  const double a = xb[0] * u[0] + xb[1] * u[1] + xb[2] * u[2] + xb[3] * u[3];
  const double w[4] = {M.rr * u[0] + M.rf * u[1] + M.ra * u[2] + M.rg * u[3],
                       M.rf * u[0] + M.ff * u[1] + M.fa * u[2] + M.fg * u[3],
                       M.ra * u[0] + M.fa * u[1] + M.aa * u[2] + M.ag * u[3],
                       M.rg * u[0] + M.fg * u[1] + M.ag * u[2] + M.gg * u[3]};
  const double b = u[0] * w[0] + u[1] * w[1] + u[2] * w[2] + u[3] * w[3];
  const double ge = (a - e) * inv;
  const double gS = (b - a * e - 0.5 * S + 0.5 * e * e) * (inv * inv);
  const double ei = e * inv, ti = 2.0 * inv;
  double gu[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) gu[i] = ei * xb[i] - ti * w[i];
  // adjoints of the predicted mean and covariance (h = [1, 0, 1, 1])
  const double xm[4] = {xb[0] - ge, xb[1], xb[2] - ge, xb[3] - ge};
  Cov4 Mm;
  Mm.rr = M.rr + gu[0] + gS;
  Mm.rf = M.rf + 0.5 * gu[1];
  Mm.ff = M.ff;
  Mm.ra = M.ra + 0.5 * (gu[0] + gu[2]) + gS;
  Mm.fa = M.fa + 0.5 * gu[1];
  Mm.aa = M.aa + gu[2] + gS;
  Mm.rg = M.rg + 0.5 * (gu[0] + gu[3]) + gS;
  Mm.fg = M.fg + 0.5 * gu[1];
  Mm.ag = M.ag + 0.5 * (gu[2] + gu[3]) + gS;
  Mm.gg = M.gg + gu[3] + gS;
  // parameters through R and Q
  G.ef2 = fma(gS, r.s2, G.ef2);
  G.eq2 += gS;
  G.v = fma(Mm.aa, -p.em * (2.0 + p.em), G.v);
  G.vc = fma(Mm.gg, r.qcu, G.vc);
  G.ss2 += Mm.rr * r.h3 + 2.0 * Mm.rf * r.h2 + Mm.ff * dt;
  // through the red-OU decay phi = F_aa: dL/dphi = xm_a x_a + 2 (Mm F P)_aa
  const double ph = p.ph;
  const double fpaa = Mm.ra * fma(dt, sp.P.fa, sp.P.ra) + Mm.fa * sp.P.fa +
                      Mm.aa * (ph * sp.P.aa) + Mm.ag * (phc * sp.P.ag);
  const double phib = fma(xm[2], sp.xa, 2.0 * fpaa);
  G.gam = fma(dt * ph, 2.0 * L.vr * ph * Mm.aa - phib, G.gam);
  // back through F: xb = F^T xm, M = F^T Mm F
  xb[0] = xm[0];
  xb[1] = fma(dt, xm[0], xm[1]);
  xb[2] = ph * xm[2];
  xb[3] = phc * xm[3];
  M.rr = Mm.rr;
  M.rf = fma(dt, Mm.rr, Mm.rf);
  M.ff = fma(dt, fma(dt, Mm.rr, 2.0 * Mm.rf), Mm.ff);
  M.ra = ph * Mm.ra;
  M.fa = ph * fma(dt, Mm.ra, Mm.fa);
  M.rg = phc * Mm.rg;
  M.fg = phc * fma(dt, Mm.rg, Mm.fg);
  M.aa = (ph * ph) * Mm.aa;
  M.ag = (ph * phc) * Mm.ag;
  M.gg = (phc * phc) * Mm.gg;
}

// Smoother: the modified Bryson-Frazier recursion. With the information
// vector lam and matrix Lam of the filtered state after a TOA (zero after
// the last TOA), the smoothed moments there are
//   E[x | y] = x - P lam,   Cov[x | y] = P - P Lam P,
// and TOA k maps the pair after it to the pair after TOA k - 1 by
//   lam <- F^T (C^T lam - h e / S),   Lam <- F^T (C^T Lam C + h h^T / S) F,
//   C = I - K h^T,  C^T Lam C = Lam - h g^T - g h^T + (K.g) h h^T,  g = Lam K.
// (In terms of the adjoints of the gradient sweep, lam = -xb and
// Lam = xb xb^T - 2 M; carrying the pair itself keeps the smoothed
// covariance free of the cancellation between xb xb^T and 2 M.)
// sp = filtered state after TOA k - 1, r = TOA k.
__device__ __forceinline__ void rev_bf(const State& sp, const TOARec& r, const LaneP& L,
                                       double lam[4], Cov4& Lm) {
  const Pred p = predict(sp, r, L);
  const double dt = r.dt, phc = r.phc, ph = p.ph;
  const double e = r.y - (p.xr + p.xa + p.xg);
  const double u[4] = {p.P.rr + p.P.ra + p.P.rg, p.P.rf + p.P.fa + p.P.fg,
                       p.P.ra + p.P.aa + p.P.ag, p.P.rg + p.P.ag + p.P.gg};
  const double S = (u[0] + u[2] + u[3]) + fma(L.efac2, r.s2, L.equad2);
  const double inv = rcp_nr(S);
  const double K[4] = {u[0] * inv, u[1] * inv, u[2] * inv, u[3] * inv};
  // C^T lam - h e / S  (h = [1, 0, 1, 1])
  const double hl = fma(K[0], lam[0], fma(K[1], lam[1], fma(K[2], lam[2], K[3] * lam[3]))) +
                    e * inv;
  const double t0 = lam[0] - hl, t1 = lam[1], t2 = lam[2] - hl, t3 = lam[3] - hl;
  // g = Lam K, C^T Lam C + h h^T / S
  const double g[4] = {Lm.rr * K[0] + Lm.rf * K[1] + Lm.ra * K[2] + Lm.rg * K[3],
                       Lm.rf * K[0] + Lm.ff * K[1] + Lm.fa * K[2] + Lm.fg * K[3],
                       Lm.ra * K[0] + Lm.fa * K[1] + Lm.aa * K[2] + Lm.ag * K[3],
                       Lm.rg * K[0] + Lm.fg * K[1] + Lm.ag * K[2] + Lm.gg * K[3]};
  const double c = fma(K[0], g[0], fma(K[1], g[1], fma(K[2], g[2], K[3] * g[3]))) + inv;
  Cov4 X;
  X.rr = Lm.rr - 2.0 * g[0] + c;
  X.rf = Lm.rf - g[1];
  X.ff = Lm.ff;
  X.ra = Lm.ra - g[2] - g[0] + c;
  X.fa = Lm.fa - g[1];
  X.aa = Lm.aa - 2.0 * g[2] + c;
  X.rg = Lm.rg - g[3] - g[0] + c;
  X.fg = Lm.fg - g[1];
  X.ag = Lm.ag - g[3] - g[2] + c;
  X.gg = Lm.gg - 2.0 * g[3] + c;
  // through F: lam = F^T t, Lam = F^T X F
  lam[0] = t0;
  lam[1] = fma(dt, t0, t1);
  lam[2] = ph * t2;
  lam[3] = phc * t3;
  Lm.rr = X.rr;
  Lm.rf = fma(dt, X.rr, X.rf);
  Lm.ff = fma(dt, fma(dt, X.rr, 2.0 * X.rf), X.ff);
  Lm.ra = ph * X.ra;
  Lm.fa = ph * fma(dt, X.ra, X.fa);
  Lm.rg = phc * X.rg;
  Lm.fg = phc * fma(dt, X.rg, X.fg);
  Lm.aa = (ph * ph) * X.aa;
  Lm.ag = (ph * phc) * X.ag;
  Lm.gg = (phc * phc) * X.gg;
}

// Smoothed moments at TOA k from the filtered state f after it and the
// information pair there: the first nc components of the mean and the
// variance diagonal at entry ((k * nc + c) * S + s); NaN when the filter
// failed.
__device__ __forceinline__ void put_smooth(const AdjArgs& a, int64_t k, int64_t s,
                                           const State& f, const double lam[4], const Cov4& Lm,
                                           bool bad) {
  const double P[4][4] = {{f.P.rr, f.P.rf, f.P.ra, f.P.rg},
                          {f.P.rf, f.P.ff, f.P.fa, f.P.fg},
                          {f.P.ra, f.P.fa, f.P.aa, f.P.ag},
                          {f.P.rg, f.P.fg, f.P.ag, f.P.gg}};
  const double x[4] = {f.xr, f.xf, f.xa, f.xg};
  double* mo = a.smean + k * a.nc * a.S + s;
  double* vo = a.svar ? a.svar + k * a.nc * a.S + s : nullptr;
  const double nan = __builtin_nan("");
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    if (c >= a.nc) break;
    // w = row c of P: mean x_c - w.lam, variance P_cc - w^T Lam w
    const double* w = P[c];
    const double m = x[c] - fma(w[0], lam[0], fma(w[1], lam[1], fma(w[2], lam[2], w[3] * lam[3])));
    const double q = fma(w[0], fma(Lm.rr, w[0], 2.0 * fma(Lm.rf, w[1], fma(Lm.ra, w[2], Lm.rg * w[3]))),
                     fma(w[1], fma(Lm.ff, w[1], 2.0 * fma(Lm.fa, w[2], Lm.fg * w[3])),
                         fma(w[2], fma(Lm.aa, w[2], 2.0 * Lm.ag * w[3]), Lm.gg * w[3] * w[3])));
    mo[c * a.S] = bad ? nan : m;
    if (vo) vo[c * a.S] = bad ? nan : P[c][c] - q;
  }
}

__device__ __forceinline__ double prm(const AdjArgs& a, int c, int64_t s) {
  const int j = a.col[c];
  return j >= 0 ? a.theta[s * a.D + j] : a.fixed[c];
}

// This lane's filter parameters for pulsar p (models 1, 2), the parameters
// the gradient's chain rule needs (model 1: t1 = EFAC; model 2: t1 =
// log10 gamma_red, t2 = EFAC, t5 = gamma), and whether one is not finite.
struct LaneTheta {
  LaneP L;
  double t1, t2, t5;
  bool pnf;
};
__device__ __forceinline__ LaneTheta lane_theta(const AdjArgs& a, int p, int64_t s) {
  // scalar locals in both branches (an aggregate assigned in each branch
  // would be merged through private memory)
  double gr, vr, vc, efac2, equad2, ss2, t1, t2, t5;
  bool pnf;
  if (a.model == 1) {
    const double t0 = prm(a, 0, s);  // log10 sigma_s
    t1 = prm(a, 1, s);               // EFAC
    pnf = !(finite_d(t0) && finite_d(t1));
    const double ss = exp10(t0);
    gr = 1.0;
    vr = vc = equad2 = 0.0;
    efac2 = t1 * t1;
    ss2 = ss * ss;
    t2 = 0.0;
    t5 = 2.0;
  } else {
    const int c0 = 4 * p, cc = 4 * a.P;
    const double t0 = prm(a, c0, s);
    t1 = prm(a, c0 + 1, s);
    t2 = prm(a, c0 + 2, s);
    const double t3 = prm(a, c0 + 3, s);
    const double t4 = prm(a, cc, s);
    t5 = prm(a, cc + 1, s);
    pnf = !(finite_d(t0) && finite_d(t1) && finite_d(t2) && finite_d(t3) && finite_d(t4) &&
            finite_d(t5));
    gr = exp10(t1);
    const double sr = exp10(t0), eq = exp10(t3);
    const double gm1 = t5 - 1.0;
    vc = exp(2.0 * kLn10 * t4 + (t5 - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
         (12.0 * kPi * kPi * gm1);
    vr = sr * sr / (2.0 * gr);
    efac2 = t2 * t2;
    equad2 = eq * eq;
    ss2 = a.mc.ss2;
  }
  return LaneTheta{LaneP{gr, vr, vc, efac2, equad2, ss2}, t1, t2, t5, pnf};
}

// What the reverse sweep carries and does per TOA. The gradient: the
// adjoints (xb, M) of the filtered state and the parameter gradient.
struct GradSweep {
  double xb[4];
  Cov4 M;
  Grad G;
  __device__ __forceinline__ void step(const State& sp, const TOARec& r, const LaneP& L) {
    rev_step(sp, r, L, xb, M, G);
  }
  __device__ __forceinline__ void emit(int, const State&) {}
};
// The smoother: the information pair (lam, Lam) of the filtered state, and
// the smoothed moments of each TOA k (within pulsar stream kb..) written out.
struct SmoothSweep {
  const AdjArgs* a;
  int kb;
  int64_t s;
  bool valid, bad;
  double lam[4];
  Cov4 Lm;
  __device__ __forceinline__ void step(const State& sp, const TOARec& r, const LaneP& L) {
    rev_bf(sp, r, L, lam, Lm);
  }
  __device__ __forceinline__ void emit(int k, const State& f) {
    if (valid) put_smooth(*a, (int64_t)kb + k, s, f, lam, Lm, bad);
  }
};

// The reverse sweep over level-1 segments sg_hi - 1 down to sg_lo of a
// pulsar's stream (ck: its level-1 checkpoints; scr: this wave's level-2
// scratch). sw holds what is carried after the last TOA of segment
// sg_hi - 1 and on return holds it before the first TOA of segment sg_lo;
// sw.emit(k, f) is called, with the filtered state f after TOA k, for every
// TOA k >= klo of the range except the last one.
// PIECES: every segment is one piece (level-1 stride 4): no level-2 pass.
template <bool PIECES, class Sweep>
__device__ __forceinline__ void reverse_segments(const RecBuf& rb, const double* ck, double* scr,
                                                 const LaneP& L, int N, int c1, int sg_lo,
                                                 int sg_hi, int klo, Sweep& sw) {
  const int lane = threadIdx.x & (kWave - 1);
  // reverse one 4-TOA piece starting at TOA ks from the state s0 before it:
  // the state before TOA i of the piece is recomputed from s0 (0..3 steps),
  // so only two states are live in registers; the piece's records are read
  // once into VGPRs (index clamped to its last TOA) and the loops are
  // unrolled so that they are addressed statically
  auto piece = [&](int ks, int nt, const State& s0) {
    TOARec q[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = load_rec_vgpr(rb, ks + (i < nt ? i : nt - 1));
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      if (i < nt) {
        State cur = s0;
#pragma unroll
        for (int j = 0; j < i; ++j) fwd_only(cur, q[j], L);
        sw.step(cur, q[i], L);
        // sw now holds the pair of the filtered state after TOA ks + i - 1
        if (ks + i > klo) sw.emit(ks + i - 1, cur);
      }
    }
  };
  for (int64_t sg = sg_hi - 1; sg >= sg_lo; --sg) {
    const int64_t k0 = sg * c1;
    const int64_t k1 = k0 + c1 < N ? k0 + c1 : N;
    if constexpr (PIECES) {
      // the piece starts from its level-1 checkpoint itself
      piece((int)k0, (int)(k1 - k0), get_state(ck + sg * kFields * kWave, lane));
      continue;
    }
    const int nsub = (int)((k1 - k0 + 3) / 4);
    // recompute the segment to level-2 checkpoints every 4 TOAs; the four
    // records of a piece are read together into VGPRs (one wait per piece)
    State cur = get_state(ck + sg * kFields * kWave, lane);
    for (int t = 0; t < nsub; ++t) {
      put_state(scr + (int64_t)t * kFields * kWave, lane, cur);
      if (t + 1 < nsub) {
        const int kk = (int)k0 + 4 * t;  // a full piece: kk + 3 < k1
        TOARec q[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) q[i] = load_rec_vgpr(rb, kk + i);
#pragma unroll
        for (int i = 0; i < 4; ++i) fwd_only(cur, q[i], L);
      }
    }
    // the pieces, last first
    for (int t = nsub - 1; t >= 0; --t) {
      const int ks = (int)k0 + 4 * t;
      piece(ks, (int)(k1 - ks < 4 ? k1 - ks : 4), get_state(scr + (int64_t)t * kFields * kWave, lane));
    }
  }
}

// SMOOTH: write the smoothed moments of every TOA instead of the gradient.
template <bool SMOOTH>
__global__ void __launch_bounds__(256) k_adjoint(AdjArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int gwave = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave));
  double* scr = a.scratch + (int64_t)gwave * a.max_sub * kFields * kWave;
  const RecPtr rec = (RecPtr)a.rec;
  for (;;) {
    int v = 0;
    if (lane == 0) v = atomicAdd(a.counter, 1);
    const int it = __builtin_amdgcn_readfirstlane(v);
    if (it >= a.n_items) break;
    const int tile = a.items[2 * it];
    const int p = a.items[2 * it + 1];
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
    const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
    const int c1 = a.c1[p];
    double* ck = a.ckpt + ((int64_t)tile * a.tot_seg + a.seg_base[p]) * kFields * kWave;

    // parameters of this lane's filter
    const LaneTheta th = lane_theta(a, p, s);
    const LaneP L = th.L;
    const double t1 = th.t1, t2 = th.t2, t5 = th.t5;
    const bool pnf = th.pnf;

    // ---------------- forward pass: log-likelihood + level-1 checkpoints
    State st{0.0, 0.0, 0.0, 0.0,
             Cov4{a.mc.s_r2, 0.0, a.mc.s_f2, 0.0, 0.0, L.vr, 0.0, 0.0, 0.0, L.vc}};
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = pnf ? kPNF : 0;
    int kc = 0;                 // position within the current segment
    double* ckw = ck;           // next level-1 checkpoint slot
    // The record of step k + 1 is fetched during step k (index clamped):
    // by the gradient variant as one 64-B scalar vector kept whole until the
    // next step, by the smoothing variant, which has no SGPRs to spare, into
    // VGPRs
    const RecVecPtr recv = (RecVecPtr)a.rec;
    const RecBuf rb = rec_buffer(a.rec + kb, N);
    RecVec vn{};
    TOARec rq{};
    if (!SMOOTH && N > 0) vn = load_rec_v(recv, kb);
    if (SMOOTH && N > 0) rq = load_rec_vgpr(rb, 0);
    for (int k = 0; k < N; ++k) {
      TOARec r;
      if (SMOOTH) {
        r = rq;
        rq = load_rec_vgpr(rb, k + 1 < N ? k + 1 : k);
      } else {
        const RecVec v = vn;
        rec_keep(v);
        vn = load_rec_v(recv, kb + (k + 1 < N ? k + 1 : k));
        r = rec_fields(v);
      }
      if (kc == 0) {
        put_state(ckw, lane, st);
        ckw += kFields * kWave;
      }
      kc = kc + 1 == c1 ? 0 : kc + 1;
      double S, e, inv;
      fwd_step(st, r, L, S, e, inv);
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
      quad = fma(e * e, inv, quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    }
    double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
    if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
    if (stat) ll = -INFINITY;

    if (valid) {
      a.part[(int64_t)p * a.S + s] = ll;
      a.pstat[(int64_t)p * a.S + s] = stat;
    }
    // ---------------- reverse sweep
    const int nseg = (N + c1 - 1) / c1;
    if constexpr (SMOOTH) {
      SmoothSweep sw{&a, kb, s, valid, stat != 0, {0.0, 0.0, 0.0, 0.0},
                     Cov4{0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
      // the last TOA's smoothed moments are its filtered ones
      if (N > 0) sw.emit(N - 1, st);
      reverse_segments<false>(rb, ck, scr, L, N, c1, 0, nseg, 0, sw);
    } else {
      GradSweep sw{{0.0, 0.0, 0.0, 0.0}, Cov4{0, 0, 0, 0, 0, 0, 0, 0, 0, 0},
                   Grad{0, 0, 0, 0, 0, 0}};
      reverse_segments<false>(rb, ck, scr, L, N, c1, 0, nseg, 0, sw);
      Grad& G = sw.G;
      // the prior P0 = diag(s_r^2, s_f^2, v_r, v_c)
      G.v += sw.M.aa;
      G.vc += sw.M.gg;
      if (!valid) continue;
      double* g = a.gpart + (int64_t)p * 6 * a.S + s;
      if (a.model == 1) {
        g[0] = G.ss2 * 2.0 * kLn10 * L.ss2;  // log10 sigma_s
        g[a.S] = G.ef2 * 2.0 * t1;           // EFAC
      } else {
        g[0] = G.v * 2.0 * kLn10 * L.vr;                                // log10 sigma_red
        g[a.S] = kLn10 * (G.gam * L.gr - G.v * L.vr);                   // log10 gamma_red
        g[2 * a.S] = G.ef2 * 2.0 * t2;                                  // EFAC
        g[3 * a.S] = G.eq2 * 2.0 * kLn10 * L.equad2;                    // log10 EQUAD
        g[4 * a.S] = G.vc * 2.0 * kLn10 * L.vc;                         // log10 A
        g[5 * a.S] = G.vc * L.vc * (a.mc.log_fyr + a.mc.log_T - 1.0 / (t5 - 1.0));  // gamma
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Time-parallel form of the smoother (models 1, 2). In the modified
// Bryson-Frazier recursion (rev_bf) TOA k maps the information pair after
// it to the pair after TOA k - 1 by
//   lam <- A^T lam - F^T h e / S,   Lam <- A^T Lam A + (F^T h)(F^T h)^T / S,
//   A = (I - K h^T) F,
// affine in lam and a congruence plus a constant in Lam. A run of TOAs
// therefore maps the pair after its last TOA to the pair before its first by
//   lam <- U lam + phi,   Lam <- U Lam U^T + Om,   U = A_1^T ... A_n^T,
// and (U, phi, Om) accumulate along the forward pass: per TOA,
//   V = U F^T, v = V h, phi -= v e / S, Om += v v^T / S, U = V - v K^T.
// An item (64-sample tile, pulsar) is split into nch chunks of whole level-1
// segments (chunk c: segments c nseg / nch .. (c + 1) nseg / nch - 1).
// k_smooth_fwd_pc (one workgroup per item) runs the forward filter over the
// whole stream (log-likelihood, level-1 checkpoints, the summaries of
// chunks 1 .. nch - 1), chains the summaries from the last chunk back (the
// pair after the last TOA is zero) and stores the pair after the last TOA
// of every chunk but the last, and the final filtered state in the last
// chunk's place. k_smooth_rev then runs the checkpointed reverse sweep of
// every (item, chunk) unit independently, longest chunks first. An item's
// serial chain drops from a forward and a reverse pass over its N TOAs to a
// forward pass over N and a reverse pass over about N / nch. This form keeps
// a checkpoint before every fourth TOA (the level-1 stride is 4, a segment is
// one reverse piece), so the reverse sweep recomputes no segment and needs no
// level-2 scratch; the store takes 112 B per four TOAs and sample (model 4:
// 160 B).
constexpr int kSum = 30;  // a chunk summary: U (16, row major), phi (4), Om (10)

__host__ __device__ constexpr int si4(int i, int j) {
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}

// The chain of the chunk summaries of one item, from the last chunk back:
// the pair after the last TOA of chunk c - 1 goes to chunk c - 1's place
// (lam, then Lam in the order of a covariance); the pair after the last TOA
// is zero. The summaries are this wave's own writes.
__device__ __forceinline__ void smooth_chain(const AdjArgs& a, int64_t base, int nch, int lane) {
  double lam[4] = {0.0, 0.0, 0.0, 0.0}, Lam[10];
#pragma unroll
  for (int i = 0; i < 10; ++i) Lam[i] = 0.0;
  for (int c = nch - 1; c >= 1; --c) {
    const double* o = a.tpsum + (base + c) * kSum * kWave + lane;
    double Uc[4][4], T[4][4], nl[4];
#pragma unroll
    for (int i = 0; i < 16; ++i) Uc[i / 4][i % 4] = o[i * kWave];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      double acc = o[(16 + i) * kWave];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        acc = fma(Uc[i][q], lam[q], acc);
        double tq = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) tq = fma(Uc[i][l], Lam[si4(l, q)], tq);
        T[i][q] = tq;
      }
      nl[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      lam[i] = nl[i];
#pragma unroll
      for (int q = 0; q <= i; ++q) {
        double acc = o[(20 + si4(i, q)) * kWave];
#pragma unroll
        for (int l = 0; l < 4; ++l) acc = fma(T[i][l], Uc[q][l], acc);
        Lam[si4(i, q)] = acc;
      }
    }
    put_state(a.tpadj + (base + c - 1) * kFields * kWave, lane,
              State{lam[0], lam[1], lam[2], lam[3],
                    Cov4{Lam[0], Lam[1], Lam[2], Lam[3], Lam[4], Lam[5], Lam[6], Lam[7], Lam[8],
                         Lam[9]}});
  }
}

// Forward pass of the time-parallel smoother: one workgroup of two waves per
// item. Wave 0 runs the filter (log-likelihood, level-1 checkpoints, final
// state) and hands, per TOA, the gain, e, 1/S, the red decay, dt and the
// common decay (kSmVals values per lane) to wave 1 through a double-buffered
// LDS ring of kSmSteps TOAs per buffer; wave 1 accumulates the chunk
// summaries one block behind and chains them. Barrier b separates wave 0's
// writes of block b from wave 1's reads of it and wave 1's reads of block
// b - 1 from wave 0's rewrite of that buffer; both waves execute nblk + 1
// barriers. The filter's serial chain carries no summary arithmetic, which
// lets its blocks be straight-line code (with the summaries inline, the
// scheduler's overlap of four steps ran out of registers).
constexpr int kSmSteps = 4, kSmVals = 9;

__global__ void __launch_bounds__(2 * kWave) k_smooth_fwd_pc(AdjArgs a) {
  __shared__ double s_ring[2 * kSmSteps * kSmVals * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int it = blockIdx.x;
  const int tile = a.items[2 * it];
  const int p = a.items[2 * it + 1];
  const int64_t s_raw = (int64_t)tile * kWave + lane;
  const bool valid = s_raw < a.S;
  const int64_t s = valid ? s_raw : a.S - 1;
  const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
  const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
  const int c1 = a.c1[p];
  const int nseg = (N + c1 - 1) / c1;
  const int nch = __builtin_amdgcn_readfirstlane(a.tp_item[2 * it]);
  const int64_t base = __builtin_amdgcn_readfirstlane(a.tp_item[2 * it + 1]);
  const int nblk = (N + kSmSteps - 1) / kSmSteps;
  double* ring = s_ring + lane;  // value v of step j of buffer b at ((b kSmSteps + j) kSmVals + v) kWave

  if (wave == 0) {
    double* ckw = a.ckpt + ((int64_t)tile * a.tot_seg + a.seg_base[p]) * kFields * kWave;
    const LaneTheta th = lane_theta(a, p, s);
    const LaneP L = th.L;
    const RecBuf rb = rec_buffer(a.rec + kb, N);
    State st{0.0, 0.0, 0.0, 0.0,
             Cov4{a.mc.s_r2, 0.0, a.mc.s_f2, 0.0, 0.0, L.vr, 0.0, 0.0, 0.0, L.vc}};
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = th.pnf ? kPNF : 0;
    // one TOA: filter step, hand-over values, log-likelihood terms
    auto step = [&](const TOARec& r, double* rv) {
      double S, e, inv, kk[4], ph;
      fwd_step(st, r, L, S, e, inv, kk, ph);
      rv[0 * kWave] = kk[0];
      rv[1 * kWave] = kk[1];
      rv[2 * kWave] = kk[2];
      rv[3 * kWave] = kk[3];
      rv[4 * kWave] = e;
      rv[5 * kWave] = inv;
      rv[6 * kWave] = ph;
      rv[7 * kWave] = r.dt;
      rv[8 * kWave] = r.phc;
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
      quad = fma(e * e, inv, quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    };
    // the records of block blk + 1 are fetched while block blk is filtered
    // (indices clamped to the last TOA); a full block is straight-line code,
    // so the steps' record-only work (the decays) overlaps the previous
    // step's chain. Level-1 segments start at block starts (c1 is a
    // multiple of kSmSteps).
    TOARec q[kSmSteps], qn[kSmSteps];
#pragma unroll
    for (int j = 0; j < kSmSteps; ++j) q[j] = load_rec_vgpr(rb, j < N ? j : (N > 0 ? N - 1 : 0));
    for (int blk = 0; blk <= nblk; ++blk) {
      double* rbuf = ring + (blk & 1) * kSmSteps * kSmVals * kWave;
      if (blk < nblk) {
        const int k0 = blk * kSmSteps;
#pragma unroll
        for (int j = 0; j < kSmSteps; ++j) {
          const int kn = k0 + kSmSteps + j;
          qn[j] = load_rec_vgpr(rb, kn < N ? kn : N - 1);
        }
        if (k0 % c1 == 0) put_state(ckw + (int64_t)(k0 / c1) * kFields * kWave, lane, st);
        if (k0 + kSmSteps <= N) {
#pragma unroll
          for (int j = 0; j < kSmSteps; ++j) step(q[j], rbuf + j * kSmVals * kWave);
        } else {
          for (int j = 0; j < N - k0; ++j) {
            // the tail: at most kSmSteps - 1 steps, records selected by index
            const TOARec r = j == 0 ? q[0] : (j == 1 ? q[1] : q[2]);
            step(r, rbuf + j * kSmVals * kWave);
          }
        }
#pragma unroll
        for (int j = 0; j < kSmSteps; ++j) q[j] = qn[j];
      }
      __syncthreads();
    }
    double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
    if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
    if (stat) ll = -INFINITY;
    if (valid) {
      a.part[(int64_t)p * a.S + s] = ll;
      a.pstat[(int64_t)p * a.S + s] = stat;
    }
    put_state(a.tpadj + (base + nch - 1) * kFields * kWave, lane, st);
  } else {
    // chunk summaries, one block behind the filter
    double U[4][4], phi[4], Om[10];
    auto reset = [&]() {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
#pragma unroll
        for (int q = 0; q < 4; ++q) U[i][q] = i == q ? 1.0 : 0.0;
        phi[i] = 0.0;
      }
#pragma unroll
      for (int i = 0; i < 10; ++i) Om[i] = 0.0;
    };
    reset();
    int c = 0;  // chunk of the next TOA and its end
    int ec = (nseg / nch) * c1 < N ? (nseg / nch) * c1 : N;
    for (int blk = 0; blk <= nblk; ++blk) {
      if (blk > 0) {
        const double* rbuf = ring + ((blk - 1) & 1) * kSmSteps * kSmVals * kWave;
#pragma unroll 1
        for (int j = 0; j < kSmSteps; ++j) {
          const int k = (blk - 1) * kSmSteps + j;
          if (k >= N) break;
          if (c > 0) {
            const double* rv = rbuf + j * kSmVals * kWave;
            const double kk[4] = {rv[0 * kWave], rv[1 * kWave], rv[2 * kWave], rv[3 * kWave]};
            const double e = rv[4 * kWave], inv = rv[5 * kWave], ph = rv[6 * kWave];
            const double dt = rv[7 * kWave], phc = rv[8 * kWave];
            const double ei = -e * inv;
            double V[4][4], v[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              V[i][0] = fma(dt, U[i][1], U[i][0]);
              V[i][1] = U[i][1];
              V[i][2] = ph * U[i][2];
              V[i][3] = phc * U[i][3];
              v[i] = V[i][0] + V[i][2] + V[i][3];
              phi[i] = fma(v[i], ei, phi[i]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const double vs = v[i] * inv;
#pragma unroll
              for (int q = 0; q <= i; ++q) Om[si4(i, q)] = fma(vs, v[q], Om[si4(i, q)]);
#pragma unroll
              for (int q = 0; q < 4; ++q) U[i][q] = fma(-v[i], kk[q], V[i][q]);
            }
          }
          if (k + 1 == ec) {
            if (c > 0) {
              double* o = a.tpsum + (base + c) * kSum * kWave + lane;
#pragma unroll
              for (int i = 0; i < 16; ++i) o[i * kWave] = U[i / 4][i % 4];
#pragma unroll
              for (int i = 0; i < 4; ++i) o[(16 + i) * kWave] = phi[i];
#pragma unroll
              for (int i = 0; i < 10; ++i) o[(20 + i) * kWave] = Om[i];
            }
            reset();
            ++c;
            const int sh = (c + 1) * nseg / nch;
            ec = sh * c1 < N ? sh * c1 : N;
          }
        }
      }
      __syncthreads();
    }
    smooth_chain(a, base, nch, lane);
  }
}

// Reverse sweep of the time-parallel smoother: one (item, chunk) unit per
// wave from a queue ordered longest chunk first; two waves per SIMD.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_smooth_rev(AdjArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int gwave = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave));
  double* scr = a.scratch + (int64_t)gwave * a.max_sub * kFields * kWave;
  for (;;) {
    int v = 0;
    if (lane == 0) v = atomicAdd(a.counter, 1);
    const int u = __builtin_amdgcn_readfirstlane(v);
    if (u >= a.n_units) break;
    const int it = a.tp_units[2 * u];
    const int c = a.tp_units[2 * u + 1];
    const int tile = a.items[2 * it];
    const int p = a.items[2 * it + 1];
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
    const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
    const int c1 = a.c1[p];
    const int nseg = (N + c1 - 1) / c1;
    const int nch = a.tp_item[2 * it];
    const int64_t base = a.tp_item[2 * it + 1];
    const int sg_lo = c * nseg / nch, sg_hi = (c + 1) * nseg / nch;
    const int k0 = sg_lo * c1, k1 = sg_hi * c1 < N ? sg_hi * c1 : N;
    const double* ck = a.ckpt + ((int64_t)tile * a.tot_seg + a.seg_base[p]) * kFields * kWave;
    const LaneP L = lane_theta(a, p, s).L;
    const RecBuf rb = rec_buffer(a.rec + kb, N);
    const bool bad = a.pstat[(int64_t)p * a.S + s] != 0;
    SmoothSweep sw{&a, kb, s, valid, bad, {0.0, 0.0, 0.0, 0.0},
                   Cov4{0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
    State fend;  // the filtered state after this chunk's last TOA
    const State slot = get_state(a.tpadj + (base + c) * kFields * kWave, lane);
    if (c == nch - 1) {
      fend = slot;
    } else {
      sw.lam[0] = slot.xr;
      sw.lam[1] = slot.xf;
      sw.lam[2] = slot.xa;
      sw.lam[3] = slot.xg;
      sw.Lm = slot.P;
      fend = get_state(ck + (int64_t)sg_hi * kFields * kWave, lane);
    }
    if (k1 > k0) sw.emit(k1 - 1, fend);
    reverse_segments<true>(rb, ck, scr, L, N, c1, sg_lo, sg_hi, k0, sw);
  }
}

// ---------------------------------------------------------------------------
// Forward-mode (tangent) gradient: the same recursion differentiated along a
// parameter direction d, carried alongside the filter. With the base step's
// F, u, S, K, e and the tangents (dx, dP) of the posterior:
//   dx- = F dx + dF x,  dP- = F dP F^T + dF P F^T + F P dF^T + dQ,
//   de = -h.dx-,  du = dP- h,  dS = h.du + dR,  dK = (du - K dS) / S,
//   dx+ = dx- + dK e + K de,
//   dP+ = dP- - du K^T - K du^T + dS K K^T  (the Joseph update's tangent at
//         the optimal gain; its dK terms cancel because u = S K),
//   dl += -1/2 (dS / S (1 - e^2 / S) + 2 e de / S).
// The parameters enter through the red-OU decay phi (its rate), the OU and
// spin noise, R and the prior. Each wave carries ND of the model's
// directions (6 for model 2: log10 sigma_red, log10 gamma_red, EFAC,
// log10 EQUAD, log10 A, gamma; 2 for model 1: log10 sigma_s, EFAC); a
// (tile, pulsar) item is split over 6 / ND waves, trading repeated base
// filters for shorter serial chains. One pass, no checkpoints.
struct TanArgs {
  const TOARec* rec;
  const double* chrom;   // [N] chromatic factor per TOA (model 4)
  const int64_t* off;
  const double* theta;
  const int32_t* col;
  const double* fixed;
  const int32_t* items;  // (tile, pulsar), longest first
  // k_tangent work units, longest first: (item index, group | ND << 8)
  const int32_t* units;
  int32_t n_units;
  int32_t* counter;
  double* part;          // [P*S]
  int32_t* pstat;        // [P*S]
  double* gpart;         // [P * 6 * S] (model 4: [P * 8 * S])
  int64_t S;
  int32_t D, P, n_items;
  ModelConst mc;
};

__device__ __forceinline__ double tprm(const TanArgs& a, int c, int64_t s) {
  const int j = a.col[c];
  return j >= 0 ? a.theta[s * a.D + j] : a.fixed[c];
}

struct Tan {
  double xr, xf, xa, xg;
  Cov4 P;
  double dl;
};

// One work unit: the base filter of (tile, pulsar) and its directions
// grp * ND .. grp * ND + ND - 1 (group 0 also writes the log-likelihood).
template <int MODEL, int ND>
__device__ __forceinline__ void tangent_unit(const TanArgs& a, const int lane, const int tile,
                                             const int p, const int grp) {
  const RecPtr rec = (RecPtr)a.rec;
  {
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
    const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;

    // parameters, base constants and each direction's sources
    double gr = 1.0, vr = 0.0, vc = 0.0, efac2, equad2 = 0.0, ss2;
    double sv[ND], sg[ND], sc[ND], sr2[ND], sq2[ND], ss[ND];
    bool pnf;
    double t1 = 0.0, t2 = 0.0, t5 = 2.0;
    if (MODEL == 1) {
      const double t0 = tprm(a, 0, s);
      t1 = tprm(a, 1, s);
      pnf = !(finite_d(t0) && finite_d(t1));
      const double sgs = exp10(t0);
      ss2 = sgs * sgs;
      efac2 = t1 * t1;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        const int dir = grp * ND + j;
        sv[j] = sg[j] = sc[j] = sq2[j] = 0.0;
        ss[j] = dir == 0 ? 2.0 * kLn10 * ss2 : 0.0;
        sr2[j] = dir == 1 ? 2.0 * t1 : 0.0;
      }
    } else {
      const int c0 = 4 * p, cc = 4 * a.P;
      const double t0 = tprm(a, c0, s);
      t1 = tprm(a, c0 + 1, s);
      t2 = tprm(a, c0 + 2, s);
      const double t3 = tprm(a, c0 + 3, s), t4 = tprm(a, cc, s);
      t5 = tprm(a, cc + 1, s);
      pnf = !(finite_d(t0) && finite_d(t1) && finite_d(t2) && finite_d(t3) && finite_d(t4) &&
              finite_d(t5));
      gr = exp10(t1);
      const double sr = exp10(t0), eq = exp10(t3);
      vr = sr * sr / (2.0 * gr);
      const double gm1 = t5 - 1.0;
      vc = exp(2.0 * kLn10 * t4 + (t5 - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
           (12.0 * kPi * kPi * gm1);
      efac2 = t2 * t2;
      equad2 = eq * eq;
      ss2 = a.mc.ss2;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        const int dir = grp * ND + j;
        sv[j] = dir == 0 ? 2.0 * kLn10 * vr : (dir == 1 ? -kLn10 * vr : 0.0);
        sg[j] = dir == 1 ? kLn10 * gr : 0.0;
        sr2[j] = dir == 2 ? 2.0 * t2 : 0.0;
        sq2[j] = dir == 3 ? 2.0 * kLn10 * equad2 : 0.0;
        sc[j] = dir == 4 ? 2.0 * kLn10 * vc
                         : (dir == 5 ? vc * (a.mc.log_fyr + a.mc.log_T - 1.0 / gm1) : 0.0);
        ss[j] = 0.0;
      }
    }

    // base filter state and the tangents (prior P0 = diag(s_r^2, s_f^2, v_r, v_c))
    State st{0.0, 0.0, 0.0, 0.0,
             Cov4{a.mc.s_r2, 0.0, a.mc.s_f2, 0.0, 0.0, vr, 0.0, 0.0, 0.0, vc}};
    Tan tg[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j)
      tg[j] = Tan{0.0, 0.0, 0.0, 0.0, Cov4{0, 0, 0, 0, 0, sv[j], 0, 0, 0, sc[j]}, 0.0};
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = pnf ? kPNF : 0;

    // Two records in flight: step k waits for the record of step k + 1,
    // computes its red decay and fetches the record of step k + 2 (index
    // clamped to the pulsar's last TOA). ss2 and the top expm1 coefficient
    // are held in VGPRs (FP64 ops with a per-TOA SGPR operand need no copy).
    ss2 = in_vgpr(ss2);
    const double c13 = in_vgpr(kExpm1Coef[11]);
    TOARec r1{}, r2{};
    double em1 = 0.0;
    if (N > 0) {
      r1 = load_rec(rec, kb);
      r2 = load_rec(rec, kb + (N > 1 ? 1 : 0));
      em1 = expm1_v(-gr * r1.dt, c13);
    }
    for (int k = 0; k < N; ++k) {
      const TOARec r = r1;
      const double em = em1;
      r1 = r2;
      sgpr_ready(r1.dt);
      r2 = load_rec(rec, kb + (k < N - 2 ? k + 2 : N - 1));
      em1 = expm1_v(-gr * r1.dt, c13);
      const double dt = r.dt, phc = r.phc;
      const double ph = 1.0 + em, qfac = -em * (2.0 + em);
      // base predict
      const Cov4& Q0 = st.P;
      const double fpra = fma(dt, Q0.fa, Q0.ra), fpfa = Q0.fa, fpaa = ph * Q0.aa,
                   fpga = phc * Q0.ag;  // (F P)_{., a} of the posterior
      const double xa0 = st.xa;
      Cov4 Pm;
      const double prf1 = fma(dt, Q0.ff, Q0.rf);
      Pm.rr = fma(dt, Q0.rf + prf1, Q0.rr) + ss2 * r.h3;
      Pm.rf = prf1 + ss2 * r.h2;
      Pm.ff = Q0.ff + ss2 * dt;
      Pm.ra = ph * fpra;
      Pm.fa = ph * fpfa;
      Pm.aa = fma(ph * ph, Q0.aa, vr * qfac);
      Pm.rg = phc * fma(dt, Q0.fg, Q0.rg);
      Pm.fg = phc * Q0.fg;
      Pm.ag = (ph * phc) * Q0.ag;
      Pm.gg = fma(phc * phc, Q0.gg, vc * r.qcu);
      const double xr = fma(dt, st.xf, st.xr), xf = st.xf, xa = ph * st.xa, xg = phc * st.xg;
      const double e = r.y - (xr + xa + xg);
      const double ur = Pm.rr + Pm.ra + Pm.rg, uf = Pm.rf + Pm.fa + Pm.fg;
      const double ua = Pm.ra + Pm.aa + Pm.ag, ug = Pm.rg + Pm.ag + Pm.gg;
      const double S = (ur + ua + ug) + fma(efac2, r.s2, equad2);
      const double inv = rcp_nr(S);
      const double kr = ur * inv, kf = uf * inv, ka = ua * inv, kg = ug * inv;
      const double ei = e * inv, hS = inv * fma(-e, ei, 1.0);  // (1 - e^2/S)/S
      // tangents
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        Tan& d = tg[j];
        const double dph = -dt * ph * sg[j];
        const double dqa = fma(sv[j], qfac, -2.0 * vr * ph * dph);
        // dx-
        const double dxr = fma(dt, d.xf, d.xr), dxf = d.xf;
        const double dxa = fma(ph, d.xa, dph * xa0), dxg = phc * d.xg;
        // dP- = F dP F^T + (dF P F^T + F P dF^T) + dQ
        const Cov4& D0 = d.P;
        Cov4 Dm;
        const double drf1 = fma(dt, D0.ff, D0.rf);
        Dm.rr = fma(dt, D0.rf + drf1, D0.rr) + ss[j] * r.h3;
        Dm.rf = drf1 + ss[j] * r.h2;
        Dm.ff = fma(ss[j], dt, D0.ff);
        Dm.ra = fma(ph, fma(dt, D0.fa, D0.ra), dph * fpra);
        Dm.fa = fma(ph, D0.fa, dph * fpfa);
        Dm.aa = fma(ph * ph, D0.aa, fma(2.0 * dph, fpaa, dqa));
        Dm.rg = phc * fma(dt, D0.fg, D0.rg);
        Dm.fg = phc * D0.fg;
        Dm.ag = fma(ph * phc, D0.ag, dph * fpga);
        Dm.gg = fma(phc * phc, D0.gg, sc[j] * r.qcu);
        // update
        const double de = -(dxr + dxa + dxg);
        const double dur = Dm.rr + Dm.ra + Dm.rg, duf = Dm.rf + Dm.fa + Dm.fg;
        const double dua = Dm.ra + Dm.aa + Dm.ag, dug = Dm.rg + Dm.ag + Dm.gg;
        const double dS = (dur + dua + dug) + fma(sr2[j], r.s2, sq2[j]);
        // x+ = x- + K e and P+ = P- - u u^T / S differentiated with no dK:
        // dx+ = dx- + du e / S + K (de - dS e / S), dP+ = dP- - w K^T - K w^T
        // with w = du - dS K / 2
        const double z = fma(-dS, ei, de), hd = -0.5 * dS;
        d.xr = fma(dur, ei, fma(kr, z, dxr));
        d.xf = fma(duf, ei, fma(kf, z, dxf));
        d.xa = fma(dua, ei, fma(ka, z, dxa));
        d.xg = fma(dug, ei, fma(kg, z, dxg));
        const double wr = fma(hd, kr, dur), wf = fma(hd, kf, duf);
        const double wa = fma(hd, ka, dua), wg = fma(hd, kg, dug);
#define TAN_UPD(dp, ki, wi, kj, wj) dp = fma(-(wi), kj, fma(-(ki), wj, dp))
        TAN_UPD(Dm.rr, kr, wr, kr, wr);
        TAN_UPD(Dm.rf, kr, wr, kf, wf);
        TAN_UPD(Dm.ff, kf, wf, kf, wf);
        TAN_UPD(Dm.ra, kr, wr, ka, wa);
        TAN_UPD(Dm.fa, kf, wf, ka, wa);
        TAN_UPD(Dm.aa, ka, wa, ka, wa);
        TAN_UPD(Dm.rg, kr, wr, kg, wg);
        TAN_UPD(Dm.fg, kf, wf, kg, wg);
        TAN_UPD(Dm.ag, ka, wa, kg, wg);
        TAN_UPD(Dm.gg, kg, wg, kg, wg);
#undef TAN_UPD
        d.P = Dm;
        d.dl = fma(-0.5, fma(dS, hS, 2.0 * ei * de), d.dl);
      }
      // base update (Joseph form, as the likelihood kernel)
      st.xr = fma(kr, e, xr);
      st.xf = fma(kf, e, xf);
      st.xa = fma(ka, e, xa);
      st.xg = fma(kg, e, xg);
      const double dr = fma(S, kr, -ur), df = fma(S, kf, -uf);
      const double da = fma(S, ka, -ua), dg = fma(S, kg, -ug);
      JOSEPH(Pm.rr, kr, ur, dr, kr);
      JOSEPH(Pm.rf, kr, uf, dr, kf);
      JOSEPH(Pm.ff, kf, uf, df, kf);
      JOSEPH(Pm.ra, kr, ua, dr, ka);
      JOSEPH(Pm.fa, kf, ua, df, ka);
      JOSEPH(Pm.aa, ka, ua, da, ka);
      JOSEPH(Pm.rg, kr, ug, dr, kg);
      JOSEPH(Pm.fg, kf, ug, df, kg);
      JOSEPH(Pm.ag, ka, ug, da, kg);
      JOSEPH(Pm.gg, kg, ug, dg, kg);
      st.P = Pm;
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
      quad = fma(e, ei, quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    }
    if (valid) {
      if (grp == 0) {
        double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
        if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
        a.part[(int64_t)p * a.S + s] = stat ? -INFINITY : ll;
        a.pstat[(int64_t)p * a.S + s] = stat;
      }
      double* g = a.gpart + (int64_t)p * 6 * a.S + s;
#pragma unroll
      for (int j = 0; j < ND; ++j) g[(int64_t)(grp * ND + j) * a.S] = tg[j].dl;
    }
  }
}

// Work units from a longest-first queue. A unit carries its own directions
// per wave, NDA or NDB: a split can give the longest pulsars fewer
// directions per wave (more waves, shorter serial chains) and the others
// more (fewer repeated base filters). NDA == NDB is a uniform split.
template <int MODEL, int NDA, int NDB>
__global__ void __launch_bounds__(256) k_tangent(TanArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  for (;;) {
    int v = 0;
    if (lane == 0) v = atomicAdd(a.counter, 1);
    const int u = __builtin_amdgcn_readfirstlane(v);
    if (u >= a.n_units) break;
    const int item = a.units[2 * u], code = a.units[2 * u + 1];
    const int grp = code & 0xff;
    const int tile = a.items[2 * item];
    const int p = a.items[2 * item + 1];
    if (NDA == NDB || (code >> 8) == NDA)
      tangent_unit<MODEL, NDA>(a, lane, tile, p, grp);
    else
      tangent_unit<MODEL, NDB>(a, lane, tile, p, grp);
  }
}

// Producer/consumer form of the model-2 tangent sweep: one workgroup of
// 1 + ceil(5 / NDC) waves per (64-sample tile, pulsar) item. Wave 0 runs the
// base filter once and hands, for every TOA, what the differentiated step
// needs from it (the red decay, the previous posterior's xa and a column,
// the gain, the innovation and 1/S: kPcVals values per lane) to the other
// waves through a double-buffered ring in LDS of kPcSteps TOAs per buffer;
// the other waves carry NDC each of five directions: the pulsar's four and
// the common variance, from which the log10 A and gamma derivatives both
// follow (NDC = 2: the red rate alone, then (log10 sigma_red, common
// variance) and (EFAC, EQUAD)). The base filter then runs once per item instead
// of once per direction group, and the serial chain of a TOA is the longer
// of the base step and an NDC-direction tangent step instead of their sum.
// Barrier b of the item separates the producer's writes of block b from the
// consumers' reads of it (in the next round) and their reads of block b - 1
// from the producer's rewrite of that buffer; every wave executes nblk + 1
// barriers. Each step differentiates the base step as tangent_unit does,
// with the update written in fewer operations (tan_dir_step).
constexpr int kPcSteps = 4;
constexpr int kPcVals = 12;

// What a consumer wave of k_tangent_pc needs from its workgroup.
struct TanPcCtx {
  const TanArgs* a;
  const double* ring;
  int N, nblk, kb, p;
  int64_t s;
  bool valid;
  double vr, gr, vc, t2, equad2, gm1;
};

// The per-TOA values shared by a consumer's directions.
struct TanPcTOA {
  double dt, phc, qcu, s2, ph, ph2, qfac, xa0, fpra, fpfa, fpaa, fpga;
  double kr, kf, ka, kg, e, inv, ei, hS;
};

// One TOA of model-2 tangent direction DIR (0 log10 sigma_red, 1
// log10 gamma_red, 2 EFAC, 3 log10 EQUAD, 4 ln of the common variance) with
// its source src (the derivative of the red variance, of the white
// variance's EFAC or EQUAD part, or of the common variance) and, for DIR 1,
// srate (of the red rate). Terms whose source is zero for DIR are left out
// at compile time: they add exact zeros. log10 A and gamma enter the filter
// only through the common variance, so both of their derivatives are
// multiples of direction 4's (see tangent_pc_consumer).
template <int DIR>
__device__ __forceinline__ void tan_dir_step(Tan& d, double src, double srate,
                                             const TanPcTOA& c, double vr) {
  constexpr bool HV = DIR <= 1, HG = DIR == 1, HR = DIR == 2, HQ = DIR == 3, HC = DIR >= 4;
  const double dt = c.dt, ph = c.ph, phc = c.phc;
  const double dph = HG ? -dt * ph * srate : 0.0;
  const double dxr = fma(dt, d.xf, d.xr), dxf = d.xf;
  const double dxa = HG ? fma(ph, d.xa, dph * c.xa0) : ph * d.xa, dxg = phc * d.xg;
  const Cov4& D0 = d.P;
  Cov4 Dm;
  const double drf1 = fma(dt, D0.ff, D0.rf);
  Dm.rr = fma(dt, D0.rf + drf1, D0.rr);
  Dm.rf = drf1;
  Dm.ff = D0.ff;
  const double ra0 = fma(dt, D0.fa, D0.ra);
  Dm.ra = HG ? fma(ph, ra0, dph * c.fpra) : ph * ra0;
  Dm.fa = HG ? fma(ph, D0.fa, dph * c.fpfa) : ph * D0.fa;
  if constexpr (HG) {
    const double dqa = fma(src, c.qfac, -2.0 * vr * ph * dph);
    Dm.aa = fma(c.ph2, D0.aa, fma(2.0 * dph, c.fpaa, dqa));
  } else if constexpr (HV) {
    Dm.aa = fma(c.ph2, D0.aa, src * c.qfac);
  } else {
    Dm.aa = c.ph2 * D0.aa;
  }
  Dm.rg = phc * fma(dt, D0.fg, D0.rg);
  Dm.fg = phc * D0.fg;
  Dm.ag = HG ? fma(ph * phc, D0.ag, dph * c.fpga) : (ph * phc) * D0.ag;
  Dm.gg = HC ? fma(phc * phc, D0.gg, src * c.qcu) : (phc * phc) * D0.gg;
  const double de = -(dxr + dxa + dxg);
  const double dur = Dm.rr + Dm.ra + Dm.rg, duf = Dm.rf + Dm.fa + Dm.fg;
  const double dua = Dm.ra + Dm.aa + Dm.ag, dug = Dm.rg + Dm.ag + Dm.gg;
  double dS = (dur + dua + dug);
  if constexpr (HR) dS += src * c.s2;
  if constexpr (HQ) dS += src;
  const double kr = c.kr, kf = c.kf, ka = c.ka, kg = c.kg, ei = c.ei;
  // x+ = x- + k e with k = u / S, so dx+ = dx- + du e / S + k (de - dS e / S)
  const double z = fma(-dS, ei, de);
  d.xr = fma(dur, ei, fma(kr, z, dxr));
  d.xf = fma(duf, ei, fma(kf, z, dxf));
  d.xa = fma(dua, ei, fma(ka, z, dxa));
  d.xg = fma(dug, ei, fma(kg, z, dxg));
  // P+ = P- - u u^T / S, so dP+ = dP- - du k^T - k du^T + dS k k^T, which is
  // dP- - w k^T - k w^T with w = du - dS k / 2
  const double hd = -0.5 * dS;
  const double wr = fma(hd, kr, dur), wf = fma(hd, kf, duf);
  const double wa = fma(hd, ka, dua), wg = fma(hd, kg, dug);
#define TAN_UPD(dp, ki, wi, kj, wj) dp = fma(-(wi), kj, fma(-(ki), wj, dp))
  TAN_UPD(Dm.rr, kr, wr, kr, wr);
  TAN_UPD(Dm.rf, kr, wr, kf, wf);
  TAN_UPD(Dm.ff, kf, wf, kf, wf);
  TAN_UPD(Dm.ra, kr, wr, ka, wa);
  TAN_UPD(Dm.fa, kf, wf, ka, wa);
  TAN_UPD(Dm.aa, ka, wa, ka, wa);
  TAN_UPD(Dm.rg, kr, wr, kg, wg);
  TAN_UPD(Dm.fg, kf, wf, kg, wg);
  TAN_UPD(Dm.ag, ka, wa, kg, wg);
  TAN_UPD(Dm.gg, kg, wg, kg, wg);
#undef TAN_UPD
  d.P = Dm;
  d.dl = fma(-0.5, fma(dS, c.hS, 2.0 * ei * de), d.dl);
}

// The source of direction DIR for this lane (see tan_dir_step) and, for the
// red rate, its second source.
template <int DIR>
__device__ __forceinline__ double tan_src(const TanPcCtx& c) {
  if constexpr (DIR == 0) return 2.0 * kLn10 * c.vr;
  if constexpr (DIR == 1) return -kLn10 * c.vr;
  if constexpr (DIR == 2) return 2.0 * c.t2;
  if constexpr (DIR == 3) return 2.0 * kLn10 * c.equad2;
  return c.vc;
}

// A consumer wave of k_tangent_pc carrying directions D0 and D1 (D1 < 0:
// D0 alone), one ring block behind the base filter wave.
template <int D0, int D1>
__device__ __forceinline__ void tangent_pc_consumer(const TanPcCtx& c) {
  const TanArgs& a = *c.a;
  const RecPtr rec = (RecPtr)a.rec;
  const double src0 = tan_src<D0>(c), srate0 = D0 == 1 ? kLn10 * c.gr : 0.0;
  const double src1 = tan_src<(D1 < 0 ? 0 : D1)>(c), srate1 = D1 == 1 ? kLn10 * c.gr : 0.0;
  // the prior's derivative: the red variance (directions 0, 1) and the
  // common variance (4) of P0
  auto prior = [](int dir, double src) {
    const double v = dir <= 1 ? src : 0.0, cc = dir >= 4 ? src : 0.0;
    return Tan{0.0, 0.0, 0.0, 0.0, Cov4{0, 0, 0, 0, 0, v, 0, 0, 0, cc}, 0.0};
  };
  Tan t0 = prior(D0, src0), t1 = prior(D1, src1);
  for (int blk = 0; blk <= c.nblk; ++blk) {
    const double* rb = c.ring + ((blk - 1) & 1) * kPcSteps * kPcVals * kWave;
#pragma unroll 1
    for (int jj = 0; jj < kPcSteps && blk > 0; ++jj) {
      const int k = (blk - 1) * kPcSteps + jj;
      if (k >= c.N) break;
      const TOARec r = load_rec(rec, c.kb + k);
      const double* rv = rb + jj * kPcVals * kWave;
      TanPcTOA o;
      const double em = rv[0 * kWave];
      o.xa0 = rv[1 * kWave];
      const double qra = rv[2 * kWave], qfa = rv[3 * kWave], qaa = rv[4 * kWave],
                   qag = rv[5 * kWave];
      o.kr = rv[6 * kWave];
      o.kf = rv[7 * kWave];
      o.ka = rv[8 * kWave];
      o.kg = rv[9 * kWave];
      o.e = rv[10 * kWave];
      o.inv = rv[11 * kWave];
      o.dt = r.dt;
      o.phc = r.phc;
      o.qcu = r.qcu;
      o.s2 = r.s2;
      o.ph = 1.0 + em;
      o.ph2 = o.ph * o.ph;
      o.qfac = -em * (2.0 + em);
      o.fpra = fma(o.dt, qfa, qra);
      o.fpfa = qfa;
      o.fpaa = o.ph * qaa;
      o.fpga = o.phc * qag;
      o.ei = o.e * o.inv;
      o.hS = o.inv * fma(-o.e, o.ei, 1.0);
      tan_dir_step<D0>(t0, src0, srate0, o, c.vr);
      if constexpr (D1 >= 0) tan_dir_step<(D1 < 0 ? 0 : D1)>(t1, src1, srate1, o, c.vr);
    }
    __syncthreads();
  }
  if (c.valid) {
    double* g = a.gpart + (int64_t)c.p * 6 * a.S + c.s;
    auto put = [&](int dir, double dl) {
      if (dir == 4) {
        // v_c = A^2 f_yr^(gamma - 3) T^(gamma - 1) / (12 pi^2 (gamma - 1)):
        // d ln v_c / d log10 A = 2 ln 10, d ln v_c / d gamma =
        // ln f_yr + ln T - 1 / (gamma - 1)
        g[4 * a.S] = 2.0 * kLn10 * dl;
        g[5 * a.S] = (a.mc.log_fyr + a.mc.log_T - 1.0 / c.gm1) * dl;
      } else {
        g[(int64_t)dir * a.S] = dl;
      }
    };
    put(D0, t0.dl);
    if constexpr (D1 >= 0) put(D1, t1.dl);
  }
}

template <int NDC>
__global__ void __launch_bounds__(kWave * (NDC == 2 ? 4 : 6)) k_tangent_pc(TanArgs a) {
  __shared__ double s_ring[2 * kPcSteps * kPcVals * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const RecPtr rec = (RecPtr)a.rec;
  const int item = blockIdx.x;
  const int tile = a.items[2 * item], p = a.items[2 * item + 1];
  const int64_t s_raw = (int64_t)tile * kWave + lane;
  const bool valid = s_raw < a.S;
  const int64_t s = valid ? s_raw : a.S - 1;
  const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
  const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
  const int nblk = (N + kPcSteps - 1) / kPcSteps;
  double* ring = s_ring + lane;  // value v of step j of buffer b at ((b kPcSteps + j) kPcVals + v) kWave

  const int c0 = 4 * p, cc = 4 * a.P;
  const double t0 = tprm(a, c0, s), t1 = tprm(a, c0 + 1, s), t2 = tprm(a, c0 + 2, s);
  const double t3 = tprm(a, c0 + 3, s), t4 = tprm(a, cc, s), t5 = tprm(a, cc + 1, s);
  const double gr = exp10(t1);
  const double sr = exp10(t0), eq = exp10(t3);
  const double vr = sr * sr / (2.0 * gr);
  const double gm1 = t5 - 1.0;
  const double vc = exp(2.0 * kLn10 * t4 + (t5 - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
                    (12.0 * kPi * kPi * gm1);

  if (wave == 0) {
    // ---- the base filter (the base part of tangent_unit, model 2)
    const bool pnf = !(finite_d(t0) && finite_d(t1) && finite_d(t2) && finite_d(t3) &&
                       finite_d(t4) && finite_d(t5));
    const double efac2 = t2 * t2, equad2 = eq * eq;
    const double ss2 = in_vgpr(a.mc.ss2);
    State st{0.0, 0.0, 0.0, 0.0,
             Cov4{a.mc.s_r2, 0.0, a.mc.s_f2, 0.0, 0.0, vr, 0.0, 0.0, 0.0, vc}};
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = pnf ? kPNF : 0;
    const double c13 = in_vgpr(kExpm1Coef[11]);
    TOARec r1{}, r2{};
    double em1 = 0.0;
    if (N > 0) {
      r1 = load_rec(rec, kb);
      r2 = load_rec(rec, kb + (N > 1 ? 1 : 0));
      em1 = expm1_v(-gr * r1.dt, c13);
    }
    for (int blk = 0; blk <= nblk; ++blk) {
      double* rb = ring + (blk & 1) * kPcSteps * kPcVals * kWave;
      for (int j = 0; j < kPcSteps && blk < nblk; ++j) {
        const int k = blk * kPcSteps + j;
        if (k >= N) break;
        const TOARec r = r1;
        const double em = em1;
        r1 = r2;
        sgpr_ready(r1.dt);
        r2 = load_rec(rec, kb + (k < N - 2 ? k + 2 : N - 1));
        em1 = expm1_v(-gr * r1.dt, c13);
        const double dt = r.dt, phc = r.phc;
        const double ph = 1.0 + em, qfac = -em * (2.0 + em);
        const Cov4& Q0 = st.P;
        double* rv = rb + j * kPcVals * kWave;
        rv[0 * kWave] = em;
        rv[1 * kWave] = st.xa;
        rv[2 * kWave] = Q0.ra;
        rv[3 * kWave] = Q0.fa;
        rv[4 * kWave] = Q0.aa;
        rv[5 * kWave] = Q0.ag;
        Cov4 Pm;
        const double prf1 = fma(dt, Q0.ff, Q0.rf);
        Pm.rr = fma(dt, Q0.rf + prf1, Q0.rr) + ss2 * r.h3;
        Pm.rf = prf1 + ss2 * r.h2;
        Pm.ff = Q0.ff + ss2 * dt;
        Pm.ra = ph * fma(dt, Q0.fa, Q0.ra);
        Pm.fa = ph * Q0.fa;
        Pm.aa = fma(ph * ph, Q0.aa, vr * qfac);
        Pm.rg = phc * fma(dt, Q0.fg, Q0.rg);
        Pm.fg = phc * Q0.fg;
        Pm.ag = (ph * phc) * Q0.ag;
        Pm.gg = fma(phc * phc, Q0.gg, vc * r.qcu);
        const double xr = fma(dt, st.xf, st.xr), xf = st.xf, xa = ph * st.xa, xg = phc * st.xg;
        const double e = r.y - (xr + xa + xg);
        const double ur = Pm.rr + Pm.ra + Pm.rg, uf = Pm.rf + Pm.fa + Pm.fg;
        const double ua = Pm.ra + Pm.aa + Pm.ag, ug = Pm.rg + Pm.ag + Pm.gg;
        const double S = (ur + ua + ug) + fma(efac2, r.s2, equad2);
        const double inv = rcp_nr(S);
        const double kr = ur * inv, kf = uf * inv, ka = ua * inv, kg = ug * inv;
        const double ei = e * inv;
        rv[6 * kWave] = kr;
        rv[7 * kWave] = kf;
        rv[8 * kWave] = ka;
        rv[9 * kWave] = kg;
        rv[10 * kWave] = e;
        rv[11 * kWave] = inv;
        st.xr = fma(kr, e, xr);
        st.xf = fma(kf, e, xf);
        st.xa = fma(ka, e, xa);
        st.xg = fma(kg, e, xg);
        const double dr = fma(S, kr, -ur), df = fma(S, kf, -uf);
        const double da = fma(S, ka, -ua), dg = fma(S, kg, -ug);
        JOSEPH(Pm.rr, kr, ur, dr, kr);
        JOSEPH(Pm.rf, kr, uf, dr, kf);
        JOSEPH(Pm.ff, kf, uf, df, kf);
        JOSEPH(Pm.ra, kr, ua, dr, ka);
        JOSEPH(Pm.fa, kf, ua, df, ka);
        JOSEPH(Pm.aa, ka, ua, da, ka);
        JOSEPH(Pm.rg, kr, ug, dr, kg);
        JOSEPH(Pm.fg, kf, ug, df, kg);
        JOSEPH(Pm.ag, ka, ug, da, kg);
        JOSEPH(Pm.gg, kg, ug, dg, kg);
        st.P = Pm;
        const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
        if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
        quad = fma(e, ei, quad);
        const double pm = lm * S;
        lm = __builtin_amdgcn_frexp_mant(pm);
        le += __builtin_amdgcn_frexp_exp(pm);
      }
      __syncthreads();
    }
    if (valid) {
      double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
      if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
      a.part[(int64_t)p * a.S + s] = stat ? -INFINITY : ll;
      a.pstat[(int64_t)p * a.S + s] = stat;
    }
  } else {
    // ---- NDC directions per wave (the tangent part of tangent_unit), each
    // wave's directions fixed at compile time
    const TanPcCtx c{&a, ring, N, nblk, kb, p, s, valid, vr, gr, vc, t2, eq * eq, gm1};
    const int grp = wave - 1;
    if constexpr (NDC == 2) {
      // the red rate's direction costs most (its decay derivative), so it
      // runs alone and the others pair up
      if (grp == 0) tangent_pc_consumer<1, -1>(c);
      else if (grp == 1) tangent_pc_consumer<0, 4>(c);
      else tangent_pc_consumer<2, 3>(c);
    } else {
      switch (grp) {
        case 0: tangent_pc_consumer<0, -1>(c); break;
        case 1: tangent_pc_consumer<1, -1>(c); break;
        case 2: tangent_pc_consumer<2, -1>(c); break;
        case 3: tangent_pc_consumer<3, -1>(c); break;
        default: tangent_pc_consumer<4, -1>(c); break;
      }
    }
  }
}

// Tangent sweep of model 4 (state [r, f, a, g, m], h = [1, 0, 1, 1, c] with
// the chromatic factor c of each TOA): the same differentiated recursion
// over five states. dF is diagonal, nonzero at a (red decay, its rate) and
// m (DM decay, its rate), so (dF P F^T + F P dF^T)_ij = dF_ii (F P)_ji +
// dF_jj (F P)_ij. Eight directions per pulsar: log10 sigma_red,
// log10 gamma_red, EFAC, log10 EQUAD, log10 sigma_dm, log10 gamma_dm,
// log10 A, gamma. Matrices are kept as lower triangles (index si(i, j)).
__host__ __device__ constexpr int si5(int i, int j) {
  return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i;
}
__device__ __forceinline__ constexpr bool h5(int i) { return i != 1; }

template <int ND>
__device__ __forceinline__ void tangent5_unit(const TanArgs& a, const int lane, const int tile,
                                              const int p, const int grp) {
  constexpr int NS = 5, NP = 15;
  const RecPtr rec = (RecPtr)a.rec;
  const ConstDPtr chrom = (ConstDPtr)a.chrom;
  {
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
    const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;

    const int c0 = 6 * p, cc = 6 * a.P;
    const double t0 = tprm(a, c0, s), t1 = tprm(a, c0 + 1, s), t2 = tprm(a, c0 + 2, s);
    const double t3 = tprm(a, c0 + 3, s), t4 = tprm(a, c0 + 4, s), t5 = tprm(a, c0 + 5, s);
    const double t6 = tprm(a, cc, s), t7 = tprm(a, cc + 1, s);
    const bool pnf = !(finite_d(t0) && finite_d(t1) && finite_d(t2) && finite_d(t3) &&
                       finite_d(t4) && finite_d(t5) && finite_d(t6) && finite_d(t7));
    const double gr = exp10(t1), sr = exp10(t0), eq = exp10(t3);
    const double gd = exp10(t5), sdm = exp10(t4);
    const double vr = sr * sr / (2.0 * gr), vd = sdm * sdm / (2.0 * gd);
    const double gm1 = t7 - 1.0;
    const double vc = exp(2.0 * kLn10 * t6 + (t7 - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
                      (12.0 * kPi * kPi * gm1);
    const double efac2 = t2 * t2, equad2 = eq * eq, ss2 = a.mc.ss2;
    // each direction's sources: variances (red, common, DM), rates (red,
    // DM), white-noise terms
    double sv[ND], sg[ND], sc[ND], sd[ND], sgd[ND], sr2[ND], sq2[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
      const int dir = grp * ND + j;
      sv[j] = dir == 0 ? 2.0 * kLn10 * vr : (dir == 1 ? -kLn10 * vr : 0.0);
      sg[j] = dir == 1 ? kLn10 * gr : 0.0;
      sr2[j] = dir == 2 ? 2.0 * t2 : 0.0;
      sq2[j] = dir == 3 ? 2.0 * kLn10 * equad2 : 0.0;
      sd[j] = dir == 4 ? 2.0 * kLn10 * vd : (dir == 5 ? -kLn10 * vd : 0.0);
      sgd[j] = dir == 5 ? kLn10 * gd : 0.0;
      sc[j] = dir == 6 ? 2.0 * kLn10 * vc
                       : (dir == 7 ? vc * (a.mc.log_fyr + a.mc.log_T - 1.0 / gm1) : 0.0);
    }
    // base state and tangents (prior P0 = diag(s_r^2, s_f^2, v_r, v_c, v_d))
    double x[NS] = {0.0, 0.0, 0.0, 0.0, 0.0}, P[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) P[i] = 0.0;
    P[si5(0, 0)] = a.mc.s_r2;
    P[si5(1, 1)] = a.mc.s_f2;
    P[si5(2, 2)] = vr;
    P[si5(3, 3)] = vc;
    P[si5(4, 4)] = vd;
    double dx[ND][NS], dP[ND][NP], dl[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) {
#pragma unroll
      for (int i = 0; i < NS; ++i) dx[j][i] = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) dP[j][i] = 0.0;
      dP[j][si5(2, 2)] = sv[j];
      dP[j][si5(3, 3)] = sc[j];
      dP[j][si5(4, 4)] = sd[j];
      dl[j] = 0.0;
    }
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = pnf ? kPNF : 0;

    // The record (one 64-B vector, kept whole until the next step) and the
    // chromatic factor of step k + 1 are fetched during step k, and the dt of
    // step k + 2 alone during step k, so both decays of step k + 1 are
    // computed without waiting (indices clamped); the top expm1 coefficient
    // is held in a VGPR
    const double c13 = in_vgpr(kExpm1Coef[11]);
    const RecVecPtr recv = (RecVecPtr)a.rec;
    const ConstDPtr dts = (ConstDPtr)a.rec;  // dt is the first of each record's 8 doubles
    RecVec vn{};
    double cn = 0.0, emn = 0.0, emdn = 0.0, dt2 = 0.0;
    if (N > 0) {
      vn = load_rec_v(recv, kb);
      cn = chrom[kb];
      dt2 = dts[8 * (int64_t)(kb + (N > 1 ? 1 : 0))];
      emn = expm1_v(-gr * vn[0], c13);
      emdn = expm1_v(-gd * vn[0], c13);
    }
    for (int k = 0; k < N; ++k) {
      const RecVec v = vn;
      const double c = cn, em = emn, emd = emdn, dt1 = dt2;
      rec_keep(v);
      sgpr_ready(dt1);
      const TOARec r = rec_fields(v);
      const int kn = kb + (k + 1 < N ? k + 1 : k);
      vn = load_rec_v(recv, kn);
      cn = chrom[kn];
      dt2 = dts[8 * (int64_t)(kb + (k < N - 2 ? k + 2 : N - 1))];
      emn = expm1_v(-gr * dt1, c13);
      emdn = expm1_v(-gd * dt1, c13);
      const double dt = r.dt;
      const double ph = 1.0 + em, phd = 1.0 + emd, phc = r.phc;
      const double qf = -em * (2.0 + em), qfd = -emd * (2.0 + emd);
      const double dg[NS] = {1.0, 1.0, ph, phc, phd};  // diagonal part of F
      // F P (posterior), needed by the tangents: row i of F times P
      double FP[NS][NS];
#pragma unroll
      for (int j = 0; j < NS; ++j) {
        FP[0][j] = fma(dt, P[si5(1, j)], P[si5(0, j)]);
#pragma unroll
        for (int i = 1; i < NS; ++i) FP[i][j] = dg[i] * P[si5(i, j)];
      }
      // base predict
      double xm[NS], Pm[NP];
      xm[0] = fma(dt, x[1], x[0]);
#pragma unroll
      for (int i = 1; i < NS; ++i) xm[i] = dg[i] * x[i];
#pragma unroll
      for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j)
          Pm[si5(i, j)] = j == 0 ? fma(dt, FP[i][1], FP[i][0]) : dg[j] * FP[i][j];
      Pm[si5(0, 0)] += ss2 * r.h3;
      Pm[si5(1, 0)] += ss2 * r.h2;
      Pm[si5(1, 1)] += ss2 * dt;
      Pm[si5(2, 2)] = fma(vr, qf, Pm[si5(2, 2)]);
      Pm[si5(3, 3)] = fma(vc, r.qcu, Pm[si5(3, 3)]);
      Pm[si5(4, 4)] = fma(vd, qfd, Pm[si5(4, 4)]);
      const double hw[NS] = {1.0, 0.0, 1.0, 1.0, c};
      double u[NS], hx = 0.0;
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        double t = 0.0;
#pragma unroll
        for (int l = 0; l < NS; ++l)
          if (h5(l)) t = fma(hw[l], Pm[si5(i, l)], t);
        u[i] = t;
        if (h5(i)) hx = fma(hw[i], xm[i], hx);
      }
      double hu = 0.0;
#pragma unroll
      for (int i = 0; i < NS; ++i)
        if (h5(i)) hu = fma(hw[i], u[i], hu);
      const double S = hu + fma(efac2, r.s2, equad2);
      const double e = r.y - hx;
      const double inv = rcp_nr(S);
      double K[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) K[i] = u[i] * inv;
      const double ei = e * inv, hS = inv * fma(-e, ei, 1.0);
      // tangents
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        const double dph = -dt * ph * sg[j], dphd = -dt * phd * sgd[j];
        const double ddg[NS] = {0.0, 0.0, dph, 0.0, dphd};  // dF (diagonal)
        // dx- = F dx + dF x
        double ddx[NS];
        ddx[0] = fma(dt, dx[j][1], dx[j][0]);
        ddx[1] = dx[j][1];
        ddx[2] = fma(ph, dx[j][2], dph * x[2]);
        ddx[3] = phc * dx[j][3];
        ddx[4] = fma(phd, dx[j][4], dphd * x[4]);
        // dP- = F dP F^T + dF_ii (F P)_qi + dF_qq (F P)_iq + dQ
        double FD[NS][NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          FD[0][q] = fma(dt, dP[j][si5(1, q)], dP[j][si5(0, q)]);
#pragma unroll
          for (int i = 1; i < NS; ++i) FD[i][q] = dg[i] * dP[j][si5(i, q)];
        }
        double D[NP];
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
          for (int q = 0; q <= i; ++q) {
            double t = q == 0 ? fma(dt, FD[i][1], FD[i][0]) : dg[q] * FD[i][q];
            if (i == 2 || i == 4) t = fma(ddg[i], FP[q][i], t);
            if (q == 2 || q == 4) t = fma(ddg[q], FP[i][q], t);
            D[si5(i, q)] = t;
          }
        D[si5(2, 2)] += fma(sv[j], qf, -2.0 * vr * ph * dph);
        D[si5(3, 3)] = fma(sc[j], r.qcu, D[si5(3, 3)]);
        D[si5(4, 4)] += fma(sd[j], qfd, -2.0 * vd * phd * dphd);
        // update
        double du[NS], de = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < NS; ++l)
            if (h5(l)) t = fma(hw[l], D[si5(i, l)], t);
          du[i] = t;
          if (h5(i)) de = fma(-hw[i], ddx[i], de);
        }
        double hdu = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i)
          if (h5(i)) hdu = fma(hw[i], du[i], hdu);
        const double dS = hdu + fma(sr2[j], r.s2, sq2[j]);
        // no dK: dx+ = dx- + du e / S + K (de - dS e / S) and
        // dP+ = dP- - w K^T - K w^T with w = du - dS K / 2
        const double z = fma(-dS, ei, de), hd = -0.5 * dS;
        double w[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          dx[j][i] = fma(du[i], ei, fma(K[i], z, ddx[i]));
          w[i] = fma(hd, K[i], du[i]);
        }
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
          for (int q = 0; q <= i; ++q)
            dP[j][si5(i, q)] = fma(-w[i], K[q], fma(-K[i], w[q], D[si5(i, q)]));
        dl[j] = fma(-0.5, fma(dS, hS, 2.0 * ei * de), dl[j]);
      }
      // base update (the likelihood kernel's Joseph form)
#pragma unroll
      for (int i = 0; i < NS; ++i) x[i] = fma(K[i], e, xm[i]);
      double dd[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) dd[i] = fma(S, K[i], -u[i]);
#pragma unroll
      for (int i = 0; i < NS; ++i)
#pragma unroll
        for (int q = 0; q <= i; ++q)
          P[si5(i, q)] = fma(dd[i], K[q], fma(-K[i], u[q], Pm[si5(i, q)]));
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
      quad = fma(e, ei, quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    }
    if (valid) {
      if (grp == 0) {
        double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
        if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
        a.part[(int64_t)p * a.S + s] = stat ? -INFINITY : ll;
        a.pstat[(int64_t)p * a.S + s] = stat;
      }
      double* g = a.gpart + (int64_t)p * 8 * a.S + s;
#pragma unroll
      for (int j = 0; j < ND; ++j) g[(int64_t)(grp * ND + j) * a.S] = dl[j];
    }
  }
}

// What a consumer wave of k_tangent5_pc needs from its workgroup.
struct Tan5PcCtx {
  const TanArgs* a;
  const double* ring;
  int N, nblk, kb, p;
  int64_t s;
  bool valid;
  double vr, gr, vd, gd, vc, t2, equad2, gm1;
};

// One model-4 direction's tangent: x (5), P (lower triangle, 15) and logL.
struct Tan5 {
  double x[5], P[15], dl;
};

// One TOA of model-4 tangent direction DIR (0 log10 sigma_red, 1
// log10 gamma_red, 2 EFAC, 3 log10 EQUAD, 4 log10 sigma_dm, 5 log10 gamma_dm,
// 6 ln of the common variance) with its source src and, for the two rate
// directions, srate. Terms whose source is zero for DIR are left out at
// compile time. The update is the derivative of the base step written as in
// tan_dir_step: dx+ = dx- + du e / S + K (de - dS e / S) and
// dP+ = dP- - w K^T - K w^T with w = du - dS K / 2.
template <int DIR>
__device__ __forceinline__ void tan5_dir_step(Tan5& d, double src, double srate, double dt,
                                              double ph, double phd, double phc, double qf,
                                              double qfd, double qcu, double s2, double x2,
                                              double x4, const double (&FP2)[5],
                                              const double (&FP4)[5], const double (&K)[5],
                                              const double (&hw)[5], double ei, double hS,
                                              double vr, double vd) {
  constexpr int NS = 5, NP = 15;
  constexpr bool HV = DIR <= 1, HG = DIR == 1, HR = DIR == 2, HQ = DIR == 3;
  constexpr bool HD = DIR == 4 || DIR == 5, HGD = DIR == 5, HC = DIR == 6;
  const double dph = HG ? -dt * ph * srate : 0.0, dphd = HGD ? -dt * phd * srate : 0.0;
  const double dg[NS] = {1.0, 1.0, ph, phc, phd};
  double ddx[NS];
  ddx[0] = fma(dt, d.x[1], d.x[0]);
  ddx[1] = d.x[1];
  ddx[2] = HG ? fma(ph, d.x[2], dph * x2) : ph * d.x[2];
  ddx[3] = phc * d.x[3];
  ddx[4] = HGD ? fma(phd, d.x[4], dphd * x4) : phd * d.x[4];
  double FD[NS][NS];
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    FD[0][q] = fma(dt, d.P[si5(1, q)], d.P[si5(0, q)]);
#pragma unroll
    for (int i = 1; i < NS; ++i) FD[i][q] = dg[i] * d.P[si5(i, q)];
  }
  // column i of F P for i = 2, 4 (the only ones a rate direction takes)
  auto fpc = [&](int row, int col) { return col == 2 ? FP2[row] : FP4[row]; };
  double D[NP];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int q = 0; q <= i; ++q) {
      double t = q == 0 ? fma(dt, FD[i][1], FD[i][0]) : dg[q] * FD[i][q];
      if (HG && i == 2) t = fma(dph, fpc(q, 2), t);
      if (HGD && i == 4) t = fma(dphd, fpc(q, 4), t);
      if (HG && q == 2) t = fma(dph, fpc(i, 2), t);
      if (HGD && q == 4) t = fma(dphd, fpc(i, 4), t);
      D[si5(i, q)] = t;
    }
  if constexpr (HG) D[si5(2, 2)] += fma(src, qf, -2.0 * vr * ph * dph);
  else if constexpr (HV) D[si5(2, 2)] = fma(src, qf, D[si5(2, 2)]);
  if constexpr (HC) D[si5(3, 3)] = fma(src, qcu, D[si5(3, 3)]);
  if constexpr (HGD) D[si5(4, 4)] += fma(src, qfd, -2.0 * vd * phd * dphd);
  else if constexpr (HD) D[si5(4, 4)] = fma(src, qfd, D[si5(4, 4)]);
  double du[NS], de = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < NS; ++l)
      if (h5(l)) t = fma(hw[l], D[si5(i, l)], t);
    du[i] = t;
    if (h5(i)) de = fma(-hw[i], ddx[i], de);
  }
  double dS = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i)
    if (h5(i)) dS = fma(hw[i], du[i], dS);
  if constexpr (HR) dS = fma(src, s2, dS);
  if constexpr (HQ) dS += src;
  const double z = fma(-dS, ei, de), hd = -0.5 * dS;
  double w[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    d.x[i] = fma(du[i], ei, fma(K[i], z, ddx[i]));
    w[i] = fma(hd, K[i], du[i]);
  }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int q = 0; q <= i; ++q)
      d.P[si5(i, q)] = fma(-w[i], K[q], fma(-K[i], w[q], D[si5(i, q)]));
  d.dl = fma(-0.5, fma(dS, hS, 2.0 * ei * de), d.dl);
}

// The source of model-4 direction DIR for this lane and, for the two rate
// directions, the rate's own source.
template <int DIR>
__device__ __forceinline__ double tan5_src(const Tan5PcCtx& c) {
  if constexpr (DIR == 0) return 2.0 * kLn10 * c.vr;
  if constexpr (DIR == 1) return -kLn10 * c.vr;
  if constexpr (DIR == 2) return 2.0 * c.t2;
  if constexpr (DIR == 3) return 2.0 * kLn10 * c.equad2;
  if constexpr (DIR == 4) return 2.0 * kLn10 * c.vd;
  if constexpr (DIR == 5) return -kLn10 * c.vd;
  return c.vc;
}
template <int DIR>
__device__ __forceinline__ double tan5_srate(const Tan5PcCtx& c) {
  if constexpr (DIR == 1) return kLn10 * c.gr;
  if constexpr (DIR == 5) return kLn10 * c.gd;
  return 0.0;
}

constexpr int kPc5Steps = 2;
constexpr int kPc5Vals = 21;

// A consumer wave of k_tangent5_pc carrying directions D0 and D1 (D1 < 0:
// D0 alone), one ring block behind the base filter wave.
template <int D0, int D1>
__device__ __forceinline__ void tangent5_pc_consumer(const Tan5PcCtx& c) {
  constexpr int NS = 5;
  constexpr int E1 = D1 < 0 ? 0 : D1;
  const TanArgs& a = *c.a;
  const RecPtr rec = (RecPtr)a.rec;
  const ConstDPtr chrom = (ConstDPtr)a.chrom;
  const double src0 = tan5_src<D0>(c), srate0 = tan5_srate<D0>(c);
  const double src1 = tan5_src<E1>(c), srate1 = tan5_srate<E1>(c);
  // the prior's derivative: the red (0, 1), common (6) or DM (4, 5) variance
  auto prior = [](int dir, double src) {
    Tan5 t;
#pragma unroll
    for (int i = 0; i < 5; ++i) t.x[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 15; ++i) t.P[i] = 0.0;
    t.P[si5(2, 2)] = dir <= 1 ? src : 0.0;
    t.P[si5(3, 3)] = dir == 6 ? src : 0.0;
    t.P[si5(4, 4)] = dir == 4 || dir == 5 ? src : 0.0;
    t.dl = 0.0;
    return t;
  };
  Tan5 t0 = prior(D0, src0), t1 = prior(E1, src1);
  for (int blk = 0; blk <= c.nblk; ++blk) {
    const double* rb = c.ring + ((blk - 1) & 1) * kPc5Steps * kPc5Vals * kWave;
#pragma unroll 1
    for (int jj = 0; jj < kPc5Steps && blk > 0; ++jj) {
      const int k = (blk - 1) * kPc5Steps + jj;
      if (k >= c.N) break;
      const TOARec r = load_rec(rec, c.kb + k);
      const double cf = chrom[c.kb + k];
      const double* rv = rb + jj * kPc5Vals * kWave;
      const double em = rv[0 * kWave], emd = rv[1 * kWave];
      const double x2 = rv[2 * kWave], x4 = rv[3 * kWave];
      double FP2[NS], FP4[NS], K[NS];
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        FP2[i] = rv[(4 + i) * kWave];
        FP4[i] = rv[(9 + i) * kWave];
        K[i] = rv[(14 + i) * kWave];
      }
      const double e = rv[19 * kWave], inv = rv[20 * kWave];
      const double ph = 1.0 + em, phd = 1.0 + emd;
      const double qf = -em * (2.0 + em), qfd = -emd * (2.0 + emd);
      const double hw[NS] = {1.0, 0.0, 1.0, 1.0, cf};
      const double ei = e * inv, hS = inv * fma(-e, ei, 1.0);
      tan5_dir_step<D0>(t0, src0, srate0, r.dt, ph, phd, r.phc, qf, qfd, r.qcu, r.s2, x2, x4,
                        FP2, FP4, K, hw, ei, hS, c.vr, c.vd);
      if constexpr (D1 >= 0)
        tan5_dir_step<E1>(t1, src1, srate1, r.dt, ph, phd, r.phc, qf, qfd, r.qcu, r.s2, x2, x4,
                          FP2, FP4, K, hw, ei, hS, c.vr, c.vd);
    }
    __syncthreads();
  }
  if (c.valid) {
    double* g = a.gpart + (int64_t)c.p * 8 * a.S + c.s;
    auto put = [&](int dir, double dl) {
      if (dir == 6) {
        // log10 A and gamma enter only through v_c (as in model 2)
        g[6 * a.S] = 2.0 * kLn10 * dl;
        g[7 * a.S] = (a.mc.log_fyr + a.mc.log_T - 1.0 / c.gm1) * dl;
      } else {
        g[(int64_t)dir * a.S] = dl;
      }
    };
    put(D0, t0.dl);
    if constexpr (D1 >= 0) put(D1, t1.dl);
  }
}

// Work units of model 4, as k_tangent: each unit carries NDA or NDB.
// Producer/consumer form of the model-4 tangent sweep, as k_tangent_pc: one
// workgroup of 1 + ceil(7 / NDC) waves per item; wave 0 runs the 5-state base
// filter once and hands per TOA the red and DM decays, the previous
// posterior's a and m states, the a and m columns of F P, the gain, the
// innovation and 1/S (kPc5Vals values per lane) through a double-buffered
// LDS ring of kPc5Steps TOAs per buffer to waves of NDC directions each.
// Each consumer step differentiates the base step (tan5_dir_step).

template <int NDC>
__global__ void __launch_bounds__(kWave * (NDC == 2 ? 5 : 8))
__attribute__((amdgpu_waves_per_eu(NDC == 2 ? 3 : 1))) k_tangent5_pc(TanArgs a) {
  constexpr int NS = 5, NP = 15;
  __shared__ double s_ring[2 * kPc5Steps * kPc5Vals * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const RecPtr rec = (RecPtr)a.rec;
  const ConstDPtr chrom = (ConstDPtr)a.chrom;
  const int item = blockIdx.x;
  const int tile = a.items[2 * item], p = a.items[2 * item + 1];
  const int64_t s_raw = (int64_t)tile * kWave + lane;
  const bool valid = s_raw < a.S;
  const int64_t s = valid ? s_raw : a.S - 1;
  const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
  const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
  const int nblk = (N + kPc5Steps - 1) / kPc5Steps;
  double* ring = s_ring + lane;  // value v of step j of buffer b at ((b kPc5Steps + j) kPc5Vals + v) kWave

  const int c0 = 6 * p, cc = 6 * a.P;
  const double t0 = tprm(a, c0, s), t1 = tprm(a, c0 + 1, s), t2 = tprm(a, c0 + 2, s);
  const double t3 = tprm(a, c0 + 3, s), t4 = tprm(a, c0 + 4, s), t5 = tprm(a, c0 + 5, s);
  const double t6 = tprm(a, cc, s), t7 = tprm(a, cc + 1, s);
  const double gr = exp10(t1), sr = exp10(t0), eq = exp10(t3);
  const double gd = exp10(t5), sdm = exp10(t4);
  const double vr = sr * sr / (2.0 * gr), vd = sdm * sdm / (2.0 * gd);
  const double gm1 = t7 - 1.0;
  const double vc = exp(2.0 * kLn10 * t6 + (t7 - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
                    (12.0 * kPi * kPi * gm1);
  const double equad2 = eq * eq;

  if (wave == 0) {
    // ---- the base filter (the base part of tangent5_unit)
    const bool pnf = !(finite_d(t0) && finite_d(t1) && finite_d(t2) && finite_d(t3) &&
                       finite_d(t4) && finite_d(t5) && finite_d(t6) && finite_d(t7));
    const double efac2 = t2 * t2, ss2 = a.mc.ss2;
    double x[NS] = {0.0, 0.0, 0.0, 0.0, 0.0}, P[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) P[i] = 0.0;
    P[si5(0, 0)] = a.mc.s_r2;
    P[si5(1, 1)] = a.mc.s_f2;
    P[si5(2, 2)] = vr;
    P[si5(3, 3)] = vc;
    P[si5(4, 4)] = vd;
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = pnf ? kPNF : 0;
    const double c13 = in_vgpr(kExpm1Coef[11]);
    const RecVecPtr recv = (RecVecPtr)a.rec;
    const ConstDPtr dts = (ConstDPtr)a.rec;
    RecVec vn{};
    double cn = 0.0, emn = 0.0, emdn = 0.0, dt2 = 0.0;
    if (N > 0) {
      vn = load_rec_v(recv, kb);
      cn = chrom[kb];
      dt2 = dts[8 * (int64_t)(kb + (N > 1 ? 1 : 0))];
      emn = expm1_v(-gr * vn[0], c13);
      emdn = expm1_v(-gd * vn[0], c13);
    }
    for (int blk = 0; blk <= nblk; ++blk) {
      double* rb = ring + (blk & 1) * kPc5Steps * kPc5Vals * kWave;
      for (int jj = 0; jj < kPc5Steps && blk < nblk; ++jj) {
        const int k = blk * kPc5Steps + jj;
        if (k >= N) break;
        const RecVec v = vn;
        const double c = cn, em = emn, emd = emdn, dt1 = dt2;
        rec_keep(v);
        sgpr_ready(dt1);
        const TOARec r = rec_fields(v);
        const int kn = kb + (k + 1 < N ? k + 1 : k);
        vn = load_rec_v(recv, kn);
        cn = chrom[kn];
        dt2 = dts[8 * (int64_t)(kb + (k < N - 2 ? k + 2 : N - 1))];
        emn = expm1_v(-gr * dt1, c13);
        emdn = expm1_v(-gd * dt1, c13);
        const double dt = r.dt;
        const double ph = 1.0 + em, phd = 1.0 + emd, phc = r.phc;
        const double qf = -em * (2.0 + em), qfd = -emd * (2.0 + emd);
        const double dg[NS] = {1.0, 1.0, ph, phc, phd};
        double FP[NS][NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          FP[0][j] = fma(dt, P[si5(1, j)], P[si5(0, j)]);
#pragma unroll
          for (int i = 1; i < NS; ++i) FP[i][j] = dg[i] * P[si5(i, j)];
        }
        double* rv = rb + jj * kPc5Vals * kWave;
        rv[0 * kWave] = em;
        rv[1 * kWave] = emd;
        rv[2 * kWave] = x[2];
        rv[3 * kWave] = x[4];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          rv[(4 + i) * kWave] = FP[i][2];
          rv[(9 + i) * kWave] = FP[i][4];
        }
        double xm[NS], Pm[NP];
        xm[0] = fma(dt, x[1], x[0]);
#pragma unroll
        for (int i = 1; i < NS; ++i) xm[i] = dg[i] * x[i];
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
          for (int j = 0; j <= i; ++j)
            Pm[si5(i, j)] = j == 0 ? fma(dt, FP[i][1], FP[i][0]) : dg[j] * FP[i][j];
        Pm[si5(0, 0)] += ss2 * r.h3;
        Pm[si5(1, 0)] += ss2 * r.h2;
        Pm[si5(1, 1)] += ss2 * dt;
        Pm[si5(2, 2)] = fma(vr, qf, Pm[si5(2, 2)]);
        Pm[si5(3, 3)] = fma(vc, r.qcu, Pm[si5(3, 3)]);
        Pm[si5(4, 4)] = fma(vd, qfd, Pm[si5(4, 4)]);
        const double hw[NS] = {1.0, 0.0, 1.0, 1.0, c};
        double u[NS], hx = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          double t = 0.0;
#pragma unroll
          for (int l = 0; l < NS; ++l)
            if (h5(l)) t = fma(hw[l], Pm[si5(i, l)], t);
          u[i] = t;
          if (h5(i)) hx = fma(hw[i], xm[i], hx);
        }
        double hu = 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i)
          if (h5(i)) hu = fma(hw[i], u[i], hu);
        const double S = hu + fma(efac2, r.s2, equad2);
        const double e = r.y - hx;
        const double inv = rcp_nr(S);
        double K[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
          K[i] = u[i] * inv;
          rv[(14 + i) * kWave] = K[i];
        }
        rv[19 * kWave] = e;
        rv[20 * kWave] = inv;
        const double ei = e * inv;
#pragma unroll
        for (int i = 0; i < NS; ++i) x[i] = fma(K[i], e, xm[i]);
        double dd[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) dd[i] = fma(S, K[i], -u[i]);
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
          for (int q = 0; q <= i; ++q)
            P[si5(i, q)] = fma(dd[i], K[q], fma(-K[i], u[q], Pm[si5(i, q)]));
        const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
        if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
        quad = fma(e, ei, quad);
        const double pm = lm * S;
        lm = __builtin_amdgcn_frexp_mant(pm);
        le += __builtin_amdgcn_frexp_exp(pm);
      }
      __syncthreads();
    }
    if (valid) {
      double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
      if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
      a.part[(int64_t)p * a.S + s] = stat ? -INFINITY : ll;
      a.pstat[(int64_t)p * a.S + s] = stat;
    }
  } else {
    // ---- NDC directions per wave, fixed at compile time: seven
    // directions (log10 A and gamma both from the common variance's)
    const Tan5PcCtx cx{&a, ring, N, nblk, kb, p, s, valid, vr, gr, vd, gd, vc, t2, equad2, gm1};
    const int grp = wave - 1;
    if constexpr (NDC == 2) {
      // each rate direction (the costliest) pairs with a white-noise one
      switch (grp) {
        case 0: tangent5_pc_consumer<1, 2>(cx); break;
        case 1: tangent5_pc_consumer<5, 3>(cx); break;
        case 2: tangent5_pc_consumer<0, 4>(cx); break;
        default: tangent5_pc_consumer<6, -1>(cx); break;
      }
    } else {
      switch (grp) {
        case 0: tangent5_pc_consumer<0, -1>(cx); break;
        case 1: tangent5_pc_consumer<1, -1>(cx); break;
        case 2: tangent5_pc_consumer<2, -1>(cx); break;
        case 3: tangent5_pc_consumer<3, -1>(cx); break;
        case 4: tangent5_pc_consumer<4, -1>(cx); break;
        case 5: tangent5_pc_consumer<5, -1>(cx); break;
        default: tangent5_pc_consumer<6, -1>(cx); break;
      }
    }
  }
}

template <int NDA, int NDB>
__global__ void __launch_bounds__(256) k_tangent5(TanArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  for (;;) {
    int v = 0;
    if (lane == 0) v = atomicAdd(a.counter, 1);
    const int u = __builtin_amdgcn_readfirstlane(v);
    if (u >= a.n_units) break;
    const int item = a.units[2 * u], code = a.units[2 * u + 1];
    const int grp = code & 0xff;
    const int tile = a.items[2 * item];
    const int p = a.items[2 * item + 1];
    if (NDA == NDB || (code >> 8) == NDA)
      tangent5_unit<NDA>(a, lane, tile, p, grp);
    else
      tangent5_unit<NDB>(a, lane, tile, p, grp);
  }
}

// ---------------------------------------------------------------------------
// Smoother of model 4 (state [r, f, a, g, m], h = [1, 0, 1, 1, c]): the
// forward filter with checkpoints as k_adjoint, and the backward recursion
// of the modified Bryson-Frazier smoother on the filtered states (no
// inverse). With (lt, Lt) the adjoint information of the filtered state
// after TOA k (zero after the last TOA), the smoothed moments of TOA k are
//   E = x+ - P+ lt,   Cov = P+ - P+ Lt P+,
// the information moves back through the update of TOA k,
//   lh = lt - h (e / S + K^T lt),
//   Lh = Lt - h (Lt K)^T - (Lt K) h^T + h h^T (K^T Lt K + 1 / S),
// and through its transition F_k to the filtered state after TOA k - 1,
//   lt = F_k^T lh,   Lt = F_k^T Lh F_k.
// The forward step is the model 4 filter step with the Joseph update in the
// W = P- - K u^T, z = R K - W h, P+ = W + z K^T form (as the model 2
// smoother). A saved state is 20 fields: x (5) and the lower triangle of P.
constexpr int kF5 = 20;

struct St5 {
  double x[5];
  double P[15];
};
struct Lane5 {
  double gr, gd, vr, vd, vc, efac2, equad2, ss2;
};

__device__ __forceinline__ void put_st5(double* base, int lane, const St5& s) {
#pragma unroll
  for (int i = 0; i < 5; ++i) base[i * kWave + lane] = s.x[i];
#pragma unroll
  for (int i = 0; i < 15; ++i) base[(5 + i) * kWave + lane] = s.P[i];
}
__device__ __forceinline__ St5 get_st5(const double* base, int lane) {
  St5 s;
#pragma unroll
  for (int i = 0; i < 5; ++i) s.x[i] = base[i * kWave + lane];
#pragma unroll
  for (int i = 0; i < 15; ++i) s.P[i] = base[(5 + i) * kWave + lane];
  return s;
}

// One filter step of TOA (record r, chromatic factor c) in place; returns
// the gain, innovation variance and innovation.
__device__ __forceinline__ void fwd5(St5& s, const TOARec& r, double c, const Lane5& L,
                                     double K[5], double& S, double& e, double& phr,
                                     double& phd) {
  constexpr int NS = 5, NP = 15;
  const double dt = r.dt;
  const double em = expm1_k(-L.gr * dt), emd = expm1_k(-L.gd * dt);
  const double dg[NS] = {1.0, 1.0, 1.0 + em, r.phc, 1.0 + emd};  // diagonal part of F
  phr = dg[2];
  phd = dg[4];
  double FP[NS][NS];
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    FP[0][j] = fma(dt, s.P[si5(1, j)], s.P[si5(0, j)]);
#pragma unroll
    for (int i = 1; i < NS; ++i) FP[i][j] = dg[i] * s.P[si5(i, j)];
  }
  double xm[NS], Pm[NP];
  xm[0] = fma(dt, s.x[1], s.x[0]);
#pragma unroll
  for (int i = 1; i < NS; ++i) xm[i] = dg[i] * s.x[i];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      Pm[si5(i, j)] = j == 0 ? fma(dt, FP[i][1], FP[i][0]) : dg[j] * FP[i][j];
  Pm[si5(0, 0)] += L.ss2 * r.h3;
  Pm[si5(1, 0)] += L.ss2 * r.h2;
  Pm[si5(1, 1)] += L.ss2 * dt;
  Pm[si5(2, 2)] = fma(L.vr, -em * (2.0 + em), Pm[si5(2, 2)]);
  Pm[si5(3, 3)] = fma(L.vc, r.qcu, Pm[si5(3, 3)]);
  Pm[si5(4, 4)] = fma(L.vd, -emd * (2.0 + emd), Pm[si5(4, 4)]);
  const double hw[NS] = {1.0, 0.0, 1.0, 1.0, c};
  double u[NS], hx = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double t = 0.0;
#pragma unroll
    for (int l = 0; l < NS; ++l)
      if (h5(l)) t = fma(hw[l], Pm[si5(i, l)], t);
    u[i] = t;
    if (h5(i)) hx = fma(hw[i], xm[i], hx);
  }
  double hu = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i)
    if (h5(i)) hu = fma(hw[i], u[i], hu);
  const double R = fma(L.efac2, r.s2, L.equad2);
  S = hu + R;
  e = r.y - hx;
  const double inv = rcp_nr(S);
#pragma unroll
  for (int i = 0; i < NS; ++i) K[i] = u[i] * inv;
#pragma unroll
  for (int i = 0; i < NS; ++i) s.x[i] = fma(K[i], e, xm[i]);
  // W = P- - K u^T (full), z = R K - W h, P+ = W + z K^T (entries i <= j)
  double W[NS][NS];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j < NS; ++j) W[i][j] = fma(-K[i], u[j], Pm[si5(i, j)]);
  double z[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double wh = 0.0;
#pragma unroll
    for (int l = 0; l < NS; ++l)
      if (h5(l)) wh = fma(hw[l], W[i][l], wh);
    z[i] = fma(R, K[i], -wh);
  }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = i; j < NS; ++j) s.P[si5(i, j)] = fma(z[i], K[j], W[i][j]);
}
__device__ __forceinline__ void fwd5(St5& s, const TOARec& r, double c, const Lane5& L,
                                     double K[5], double& S, double& e) {
  double phr, phd;
  fwd5(s, r, c, L, K, S, e, phr, phd);
}

// Smoothed mean and variance of TOA k from its filtered state and the
// adjoint information (lt, Lt); NaN when the filter failed.
__device__ __forceinline__ void put_smooth5(const AdjArgs& a, int64_t k, int64_t s,
                                            const St5& f, const double lt[5],
                                            const double Lt[15], bool bad) {
  constexpr int NS = 5;
  double* mo = a.smean + k * NS * a.S + s;
  double* vo = a.svar ? a.svar + k * NS * a.S + s : nullptr;
  const double nan = __builtin_nan("");
#pragma unroll
  for (int c = 0; c < NS; ++c) {
    double m = f.x[c], v = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      m = fma(-f.P[si5(c, i)], lt[i], m);
      double lp = 0.0;  // (Lt P+)_{i c}
#pragma unroll
      for (int j = 0; j < NS; ++j) lp = fma(Lt[si5(i, j)], f.P[si5(j, c)], lp);
      v = fma(f.P[si5(c, i)], lp, v);
    }
    mo[c * a.S] = bad ? nan : m;
    if (vo) vo[c * a.S] = bad ? nan : f.P[si5(c, c)] - v;
  }
}

// The adjoint information moved back through the update of TOA k (gain K,
// innovation variance S, innovation e, chromatic factor c) and through its
// transition (record r) to the filtered state after TOA k - 1.
__device__ __forceinline__ void bwd5(double lt[5], double Lt[15], const double K[5], double S,
                                     double e, double c, const TOARec& r, const Lane5& L) {
  constexpr int NS = 5, NP = 15;
  const double hw[NS] = {1.0, 0.0, 1.0, 1.0, c};
  const double inv = rcp_nr(S);
  double ktl = 0.0, LK[NS], klk = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i) ktl = fma(K[i], lt[i], ktl);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < NS; ++j) t = fma(Lt[si5(i, j)], K[j], t);
    LK[i] = t;
    klk = fma(K[i], t, klk);
  }
  const double g = fma(e, inv, ktl), q = klk + inv;
  double lh[NS], Lh[NP];
#pragma unroll
  for (int i = 0; i < NS; ++i) lh[i] = h5(i) ? fma(-hw[i], g, lt[i]) : lt[i];
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double v = Lt[si5(i, j)];
      if (h5(i)) v = fma(-hw[i], LK[j], v);
      if (h5(j)) v = fma(-LK[i], hw[j], v);
      if (h5(i) && h5(j)) v = fma(hw[i] * hw[j], q, v);
      Lh[si5(i, j)] = v;
    }
  // F = diag(1, 1, phi_r, phi_c, phi_d) + dt e_0 e_1^T for the interval
  // ending at TOA k: lt = F^T lh, Lt = F^T Lh F
  const double dt = r.dt;
  const double dg[NS] = {1.0, 1.0, 1.0 + expm1_k(-L.gr * dt), r.phc, 1.0 + expm1_k(-L.gd * dt)};
  lt[0] = lh[0];
  lt[1] = fma(dt, lh[0], lh[1]);
#pragma unroll
  for (int i = 2; i < NS; ++i) lt[i] = dg[i] * lh[i];
  double G[NS][NS];  // Lh F
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    G[i][0] = Lh[si5(i, 0)];
    G[i][1] = fma(dt, Lh[si5(i, 0)], Lh[si5(i, 1)]);
#pragma unroll
    for (int k = 2; k < NS; ++k) G[i][k] = dg[k] * Lh[si5(i, k)];
  }
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int k = 0; k <= i; ++k)
      Lt[si5(i, k)] = i == 0 ? G[0][k] : (i == 1 ? fma(dt, G[0][k], G[1][k]) : dg[i] * G[i][k]);
}

// The model-4 backward pass over level-1 segments sg_hi - 1 down to sg_lo
// (ck: the level-1 checkpoints; scr: this wave's level-2 scratch), from the
// pair (lt, Lt) after the last TOA of segment sg_hi - 1: each segment is
// recomputed to level-2 checkpoints every 4 TOAs, then its 4-TOA pieces are
// taken last first, each TOA's filtered state recomputed from its piece's
// checkpoint and its smoothed moments written. A piece's records and
// chromatic factors are read once into VGPRs (index clamped to its last
// TOA), so the unrolled loops address them statically. PIECES: every
// segment is one piece (level-1 stride 4): no level-2 pass.
template <bool PIECES>
__device__ __forceinline__ void reverse5(const AdjArgs& a, const RecBuf& rb,
                                         const double* chr, const double* ck, double* scr,
                                         const Lane5& L, int kb, int N, int c1, int sg_lo,
                                         int sg_hi, int64_t s, bool valid, bool bad, double lt[5],
                                         double Lt[15]) {
  constexpr int NS = 5;
  const int lane = threadIdx.x & (kWave - 1);
  // one 4-TOA piece starting at TOA ks from the state s0 before it
  auto piece = [&](int ks, int nt, const St5& s0) {
    TOARec q[4];
    double cq[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = ks + (i < nt ? i : nt - 1);
      q[i] = load_rec_vgpr(rb, k);
      cq[i] = chr[k];
    }
#pragma unroll
    for (int i = 3; i >= 0; --i) {
      if (i < nt) {
        St5 c = s0;
        double K[NS], S, e;
#pragma unroll
        for (int j = 0; j < i; ++j) fwd5(c, q[j], cq[j], L, K, S, e);
        fwd5(c, q[i], cq[i], L, K, S, e);
        if (valid) put_smooth5(a, kb + ks + i, s, c, lt, Lt, bad);
        bwd5(lt, Lt, K, S, e, cq[i], q[i], L);
      }
    }
  };
  for (int sg = sg_hi - 1; sg >= sg_lo; --sg) {
    const int k0 = sg * c1;
    const int k1 = k0 + c1 < N ? k0 + c1 : N;
    if constexpr (PIECES) {
      // the piece starts from its level-1 checkpoint itself
      piece(k0, k1 - k0, get_st5(ck + (int64_t)sg * kF5 * kWave, lane));
      continue;
    }
    const int nsub = (k1 - k0 + 3) / 4;
    St5 cur = get_st5(ck + (int64_t)sg * kF5 * kWave, lane);
    for (int t = 0; t < nsub; ++t) {
      put_st5(scr + (int64_t)t * kF5 * kWave, lane, cur);
      if (t + 1 < nsub) {
        const int kk = k0 + 4 * t;  // a full piece
        TOARec q[4];
        double cq[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          q[i] = load_rec_vgpr(rb, kk + i);
          cq[i] = chr[kk + i];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          double K[NS], S, e;
          fwd5(cur, q[i], cq[i], L, K, S, e);
        }
      }
    }
    for (int t = nsub - 1; t >= 0; --t) {
      const int ks = k0 + 4 * t;
      piece(ks, k1 - ks < 4 ? k1 - ks : 4, get_st5(scr + (int64_t)t * kF5 * kWave, lane));
    }
  }
}

// This lane's model-4 parameters for pulsar p, and whether one is not finite.
__device__ __forceinline__ Lane5 lane5(const AdjArgs& a, int p, int64_t s, bool& pnf) {
  const int c0 = 6 * p, cc = 6 * a.P;
  const double t0 = prm(a, c0, s), t1 = prm(a, c0 + 1, s), t2 = prm(a, c0 + 2, s);
  const double t3 = prm(a, c0 + 3, s), t4 = prm(a, c0 + 4, s), t5 = prm(a, c0 + 5, s);
  const double t6 = prm(a, cc, s), t7 = prm(a, cc + 1, s);
  pnf = !(finite_d(t0) && finite_d(t1) && finite_d(t2) && finite_d(t3) && finite_d(t4) &&
          finite_d(t5) && finite_d(t6) && finite_d(t7));
  Lane5 L;
  L.gr = exp10(t1);
  L.gd = exp10(t5);
  const double sr = exp10(t0), sdm = exp10(t4), eq = exp10(t3);
  L.vr = sr * sr / (2.0 * L.gr);
  L.vd = sdm * sdm / (2.0 * L.gd);
  const double gm1 = t7 - 1.0;
  L.vc = exp(2.0 * kLn10 * t6 + (t7 - 3.0) * a.mc.log_fyr + gm1 * a.mc.log_T) /
         (12.0 * kPi * kPi * gm1);
  L.efac2 = t2 * t2;
  L.equad2 = eq * eq;
  L.ss2 = a.mc.ss2;
  return L;
}

// The prior state of model 4: zero mean, P0 = diag(s_r^2, s_f^2, v_r, v_c, v_d).
__device__ __forceinline__ St5 prior5(const AdjArgs& a, const Lane5& L) {
  St5 st;
#pragma unroll
  for (int i = 0; i < 5; ++i) st.x[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 15; ++i) st.P[i] = 0.0;
  st.P[si5(0, 0)] = a.mc.s_r2;
  st.P[si5(1, 1)] = a.mc.s_f2;
  st.P[si5(2, 2)] = L.vr;
  st.P[si5(3, 3)] = L.vc;
  st.P[si5(4, 4)] = L.vd;
  return st;
}

__global__ void __launch_bounds__(256) k_smooth5(AdjArgs a) {
  constexpr int NS = 5, NP = 15;
  const int lane = threadIdx.x & (kWave - 1);
  const int gwave = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave));
  double* scr = a.scratch + (int64_t)gwave * a.max_sub * kF5 * kWave;
  for (;;) {
    int v = 0;
    if (lane == 0) v = atomicAdd(a.counter, 1);
    const int it = __builtin_amdgcn_readfirstlane(v);
    if (it >= a.n_items) break;
    const int tile = a.items[2 * it];
    const int p = a.items[2 * it + 1];
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
    const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
    const int c1 = a.c1[p];
    double* ck = a.ckpt + ((int64_t)tile * a.tot_seg + a.seg_base[p]) * kF5 * kWave;

    bool pnf;
    const Lane5 L = lane5(a, p, s, pnf);

    // forward pass: log-likelihood and level-1 checkpoints (the state
    // before the first TOA of each segment of c1 TOAs); the record and
    // chromatic factor of TOA k + 1 are fetched during step k
    const RecBuf rb = rec_buffer(a.rec + kb, N);
    const double* chr = a.chrom + kb;
    St5 st = prior5(a, L);
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = pnf ? kPNF : 0;
    TOARec rq{};
    double cqn = 0.0;
    if (N > 0) {
      rq = load_rec_vgpr(rb, 0);
      cqn = chr[0];
    }
    for (int k = 0; k < N; ++k) {
      const TOARec r = rq;
      const double ch = cqn;
      const int kn = k + 1 < N ? k + 1 : k;
      rq = load_rec_vgpr(rb, kn);
      cqn = chr[kn];
      if (k % c1 == 0) put_st5(ck + (int64_t)(k / c1) * kF5 * kWave, lane, st);
      double K[NS], S, e;
      fwd5(st, r, ch, L, K, S, e);
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
      quad = fma(e * e, rcp_nr(S), quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    }
    double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
    if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
    if (stat) ll = -INFINITY;

    // backward pass over all segments from a zero pair
    double lt[NS], Lt[NP];
#pragma unroll
    for (int i = 0; i < NS; ++i) lt[i] = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) Lt[i] = 0.0;
    reverse5<false>(a, rb, chr, ck, scr, L, kb, N, c1, 0, (N + c1 - 1) / c1, s, valid, stat != 0, lt,
             Lt);
    if (valid) {
      a.part[(int64_t)p * a.S + s] = ll;
      a.pstat[(int64_t)p * a.S + s] = stat;
    }
  }
}

// Time-parallel form of the model-4 smoother, as k_smooth_fwd_pc / k_smooth_rev
// for models 1 and 2: the summary of a chunk is U (5 x 5, row major), phi (5)
// and Om (15) with F = diag(1, 1, phi_r, phi_c, phi_d) + dt e_0 e_1^T and
// h = [1, 0, 1, 1, c] per TOA; a chunk's place holds the pair (lt, Lt) after
// its last TOA as a saved state's 20 fields (the last chunk starts from zero
// and, like k_smooth5, recomputes each TOA's filtered state itself).
constexpr int kSum5 = 45;

// The chain of one item's model-4 chunk summaries from the last chunk back,
// as smooth_chain; the pair (lt, Lt) after the last TOA of chunk c - 1 goes
// to chunk c - 1's place in a saved state's fields.
__device__ __forceinline__ void smooth5_chain(const AdjArgs& a, int64_t base, int nch,
                                              int lane) {
  constexpr int NS = 5, NP = 15;
  St5 pr;  // (lt, Lt) in a saved state's fields
#pragma unroll
  for (int i = 0; i < NS; ++i) pr.x[i] = 0.0;
#pragma unroll
  for (int i = 0; i < NP; ++i) pr.P[i] = 0.0;
  for (int c = nch - 1; c >= 1; --c) {
    const double* o = a.tpsum + (base + c) * kSum5 * kWave + lane;
    double Uc[NS][NS], T[NS][NS], nl[NS];
#pragma unroll
    for (int i = 0; i < NS * NS; ++i) Uc[i / NS][i % NS] = o[i * kWave];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      double acc = o[(NS * NS + i) * kWave];
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        acc = fma(Uc[i][q], pr.x[q], acc);
        double tq = 0.0;
#pragma unroll
        for (int l = 0; l < NS; ++l) tq = fma(Uc[i][l], pr.P[si5(l, q)], tq);
        T[i][q] = tq;
      }
      nl[i] = acc;
    }
    double nL[NP];
#pragma unroll
    for (int i = 0; i < NS; ++i)
#pragma unroll
      for (int q = 0; q <= i; ++q) {
        double acc = o[(30 + si5(i, q)) * kWave];
#pragma unroll
        for (int l = 0; l < NS; ++l) acc = fma(T[i][l], Uc[q][l], acc);
        nL[si5(i, q)] = acc;
      }
#pragma unroll
    for (int i = 0; i < NS; ++i) pr.x[i] = nl[i];
#pragma unroll
    for (int i = 0; i < NP; ++i) pr.P[i] = nL[i];
    put_st5(a.tpadj + (base + c - 1) * kF5 * kWave, lane, pr);
  }
}

// Forward pass of the model-4 time-parallel smoother, as k_smooth_fwd_pc:
// wave 0 filters (blocks of kSmSteps TOAs, full blocks straight-line) and
// hands per TOA the gain, e, 1/S, dt, the three decays and the chromatic
// factor (kSm5Vals values) to wave 1, which accumulates the chunk summaries
// one block behind and chains them.
constexpr int kSm5Vals = 12;

__global__ void __launch_bounds__(2 * kWave) __attribute__((amdgpu_waves_per_eu(2)))
k_smooth5_fwd_pc(AdjArgs a) {
  constexpr int NS = 5, NP = 15;
  __shared__ double s_ring[2 * kSmSteps * kSm5Vals * kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int it = blockIdx.x;
  const int tile = a.items[2 * it];
  const int p = a.items[2 * it + 1];
  const int64_t s_raw = (int64_t)tile * kWave + lane;
  const bool valid = s_raw < a.S;
  const int64_t s = valid ? s_raw : a.S - 1;
  const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
  const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
  const int c1 = a.c1[p];
  const int nseg = (N + c1 - 1) / c1;
  const int nch = __builtin_amdgcn_readfirstlane(a.tp_item[2 * it]);
  const int64_t base = __builtin_amdgcn_readfirstlane(a.tp_item[2 * it + 1]);
  const int nblk = (N + kSmSteps - 1) / kSmSteps;
  double* ring = s_ring + lane;  // value v of step j of buffer b at ((b kSmSteps + j) kSm5Vals + v) kWave

  if (wave == 0) {
    double* ck = a.ckpt + ((int64_t)tile * a.tot_seg + a.seg_base[p]) * kF5 * kWave;
    bool pnf;
    const Lane5 L = lane5(a, p, s, pnf);
    const RecBuf rb = rec_buffer(a.rec + kb, N);
    const double* chr = a.chrom + kb;
    St5 st = prior5(a, L);
    double quad = 0.0, lm = 1.0;
    int le = 0, stat = pnf ? kPNF : 0;
    auto step = [&](const TOARec& r, double ch, double* rv) {
      double K[NS], S, e, phr, phd;
      fwd5(st, r, ch, L, K, S, e, phr, phd);
      const double inv = rcp_nr(S);
#pragma unroll
      for (int i = 0; i < NS; ++i) rv[i * kWave] = K[i];
      rv[5 * kWave] = e;
      rv[6 * kWave] = inv;
      rv[7 * kWave] = r.dt;
      rv[8 * kWave] = phr;
      rv[9 * kWave] = r.phc;
      rv[10 * kWave] = phd;
      rv[11 * kWave] = ch;
      const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
      if (!good && stat == 0) stat = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
      quad = fma(e * e, inv, quad);
      const double pm = lm * S;
      lm = __builtin_amdgcn_frexp_mant(pm);
      le += __builtin_amdgcn_frexp_exp(pm);
    };
    for (int blk = 0; blk <= nblk; ++blk) {
      double* rbuf = ring + (blk & 1) * kSmSteps * kSm5Vals * kWave;
      if (blk < nblk) {
        // the block's records and chromatic factors, read together (index
        // clamped to the last TOA); a full block is straight-line code, two
        // steps at a time (four at once need more registers than two waves
        // per SIMD leave)
        const int k0 = blk * kSmSteps;
        TOARec q[kSmSteps];
        double cq[kSmSteps];
#pragma unroll
        for (int j = 0; j < kSmSteps; ++j) {
          const int k = k0 + j < N ? k0 + j : N - 1;
          q[j] = load_rec_vgpr(rb, k);
          cq[j] = chr[k];
        }
        if (k0 % c1 == 0) put_st5(ck + (int64_t)(k0 / c1) * kF5 * kWave, lane, st);
        if (k0 + kSmSteps <= N) {
#pragma unroll
          for (int j = 0; j < kSmSteps; ++j) {
            step(q[j], cq[j], rbuf + j * kSm5Vals * kWave);
            if (j % 2 == 1) __builtin_amdgcn_sched_barrier(0);
          }
        } else {
          for (int j = 0; j < N - k0; ++j) {
            const TOARec r = j == 0 ? q[0] : (j == 1 ? q[1] : q[2]);
            const double ch = j == 0 ? cq[0] : (j == 1 ? cq[1] : cq[2]);
            step(r, ch, rbuf + j * kSm5Vals * kWave);
          }
        }
      }
      __syncthreads();
    }
    double ll = -0.5 * ((double)N * kLn2Pi + (log(lm) + (double)le * kLn2) + quad);
    if (stat == 0 && !finite_d(ll)) stat = kNonFinite;
    if (stat) ll = -INFINITY;
    if (valid) {
      a.part[(int64_t)p * a.S + s] = ll;
      a.pstat[(int64_t)p * a.S + s] = stat;
    }
  } else {
    double U[NS][NS], phi[NS], Om[NP];
    auto reset = [&]() {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
#pragma unroll
        for (int q = 0; q < NS; ++q) U[i][q] = i == q ? 1.0 : 0.0;
        phi[i] = 0.0;
      }
#pragma unroll
      for (int i = 0; i < NP; ++i) Om[i] = 0.0;
    };
    reset();
    int c = 0;  // chunk of the next TOA and its end
    int ec = (nseg / nch) * c1 < N ? (nseg / nch) * c1 : N;
    for (int blk = 0; blk <= nblk; ++blk) {
      if (blk > 0) {
        const double* rbuf = ring + ((blk - 1) & 1) * kSmSteps * kSm5Vals * kWave;
#pragma unroll 1
        for (int j = 0; j < kSmSteps; ++j) {
          const int k = (blk - 1) * kSmSteps + j;
          if (k >= N) break;
          if (c > 0) {
            const double* rv = rbuf + j * kSm5Vals * kWave;
            double K[NS];
#pragma unroll
            for (int i = 0; i < NS; ++i) K[i] = rv[i * kWave];
            const double e = rv[5 * kWave], inv = rv[6 * kWave], dt = rv[7 * kWave];
            const double dg[NS] = {1.0, 1.0, rv[8 * kWave], rv[9 * kWave], rv[10 * kWave]};
            const double ch = rv[11 * kWave];
            const double ei = -e * inv;
            double V[NS][NS], v[NS];
#pragma unroll
            for (int i = 0; i < NS; ++i) {
              V[i][0] = fma(dt, U[i][1], U[i][0]);
              V[i][1] = U[i][1];
#pragma unroll
              for (int q = 2; q < NS; ++q) V[i][q] = dg[q] * U[i][q];
              v[i] = fma(ch, V[i][4], V[i][0] + V[i][2] + V[i][3]);
              phi[i] = fma(v[i], ei, phi[i]);
            }
#pragma unroll
            for (int i = 0; i < NS; ++i) {
              const double vs = v[i] * inv;
#pragma unroll
              for (int q = 0; q <= i; ++q) Om[si5(i, q)] = fma(vs, v[q], Om[si5(i, q)]);
#pragma unroll
              for (int q = 0; q < NS; ++q) U[i][q] = fma(-v[i], K[q], V[i][q]);
            }
          }
          if (k + 1 == ec) {
            if (c > 0) {
              double* o = a.tpsum + (base + c) * kSum5 * kWave + lane;
#pragma unroll
              for (int i = 0; i < NS * NS; ++i) o[i * kWave] = U[i / NS][i % NS];
#pragma unroll
              for (int i = 0; i < NS; ++i) o[(NS * NS + i) * kWave] = phi[i];
#pragma unroll
              for (int i = 0; i < NP; ++i) o[(30 + i) * kWave] = Om[i];
            }
            reset();
            ++c;
            const int sh = (c + 1) * nseg / nch;
            ec = sh * c1 < N ? sh * c1 : N;
          }
        }
      }
      __syncthreads();
    }
    smooth5_chain(a, base, nch, lane);
  }
}

// One wave per SIMD: at two, the piece's records in VGPRs no longer fit
// without spills (measured slower).
__global__ void __launch_bounds__(256) k_smooth5_rev(AdjArgs a) {
  constexpr int NS = 5, NP = 15;
  const int lane = threadIdx.x & (kWave - 1);
  const int gwave = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave));
  double* scr = a.scratch + (int64_t)gwave * a.max_sub * kF5 * kWave;
  for (;;) {
    int v = 0;
    if (lane == 0) v = atomicAdd(a.counter, 1);
    const int u = __builtin_amdgcn_readfirstlane(v);
    if (u >= a.n_units) break;
    const int it = a.tp_units[2 * u];
    const int cch = a.tp_units[2 * u + 1];
    const int tile = a.items[2 * it];
    const int p = a.items[2 * it + 1];
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
    const int N = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]) - kb;
    const int c1 = a.c1[p];
    const int nseg = (N + c1 - 1) / c1;
    const int nch = a.tp_item[2 * it];
    const int64_t base = a.tp_item[2 * it + 1];
    const int sg_lo = cch * nseg / nch, sg_hi = (cch + 1) * nseg / nch;
    const double* ck = a.ckpt + ((int64_t)tile * a.tot_seg + a.seg_base[p]) * kF5 * kWave;
    bool pnf;
    const Lane5 L = lane5(a, p, s, pnf);
    const bool bad = a.pstat[(int64_t)p * a.S + s] != 0;
    double lt[NS], Lt[NP];
    if (cch == nch - 1) {
#pragma unroll
      for (int i = 0; i < NS; ++i) lt[i] = 0.0;
#pragma unroll
      for (int i = 0; i < NP; ++i) Lt[i] = 0.0;
    } else {
      const St5 pr = get_st5(a.tpadj + (base + cch) * kF5 * kWave, lane);
#pragma unroll
      for (int i = 0; i < NS; ++i) lt[i] = pr.x[i];
#pragma unroll
      for (int i = 0; i < NP; ++i) Lt[i] = pr.P[i];
    }
    reverse5<true>(a, rec_buffer(a.rec + kb, N), a.chrom + kb, ck, scr, L, kb, N, c1, sg_lo, sg_hi, s,
             valid, bad, lt, Lt);
  }
}

// grad[s, c] from the per-pulsar parts, one thread per element (consecutive
// threads on consecutive columns of a row, so the rows are written whole): a
// pulsar's own parameters from its filter, the common ones summed over
// pulsars in index order; rows of failed samples are zero.
__global__ void __launch_bounds__(256) k_grad_reduce(const double* gpart, const int32_t* status,
                                                     const int32_t* icol, double* grad, int64_t S,
                                                     int D, int P, int model) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S * D) return;
  const int64_t s = i / D;
  const int c = (int)(i - s * D);
  const int k = icol[c];  // canonical parameter of column c
  double v;
  // per pulsar: kp own parameters, np gradient parts (own + the two common)
  const int kp = model == 4 ? 6 : 4, np = kp + 2;
  if (model == 1) {
    v = gpart[(int64_t)k * S + s];
  } else if (k < kp * P) {
    v = gpart[((int64_t)(k / kp) * np + (k % kp)) * S + s];
  } else {
    const int j = k - kp * P;
    v = 0.0;
    for (int p = 0; p < P; ++p) v += gpart[((int64_t)p * np + kp + j) * S + s];
  }
  grad[i] = status[s] != 0 ? 0.0 : v;
}

}  // namespace

namespace {

// Per-sample log-likelihood, status and gradient rows from the per-pulsar
// parts (shared by both gradient sweeps).
int grad_finish(argus_dataset* ds, Workspace* w, int64_t S, double* logl, double* grad,
                int32_t* status, hipStream_t st) {
  int32_t* stat = status ? status : w->stat_tmp.as<int32_t>();
  ReduceArgs r{w->part.as<double>(), w->pstat.as<int32_t>(), logl, stat,
               w->counter.as<int32_t>(), S, ds->P};
  HIPCHK(launch_reduce(r, st));
  const int blk = 256;
  if (ds->D > 0)
    hipLaunchKernelGGL(k_grad_reduce, dim3((unsigned)((S * ds->D + blk - 1) / blk)), dim3(blk), 0,
                       st, w->gpart.as<double>(), stat, ds->icol.as<int32_t>(), grad, S, ds->D,
                       ds->P, ds->model);
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

// Work units of a split: every item (tile, pulsar) in the
// longest-first order, cut into ndir / nd groups with nd = nda for pulsars
// of at least thresh TOAs and ndb for the others.
int tangent_units(argus_dataset* ds, Workspace* w, int nda, int ndb, int64_t thresh) {
  if (w->units_nda == nda && w->units_ndb == ndb && w->units_thresh == thresh) return ARGUS_OK;
  const int ndir = ds->model == 1 ? 2 : (ds->model == 4 ? 8 : 6);
  std::vector<int32_t> u;
  for (int i = 0; i < w->n_items; ++i) {
    const int p = w->items_host[2 * i + 1];
    const int nd = ds->counts[p] >= thresh ? nda : ndb;
    for (int g = 0; g < ndir / nd; ++g) {
      u.push_back(i);
      u.push_back(g | nd << 8);
    }
  }
  w->n_tan_units = (int)(u.size() / 2);
  if (u.empty()) u.assign(2, 0);  // keep the buffer non-empty
  const int rc = w->tan_units.upload(u.data(), u.size() * sizeof(int32_t));
  if (rc) return rc;
  w->units_nda = nda;
  w->units_ndb = ndb;
  w->units_thresh = thresh;
  return ARGUS_OK;
}

int launch_tangent(argus_dataset* ds, Workspace* w, const double* theta, int nda, int ndb,
                   int64_t thresh, hipStream_t st) {
  TanArgs a{};
  a.rec = ds->rec.as<TOARec>();
  a.chrom = ds->chrom.as<double>();
  a.off = ds->off.as<int64_t>();
  a.theta = theta;
  a.col = ds->col.as<int32_t>();
  a.fixed = ds->fixed.as<double>();
  a.items = w->items.as<int32_t>();
  a.counter = w->counter.as<int32_t>();
  a.part = w->part.as<double>();
  a.pstat = w->pstat.as<int32_t>();
  a.gpart = w->gpart.as<double>();
  a.S = w->S;
  a.D = ds->D;
  a.P = ds->P;
  a.n_items = w->n_items;
  a.mc = ds->mc;
  if (thresh < 0) {
    // the producer/consumer forms: one workgroup of 1 + ceil(ndir / nda)
    // waves per item (model 2: 5 directions, model 4: 7)
    const dim3 grid((unsigned)w->n_items);
    if (ds->model == 2 && nda == 2)
      hipLaunchKernelGGL(k_tangent_pc<2>, grid, dim3(4 * kWave), 0, st, a);
    else if (ds->model == 2 && nda == 1)
      hipLaunchKernelGGL(k_tangent_pc<1>, grid, dim3(6 * kWave), 0, st, a);
    else if (ds->model == 4 && nda == 2)
      hipLaunchKernelGGL(k_tangent5_pc<2>, grid, dim3(5 * kWave), 0, st, a);
    else if (ds->model == 4 && nda == 1)
      hipLaunchKernelGGL(k_tangent5_pc<1>, grid, dim3(8 * kWave), 0, st, a);
    else
      return fail(ARGUS_E_INVAL, "unsupported tangent split");
    HIPCHK(hipGetLastError());
    return ARGUS_OK;
  }
  int rc = tangent_units(ds, w, nda, ndb, thresh);
  if (rc) return rc;
  a.units = w->tan_units.as<int32_t>();
  a.n_units = w->n_tan_units;
  const int64_t waves = std::max<int64_t>(4, std::min<int64_t>(a.n_units, 8LL * ds->n_cu));
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
  const int key = nda * 10 + ndb;
  if (ds->model == 4) {
    if (key == 44)
      hipLaunchKernelGGL((k_tangent5<4, 4>), grid, block, 0, st, a);
    else if (key == 22)
      hipLaunchKernelGGL((k_tangent5<2, 2>), grid, block, 0, st, a);
    else if (key == 11)
      hipLaunchKernelGGL((k_tangent5<1, 1>), grid, block, 0, st, a);
    else if (key == 12)
      hipLaunchKernelGGL((k_tangent5<1, 2>), grid, block, 0, st, a);
    else if (key == 14)
      hipLaunchKernelGGL((k_tangent5<1, 4>), grid, block, 0, st, a);
    else if (key == 24)
      hipLaunchKernelGGL((k_tangent5<2, 4>), grid, block, 0, st, a);
    else
      return fail(ARGUS_E_INVAL, "unsupported tangent split");
  } else if (ds->model == 1)
    hipLaunchKernelGGL((k_tangent<1, 2, 2>), grid, block, 0, st, a);
  else if (key == 66)
    hipLaunchKernelGGL((k_tangent<2, 6, 6>), grid, block, 0, st, a);
  else if (key == 33)
    hipLaunchKernelGGL((k_tangent<2, 3, 3>), grid, block, 0, st, a);
  else if (key == 22)
    hipLaunchKernelGGL((k_tangent<2, 2, 2>), grid, block, 0, st, a);
  else if (key == 11)
    hipLaunchKernelGGL((k_tangent<2, 1, 1>), grid, block, 0, st, a);
  else if (key == 12)
    hipLaunchKernelGGL((k_tangent<2, 1, 2>), grid, block, 0, st, a);
  else if (key == 13)
    hipLaunchKernelGGL((k_tangent<2, 1, 3>), grid, block, 0, st, a);
  else if (key == 23)
    hipLaunchKernelGGL((k_tangent<2, 2, 3>), grid, block, 0, st, a);
  else
    return fail(ARGUS_E_INVAL, "unsupported tangent split");
  HIPCHK(hipGetLastError());
  return ARGUS_OK;
}

}  // namespace

// Tangent-mode gradient (the default): one streaming pass per direction
// group; on the first call for a sample count the directions per wave are
// chosen by timing (model 2: 6, 3, 2 or 1 for every pulsar, or fewer for
// the longest pulsars than for the others).
int tangent_loglike(argus_dataset* ds, const double* theta, int64_t S, double* logl,
                    double* grad, int32_t* status, hipStream_t st) {
  int rc = ARGUS_OK;
  Workspace* w = get_workspace(ds, S, &rc);
  if (!w) return rc;
  const int gstride = ds->model == 4 ? 8 : 6;  // gradient parts per pulsar
  if (w->gpart.p == nullptr &&
      (rc = w->gpart.alloc((size_t)ds->P * gstride * S * sizeof(double))))
    return rc;
  if (w->tan_nda == 0) {
    // a forced split: "nd" (uniform), "nda,ndb,thresh", or "pc" / "pc1"
    // (models 2, 4: the producer/consumer form with 2 / 1 directions per
    // wave)
    const char* forced = std::getenv("ARGUS_TAN_ND");
    int fa = 0, fb = 0;
    long long ft = 0;
    const bool fpc = forced && (ds->model == 2 || ds->model == 4) &&
                     (std::strcmp(forced, "pc") == 0 || std::strcmp(forced, "pc1") == 0);
    const int nf = forced && !fpc ? std::sscanf(forced, "%d,%d,%lld", &fa, &fb, &ft) : 0;
    if (nf == 1) fb = fa;
    if (ds->model == 1) fa = fb = 2;
    const bool uni = fa == fb;
    const int fk = fa * 10 + fb;
    const bool ok = ds->model == 4
                        ? (uni ? (fa == 1 || fa == 2 || fa == 4)
                               : nf == 3 && ft >= 0 && (fk == 12 || fk == 14 || fk == 24))
                        : (uni ? (fa == 1 || fa == 2 || fa == 3 || fa == 6)
                               : nf == 3 && ft >= 0 && (fk == 12 || fk == 13 || fk == 23));
    if (fpc) {
      w->tan_nda = w->tan_ndb = std::strcmp(forced, "pc1") == 0 ? 1 : 2;
      w->tan_thresh = -1;
    } else if (ok) {
      w->tan_nda = fa;
      w->tan_ndb = fb;
      w->tan_thresh = uni ? 0 : ft;
    } else {
      // timed candidates: uniform splits, and (models 2, 4) mixed ones that
      // give the pulsars of at least 1/2, 3/4 or 7/8 of the longest
      // pulsar's TOAs fewer directions per wave
      struct Cand {
        int a, b;
        int64_t t;
      };
      std::vector<Cand> cand;
      std::vector<std::pair<int, int>> mixed;
      if (ds->model == 4) {
        for (int c : {4, 2, 1}) cand.push_back({c, c, 0});
        mixed = {{1, 2}, {1, 4}, {2, 4}};
      } else if (ds->model == 2) {
        for (int c : {6, 3, 2, 1}) cand.push_back({c, c, 0});
        mixed = {{1, 2}, {1, 3}, {2, 3}};
      } else {
        cand.push_back({2, 2, 0});
      }
      const int64_t nmax = ds->counts.empty()
                               ? 0
                               : *std::max_element(ds->counts.begin(), ds->counts.end());
      for (int64_t t : {nmax / 2, (3 * nmax) / 4, (7 * nmax) / 8})
        for (auto ab : mixed)
          if (t > 0) cand.push_back({ab.first, ab.second, t});
      if (ds->model == 2 || ds->model == 4)  // producer/consumer forms
        for (int c : {2, 1}) cand.push_back({c, c, -1});
      hipEvent_t e0, e1;
      HIPCHK(hipEventCreate(&e0));
      HIPCHK(hipEventCreate(&e1));
      float best = 1e30f;
      Cand pick = cand[0];
      w->grad_log.clear();
      for (const Cand& c : cand) {
        float m = 1e30f;
        for (int rep = 0; rep < 3 && rc == ARGUS_OK; ++rep) {
          if (hipEventRecord(e0, st) != hipSuccess) rc = fail(ARGUS_E_HIP, "event");
          if (!rc) rc = launch_tangent(ds, w, theta, c.a, c.b, c.t, st);
          if (!rc) rc = grad_finish(ds, w, S, logl, grad, status, st);
          if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = fail(ARGUS_E_HIP, "event");
          if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(ARGUS_E_HIP, "sync");
          float ms = 0;
          if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(ARGUS_E_HIP, "t");
          if (rep > 0) m = std::min(m, ms);
        }
        if (rc) break;
        char b[160];
        if (c.t < 0)
          std::snprintf(b, sizeof b, "tangent producer/consumer (%s): %.4f ms\n",
                        tangent_pc_layout(ds->model, c.a), m);
        else if (c.a == c.b)
          std::snprintf(b, sizeof b, "tangent directions per wave %d: %.4f ms\n", c.a, m);
        else
          std::snprintf(b, sizeof b, "tangent directions per wave %d (>= %lld TOAs) / %d: %.4f ms\n",
                        c.a, (long long)c.t, c.b, m);
        w->grad_log += b;
        if (m < best) {
          best = m;
          pick = c;
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (rc) return rc;
      w->tan_nda = pick.a;
      w->tan_ndb = pick.b;
      w->tan_thresh = pick.t;
    }
  }
  if ((rc = launch_tangent(ds, w, theta, w->tan_nda, w->tan_ndb, w->tan_thresh, st))) return rc;
  return grad_finish(ds, w, S, logl, grad, status, st);
}

namespace {

// Checkpoint layout of the reverse sweep for one sample count: level-1
// strides ceil(sqrt(N_p)) rounded up to a multiple of 4, segment offsets,
// the level-1 store and the per-wave level-2 scratch.
int adjoint_setup(argus_dataset* ds, Workspace* w, int64_t S) {
  if (w->grad_ready) return ARGUS_OK;
  // the reverse sweep reads a pulsar's records through one buffer
  // descriptor, whose byte range is 31 bits
  for (const int64_t n : ds->counts)
    if (n > INT32_MAX / 64)
      return fail(ARGUS_E_UNSUPPORTED, "the reverse sweep takes at most 33554431 TOAs per pulsar");
  const int64_t tiles = (S + kWave - 1) / kWave;
  std::vector<int32_t> c1(ds->P);
  std::vector<int64_t> base(ds->P);
  int64_t tot = 0;
  int cmax = 4;
  for (int p = 0; p < ds->P; ++p) {
    const int64_t n = ds->counts[p];
    int64_t r = (int64_t)std::ceil(std::sqrt((double)std::max<int64_t>(n, 1)));
    r = ((r + 3) / 4) * 4;
    c1[p] = (int32_t)r;
    cmax = std::max<int>(cmax, (int)r);
    base[p] = tot;
    tot += (n + r - 1) / r;
  }
  w->tot_seg = tot;
  w->max_sub = cmax / 4;
  const int fields = ds->model == 4 ? kF5 : kFields;  // doubles per saved state
  w->grad_waves = (int)std::min<int64_t>(w->n_items, 8LL * ds->n_cu);
  w->grad_waves = ((w->grad_waves + 3) / 4) * 4;
  int rc;
  if ((rc = w->c1.upload(c1.data(), c1.size() * sizeof(int32_t))) ||
      (rc = w->seg_base.upload(base.data(), base.size() * sizeof(int64_t))) ||
      (rc = w->ckpt.alloc((size_t)std::max<int64_t>(tiles * tot, 1) * fields * kWave *
                          sizeof(double))) ||
      (rc = w->scratch.alloc((size_t)w->grad_waves * w->max_sub * fields * kWave *
                             sizeof(double))))
    return rc;
  w->grad_ready = true;
  return ARGUS_OK;
}

AdjArgs adjoint_args(argus_dataset* ds, Workspace* w, const double* theta, int64_t S) {
  AdjArgs a{};
  a.rec = ds->rec.as<TOARec>();
  a.chrom = ds->chrom.as<double>();
  a.off = ds->off.as<int64_t>();
  a.theta = theta;
  a.col = ds->col.as<int32_t>();
  a.fixed = ds->fixed.as<double>();
  a.items = w->items.as<int32_t>();
  a.counter = w->counter.as<int32_t>();
  a.c1 = w->c1.as<int32_t>();
  a.seg_base = w->seg_base.as<int64_t>();
  a.ckpt = w->ckpt.as<double>();
  a.scratch = w->scratch.as<double>();
  a.part = w->part.as<double>();
  a.pstat = w->pstat.as<int32_t>();
  a.S = S;
  a.tot_seg = w->tot_seg;
  a.D = ds->D;
  a.P = ds->P;
  a.n_items = w->n_items;
  a.max_sub = w->max_sub;
  a.model = ds->model;
  a.nc = ds->model == 1 ? 2 : (ds->model == 4 ? 5 : 4);
  a.mc = ds->mc;
  return a;
}

}  // namespace

int grad_loglike(argus_dataset* ds, const double* theta, int64_t S, double* logl, double* grad,
                 int32_t* status, hipStream_t st) {
  const char* mode = std::getenv("ARGUS_GRAD");
  if (!(mode && std::strcmp(mode, "adjoint") == 0) || ds->model == 4)
    return tangent_loglike(ds, theta, S, logl, grad, status, st);
  int rc = ARGUS_OK;
  Workspace* w = get_workspace(ds, S, &rc);
  if (!w) return rc;
  if ((rc = adjoint_setup(ds, w, S))) return rc;
  if (w->gpart.p == nullptr && (rc = w->gpart.alloc((size_t)ds->P * 6 * S * sizeof(double))))
    return rc;
  AdjArgs a = adjoint_args(ds, w, theta, S);
  a.gpart = w->gpart.as<double>();
  hipLaunchKernelGGL(k_adjoint<false>, dim3(w->grad_waves / 4), dim3(256), 0, st, a);
  HIPCHK(hipGetLastError());
  return grad_finish(ds, w, S, logl, grad, status, st);
}

namespace {

// Chunks of the time-parallel smoother for K chunks of the longest pulsar:
// a pulsar of N TOAs gets ceil(N / ceil(N_max / K)) chunks (at most one per
// level-1 segment); per item its chunk count and first slot, and the (item,
// chunk) units ordered by chunk length, longest first. Buffers grow to fit.
int smooth_tp_setup(argus_dataset* ds, Workspace* w, int K) {
  if (w->tp_built_k == K) return ARGUS_OK;
  const bool m4 = ds->model == 4;
  const int fields = m4 ? kF5 : kFields;
  int rc;
  if (w->tp_ck.p == nullptr) {
    // the checkpoint layout of the time-parallel form: the state before
    // every fourth TOA, so that the reverse sweep recomputes at most three
    // steps per TOA and no segment
    std::vector<int32_t> c1(ds->P, 4);
    std::vector<int64_t> seg(ds->P);
    int64_t tot = 0;
    for (int p = 0; p < ds->P; ++p) {
      seg[p] = tot;
      tot += (ds->counts[p] + 3) / 4;
    }
    const int64_t tiles = (w->S + kWave - 1) / kWave;
    if ((rc = w->tp_c1.upload(c1.data(), c1.size() * sizeof(int32_t))) ||
        (rc = w->tp_seg.upload(seg.data(), seg.size() * sizeof(int64_t))) ||
        (rc = w->tp_ck.alloc((size_t)std::max<int64_t>(tiles * tot, 1) * fields * kWave *
                             sizeof(double))))
      return rc;
    w->tp_tot_seg = tot;
  }
  const int64_t nmax =
      ds->counts.empty() ? 1 : std::max<int64_t>(1, *std::max_element(ds->counts.begin(),
                                                                       ds->counts.end()));
  const int64_t lc = (nmax + K - 1) / K;
  std::vector<int32_t> item(2 * (size_t)w->n_items);
  std::vector<std::pair<int64_t, int64_t>> units;  // (-chunk length, item * 65536 + chunk)
  int64_t slots = 0;
  for (int i = 0; i < w->n_items; ++i) {
    const int p = w->items_host[2 * i + 1];
    const int64_t n = ds->counts[p];
    const int64_t c1 = 4;
    const int64_t nseg = (n + c1 - 1) / c1;
    int64_t nch = (n + lc - 1) / lc;
    nch = std::max<int64_t>(1, std::min<int64_t>(nch, std::max<int64_t>(nseg, 1)));
    nch = std::min<int64_t>(nch, 65535);
    item[2 * i] = (int32_t)nch;
    item[2 * i + 1] = (int32_t)slots;
    for (int64_t c = 0; c < nch; ++c) {
      const int64_t lo = std::min(n, (c * nseg / nch) * c1);
      const int64_t hi = std::min(n, ((c + 1) * nseg / nch) * c1);
      units.push_back({-(hi - lo), (int64_t)i * 65536 + c});
    }
    slots += nch;
  }
  if (slots > INT32_MAX) return fail(ARGUS_E_UNSUPPORTED, "time-parallel smoother: too many chunks");
  std::stable_sort(units.begin(), units.end(),
                   [](const auto& x, const auto& y) { return x.first < y.first; });
  std::vector<int32_t> uh(2 * units.size());
  for (size_t u = 0; u < units.size(); ++u) {
    uh[2 * u] = (int32_t)(units[u].second / 65536);
    uh[2 * u + 1] = (int32_t)(units[u].second % 65536);
  }
  // resident reverse waves: two per SIMD for models 1 and 2, one for model 4
  const int waves = (int)std::min<int64_t>((int64_t)units.size(),
                                           (ds->model == 4 ? 4LL : 8LL) * ds->n_cu);
  w->tp_waves = ((std::max(waves, 1) + 3) / 4) * 4;
  const size_t need_sum =
      (size_t)std::max<int64_t>(slots, 1) * (m4 ? kSum5 : kSum) * kWave * sizeof(double);
  const size_t need_adj =
      (size_t)std::max<int64_t>(slots, 1) * (m4 ? kF5 : kFields) * kWave * sizeof(double);
  // level-2 scratch of one state per wave (segments of one piece need none)
  const size_t need_scr = (size_t)w->tp_waves * fields * kWave * sizeof(double);
  if ((rc = w->tp_item.upload(item.data(), item.size() * sizeof(int32_t))) ||
      (rc = w->tp_units.upload(uh.data(), uh.size() * sizeof(int32_t))))
    return rc;
  if (w->tp_sum.bytes < need_sum && (rc = w->tp_sum.alloc(need_sum))) return rc;
  if (w->tp_adj.bytes < need_adj && (rc = w->tp_adj.alloc(need_adj))) return rc;
  if (w->tp_scr.bytes < need_scr && (rc = w->tp_scr.alloc(need_scr))) return rc;
  w->n_tp_units = (int)units.size();
  w->tp_built_k = K;
  return ARGUS_OK;
}

// One smoother launch of the given form (1: one wave per item; K > 1: the
// time-parallel form, the longest pulsars in K chunks) and the reduction of
// the log-likelihood terms.
int smooth_once(argus_dataset* ds, Workspace* w, const AdjArgs& a, int nw, int64_t S,
                double* logl, int32_t* status, hipStream_t st) {
  int rc;
  if (nw == 1) {
    if (ds->model == 4)
      hipLaunchKernelGGL(k_smooth5, dim3(w->grad_waves / 4), dim3(256), 0, st, a);
    else
      hipLaunchKernelGGL(k_adjoint<true>, dim3(w->grad_waves / 4), dim3(256), 0, st, a);
    HIPCHK(hipGetLastError());
  } else {
    if ((rc = smooth_tp_setup(ds, w, nw))) return rc;
    AdjArgs b = a;
    b.tp_item = w->tp_item.as<int32_t>();
    b.tp_units = w->tp_units.as<int32_t>();
    b.tpsum = w->tp_sum.as<double>();
    b.tpadj = w->tp_adj.as<double>();
    b.scratch = w->tp_scr.as<double>();
    b.n_units = w->n_tp_units;
    b.ckpt = w->tp_ck.as<double>();
    b.c1 = w->tp_c1.as<int32_t>();
    b.seg_base = w->tp_seg.as<int64_t>();
    b.tot_seg = w->tp_tot_seg;
    b.max_sub = 1;
    if (ds->model == 4) {
      hipLaunchKernelGGL(k_smooth5_fwd_pc, dim3(w->n_items), dim3(2 * kWave), 0, st, b);
      HIPCHK(hipGetLastError());
      hipLaunchKernelGGL(k_smooth5_rev, dim3(w->tp_waves / 4), dim3(256), 0, st, b);
    } else {
      hipLaunchKernelGGL(k_smooth_fwd_pc, dim3(w->n_items), dim3(2 * kWave), 0, st, b);
      HIPCHK(hipGetLastError());
      hipLaunchKernelGGL(k_smooth_rev, dim3(w->tp_waves / 4), dim3(256), 0, st, b);
    }
    HIPCHK(hipGetLastError());
  }
  double* ll = logl ? logl : w->logl_tmp.as<double>();
  int32_t* stat = status ? status : w->stat_tmp.as<int32_t>();
  ReduceArgs r{w->part.as<double>(), w->pstat.as<int32_t>(), ll, stat, w->counter.as<int32_t>(),
               S, ds->P};
  HIPCHK(launch_reduce(r, st));
  return ARGUS_OK;
}

}  // namespace

// Smoothed latent states: the filter pass with checkpoints and the
// Bryson-Frazier recursion back over it. The first call per sample count
// times the one-wave-per-item sweep against the time-parallel form
// with the longest pulsars in 2, 4, 8 and 16 chunks and keeps the fastest;
// ARGUS_SMOOTH = seq | tp2 | tp4 | tp8 | tp16 forces a form.
int smooth_states(argus_dataset* ds, const double* theta, int64_t S, double* mean, double* var,
                  double* logl, int32_t* status, hipStream_t st) {
  int rc = ARGUS_OK;
  Workspace* w = get_workspace(ds, S, &rc);
  if (!w) return rc;
  if ((rc = adjoint_setup(ds, w, S))) return rc;
  AdjArgs a = adjoint_args(ds, w, theta, S);
  a.smean = mean;
  a.svar = var;
  const char* force = std::getenv("ARGUS_SMOOTH");
  int forced = 0;
  if (force && *force) {
    if (!std::strcmp(force, "seq")) forced = 1;
    else if (!std::strcmp(force, "tp2")) forced = 2;
    else if (!std::strcmp(force, "tp4")) forced = 4;
    else if (!std::strcmp(force, "tp8")) forced = 8;
    else if (!std::strcmp(force, "tp16")) forced = 16;
    else return fail(ARGUS_E_INVAL, "ARGUS_SMOOTH: seq, tp2, tp4, tp8 or tp16");
  }
  if (forced) return smooth_once(ds, w, a, forced, S, logl, status, st);
  if (!w->smooth_k) {
    const std::vector<int> cand = {1, 2, 4, 8, 16};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 1e30f;
    int pick = 1;
    w->smooth_log.clear();
    for (int nw : cand) {
      float m = 1e30f;
      for (int rep = 0; rep < 2 && rc == ARGUS_OK; ++rep) {
        if (hipEventRecord(e0, st) != hipSuccess) rc = fail(ARGUS_E_HIP, "event");
        if (!rc) rc = smooth_once(ds, w, a, nw, S, logl, status, st);
        if (!rc && hipEventRecord(e1, st) != hipSuccess) rc = fail(ARGUS_E_HIP, "event");
        if (!rc && hipEventSynchronize(e1) != hipSuccess) rc = fail(ARGUS_E_HIP, "sync");
        float ms = 0;
        if (!rc && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(ARGUS_E_HIP, "t");
        if (!rc) m = std::min(m, ms);
      }
      if (rc == ARGUS_E_NOMEM && nw > 1) {
        // the time-parallel form's checkpoint store did not fit: drop the
        // form (its buffers too) and keep timing the others
        w->tp_ck.release();
        w->tp_sum.release();
        w->tp_adj.release();
        w->tp_built_k = 0;
        char line[96];
        std::snprintf(line, sizeof line, "  smoother tp%d: not enough device memory\n", nw);
        w->smooth_log += line;
        rc = ARGUS_OK;
        continue;
      }
      if (rc) break;
      char line[96];
      std::snprintf(line, sizeof line, "  smoother %s%d: %.3f ms\n", nw == 1 ? "seq" : "tp", nw,
                    m);
      w->smooth_log += line;
      if (m < best) {
        best = m;
        pick = nw;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    w->smooth_k = pick;
  }
  return smooth_once(ds, w, a, w->smooth_k, S, logl, status, st);
}

}  // namespace argus
