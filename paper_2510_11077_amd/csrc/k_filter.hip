// Batched Kalman filters of independent pulsars (models 1 and 2), the
// per-TOA staging kernel, the Hellings-Downs matrix, the per-sample
// reduction, and the plain per-sample baseline filter.
//
// Method (paper: Functionality, "Kalman filter likelihood evaluation"): for
// each TOA the filter discretises the SDEs over the interval since the
// previous TOA (transition F, process noise Q), predicts, forms the
// innovation e and its variance S, updates the state and covariance, and
// accumulates -1/2 (ln 2 pi + ln S + e^2 / S).
//
// Mapping on CDNA4: one wavefront owns one (64-sample tile, pulsar) filter:
// lane = sample. All lanes walk the same TOA stream, so every per-TOA value
// is wave-uniform and is read with scalar loads from one 64-B record; each
// lane keeps its 4-state mean and the 10 unique covariance entries in VGPRs.
// The covariance update is the Joseph form written as the symmetric rank-2
// expression P - K u^T - u K^T + S K K^T (u = P H^T), which equals
// (I - K H) P (I - K H)^T + K R K^T for any gain K. ln S is accumulated as a
// product of mantissas with exponent extraction (frexp), one log per filter.
// Waves take work items from a longest-first queue (atomic head) so pulsars
// of uneven length balance across the 1024 SIMDs.
#include "argus_internal.h"

namespace argus {

namespace {

__device__ __forceinline__ bool finite_d(double v) {
  return __builtin_amdgcn_class(v, 0x1F8);  // -normal..+normal incl. zeros
}

// First-failure classification, same order of tests as the definition:
// a non-finite S or e is NONFINITE, otherwise S <= 0 is NONPD. The common
// case (S positive and finite, e finite) costs two class tests.
__device__ __forceinline__ void step_status(int& st, double S, double e) {
  const bool good = __builtin_amdgcn_class(S, 0x180) & finite_d(e);
  if (__builtin_expect(!good, 0)) {
    if (st == 0) st = (!finite_d(S) || !finite_d(e)) ? kNonFinite : kNonPD;
  }
}

struct LogAcc {
  double m;
  int e;
};
__device__ __forceinline__ void acc_mul(LogAcc& L, double S) {
  const double p = L.m * S;
  L.m = __builtin_amdgcn_frexp_mant(p);
  L.e += __builtin_amdgcn_frexp_exp(p);
}
__device__ __forceinline__ double acc_log(const LogAcc& L) {
  return log(L.m) + (double)L.e * kLn2;
}

__device__ __forceinline__ double load_param(const FilterArgs& a, int c,
                                             int64_t s) {
  const int j = a.col[c];
  return j >= 0 ? a.theta[s * a.D + j] : a.fixed[c];
}

// Stationary variance of the common OU process from the power law (log10 A,
// gamma): A^2 f_yr^(gamma-3) T^(gamma-1) / (12 pi^2 (gamma-1)).
__device__ __forceinline__ double common_var(double la, double gc,
                                             const ModelConst& mc) {
  const double gm1 = gc - 1.0;
  return exp(2.0 * kLn10 * la + (gc - 3.0) * mc.log_fyr + gm1 * mc.log_T) /
         (12.0 * kPi * kPi * gm1);
}

// Joseph update of one covariance entry. The symmetric rank-2 form
// P - K u^T - u K^T + S K K^T is regrouped as P - K u^T + (S K - u) K^T,
// the same expression for any gain K; d = S K - u is formed with one
// rounding (fma), so the small residual of the optimal gain is not lost to
// cancellation.
#define JOSEPH(pij, ki, uj, di, kj) pij = fma(di, kj, fma(-(ki), uj, pij))

// ------------------------------------------------------------ model 2 step
struct F4 {
  double xr, xf, xa, xg;
  double prr, prf, pff, pra, pfa, paa, prg, pfg, pag, pgg;
  double quad;
  LogAcc L;
  int st;
};

// em = expm1(-rate dt) for this record (computed a step ahead by the caller:
// it does not depend on the state, so it overlaps the previous step's chain)
__device__ __forceinline__ void step4(F4& f, const TOARec r, double em,
                                      double vr, double vc, double efac2,
                                      double equad2, double ss2) {
  const double dt = r.dt;
  // red OU over dt for this lane's rate: phi = 1 + expm1(-g dt),
  // q = v (1 - phi^2) = -v em (2 + em) without cancellation
  const double phr = 1.0 + em;
  const double qr = vr * (-em * (2.0 + em));
  const double phc = r.phc;
  const double qc = vc * r.qcu;
  // predict mean
  f.xr = fma(dt, f.xf, f.xr);
  f.xa *= phr;
  f.xg *= phc;
  // predict covariance F P F^T + Q
  const double prf1 = fma(dt, f.pff, f.prf);
  f.prr = fma(dt, f.prf + prf1, f.prr) + ss2 * r.h3;
  f.prf = prf1 + ss2 * r.h2;
  f.pff = f.pff + ss2 * dt;
  f.pra = phr * fma(dt, f.pfa, f.pra);
  f.pfa = phr * f.pfa;
  f.paa = fma(phr * phr, f.paa, qr);
  f.prg = phc * fma(dt, f.pfg, f.prg);
  f.pfg = phc * f.pfg;
  f.pag = (phr * phc) * f.pag;
  f.pgg = fma(phc * phc, f.pgg, qc);
  // innovation, H = [1, 0, 1, 1]
  const double e = r.y - (f.xr + f.xa + f.xg);
  const double ur = f.prr + f.pra + f.prg;
  const double uf = f.prf + f.pfa + f.pfg;
  const double ua = f.pra + f.paa + f.pag;
  const double ug = f.prg + f.pag + f.pgg;
  const double S = (ur + ua + ug) + fma(efac2, r.s2, equad2);
  step_status(f.st, S, e);
  const double inv = rcp_nr(S);
  const double kr = ur * inv, kf = uf * inv, ka = ua * inv, kg = ug * inv;
  f.xr = fma(kr, e, f.xr);
  f.xf = fma(kf, e, f.xf);
  f.xa = fma(ka, e, f.xa);
  f.xg = fma(kg, e, f.xg);
  const double dr = fma(S, kr, -ur), df = fma(S, kf, -uf);
  const double da = fma(S, ka, -ua), dg = fma(S, kg, -ug);
  JOSEPH(f.prr, kr, ur, dr, kr);
  JOSEPH(f.prf, kr, uf, dr, kf);
  JOSEPH(f.pff, kf, uf, df, kf);
  JOSEPH(f.pra, kr, ua, dr, ka);
  JOSEPH(f.pfa, kf, ua, df, ka);
  JOSEPH(f.paa, ka, ua, da, ka);
  JOSEPH(f.prg, kr, ug, dr, kg);
  JOSEPH(f.pfg, kf, ug, df, kg);
  JOSEPH(f.pag, ka, ug, da, kg);
  JOSEPH(f.pgg, kg, ug, dg, kg);
  f.quad = fma(e * e, inv, f.quad);
  acc_mul(f.L, S);
}

// ------------------------------------------------- model 2 step, fast form
// The same recursion as step4 with fewer instructions for the common case:
// no per-step failure classification and no per-step exponent extraction.
// ln S is accumulated as a plain product of S over groups of kGroup steps,
// its exponent extracted once per group (group_end), and every S compared
// with 2^-120; a filter whose S ever falls below 2^-120 (including S <= 0), whose
// product leaves the positive normal range, or whose result is not finite is
// re-run by the caller with step4, whose per-step tests decide the status
// word. The red-OU decay comes from expm1_fast, which needs |rate dt| <=
// 2^30 ln 2 (the caller checks every item against its pulsar's largest
// interval). With S >= 2^-120 a group's partial products stay above
// 2^-961, so no product passes through the subnormal range.
constexpr int kGroup = 8;

struct F4f {
  double xr, xf, xa, xg;
  double prr, prf, pff, pra, pfa, paa, prg, pfg, pag, pgg;
  double quad, lm;
  int le;
};

// Coefficients of H(u) = (expm1(u ln 2) - u ln 2) / u^2 on |u| <= 1/2,
// highest degree first: its 10-term Chebyshev fit (expm1_coef.py beside this
// file); the fit's own error contributes at most 3.7e-17 relative to expm1.
__constant__ double kExpm1H[10] = {
    0.000000000445410341058704017628, 0.00000000707097786650813855584,
    0.000000101780672674494267932,    0.00000132154516332214343743,
    0.0000152527338207958030237,      0.000154035304247765275866,
    0.0013333558146423213121,         0.00961812910761866557058,
    0.0555041086648215825683,         0.240226506959100761392};

// the coefficients, ln 2 and the rounding constant 1.5 * 2^52, all in VGPRs
// (an FP64 instruction reads at most one SGPR, and the step's other operands
// are the record's SGPRs)
struct Expm1H {
  double c[10];
  double ln2, magic;
};
__device__ __forceinline__ Expm1H expm1h_vgpr() {
  Expm1H k;
#pragma unroll
  for (int i = 0; i < 10; ++i) {
    k.c[i] = kExpm1H[i];
    asm volatile("" : "+v"(k.c[i]));
  }
  k.ln2 = in_vgpr(kLn2);
  k.magic = in_vgpr(6755399441055744.0);
  return k;
}

// expm1(-g dt) for gl = g / ln 2 with 0 <= gl dt <= 2^30. Adding
// 1.5 * 2^52 rounds -gl dt to the nearest integer k (ties to even), and the
// low 32 bits of that sum are k itself (|k| < 2^31); u = -gl dt - k is
// formed with one rounding (exact product in the fma), |u| <= 1/2;
// expm1(u ln 2) = u (ln 2 + u H(u)); expm1(-g dt) = 2^k expm1(u ln 2) +
// (2^k - 1), where 2^k underflows to 0 (the result -1) below k = -1074.
__device__ __forceinline__ double expm1_fast(double gl, double dt, const Expm1H& h) {
  const double t = __builtin_fma(-gl, dt, h.magic);
  const double kf = t - h.magic;
  const double u = __builtin_fma(-gl, dt, -kf);
  double q = __builtin_fma(h.c[0], u, h.c[1]);
#pragma unroll
  for (int i = 2; i < 10; ++i) q = __builtin_fma(q, u, h.c[i]);
  const double p = u * __builtin_fma(q, u, h.ln2);
  const int k = (int)(uint32_t)__builtin_bit_cast(uint64_t, t);
  const double tk = __builtin_ldexp(1.0, k);
  return __builtin_fma(tk, p, tk - 1.0);
}

__device__ __forceinline__ void step4_fast(F4f& f, double dt, double h2, double h3, double phc,
                                           double qcu, double y, double s2, double phc2,
                                           double em, double vr, double vr2, double vc,
                                           double efac2, double equad2, double ss2, bool& ok) {
  const double phr = 1.0 + em;
  // vr (1 - phr^2) = -vr em (2 + em) = -em (vr em + 2 vr)
  const double qr = -em * fma(vr, em, vr2);
  const double qc = vc * qcu;
  f.xr = fma(dt, f.xf, f.xr);
  f.xa *= phr;
  f.xg *= phc;
  const double prf1 = fma(dt, f.pff, f.prf);
  f.prr = fma(dt, f.prf + prf1, f.prr) + ss2 * h3;
  f.prf = prf1 + ss2 * h2;
  f.pff = f.pff + ss2 * dt;
  f.pra = phr * fma(dt, f.pfa, f.pra);
  f.pfa = phr * f.pfa;
  f.paa = fma(phr * phr, f.paa, qr);
  f.prg = phc * fma(dt, f.pfg, f.prg);
  f.pfg = phc * f.pfg;
  f.pag = (phr * phc) * f.pag;
  f.pgg = fma(phc2, f.pgg, qc);
  const double e = y - (f.xr + f.xa + f.xg);
  const double ur = f.prr + f.pra + f.prg;
  const double uf = f.prf + f.pfa + f.pfg;
  const double ua = f.pra + f.paa + f.pag;
  const double ug = f.prg + f.pag + f.pgg;
  const double S = (ur + ua + ug) + fma(efac2, s2, equad2);
  const double inv = rcp_nr(S);
  const double kr = ur * inv, kf = uf * inv, ka = ua * inv, kg = ug * inv;
  f.xr = fma(kr, e, f.xr);
  f.xf = fma(kf, e, f.xf);
  f.xa = fma(ka, e, f.xa);
  f.xg = fma(kg, e, f.xg);
  const double dr = fma(S, kr, -ur), df = fma(S, kf, -uf);
  const double da = fma(S, ka, -ua), dg = fma(S, kg, -ug);
  JOSEPH(f.prr, kr, ur, dr, kr);
  JOSEPH(f.prf, kr, uf, dr, kf);
  JOSEPH(f.pff, kf, uf, df, kf);
  JOSEPH(f.pra, kr, ua, dr, ka);
  JOSEPH(f.pfa, kf, ua, df, ka);
  JOSEPH(f.paa, ka, ua, da, ka);
  JOSEPH(f.prg, kr, ug, dr, kg);
  JOSEPH(f.pfg, kf, ug, df, kg);
  JOSEPH(f.pag, ka, ug, da, kg);
  JOSEPH(f.pgg, kg, ug, dg, kg);
  f.quad = fma(e * e, inv, f.quad);
  f.lm *= S;
  ok = ok && S >= 0x1p-120;
}

// end of a group: the product must be a positive normal number; its
// exponent moves to the integer accumulator
__device__ __forceinline__ void group_end(F4f& f, bool& ok) {
  ok = ok && __builtin_amdgcn_class(f.lm, 0x100);
  f.le += __builtin_amdgcn_frexp_exp(f.lm);
  f.lm = __builtin_amdgcn_frexp_mant(f.lm);
}

// ------------------------------------------------------------ model 4 step
// The model 2 state plus m, the DM delay at the reference frequency (an OU
// process), observed with the chromatic factor c = (nu_ref / nu)^2 of the
// TOA: h = [1, 0, 1, 1, c].
struct F5 {
  double xr, xf, xa, xg, xm;
  double prr, prf, pff, pra, pfa, paa, prg, pfg, pag, pgg, prm, pfm, pam, pgm, pmm;
  double quad;
  LogAcc L;
  int st;
};

// em, emd = expm1(-rate dt) of the red and DM processes for this record
__device__ __forceinline__ void step5(F5& f, const TOARec r, double c, double em, double emd,
                                      double vr, double vc, double vd, double efac2,
                                      double equad2, double ss2) {
  const double dt = r.dt;
  const double phr = 1.0 + em, phd = 1.0 + emd;
  const double qr = vr * (-em * (2.0 + em));
  const double qd = vd * (-emd * (2.0 + emd));
  const double phc = r.phc;
  const double qc = vc * r.qcu;
  f.xr = fma(dt, f.xf, f.xr);
  f.xa *= phr;
  f.xg *= phc;
  f.xm *= phd;
  const double prf1 = fma(dt, f.pff, f.prf);
  f.prr = fma(dt, f.prf + prf1, f.prr) + ss2 * r.h3;
  f.prf = prf1 + ss2 * r.h2;
  f.pff = f.pff + ss2 * dt;
  f.pra = phr * fma(dt, f.pfa, f.pra);
  f.pfa = phr * f.pfa;
  f.paa = fma(phr * phr, f.paa, qr);
  f.prg = phc * fma(dt, f.pfg, f.prg);
  f.pfg = phc * f.pfg;
  f.pag = (phr * phc) * f.pag;
  f.pgg = fma(phc * phc, f.pgg, qc);
  f.prm = phd * fma(dt, f.pfm, f.prm);
  f.pfm = phd * f.pfm;
  f.pam = (phr * phd) * f.pam;
  f.pgm = (phc * phd) * f.pgm;
  f.pmm = fma(phd * phd, f.pmm, qd);
  const double e = r.y - fma(c, f.xm, f.xr + f.xa + f.xg);
  const double ur = fma(c, f.prm, f.prr + f.pra + f.prg);
  const double uf = fma(c, f.pfm, f.prf + f.pfa + f.pfg);
  const double ua = fma(c, f.pam, f.pra + f.paa + f.pag);
  const double ug = fma(c, f.pgm, f.prg + f.pag + f.pgg);
  const double um = fma(c, f.pmm, f.prm + f.pam + f.pgm);
  const double S = fma(c, um, ur + ua + ug) + fma(efac2, r.s2, equad2);
  step_status(f.st, S, e);
  const double inv = rcp_nr(S);
  const double kr = ur * inv, kf = uf * inv, ka = ua * inv, kg = ug * inv, km = um * inv;
  f.xr = fma(kr, e, f.xr);
  f.xf = fma(kf, e, f.xf);
  f.xa = fma(ka, e, f.xa);
  f.xg = fma(kg, e, f.xg);
  f.xm = fma(km, e, f.xm);
  const double dr = fma(S, kr, -ur), df = fma(S, kf, -uf);
  const double da = fma(S, ka, -ua), dg = fma(S, kg, -ug), dm = fma(S, km, -um);
  JOSEPH(f.prr, kr, ur, dr, kr);
  JOSEPH(f.prf, kr, uf, dr, kf);
  JOSEPH(f.pff, kf, uf, df, kf);
  JOSEPH(f.pra, kr, ua, dr, ka);
  JOSEPH(f.pfa, kf, ua, df, ka);
  JOSEPH(f.paa, ka, ua, da, ka);
  JOSEPH(f.prg, kr, ug, dr, kg);
  JOSEPH(f.pfg, kf, ug, df, kg);
  JOSEPH(f.pag, ka, ug, da, kg);
  JOSEPH(f.pgg, kg, ug, dg, kg);
  JOSEPH(f.prm, kr, um, dr, km);
  JOSEPH(f.pfm, kf, um, df, km);
  JOSEPH(f.pam, ka, um, da, km);
  JOSEPH(f.pgm, kg, um, dg, km);
  JOSEPH(f.pmm, km, um, dm, km);
  f.quad = fma(e * e, inv, f.quad);
  acc_mul(f.L, S);
}

// ------------------------------------------------------------ model 1 step
struct F2 {
  double xr, xf, prr, prf, pff, quad;
  LogAcc L;
  int st;
};

__device__ __forceinline__ void step2(F2& f, const TOARec r, double ss2,
                                      double efac2) {
  const double dt = r.dt;
  f.xr = fma(dt, f.xf, f.xr);
  const double prf1 = fma(dt, f.pff, f.prf);
  f.prr = fma(dt, f.prf + prf1, f.prr) + ss2 * r.h3;
  f.prf = prf1 + ss2 * r.h2;
  f.pff = f.pff + ss2 * dt;
  const double e = r.y - f.xr;
  const double ur = f.prr, uf = f.prf;
  const double S = ur + efac2 * r.s2;
  step_status(f.st, S, e);
  const double inv = rcp_nr(S);
  const double kr = ur * inv, kf = uf * inv;
  f.xr = fma(kr, e, f.xr);
  f.xf = fma(kf, e, f.xf);
  const double dr = fma(S, kr, -ur), df = fma(S, kf, -uf);
  JOSEPH(f.prr, kr, ur, dr, kr);
  JOSEPH(f.prf, kr, uf, dr, kf);
  JOSEPH(f.pff, kf, uf, df, kf);
  f.quad = fma(e * e, inv, f.quad);
  acc_mul(f.L, S);
}

__device__ __forceinline__ double finish(double n, double quad,
                                         const LogAcc& L, int& st) {
  double ll = -0.5 * (n * kLn2Pi + acc_log(L) + quad);
  if (st == 0 && !finite_d(ll)) st = kNonFinite;
  return st ? -INFINITY : ll;
}

// MAXT: launch bound (256, or 1024 for the one-block-per-CU layout).
// FAST (model 2): the fast loop only; an item it cannot decide is marked in
// a.redo (one flag per item, written for every item) and left to the general
// loop, which a second launch (FAST = false with a.redo set) runs on the
// marked items only.
template <int MODEL, int MAXT, bool FAST>
__global__ void __launch_bounds__(MAXT) k_filter(FilterArgs a) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wpb = blockDim.x / kWave;
  const int gwave = __builtin_amdgcn_readfirstlane(
      (int)(blockIdx.x * wpb + (threadIdx.x / kWave)));
  const int nwaves = gridDim.x * wpb;
  // per-SIMD queues (one block per CU): the host splits the items into one
  // list per SIMD of about equal TOA steps; a wave reads which SIMD it runs
  // on and takes items, longest first, from that SIMD's list, then from the
  // other three, so every item is taken wherever the waves were placed. A
  // SIMD issues from its older waves first, so what sets its finishing time
  // is the total it is given, which is what the lists balance.
  __shared__ int q_head[4];
  int simd = 0, q_sl = 0, q_lo = 0, q_hi = 0;
  if (a.dynamic == 2) {
    if (threadIdx.x < 4) q_head[threadIdx.x] = 0;
    __syncthreads();
    simd = (int)((__builtin_amdgcn_s_getreg((31 << 11) | 4) >> 4) & 3);  // HW_ID.SIMD_ID
    q_lo = a.bin_off[4 * blockIdx.x + simd];
    q_hi = a.bin_off[4 * blockIdx.x + simd + 1];
  }
  int next = gwave;
  for (;;) {
    int it;
    if (a.dynamic == 1) {
      int v = 0;
      if (lane == 0) v = atomicAdd(a.counter, 1);
      it = __builtin_amdgcn_readfirstlane(v);
    } else if (a.dynamic == 2) {
      // next item of list (simd + q_sl) % 4; an exhausted list moves on
      for (;;) {
        int v = 0;
        if (lane == 0) v = atomicAdd(&q_head[(simd + q_sl) & 3], 1);
        it = q_lo + __builtin_amdgcn_readfirstlane(v);
        if (it < q_hi || ++q_sl == 4) break;
        const int sl = (simd + q_sl) & 3;
        q_lo = a.bin_off[4 * blockIdx.x + sl];
        q_hi = a.bin_off[4 * blockIdx.x + sl + 1];
      }
      if (it >= q_hi) break;
    } else {
      it = next;
      next += nwaves;
    }
    if (a.dynamic != 2 && it >= a.n_items) break;
    // general form after the fast one (model 2): the marked items only
    if (MODEL == 2 && !FAST && a.redo && !a.redo[it]) continue;
    const int tile = a.items ? a.items[2 * it] : it % a.tiles;
    const int p = a.items ? a.items[2 * it + 1] : a.porder[it / a.tiles];
    const int64_t s_raw = (int64_t)tile * kWave + lane;
    const bool valid = s_raw < a.S;
    const int64_t s = valid ? s_raw : a.S - 1;
    // TOA range of the pulsar (wave-uniform; the host bounds N below 2^31),
    // so the record index and loop control live in SGPRs
    const int kb = __builtin_amdgcn_readfirstlane((int)a.off[p]);
    const int ke = __builtin_amdgcn_readfirstlane((int)a.off[p + 1]);
    double ll;
    int st;
    if (MODEL == 1) {
      const double lss = load_param(a, 0, s), efac = load_param(a, 1, s);
      const bool pnf = !(finite_d(lss) && finite_d(efac));
      const double ss = exp10(lss);
      const double ss2 = ss * ss, efac2 = efac * efac;
      F2 f{0.0, 0.0, a.mc.s_r2, 0.0, a.mc.s_f2, 0.0, {1.0, 0}, pnf ? kPNF : 0};
      const RecPtr rec = (RecPtr)a.rec;
      // the next record is fetched one step ahead (index clamped)
      TOARec rn{};
      if (kb < ke) rn = load_rec(rec, kb);
      for (int k = kb; k < ke; ++k) {
        const TOARec r = rn;
        rn = load_rec(rec, k + 1 < ke ? k + 1 : k);
        step2(f, r, ss2, efac2);
      }
      st = f.st;
      ll = finish((double)(ke - kb), f.quad, f.L, st);
    } else if (MODEL == 4) {
      const int c0 = 6 * p, cc = 6 * a.P;
      const double lsr = load_param(a, c0, s), lgr = load_param(a, c0 + 1, s);
      const double efac = load_param(a, c0 + 2, s), leq = load_param(a, c0 + 3, s);
      const double lsd = load_param(a, c0 + 4, s), lgd = load_param(a, c0 + 5, s);
      const double la = load_param(a, cc, s), gc = load_param(a, cc + 1, s);
      const bool pnf = !(finite_d(lsr) && finite_d(lgr) && finite_d(efac) && finite_d(leq) &&
                         finite_d(lsd) && finite_d(lgd) && finite_d(la) && finite_d(gc));
      const double gr = exp10(lgr), sr = exp10(lsr), eq = exp10(leq);
      const double gd = exp10(lgd), sd = exp10(lsd);
      const double vr = sr * sr / (2.0 * gr), vd = sd * sd / (2.0 * gd);
      const double vc = common_var(la, gc, a.mc);
      const double efac2 = efac * efac, equad2 = eq * eq;
      F5 f{};
      f.prr = a.mc.s_r2;
      f.pff = a.mc.s_f2;
      f.paa = vr;
      f.pgg = vc;
      f.pmm = vd;
      f.L = {1.0, 0};
      f.st = pnf ? kPNF : 0;
      const double ss2 = a.mc.ss2;
      const RecPtr rec = (RecPtr)a.rec;
      const ConstDPtr chrom = (ConstDPtr)a.chrom;
      const double ss2v = in_vgpr(ss2), c13 = in_vgpr(kExpm1Coef[11]);
      // The record and chromatic factor of step k + 1 are fetched during
      // step k; both decays of step k + 1 are computed during step k from
      // its dt, which was fetched alone (8 B) during step k - 1, so no value
      // is used in the step that fetches it (indices clamped).
      const RecVecPtr recv = (RecVecPtr)a.rec;
      const ConstDPtr dts = (ConstDPtr)a.rec;  // dt is the first of each record's 8 doubles
      RecVec vn{};
      double cn = 0.0, emn = 0.0, emdn = 0.0, dt2 = 0.0;
      if (kb < ke) {
        vn = load_rec_v(recv, kb);
        cn = chrom[kb];
        dt2 = dts[8 * (int64_t)(kb + 1 < ke ? kb + 1 : kb)];
        emn = expm1_v(-gr * vn[0], c13);
        emdn = expm1_v(-gd * vn[0], c13);
      }
      for (int k = kb; k < ke; ++k) {
        const RecVec v = vn;
        const double c = cn, em = emn, emd = emdn, dt1 = dt2;
        rec_keep(v);
        sgpr_ready(dt1);
        const TOARec r = rec_fields(v);
        const int kn = k + 1 < ke ? k + 1 : k;
        vn = load_rec_v(recv, kn);
        cn = chrom[kn];
        dt2 = dts[8 * (int64_t)(k < ke - 2 ? k + 2 : ke - 1)];
        emn = expm1_v(-gr * dt1, c13);
        emdn = expm1_v(-gd * dt1, c13);
        step5(f, r, c, em, emd, vr, vc, vd, efac2, equad2, ss2v);
      }
      st = f.st;
      ll = finish((double)(ke - kb), f.quad, f.L, st);
    } else {
      const int c0 = 4 * p, cc = 4 * a.P;
      const double lsr = load_param(a, c0, s), lgr = load_param(a, c0 + 1, s);
      const double efac = load_param(a, c0 + 2, s);
      const double leq = load_param(a, c0 + 3, s);
      const double la = load_param(a, cc, s), gc = load_param(a, cc + 1, s);
      const bool pnf = !(finite_d(lsr) && finite_d(lgr) && finite_d(efac) &&
                         finite_d(leq) && finite_d(la) && finite_d(gc));
      const double gr = exp10(lgr), sr = exp10(lsr), eq = exp10(leq);
      const double vr = sr * sr / (2.0 * gr);
      const double vc = common_var(la, gc, a.mc);
      const double efac2 = efac * efac, equad2 = eq * eq;
      const double ss2 = a.mc.ss2;
      const RecPtr rec = (RecPtr)a.rec;
      const double ss2v = in_vgpr(ss2);
      // fast form unless a parameter is not finite or the red-OU exponent
      // could leave expm1_fast's range on this pulsar
      const double gl = gr * 1.44269504088896338700;
      const bool fast_lane = !pnf && gl * a.maxdt[p] <= 0x1p30;
      bool done = false;
      if (FAST && __builtin_amdgcn_ballot_w64(!fast_lane) == 0) {
        const Expm1H hc = expm1h_vgpr();
        const double vr2 = 2.0 * vr;
        F4f g{};
        g.prr = a.mc.s_r2;
        g.pff = a.mc.s_f2;
        g.paa = vr;
        g.pgg = vc;
        g.lm = 1.0;
        bool ok = true;
        // The record of step k + 1 is fetched during step k (as one 64-B
        // scalar vector, its last double phc^2); the red decay of step k + 1
        // is computed during step k from its dt, fetched alone during step
        // k - 1 (indices clamped), so no value is used in the step that
        // fetches it.
        const RecVecPtr recv = (RecVecPtr)a.rec;
        const ConstDPtr dts = (ConstDPtr)a.rec;  // dt: first double of each record
        RecVec vn{};
        double emn = 0.0, dt2 = 0.0;
        if (kb < ke) {
          vn = load_rec_v(recv, kb);
          dt2 = dts[8 * (int64_t)(kb + 1 < ke ? kb + 1 : kb)];
          emn = expm1_fast(gl, vn[0], hc);
        }
        auto one = [&](int k) {
          const RecVec v = vn;
          const double em = emn, dt1 = dt2;
          rec_keep(v);
          sgpr_ready(dt1);
          vn = load_rec_v(recv, k + 1 < ke ? k + 1 : k);
          dt2 = dts[8 * (int64_t)(k < ke - 2 ? k + 2 : ke - 1)];
          emn = expm1_fast(gl, dt1, hc);
          step4_fast(g, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], em, vr, vr2, vc, efac2,
                     equad2, ss2v, ok);
        };
        int k = kb;
        for (; k + kGroup <= ke; k += kGroup) {
#pragma unroll 2
          for (int j = 0; j < kGroup; ++j) one(k + j);
          group_end(g, ok);
        }
        if (k < ke) {
          for (; k < ke; ++k) one(k);
          group_end(g, ok);
        }
        ll = -0.5 * ((double)(ke - kb) * kLn2Pi + (log(g.lm) + (double)g.le * kLn2) + g.quad);
        st = 0;
        const bool bad = !ok || !finite_d(ll);
        done = __builtin_amdgcn_ballot_w64(bad) == 0;
      }
      if (FAST) {
        if (lane == 0) a.redo[it] = done ? 0 : 1;
        if (!done) continue;
      } else {
      F4 f{};
      f.prr = a.mc.s_r2;
      f.pff = a.mc.s_f2;
      f.paa = vr;
      f.pgg = vc;
      f.L = {1.0, 0};
      f.st = pnf ? kPNF : 0;
      const Expm1Coef kc = expm1_coef_vgpr();
      // Two records in flight: step k waits for the record of step k + 1
      // (fetched during step k - 1), evaluates its red decay, and fetches
      // the record of step k + 2, so every scalar load has a whole step to
      // arrive; the last steps refetch the final record (index clamped).
      TOARec r1{}, r2{};
      double em1 = 0.0;
      if (kb < ke) {
        r1 = load_rec(rec, kb);
        r2 = load_rec(rec, kb + 1 < ke ? kb + 1 : kb);
        em1 = expm1_c(-gr * r1.dt, kc);
      }
      for (int k = kb; k < ke; ++k) {
        const TOARec r = r1;
        const double em = em1;
        r1 = r2;
        sgpr_ready(r1.dt);
        r2 = load_rec(rec, k < ke - 2 ? k + 2 : ke - 1);
        em1 = expm1_c(-gr * r1.dt, kc);
        step4(f, r, em, vr, vc, efac2, equad2, ss2v);
      }
      st = f.st;
      ll = finish((double)(ke - kb), f.quad, f.L, st);
      }
    }
    if (valid) {
      a.part[(int64_t)p * a.S + s] = ll;
      a.pstat[(int64_t)p * a.S + s] = st;
    }
  }
}

// logL[s] = sum over pulsars in index order; status = first failure in
// pulsar order, NONFINITE if any parameter of the row is not finite.
__global__ void k_reduce(ReduceArgs a) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (blockIdx.x == 0 && threadIdx.x == 0 && a.counter) *a.counter = 0;
  if (s >= a.S) return;
  double acc = 0.0;
  int st = 0;
  bool pnf = false;
  // pulsars in batches: a batch's loads are all issued before its sums, so
  // a thread waits once per batch instead of once per pulsar; the sum is
  // still taken in pulsar order
  constexpr int kBatch = 16;
  for (int p0 = 0; p0 < a.P; p0 += kBatch) {
    double v[kBatch];
    int c[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int p = p0 + j;
      v[j] = p < a.P ? a.part[(int64_t)p * a.S + s] : 0.0;
      c[j] = p < a.P ? a.pstat[(int64_t)p * a.S + s] : 0;
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      if (p0 + j >= a.P) break;
      acc += v[j];
      if (c[j] & kPNF)
        pnf = true;
      else if (c[j] && !st)
        st = c[j];
    }
  }
  if (pnf) st = kNonFinite;
  a.logl[s] = st ? -INFINITY : acc;
  if (a.status) a.status[s] = st;
}

__global__ void k_stage(StageArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.N) return;
  const int64_t j = a.src[k], pj = a.prev[k];
  const double dt = a.t[j] - (pj >= 0 ? a.t[pj] : 0.0);
  TOARec r;
  r.dt = dt;
  r.h2 = dt * dt * 0.5;
  r.h3 = dt * dt * dt / 3.0;
  const double em = expm1(-a.lam * dt);
  r.phc = 1.0 + em;
  r.qcu = -em * (2.0 + em);
  r.y = a.y[j];
  const double sg = a.sig[j];
  r.s2 = sg * sg;
  if (a.merged) {
    r.psr = a.psr[k];
    r.pad = 0;
  } else {
    const double p2 = r.phc * r.phc;
    __builtin_memcpy(&r.psr, &p2, sizeof p2);
  }
  a.rec[k] = r;
}

// Hellings & Downs (1983) correlation with the pulsar term on the diagonal:
// G_ab = 3/2 x ln x - x/4 + 1/2 + delta_ab/2, x = (1 - cos zeta_ab)/2.
__global__ void k_hd(const double* pos, int P, double* G) {
  const int a = blockIdx.x;
  if (a >= P) return;
  for (int b = threadIdx.x; b < P; b += blockDim.x) {
    const double c = pos[3 * a] * pos[3 * b] + pos[3 * a + 1] * pos[3 * b + 1] +
                     pos[3 * a + 2] * pos[3 * b + 2];
    double x = a == b ? 0.0 : 0.5 * (1.0 - c);
    x = x < 0.0 ? 0.0 : x;
    const double xl = x > 0.0 ? x * log(x) : 0.0;
    G[a * P + b] = 1.5 * xl - 0.25 * x + 0.5 + (a == b ? 0.5 : 0.0);
  }
}

// ------------------------------------------------ plain per-sample baseline
// One thread per pulsar filter of one sample: textbook dense recursion with
// the transition and noise rebuilt from exp/expm1 at every TOA, Joseph form
// via explicit (I - K H), one log and one division per TOA.
template <int N>
__device__ double plain_filter(const PlainArgs& a, int p, int& st) {
  double lss = 0, efac, leq = 0, lsr = 0, lgr = 0, la = 0, gc = 2;
  auto prm = [&](int c) {
    const int j = a.col[c];
    return j >= 0 ? a.theta_row[j] : a.fixed[c];
  };
  if (N == 2) {
    lss = prm(0);
    efac = prm(1);
  } else {
    lsr = prm(4 * p);
    lgr = prm(4 * p + 1);
    efac = prm(4 * p + 2);
    leq = prm(4 * p + 3);
    la = prm(4 * a.P);
    gc = prm(4 * a.P + 1);
  }
  st = 0;
  if (!(finite_d(lss) && finite_d(efac) && finite_d(leq) && finite_d(lsr) &&
        finite_d(lgr) && finite_d(la) && finite_d(gc))) {
    st = kPNF;
    return -INFINITY;
  }
  const double ss2 = N == 2 ? pow(10.0, 2.0 * lss) : a.mc.ss2;
  const double gr = pow(10.0, lgr);
  const double vr = pow(10.0, 2.0 * lsr) / (2.0 * gr);
  const double equad2 = N == 2 ? 0.0 : pow(10.0, 2.0 * leq);
  const double vc = N == 2 ? 0.0
                           : pow(10.0, 2.0 * la) * pow(1.0 / kYear, gc - 3.0) *
                                 exp((gc - 1.0) * a.mc.log_T) /
                                 (12.0 * kPi * kPi * (gc - 1.0));
  double x[N] = {}, P[N][N] = {};
  P[0][0] = a.mc.s_r2;
  P[1][1] = a.mc.s_f2;
  if constexpr (N == 4) {
    P[2][2] = vr;
    P[3][3] = vc;
  }
  double H[N] = {};
  H[0] = 1.0;
  if constexpr (N == 4) H[2] = H[3] = 1.0;
  double ll = 0.0, tprev = 0.0;
  for (int64_t j = a.off[p]; j < a.off[p + 1]; ++j) {
    const double dt = a.t[j] - tprev;
    tprev = a.t[j];
    double F[N][N] = {}, Q[N][N] = {};
    F[0][0] = F[1][1] = 1.0;
    F[0][1] = dt;
    Q[0][0] = ss2 * dt * dt * dt / 3.0;
    Q[0][1] = Q[1][0] = ss2 * dt * dt / 2.0;
    Q[1][1] = ss2 * dt;
    if constexpr (N == 4) {
      F[2][2] = exp(-gr * dt);
      Q[2][2] = -vr * expm1(-2.0 * gr * dt);
      F[3][3] = exp(-a.mc.lam * dt);
      Q[3][3] = -vc * expm1(-2.0 * a.mc.lam * dt);
    }
    double xp[N], T[N][N], Pp[N][N];
    for (int i = 0; i < N; ++i) {
      xp[i] = 0;
      for (int m = 0; m < N; ++m) xp[i] += F[i][m] * x[m];
    }
    for (int i = 0; i < N; ++i)
      for (int m = 0; m < N; ++m) {
        T[i][m] = 0;
        for (int l = 0; l < N; ++l) T[i][m] += F[i][l] * P[l][m];
      }
    for (int i = 0; i < N; ++i)
      for (int m = 0; m < N; ++m) {
        Pp[i][m] = Q[i][m];
        for (int l = 0; l < N; ++l) Pp[i][m] += T[i][l] * F[m][l];
      }
    const double sg = a.sig[j];
    const double R = efac * efac * sg * sg + equad2;
    double hx = 0, u[N], S = R;
    for (int i = 0; i < N; ++i) hx += H[i] * xp[i];
    const double e = a.y[j] - hx;
    for (int i = 0; i < N; ++i) {
      u[i] = 0;
      for (int m = 0; m < N; ++m) u[i] += Pp[i][m] * H[m];
      S += H[i] * u[i];
    }
    step_status(st, S, e);
    double K[N], A[N][N];
    for (int i = 0; i < N; ++i) {
      K[i] = u[i] / S;
      x[i] = xp[i] + K[i] * e;
    }
    for (int i = 0; i < N; ++i)
      for (int m = 0; m < N; ++m) A[i][m] = (i == m ? 1.0 : 0.0) - K[i] * H[m];
    for (int i = 0; i < N; ++i)
      for (int m = 0; m < N; ++m) {
        T[i][m] = 0;
        for (int l = 0; l < N; ++l) T[i][m] += A[i][l] * Pp[l][m];
      }
    for (int i = 0; i < N; ++i)
      for (int m = 0; m < N; ++m) {
        P[i][m] = K[i] * R * K[m];
        for (int l = 0; l < N; ++l) P[i][m] += T[i][l] * A[m][l];
      }
    for (int i = 0; i < N; ++i)
      for (int m = i + 1; m < N; ++m) P[i][m] = P[m][i] = 0.5 * (P[i][m] + P[m][i]);
    ll += -0.5 * (kLn2Pi + log(S) + e * e / S);
  }
  if (st == 0 && !finite_d(ll)) st = kNonFinite;
  return st ? -INFINITY : ll;
}

__global__ void __launch_bounds__(64) k_plain(PlainArgs a) {
  __shared__ double lls[64];
  __shared__ int sts[64];
  double acc = 0.0;
  int st = 0;
  bool pnf = false;
  for (int base = 0; base < a.P; base += 64) {
    const int p = base + threadIdx.x;
    if (p < a.P) {
      int s = 0;
      lls[threadIdx.x] = a.model == 1 ? plain_filter<2>(a, p, s)
                                      : plain_filter<4>(a, p, s);
      sts[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int n = a.P - base < 64 ? a.P - base : 64;
      for (int q = 0; q < n; ++q) {
        acc += lls[q];
        if (sts[q] & kPNF)
          pnf = true;
        else if (sts[q] && !st)
          st = sts[q];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (pnf) st = kNonFinite;
    *a.logl = st ? -INFINITY : acc;
    if (a.status) *a.status = st;
  }
}

}  // namespace

hipError_t launch_stage(const StageArgs& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  const int blk = 256;
  const int64_t grid = (a.N + blk - 1) / blk;
  hipLaunchKernelGGL(k_stage, dim3((unsigned)grid), dim3(blk), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_hd(const double* pos, int P, double* G, hipStream_t st) {
  hipLaunchKernelGGL(k_hd, dim3(P), dim3(64), 0, st, pos, P, G);
  return hipGetLastError();
}

hipError_t launch_filter(int model, const FilterArgs& a, int grid, int block,
                         hipStream_t st, bool with_redo) {
  const bool big = block > 256;
  if (model == 4 && !big)
    hipLaunchKernelGGL((k_filter<4, 256, false>), dim3(grid), dim3(block), 0, st, a);
  else if (model == 4)
    hipLaunchKernelGGL((k_filter<4, 1024, false>), dim3(grid), dim3(block), 0, st, a);
  else if (model == 1 && !big)
    hipLaunchKernelGGL((k_filter<1, 256, false>), dim3(grid), dim3(block), 0, st, a);
  else if (model == 1)
    hipLaunchKernelGGL((k_filter<1, 1024, false>), dim3(grid), dim3(block), 0, st, a);
  else {
    // model 2: the fast form over all items, then the general form over the
    // items it marked (without marks every wave only reads its flag)
    if (!big)
      hipLaunchKernelGGL((k_filter<2, 256, true>), dim3(grid), dim3(block), 0, st, a);
    else if (block <= 512)
      hipLaunchKernelGGL((k_filter<2, 512, true>), dim3(grid), dim3(block), 0, st, a);
    else
      hipLaunchKernelGGL((k_filter<2, 1024, true>), dim3(grid), dim3(block), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !with_redo) return e;
    // One wave per item (statically assigned), each reading its own flag,
    // so that many marked items run in parallel; with per-SIMD lists,
    // a.items and a.n_items are those lists, which is what the fast form's
    // item indices refer to.
    FilterArgs b = a;
    b.dynamic = 0;
    const int rg = b.n_items > 0 ? (b.n_items + 3) / 4 : 1;
    hipLaunchKernelGGL((k_filter<2, 256, false>), dim3(rg), dim3(256), 0, st, b);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st) {
  const int blk = 256;
  const int64_t grid = a.S > 0 ? (a.S + blk - 1) / blk : 1;
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)grid), dim3(blk), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_plain(const PlainArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_plain, dim3(1), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace argus
