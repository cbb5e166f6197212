// Host side of libargus: the C ABI declared in include/argus.h, dataset
// staging, per-sample-count workspaces, the launch autotuner and hipGraph
// capture/replay of the batched likelihood.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <numeric>
#include <queue>
#include <string>
#include <vector>

#include "argus.h"
#include "argus_internal.h"
#include "argus_host.h"

using namespace argus;

namespace argus {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

int DevBuf::alloc(size_t nbytes) {
  release();
  if (nbytes == 0) nbytes = 64;
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    (void)hipGetLastError();  // a later launch check must not see this failure
    return fail(ARGUS_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  bytes = nbytes;
  return ARGUS_OK;
}

int DevBuf::upload(const void* src, size_t nbytes) {
  int rc = alloc(nbytes);
  if (rc) return rc;
  if (nbytes && src) HIPCHK(hipMemcpy(p, src, nbytes, hipMemcpyHostToDevice));
  return ARGUS_OK;
}

Workspace::~Workspace() {
  if (has_graph) (void)hipGraphExecDestroy(exec);
}

int check_device(const argus_dataset* ds) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != ds->device)
    return fail(ARGUS_E_INVAL, "dataset was created on device " +
                                   std::to_string(ds->device) +
                                   " but the current device is " +
                                   std::to_string(dev));
  return ARGUS_OK;
}

}  // namespace argus

namespace {

bool finite(double v) { return std::isfinite(v); }

int validate(const argus_dataset_desc* d) {
  if (!d) return fail(ARGUS_E_INVAL, "desc is NULL");
  if (d->model < 1 || d->model > 4) return fail(ARGUS_E_INVAL, "unknown model");
  if (d->n_psr < 1) return fail(ARGUS_E_INVAL, "n_psr must be >= 1");
  if (d->model == ARGUS_M1_SPIN && d->n_psr != 1)
    return fail(ARGUS_E_INVAL, "model 1 takes exactly one pulsar");
  if (d->model == ARGUS_M3_JOINT_HD && d->n_psr > kJointMaxPsr)
    return fail(ARGUS_E_UNSUPPORTED,
                "joint model supports at most " + std::to_string(kJointMaxPsr) + " pulsars");
  if (!d->toa_off) return fail(ARGUS_E_INVAL, "toa_off is NULL");
  if (d->toa_off[0] != 0) return fail(ARGUS_E_INVAL, "toa_off[0] must be 0");
  for (int p = 0; p < d->n_psr; ++p)
    if (d->toa_off[p + 1] < d->toa_off[p])
      return fail(ARGUS_E_INVAL, "toa_off must be non-decreasing");
  const int64_t N = d->toa_off[d->n_psr];
  if (N > INT32_MAX) return fail(ARGUS_E_UNSUPPORTED, "too many TOAs (at most 2^31 - 1)");
  if (N > 0 && (!d->t || !d->y || !d->sigma))
    return fail(ARGUS_E_INVAL, "t, y and sigma are required");
  for (int p = 0; p < d->n_psr; ++p)
    for (int64_t k = d->toa_off[p]; k < d->toa_off[p + 1]; ++k) {
      if (!finite(d->t[k]) || d->t[k] < 0.0)
        return fail(ARGUS_E_INVAL, "t must be finite and >= 0 (epoch t0 = 0)");
      if (k > d->toa_off[p] && !(d->t[k] > d->t[k - 1]))
        return fail(ARGUS_E_INVAL, "t must be strictly ascending within a pulsar");
      if (!finite(d->y[k])) return fail(ARGUS_E_INVAL, "y must be finite");
      if (!finite(d->sigma[k]) || !(d->sigma[k] > 0.0))
        return fail(ARGUS_E_INVAL, "sigma must be finite and > 0");
    }
  if (d->model == ARGUS_M4_PSR5_DM) {
    if (N > 0 && !d->freq) return fail(ARGUS_E_INVAL, "freq is required for model 4");
    for (int64_t k = 0; k < N; ++k)
      if (!finite(d->freq[k]) || !(d->freq[k] > 0.0))
        return fail(ARGUS_E_INVAL, "freq must be finite and > 0");
  }
  if (d->model == ARGUS_M3_JOINT_HD) {
    if (!d->pos) return fail(ARGUS_E_INVAL, "pos is required for the joint model");
    for (int i = 0; i < 3 * d->n_psr; ++i)
      if (!finite(d->pos[i])) return fail(ARGUS_E_INVAL, "pos must be finite");
  }
  if (!finite(d->t_span) || !(d->t_span > 0.0))
    return fail(ARGUS_E_INVAL, "t_span must be > 0");
  if (!finite(d->s_r) || !finite(d->s_f) || !finite(d->sigma_s) || d->s_r < 0 ||
      d->s_f < 0 || d->sigma_s < 0)
    return fail(ARGUS_E_INVAL, "s_r, s_f, sigma_s must be finite and >= 0");
  const int C = d->model == ARGUS_M1_SPIN ? 2 : (d->model == ARGUS_M4_PSR5_DM ? 6 : 4) * d->n_psr + 2;
  for (int c = 0; c < C; ++c) {
    const bool fr = d->free_mask ? d->free_mask[c] != 0 : true;
    if (!fr && (!d->fixed || !finite(d->fixed[c])))
      return fail(ARGUS_E_INVAL, "fixed values of non-free params must be finite");
  }
  return ARGUS_OK;
}

// Work items (64-sample tile, pulsar) in longest-first order.
std::vector<int32_t> make_items(const std::vector<int64_t>& counts, int64_t S) {
  const int64_t tiles = (S + kWave - 1) / kWave;
  std::vector<int> order(counts.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return counts[a] > counts[b]; });
  std::vector<int32_t> it;
  it.reserve(2 * tiles * counts.size());
  for (int p : order)
    for (int64_t t = 0; t < tiles; ++t) {
      it.push_back((int32_t)t);
      it.push_back(p);
    }
  return it;
}

// Items (tile, pulsar) split into n_bins lists of about equal total TOA
// steps (longest item first to the least-loaded list), each list longest
// first, concatenated; off[b]..off[b+1] is list b. Lists 4c..4c+3 are the
// four SIMDs of block c, one block per CU.
std::vector<int32_t> make_items_binned(const std::vector<int64_t>& counts, int64_t S,
                                       int n_bins, std::vector<int32_t>* off) {
  const int64_t tiles = (S + kWave - 1) / kWave;
  std::vector<int> order(counts.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return counts[a] > counts[b]; });
  std::vector<std::vector<int32_t>> bins(n_bins);
  using E = std::pair<int64_t, int>;
  std::priority_queue<E, std::vector<E>, std::greater<E>> heap;
  for (int b = 0; b < n_bins; ++b) heap.push({0, b});
  for (int p : order)
    for (int64_t t = 0; t < tiles; ++t) {
      const E e = heap.top();
      heap.pop();
      bins[e.second].push_back((int32_t)t);
      bins[e.second].push_back(p);
      heap.push({e.first + std::max<int64_t>(counts[p], 1), e.second});
    }
  std::vector<int32_t> it;
  off->assign(1, 0);
  for (auto& b : bins) {
    it.insert(it.end(), b.begin(), b.end());
    off->push_back((int32_t)(it.size() / 2));
  }
  return it;
}

FilterArgs filter_args(argus_dataset* ds, Workspace* w, const double* theta,
                       const TuneCfg& cfg);

int launch_loglike_seq(argus_dataset* ds, Workspace* w, const double* theta,
                       double* logl, int32_t* status, const TuneCfg& cfg,
                       hipStream_t st) {
  const FilterArgs a = filter_args(ds, w, theta, cfg);
  if (cfg.order == 2)
    HIPCHK(launch_scan(ds->model, a, cfg.grid, cfg.block / kWave, st));
  else
    HIPCHK(launch_filter(ds->model, a, cfg.grid, cfg.block, st));
  ReduceArgs r{w->part.as<double>(), w->pstat.as<int32_t>(), logl, status,
               w->counter.as<int32_t>(), w->S, ds->P};
  HIPCHK(launch_reduce(r, st));
  return ARGUS_OK;
}

FilterArgs filter_args(argus_dataset* ds, Workspace* w, const double* theta,
                       const TuneCfg& cfg) {
  FilterArgs a{};
  a.rec = ds->rec.as<TOARec>();
  a.chrom = ds->chrom.as<double>();
  a.off = ds->off.as<int64_t>();
  a.maxdt = ds->maxdt.as<double>();
  a.theta = theta;
  a.col = ds->col.as<int32_t>();
  a.fixed = ds->fixed.as<double>();
  const bool bal = cfg.order == 1;
  a.items = (bal ? w->items_bal : w->items).as<int32_t>();
  a.bin_off = bal ? w->bin_off.as<int32_t>() : nullptr;
  a.counter = w->counter.as<int32_t>();
  a.redo = w->redo.as<int32_t>();
  a.part = w->part.as<double>();
  a.pstat = w->pstat.as<int32_t>();
  a.S = w->S;
  a.D = ds->D;
  a.P = ds->P;
  a.n_items = bal ? w->n_items_bal : w->n_items;
  a.dynamic = bal ? 2 : cfg.dynamic;
  a.mc = ds->mc;
  return a;
}

std::vector<TuneCfg> candidates(const argus_dataset* ds, const Workspace* w) {
  const int simd = 4 * ds->n_cu;
  std::vector<TuneCfg> c;
  auto add = [&](int block, int64_t waves, int dyn) {
    const int wpb = block / kWave;
    waves = std::min<int64_t>(waves, w->n_items);
    waves = std::max<int64_t>(waves, 1);
    const int64_t grid = (waves + wpb - 1) / wpb;
    for (auto& x : c)
      if (x.block == block && x.grid == grid && x.dynamic == dyn) return;
    c.push_back({block, (int)grid, dyn, 0, 0.f});
  };
  add(64, w->n_items, 0);
  add(256, w->n_items, 0);
  if (w->n_items_bal > 0)
    for (int b : {256, 512, 1024}) c.push_back({b, w->n_bins, 0, 1, 0.f});
  for (int k : {1, 2, 3, 4, 6}) add(64, (int64_t)simd * k, 1);
  for (int k : {2, 4}) add(256, (int64_t)simd * k, 1);
  // time-parallel filter, one workgroup of nw waves per item: only when the
  // items leave most SIMDs idle
  if (ds->model != ARGUS_M4_PSR5_DM && (int64_t)w->n_items * 4 <= simd)
    for (int nw : {4, 8, 16}) c.push_back({nw * kWave, w->n_items, 0, 2, 0.f});
  return c;
}

int autotune(argus_dataset* ds, Workspace* w, const double* theta, double* logl,
             int32_t* status, hipStream_t st) {
  const char* forced = std::getenv("ARGUS_CFG");
  if (forced) {
    int b = 0, g = 0, dyn = 0, ord = 0;
    const int nf = std::sscanf(forced, "%d,%d,%d,%d", &b, &g, &dyn, &ord);
    const bool ok0 = ord == 0 && b >= 64 && b <= 256 && (dyn == 0 || dyn == 1);
    const bool ok1 = ord == 1 && b >= 64 && b <= 1024 && w->n_items_bal > 0;
    const bool ok2 = ord == 2 && (b == 256 || b == 512 || b == 1024) &&
                     ds->model != ARGUS_M4_PSR5_DM;
    if (nf >= 3 && b % 64 == 0 && g >= 1 && (ok0 || ok1 || ok2)) {
      w->cfg = {b, ord == 1 ? w->n_bins : g, ord == 0 ? dyn : 0, ord, 0.f};
      w->tuned = true;
      return ARGUS_OK;
    }
    return fail(ARGUS_E_INVAL,
                "ARGUS_CFG must be 'block,grid,dynamic[,order]' (order 0: block <= 256; "
                "order 1: per-SIMD lists, block <= 1024, grid ignored; order 2: "
                "time-parallel filter, block 256, 512 or 1024 = 4, 8 or 16 chunks)");
  }
  const char* en = std::getenv("ARGUS_TUNE");
  if (en && std::strcmp(en, "0") == 0) {
    const int wpb = 1;
    w->cfg = {64 * wpb, (int)std::min<int64_t>(w->n_items, 8LL * ds->n_cu), 1, 0, 0.f};
    w->tuned = true;
    return ARGUS_OK;
  }
  std::vector<TuneCfg> cand = candidates(ds, w);
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  int rc = ARGUS_OK;
  // one sample: eight launches back to back, as a caller replays them (a
  // launch timed alone, after a synchronisation, runs at another clock and
  // ranks the layouts differently)
  auto time_one = [&](const TuneCfg& c, float* ms) -> int {
    constexpr int kBack = 8;
    if (hipEventRecord(e0, st) != hipSuccess) return fail(ARGUS_E_HIP, "event");
    for (int i = 0; i < kBack; ++i) {
      const int r = launch_loglike_seq(ds, w, theta, logl, status, c, st);
      if (r) return r;
    }
    if (hipEventRecord(e1, st) != hipSuccess) return fail(ARGUS_E_HIP, "event");
    if (hipEventSynchronize(e1) != hipSuccess) return fail(ARGUS_E_HIP, "sync");
    if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return fail(ARGUS_E_HIP, "elapsed");
    *ms /= kBack;
    return ARGUS_OK;
  };
  // Candidates are timed in interleaved rounds (round 0 warms caches), each
  // keeping its best, so that a drift of the clock between candidates does
  // not decide; the three best then get more interleaved rounds.
  for (auto& c : cand) c.ms = 1e30f;
  for (int round = 0; round < 4 && !rc; ++round)
    for (auto& c : cand) {
      float ms = 0;
      if ((rc = time_one(c, &ms))) break;
      if (round > 0) c.ms = std::min(c.ms, ms);
    }
  if (!rc && cand.size() > 3) {
    std::vector<TuneCfg*> top;
    for (auto& c : cand) top.push_back(&c);
    std::partial_sort(top.begin(), top.begin() + 3, top.end(),
                      [](const TuneCfg* a, const TuneCfg* b) { return a->ms < b->ms; });
    for (int round = 0; round < 8 && !rc; ++round)
      for (int i = 0; i < 3; ++i) {
        float ms = 0;
        if ((rc = time_one(*top[i], &ms))) break;
        top[i]->ms = std::min(top[i]->ms, ms);
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  // Candidates within 3 % of the fastest are ties, and a tie goes to the
  // layout with more resident waves: the tuning samples are short, and
  // under sustained load (lower clock) layouts with fewer waves per SIMD
  // lose more (measured on the 47-pulsar workload: 2 waves per SIMD 0.59 ms
  // in tuning but 0.67-0.71 ms over 50 calls, 4 waves per SIMD 0.60 and
  // 0.62-0.63 ms).
  const float fastest =
      std::min_element(cand.begin(), cand.end(),
                       [](const TuneCfg& a, const TuneCfg& b) { return a.ms < b.ms; })
          ->ms;
  auto waves = [&](const TuneCfg& c) {
    return std::min<int64_t>((int64_t)c.grid * (c.block / kWave),
                             c.order == 2 ? (int64_t)c.grid * (c.block / kWave)
                                          : (int64_t)std::max(w->n_items, w->n_items_bal));
  };
  const TuneCfg* pick = nullptr;
  for (const auto& c : cand) {
    if (c.ms > 1.03f * fastest) continue;
    if (!pick || waves(c) > waves(*pick) || (waves(c) == waves(*pick) && c.ms < pick->ms))
      pick = &c;
  }
  w->cfg = *pick;
  w->tuned = true;
  w->tune_log.clear();
  for (auto& c : cand) {
    char b[128];
    std::snprintf(b, sizeof b, "block=%d grid=%d dyn=%d order=%d: %.4f ms\n", c.block, c.grid,
                  c.dynamic, c.order, c.ms);
    w->tune_log += b;
  }
  return ARGUS_OK;
}

}  // namespace

namespace argus {

Workspace* get_workspace(argus_dataset* ds, int64_t S, int* rc) {
  auto it = ds->ws.find(S);
  if (it != ds->ws.end()) return it->second.get();
  auto w = std::make_unique<Workspace>();
  w->S = S;
  const size_t ps = (size_t)ds->P * (size_t)S;
  if ((*rc = w->part.alloc(ps * sizeof(double)))) return nullptr;
  if ((*rc = w->pstat.alloc(ps * sizeof(int32_t)))) return nullptr;
  if ((*rc = w->logl_tmp.alloc((size_t)S * sizeof(double)))) return nullptr;
  if ((*rc = w->counter.alloc(64))) return nullptr;
  if ((*rc = w->stat_tmp.alloc((size_t)S * sizeof(int32_t)))) return nullptr;
  if (hipMemset(w->counter.p, 0, 64) != hipSuccess) {
    *rc = fail(ARGUS_E_HIP, "hipMemset");
    return nullptr;
  }
  if (ds->model != ARGUS_M3_JOINT_HD) {
    std::vector<int32_t> items = make_items(ds->counts, S);
    w->n_items = (int)(items.size() / 2);
    if ((*rc = w->items.upload(items.data(), items.size() * sizeof(int32_t)))) return nullptr;
    w->items_host = items;
    std::vector<int32_t> boff;
    std::vector<int32_t> bal = make_items_binned(ds->counts, S, 4 * ds->n_cu, &boff);
    w->n_items_bal = (int)(bal.size() / 2);
    w->n_bins = ds->n_cu;  // blocks
    if (bal.empty()) bal.assign(2, -1);  // keep the buffer non-empty
    if ((*rc = w->items_bal.upload(bal.data(), bal.size() * sizeof(int32_t))) ||
        (*rc = w->bin_off.upload(boff.data(), boff.size() * sizeof(int32_t))) ||
        (*rc = w->redo.alloc((size_t)std::max(w->n_items, w->n_items_bal) * sizeof(int32_t))))
      return nullptr;
  }
  Workspace* raw = w.get();
  ds->ws[S] = std::move(w);
  *rc = ARGUS_OK;
  return raw;
}

}  // namespace argus

// ======================================================================= ABI
extern "C" {

const char* argus_last_error(void) { return g_err.c_str(); }

int argus_dataset_create(const argus_dataset_desc* d, argus_dataset_t* out) {
  if (!out) return fail(ARGUS_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(d);
  if (rc) return rc;
  auto ds = std::make_unique<argus_dataset>();
  ds->model = d->model;
  ds->P = d->n_psr;
  ds->C = d->model == ARGUS_M1_SPIN ? 2 : (d->model == ARGUS_M4_PSR5_DM ? 6 : 4) * d->n_psr + 2;
  ds->N = d->toa_off[d->n_psr];
  HIPCHK(hipGetDevice(&ds->device));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, ds->device));
  ds->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  ds->mc.s_r2 = d->s_r * d->s_r;
  ds->mc.s_f2 = d->s_f * d->s_f;
  ds->mc.ss2 = d->sigma_s * d->sigma_s;
  ds->mc.log_fyr = std::log(1.0 / kYear);
  ds->mc.log_T = std::log(d->t_span);
  ds->mc.lam = 2.0 * kPi / d->t_span;
  // free parameters -> theta columns in canonical order
  std::vector<int32_t> col(ds->C);
  std::vector<double> fixed(ds->C, 0.0);
  int D = 0;
  for (int c = 0; c < ds->C; ++c) {
    const bool fr = d->free_mask ? d->free_mask[c] != 0 : true;
    col[c] = fr ? D++ : -1;
    if (d->fixed) fixed[c] = d->fixed[c];
  }
  ds->D = D;
  std::vector<int32_t> icol(D > 0 ? D : 1, 0);
  for (int c = 0; c < ds->C; ++c)
    if (col[c] >= 0) icol[col[c]] = c;
  ds->off_h.assign(d->toa_off, d->toa_off + ds->P + 1);
  ds->counts.resize(ds->P);
  for (int p = 0; p < ds->P; ++p) ds->counts[p] = d->toa_off[p + 1] - d->toa_off[p];
  // stream order: per-pulsar CSR, or merged by (t, pulsar) for the joint model
  const int64_t N = ds->N;
  std::vector<int64_t> src(N), prev(N);
  std::vector<int32_t> psr(N);
  if (d->model == ARGUS_M3_JOINT_HD) {
    std::vector<std::pair<double, int32_t>> key(N);
    std::vector<int64_t> ord(N);
    for (int p = 0; p < ds->P; ++p)
      for (int64_t k = d->toa_off[p]; k < d->toa_off[p + 1]; ++k) key[k] = {d->t[k], p};
    std::iota(ord.begin(), ord.end(), 0);
    std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
      return key[a].first != key[b].first ? key[a].first < key[b].first
                                          : key[a].second < key[b].second;
    });
    for (int64_t k = 0; k < N; ++k) {
      src[k] = ord[k];
      prev[k] = k ? ord[k - 1] : -1;
      psr[k] = key[ord[k]].second;
    }
  } else {
    for (int p = 0; p < ds->P; ++p)
      for (int64_t k = d->toa_off[p]; k < d->toa_off[p + 1]; ++k) {
        src[k] = k;
        prev[k] = k > d->toa_off[p] ? k - 1 : -1;
        psr[k] = p;
      }
  }
  DevBuf dsrc, dprev, dpsr;
  if ((rc = ds->t.upload(d->t, N * sizeof(double))) ||
      (rc = ds->y.upload(d->y, N * sizeof(double))) ||
      (rc = ds->sig.upload(d->sigma, N * sizeof(double))) ||
      (rc = dsrc.upload(src.data(), N * sizeof(int64_t))) ||
      (rc = dprev.upload(prev.data(), N * sizeof(int64_t))) ||
      (rc = dpsr.upload(psr.data(), N * sizeof(int32_t))) ||
      (rc = ds->rec.alloc(N * sizeof(TOARec))) ||
      (rc = ds->off.upload(d->toa_off, (ds->P + 1) * sizeof(int64_t))) ||
      (rc = ds->col.upload(col.data(), ds->C * sizeof(int32_t))) ||
      (rc = ds->icol.upload(icol.data(), icol.size() * sizeof(int32_t))) ||
      (rc = ds->fixed.upload(fixed.data(), ds->C * sizeof(double))))
    return rc;
  if (d->model == ARGUS_M4_PSR5_DM) {
    std::vector<double> ch(N > 0 ? N : 1, 0.0);
    for (int64_t k = 0; k < N; ++k) {
      const double r = kNuRef / d->freq[k];
      ch[k] = r * r;
    }
    if ((rc = ds->chrom.upload(ch.data(), ch.size() * sizeof(double)))) return rc;
  }
  if (d->model != ARGUS_M3_JOINT_HD) {
    std::vector<int32_t> po(ds->P);
    std::iota(po.begin(), po.end(), 0);
    std::stable_sort(po.begin(), po.end(),
                     [&](int a, int b) { return ds->counts[a] > ds->counts[b]; });
    if ((rc = ds->porder.upload(po.data(), po.size() * sizeof(int32_t)))) return rc;
    std::vector<double> mdt(ds->P, 0.0);
    for (int p = 0; p < ds->P; ++p)
      for (int64_t k = d->toa_off[p]; k < d->toa_off[p + 1]; ++k)
        mdt[p] = std::max(mdt[p], d->t[k] - (k > d->toa_off[p] ? d->t[k - 1] : 0.0));
    if ((rc = ds->maxdt.upload(mdt.data(), mdt.size() * sizeof(double)))) return rc;
  }
  StageArgs sa{ds->t.as<double>(), ds->y.as<double>(), ds->sig.as<double>(),
               dsrc.as<int64_t>(), dprev.as<int64_t>(), dpsr.as<int32_t>(),
               ds->rec.as<TOARec>(), N, ds->mc.lam, d->model == ARGUS_M3_JOINT_HD ? 1 : 0};
  HIPCHK(launch_stage(sa, 0));
  if (d->model == ARGUS_M3_JOINT_HD) {
    DevBuf dpos;
    if ((rc = dpos.upload(d->pos, 3 * ds->P * sizeof(double))) ||
        (rc = ds->hd.alloc((size_t)ds->P * ds->P * sizeof(double))))
      return rc;
    HIPCHK(launch_hd(dpos.as<double>(), ds->P, ds->hd.as<double>(), 0));
    HIPCHK(hipDeviceSynchronize());
  }
  HIPCHK(hipDeviceSynchronize());
  HIPCHK(hipStreamCreateWithFlags(&ds->cap_stream, hipStreamNonBlocking));
  *out = ds.release();
  return ARGUS_OK;
}

int argus_dataset_destroy(argus_dataset_t ds) {
  if (!ds) return ARGUS_OK;
  (void)hipDeviceSynchronize();
  if (ds->cap_stream) (void)hipStreamDestroy(ds->cap_stream);
  delete ds;
  return ARGUS_OK;
}

int argus_dataset_n_params(argus_dataset_t ds, int32_t* D) {
  if (!ds || !D) return fail(ARGUS_E_INVAL, "NULL argument");
  *D = ds->D;
  return ARGUS_OK;
}

static int check_call(argus_dataset_t ds, const double* theta, int64_t S, const void* out) {
  if (!ds) return fail(ARGUS_E_INVAL, "dataset is NULL");
  if (S < 0) return fail(ARGUS_E_INVAL, "S must be >= 0");
  if (S > ((int64_t)1 << 30)) return fail(ARGUS_E_UNSUPPORTED, "S too large");
  if (S > 0 && ds->D > 0 && !theta) return fail(ARGUS_E_INVAL, "theta is NULL");
  if (S > 0 && !out) return fail(ARGUS_E_INVAL, "output is NULL");
  return check_device(ds);
}

int argus_loglike(argus_dataset_t ds, const double* theta, int64_t S, double* logl,
                  int32_t* status, void* stream) {
  int rc = check_call(ds, theta, S, logl);
  if (rc || S == 0) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (ds->model == ARGUS_M3_JOINT_HD) return joint_loglike(ds, theta, S, logl, status, st);
  Workspace* w = get_workspace(ds, S, &rc);
  if (!w) return rc;
  if (!w->tuned && (rc = autotune(ds, w, theta, logl, status, st))) return rc;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(st, &cs));
  const char* ng = std::getenv("ARGUS_NO_GRAPH");
  const bool stable = w->last_theta == theta && w->last_out == logl && w->last_status == status;
  w->last_theta = theta;
  w->last_out = logl;
  w->last_status = status;
  if (cs != hipStreamCaptureStatusNone || (ng && std::strcmp(ng, "1") == 0) || !stable)
    return launch_loglike_seq(ds, w, theta, logl, status, w->cfg, st);
  if (!w->has_graph || w->g_theta != theta || w->g_out != logl || w->g_status != status) {
    if (w->has_graph) {
      HIPCHK(hipGraphExecDestroy(w->exec));
      w->has_graph = false;
    }
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(ds->cap_stream, hipStreamCaptureModeThreadLocal));
    rc = launch_loglike_seq(ds, w, theta, logl, status, w->cfg, ds->cap_stream);
    hipError_t e = hipStreamEndCapture(ds->cap_stream, &g);
    if (rc) return rc;
    if (e != hipSuccess) return fail(ARGUS_E_HIP, "hipStreamEndCapture failed");
    e = hipGraphInstantiate(&w->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(ARGUS_E_HIP, "hipGraphInstantiate failed");
    w->has_graph = true;
    w->g_theta = theta;
    w->g_out = logl;
    w->g_status = status;
  }
  HIPCHK(hipGraphLaunch(w->exec, st));
  return ARGUS_OK;
}

int argus_loglike_terms(argus_dataset_t ds, const double* theta, int64_t S, double* terms,
                        int32_t* status, void* stream) {
  int rc = check_call(ds, theta, S, terms);
  if (rc || S == 0) return rc;
  if (ds->model == ARGUS_M3_JOINT_HD)
    return fail(ARGUS_E_UNSUPPORTED, "per-pulsar terms exist for models 1, 2 and 4 only");
  hipStream_t st = (hipStream_t)stream;
  Workspace* w = get_workspace(ds, S, &rc);
  if (!w) return rc;
  if (!w->tuned && (rc = autotune(ds, w, theta, w->logl_tmp.as<double>(), status, st)))
    return rc;
  if ((rc = launch_loglike_seq(ds, w, theta, w->logl_tmp.as<double>(), status, w->cfg, st)))
    return rc;
  HIPCHK(hipMemcpyAsync(terms, w->part.p, (size_t)ds->P * S * sizeof(double),
                        hipMemcpyDeviceToDevice, st));
  return ARGUS_OK;
}

int argus_loglike_plain(argus_dataset_t ds, const double* theta, int64_t S, double* logl,
                        int32_t* status, void* stream) {
  int rc = check_call(ds, theta, S, logl);
  if (rc || S == 0) return rc;
  if (ds->model == ARGUS_M3_JOINT_HD || ds->model == ARGUS_M4_PSR5_DM)
    return fail(ARGUS_E_UNSUPPORTED, "the plain baseline covers models 1 and 2");
  hipStream_t st = (hipStream_t)stream;
  for (int64_t s = 0; s < S; ++s) {
    PlainArgs a{ds->t.as<double>(), ds->y.as<double>(), ds->sig.as<double>(),
                ds->off.as<int64_t>(), theta ? theta + s * ds->D : nullptr,
                ds->col.as<int32_t>(), ds->fixed.as<double>(), logl + s,
                status ? status + s : nullptr, ds->D, ds->P, ds->model, ds->mc};
    HIPCHK(launch_plain(a, st));
  }
  return ARGUS_OK;
}

int argus_filter_kernel_ms(argus_dataset_t ds, const double* theta, int64_t S, int32_t reps,
                           double* ms, void* stream) {
  int rc = check_call(ds, theta, S, ms);
  if (rc) return rc;
  if (!ms || reps < 1 || S < 1) return fail(ARGUS_E_INVAL, "need ms, reps >= 1 and S >= 1");
  if (ds->model == ARGUS_M3_JOINT_HD)
    return fail(ARGUS_E_UNSUPPORTED, "the joint model has one kernel per call: time the call");
  auto it = ds->ws.find(S);
  if (it == ds->ws.end() || !it->second->tuned)
    return fail(ARGUS_E_INVAL, "call argus_loglike for this S first (the launch is tuned there)");
  Workspace* w = it->second.get();
  hipStream_t st = (hipStream_t)stream;
  const FilterArgs a = filter_args(ds, w, theta, w->cfg);
  // one pair of events around each launch; the work-queue head of the
  // atomic-queue layout is cleared between launches, outside the pairs
  std::vector<hipEvent_t> ev(2 * (size_t)reps, nullptr);
  hipError_t e = hipSuccess;
  for (auto& x : ev)
    if (e == hipSuccess) e = hipEventCreate(&x);
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    if (w->cfg.dynamic == 1 && w->cfg.order == 0) e = hipMemsetAsync(w->counter.p, 0, 4, st);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * i], st);
    if (e == hipSuccess)
      e = w->cfg.order == 2 ? launch_scan(ds->model, a, w->cfg.grid, w->cfg.block / kWave, st)
                            : launch_filter(ds->model, a, w->cfg.grid, w->cfg.block, st, false);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * i + 1], st);
  }
  if (e == hipSuccess) e = hipEventSynchronize(ev.back());
  double tot = 0.0;
  for (int i = 0; i < reps && e == hipSuccess; ++i) {
    float t = 0.f;
    e = hipEventElapsedTime(&t, ev[2 * i], ev[2 * i + 1]);
    tot += t;
  }
  for (auto& x : ev)
    if (x) (void)hipEventDestroy(x);
  if (w->cfg.dynamic == 1 && w->cfg.order == 0 && e == hipSuccess)
    e = hipMemsetAsync(w->counter.p, 0, 4, st);
  if (e != hipSuccess) return fail(ARGUS_E_HIP, std::string("timing: ") + hipGetErrorString(e));
  *ms = tot / reps;
  return ARGUS_OK;
}

int argus_tune_info(argus_dataset_t ds, int64_t S, char* buf, int32_t len) {
  if (!ds || !buf || len <= 0) return fail(ARGUS_E_INVAL, "bad argument");
  auto it = ds->ws.find(S);
  std::string s;
  const Workspace* w = it == ds->ws.end() ? nullptr : it->second.get();
  char b[160];
  if (!w || !w->tuned) {
    s = "likelihood launch not tuned\n";
  } else {
    std::snprintf(b, sizeof b, "chosen block=%d grid=%d dyn=%d order=%d items=%d\n",
                  w->cfg.block, w->cfg.grid, w->cfg.dynamic, w->cfg.order,
                  w->cfg.order == 1 ? w->n_items_bal : w->n_items);
    s = b + w->tune_log;
  }
  if (w && w->tan_nda) {
    if (w->tan_thresh < 0)
      std::snprintf(b, sizeof b, "gradient: tangent sweep, producer/consumer form (%s per item)\n",
                    tangent_pc_layout(ds->model, w->tan_nda));
    else if (w->tan_nda == w->tan_ndb)
      std::snprintf(b, sizeof b, "gradient: tangent sweep, %d directions per wave\n", w->tan_nda);
    else
      std::snprintf(b, sizeof b,
                    "gradient: tangent sweep, %d directions per wave for pulsars of >= %lld "
                    "TOAs, %d for the others\n",
                    w->tan_nda, (long long)w->tan_thresh, w->tan_ndb);
    s += b + w->grad_log;
  }
  if (w && w->smooth_k) {
    if (w->smooth_k == 1)
      std::snprintf(b, sizeof b, "smoother: one wave per item\n");
    else
      std::snprintf(b, sizeof b,
                    "smoother: time-parallel form, the longest pulsars in %d chunks\n",
                    w->smooth_k);
    s += b + w->smooth_log;
  }
  std::snprintf(buf, len, "%s", s.c_str());
  return ARGUS_OK;
}

}  // extern "C"
extern "C" int argus_loglike_grad(argus_dataset_t ds, const double* theta, int64_t S,
                                  double* logl, double* grad, int32_t* status, void* stream) {
  int rc = check_call(ds, theta, S, logl);
  if (rc || S == 0) return rc;
  if (ds->D > 0 && !grad) return fail(ARGUS_E_INVAL, "grad is NULL");
  if (ds->model == ARGUS_M3_JOINT_HD)
    return fail(ARGUS_E_UNSUPPORTED, "the gradient covers models 1, 2 and 4");
  return grad_loglike(ds, theta, S, logl, grad, status, (hipStream_t)stream);
}

extern "C" int argus_hmc_step(argus_dataset_t ds, int64_t S, int32_t n_leapfrog,
                              const double* eps, const double* inv_mass, const double* lo,
                              const double* hi, const double* z, const double* logu,
                              double* theta, double* logl, double* grad, int32_t* accepted,
                              double* energy_err, void* stream) {
  int rc = check_call(ds, theta, S, logl);
  if (rc || S == 0) return rc;
  if (ds->model == ARGUS_M3_JOINT_HD)
    return fail(ARGUS_E_UNSUPPORTED, "HMC needs the gradient (models 1, 2 and 4)");
  if (ds->D < 1) return fail(ARGUS_E_INVAL, "HMC needs at least one free parameter");
  if (n_leapfrog < 1) return fail(ARGUS_E_INVAL, "n_leapfrog must be >= 1");
  if (!eps || !inv_mass || !lo || !hi || !z || !logu || !grad || !accepted)
    return fail(ARGUS_E_INVAL, "a required HMC pointer is NULL");
  return hmc_step(ds, S, n_leapfrog, eps, inv_mass, lo, hi, z, logu, theta, logl, grad,
                  accepted, energy_err, (hipStream_t)stream);
}

extern "C" int argus_nuts_step(argus_dataset_t ds, int64_t S, int32_t max_depth,
                               const double* eps, const double* inv_mass, const double* lo,
                               const double* hi, const double* z, const int32_t* dirs,
                               const double* u_top, const double* u_sub, double* theta,
                               double* logl, double* grad, int32_t* depth, int32_t* n_leapfrog,
                               int32_t* divergent, double* accept_stat, void* stream) {
  int rc = check_call(ds, theta, S, logl);
  if (rc || S == 0) return rc;
  if (ds->model == ARGUS_M3_JOINT_HD)
    return fail(ARGUS_E_UNSUPPORTED, "NUTS needs the gradient (models 1, 2 and 4)");
  if (ds->D < 1) return fail(ARGUS_E_INVAL, "NUTS needs at least one free parameter");
  if (max_depth < 1 || max_depth > 10) return fail(ARGUS_E_INVAL, "max_depth must be in [1, 10]");
  if (!eps || !inv_mass || !lo || !hi || !z || !dirs || !u_top || !u_sub || !grad || !depth ||
      !n_leapfrog || !divergent)
    return fail(ARGUS_E_INVAL, "a required NUTS pointer is NULL");
  return nuts_step(ds, S, max_depth, eps, inv_mass, lo, hi, z, dirs, u_top, u_sub, theta, logl,
                   grad, depth, n_leapfrog, divergent, accept_stat, (hipStream_t)stream);
}

extern "C" int argus_fp64_rate(int32_t waves_per_simd, double* tflops, double* clock_mhz,
                               void* stream) {
  if (!tflops || !clock_mhz) return fail(ARGUS_E_INVAL, "tflops and clock_mhz are required");
  if (waves_per_simd < 1 || waves_per_simd > 4)
    return fail(ARGUS_E_INVAL, "waves_per_simd must be 1..4");
  // about 1 ms of FMAs at one wave per SIMD
  return device_rate(0, waves_per_simd, 2000 / waves_per_simd, tflops, clock_mhz,
                     (hipStream_t)stream);
}

extern "C" int argus_mfma_rate(int32_t kind, int32_t waves_per_simd, double* tflops,
                               double* clock_mhz, void* stream) {
  if (!tflops || !clock_mhz) return fail(ARGUS_E_INVAL, "tflops and clock_mhz are required");
  if (kind != 1 && kind != 2) return fail(ARGUS_E_INVAL, "kind must be 1 (FP64) or 2 (BF16)");
  if (waves_per_simd < 1 || waves_per_simd > 4)
    return fail(ARGUS_E_INVAL, "waves_per_simd must be 1..4");
  // about 1 ms of matrix instructions at one wave per SIMD
  const int iters = (kind == 1 ? 4000 : 2000) / waves_per_simd;
  return device_rate(kind, waves_per_simd, iters, tflops, clock_mhz, (hipStream_t)stream);
}

extern "C" int argus_smooth(argus_dataset_t ds, const double* theta, int64_t S, double* mean,
                            double* var, double* logl, int32_t* status, void* stream) {
  int rc = check_call(ds, theta, S, mean);
  if (rc || S == 0) return rc;
  if (ds->model == ARGUS_M3_JOINT_HD)
    return fail(ARGUS_E_UNSUPPORTED, "the smoother covers models 1, 2 and 4");
  const uint64_t nc = ds->model == ARGUS_M1_SPIN ? 2 : (ds->model == ARGUS_M4_PSR5_DM ? 5 : 4);
  if (ds->N > 0 && (uint64_t)ds->N * nc * (uint64_t)S > ((uint64_t)1 << 40))
    return fail(ARGUS_E_UNSUPPORTED, "N * nc * S too large for one call");
  return smooth_states(ds, theta, S, mean, var, logl, status, (hipStream_t)stream);
}
