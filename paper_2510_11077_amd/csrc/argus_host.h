// Host-side state of libargus (dataset handles, workspaces, error helpers).
#pragma once

#include <map>
#include <memory>
#include <string>
#include <vector>

#include "argus.h"
#include "argus_internal.h"

namespace argus {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);

#define HIPCHK(x)                                                          \
  do {                                                                     \
    hipError_t e_ = (x);                                                   \
    if (e_ != hipSuccess)                                                  \
      return ::argus::fail(ARGUS_E_HIP,                                    \
                           std::string(#x ": ") + hipGetErrorString(e_));  \
  } while (0)

// Joint model sizes. The blocked kernel (one 16-wave workgroup per sample)
// keeps the 4P-state covariance, padded to 96 rows, in the workgroup's LDS
// with 48 rows of G on each of its two elimination waves, and the
// transition of the covariance gives each of its 384 lanes at most 3 of the
// 2 P (P + 1) column segments, so P <= 22. Above that the sequential kernel
// spreads the covariance's P (P + 1) / 2 lower 4x4 pulsar blocks over the
// registers of one workgroup, at most 2048 blocks (512 threads, 4 each):
// P <= 63.
constexpr int kJointBlockedMaxPsr = 22;
constexpr int kJointMaxPsr = 63;

// The wave layout of the producer/consumer tangent sweep (k_tangent_pc,
// k_tangent5_pc) for tuning logs: one base-filter wave, then the direction
// waves (model 2: five directions, model 4: seven; log10 A and gamma both
// come from the common variance's tangent).
inline const char* tangent_pc_layout(int model, int nda) {
  if (model == 4)
    return nda == 2 ? "base wave + 3 waves of 2 directions + the common variance's wave"
                    : "base wave + 7 waves of 1 direction";
  return nda == 2 ? "base wave + the red rate's wave + 2 waves of 2 directions"
                  : "base wave + 5 waves of 1 direction";
}

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release();
  int alloc(size_t nbytes);
  int upload(const void* src, size_t nbytes);
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct TuneCfg {
  int block = 64;
  int grid = 1;
  int dynamic = 1;
  int order = 0;  // 0: items longest-first; 1: one block per CU, per-SIMD item lists;
                  // 2: time-parallel filter, block / 64 chunks per item
  float ms = 0.f;
};

// Per-sample-count state of a dataset.
struct Workspace {
  int64_t S = 0;
  DevBuf part, pstat, logl_tmp, items, counter;
  DevBuf redo;  // model 2: per-item flags of the fast form (max of both item counts)
  int n_items = 0;
  // the same items in one list per SIMD (4 per CU) with about equal TOA
  // steps per list
  DevBuf items_bal, bin_off;
  int n_items_bal = 0, n_bins = 0;
  TuneCfg cfg;
  bool tuned = false;
  std::string tune_log;
  // captured launch sequence, valid for the pointers it was captured with
  hipGraphExec_t exec{};
  bool has_graph = false;
  const void* g_theta = nullptr;
  const void* g_out = nullptr;
  const void* g_status = nullptr;
  // pointers of the previous call: a graph is captured and replayed only
  // for pointers seen on two consecutive calls
  const void* last_theta = nullptr;
  const void* last_out = nullptr;
  const void* last_status = nullptr;
  // gradient workspace: level-1 checkpoints, per-wave level-2 scratch,
  // per-pulsar gradient parts
  DevBuf ckpt, scratch, gpart, c1, seg_base, stat_tmp;
  int64_t tot_seg = 0;
  int max_sub = 0, grad_waves = 0;
  bool grad_ready = false;
  // tangent-mode gradient: directions per wave, tan_nda for pulsars of at
  // least tan_thresh TOAs and tan_ndb for the others (0 = not tuned yet;
  // tan_thresh < 0: the producer/consumer form of model 2), and the work
  // units of the split they were built for
  int tan_nda = 0, tan_ndb = 0;
  int64_t tan_thresh = 0;
  DevBuf tan_units;
  int n_tan_units = 0, units_nda = 0, units_ndb = 0;
  int64_t units_thresh = -1;
  std::vector<int32_t> items_host;  // the items, as uploaded
  std::string grad_log;
  // smoother of models 1, 2: 1 = one wave per item, K > 1 = the
  // time-parallel form with chunks of about 1 / K of the longest pulsar
  // (0 = not tuned yet); the per-item chunk counts and slots, the (item,
  // chunk) units and the chunk count they were built for, chunk summaries,
  // hand-over states and the reverse waves' level-2 scratch
  int smooth_k = 0, tp_built_k = 0, n_tp_units = 0, tp_waves = 0;
  DevBuf tp_item, tp_units, tp_sum, tp_adj, tp_scr;
  // its checkpoints: the filtered state before every fourth TOA (per-pulsar
  // stride 4, segment bases, the store)
  DevBuf tp_c1, tp_seg, tp_ck;
  int64_t tp_tot_seg = 0;
  std::string smooth_log;
  // HMC: proposal position, momentum, gradient, logL, initial energy, flags
  DevBuf hmc_x, hmc_p, hmc_g, hmc_l, hmc_h0, hmc_ok;
  // NUTS: trajectory, cursor and subtree-stack buffers for depth <= nuts_md
  DevBuf nuts_f, nuts_i;
  int nuts_md = 0;
  ~Workspace();
};

}  // namespace argus

struct argus_dataset {
  int model = 0, P = 0, C = 0, D = 0;
  int64_t N = 0;
  int device = 0, n_cu = 256;
  argus::ModelConst mc{};
  argus::DevBuf rec, off, col, icol, fixed, hd, t, y, sig;  // icol: theta column -> canonical
  argus::DevBuf chrom;  // model 4: (nu_ref / nu)^2 per TOA
  argus::DevBuf porder; // models 1, 2, 4: pulsars by TOA count, longest first
  argus::DevBuf maxdt;  // models 1, 2, 4: largest TOA interval of each pulsar
  std::vector<int64_t> off_h, counts;
  std::map<int64_t, std::unique_ptr<argus::Workspace>> ws;
  hipStream_t cap_stream = nullptr;
};

namespace argus {
int check_device(const argus_dataset* ds);
Workspace* get_workspace(argus_dataset* ds, int64_t S, int* rc);
int joint_loglike(argus_dataset* ds, const double* theta, int64_t S, double* logl,
                  int32_t* status, hipStream_t st);
int grad_loglike(argus_dataset* ds, const double* theta, int64_t S, double* logl, double* grad,
                 int32_t* status, hipStream_t st);
int smooth_states(argus_dataset* ds, const double* theta, int64_t S, double* mean, double* var,
                  double* logl, int32_t* status, hipStream_t st);
int nuts_step(argus_dataset* ds, int64_t S, int32_t max_depth, const double* eps,
              const double* m_inv, const double* lo, const double* hi, const double* z,
              const int32_t* dirs, const double* u_top, const double* u_sub, double* theta,
              double* logl, double* grad, int32_t* depth, int32_t* n_leapfrog,
              int32_t* divergent, double* accept_stat, hipStream_t st);
int device_rate(int kind, int waves_per_simd, int iters, double* tflops, double* clock_mhz,
                hipStream_t st);
int hmc_step(argus_dataset* ds, int64_t S, int32_t n_leapfrog, const double* eps,
             const double* m_inv, const double* lo, const double* hi, const double* z,
             const double* logu, double* theta, double* logl, double* grad,
             int32_t* accepted, double* dh, hipStream_t st);
}  // namespace argus
