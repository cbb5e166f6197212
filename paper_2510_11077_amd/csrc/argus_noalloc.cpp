// The batched likelihood without device allocation: argus_loglike_noalloc.
//
// Same kernels as argus_loglike (the per-pulsar filter, then the fixed-order
// reduction over pulsars), launched in one fixed layout (no autotuning, no
// graph), with the per-(pulsar, sample) partial terms and status words kept
// in a file-scope device array instead of a per-sample-count workspace.
// Host code never passes that array's name to a kernel or a copy: in host
// code the name stands for a host-side shadow, not a device address. Its
// device address is looked up once per device with hipGetSymbolAddress (each
// device holds its own copy of the array) and only that address is used.
#include <algorithm>
#include <mutex>
#include <string>

#include "argus.h"
#include "argus_host.h"
#include "argus_internal.h"

using namespace argus;

namespace {

constexpr size_t kScratchBytes = size_t(8) << 20;
constexpr int kMaxDevices = 64;

// partial logL terms [P * S] doubles, status words [P * S] int32 and the
// per-item flags of the fast model 2 loop [P * ceil(S / 64)] int32, each
// part starting on a 256-B boundary
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array, looked up on
// the first call on the device (the current device).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return fail(ARGUS_E_UNSUPPORTED, "device index beyond the no-allocation table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ARGUS_E_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                   hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ARGUS_OK;
}

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t scratch_need(int P, int64_t S) {
  const size_t ps = (size_t)P * (size_t)S, items = (size_t)P * (size_t)((S + 63) / 64);
  return round_up(ps * 8, 256) + round_up(ps * 4, 256) + items * 4;
}

// largest S whose parts fit the array
int64_t max_samples(int P) {
  int64_t s = (int64_t)(kScratchBytes / (12 * (size_t)P));
  while (s > 0 && scratch_need(P, s) > kScratchBytes) --s;
  return s;
}

}  // namespace

extern "C" int argus_loglike_noalloc(argus_dataset_t ds, const double* theta, int64_t S,
                                     double* logl, int32_t* status, void* stream) {
  if (!ds) return fail(ARGUS_E_INVAL, "dataset is NULL");
  if (S < 0) return fail(ARGUS_E_INVAL, "S must be >= 0");
  if (S > 0 && ds->D > 0 && !theta) return fail(ARGUS_E_INVAL, "theta is NULL");
  if (S > 0 && !logl) return fail(ARGUS_E_INVAL, "output is NULL");
  if (ds->model == ARGUS_M3_JOINT_HD)
    return fail(ARGUS_E_UNSUPPORTED, "the no-allocation likelihood covers models 1, 2 and 4");
  int rc = check_device(ds);
  if (rc || S == 0) return rc;
  const size_t ps = (size_t)ds->P * (size_t)S;
  const size_t part_bytes = round_up(ps * sizeof(double), 256);
  const size_t stat_bytes = round_up(ps * sizeof(int32_t), 256);
  if (S > ((int64_t)1 << 30) || scratch_need(ds->P, S) > kScratchBytes) {
    return fail(ARGUS_E_INVAL, "S = " + std::to_string(S) + " exceeds the no-allocation scratch (" +
                                   std::to_string(kScratchBytes >> 20) + " MiB: at most " +
                                   std::to_string(max_samples(ds->P)) + " samples for " +
                                   std::to_string(ds->P) + " pulsars)");
  }
  void* base = nullptr;
  if ((rc = scratch_address(ds->device, &base))) return rc;
  double* part = static_cast<double*>(base);
  int32_t* pstat = reinterpret_cast<int32_t*>(static_cast<unsigned char*>(base) + part_bytes);
  int32_t* redo =
      reinterpret_cast<int32_t*>(static_cast<unsigned char*>(base) + part_bytes + stat_bytes);
  hipStream_t st = (hipStream_t)stream;
  // every (pulsar, sample) term and every item flag is written by the
  // filter before it is read, so nothing needs clearing; no work-queue
  // counter
  FilterArgs a{};
  a.rec = ds->rec.as<TOARec>();
  a.chrom = ds->chrom.as<double>();
  a.off = ds->off.as<int64_t>();
  a.maxdt = ds->maxdt.as<double>();
  a.theta = theta;
  a.col = ds->col.as<int32_t>();
  a.fixed = ds->fixed.as<double>();
  a.items = nullptr;
  a.porder = ds->porder.as<int32_t>();
  a.tiles = (int32_t)((S + kWave - 1) / kWave);
  a.bin_off = nullptr;
  a.counter = nullptr;
  a.redo = redo;
  a.part = part;
  a.pstat = pstat;
  a.S = S;
  a.D = ds->D;
  a.P = ds->P;
  a.n_items = a.tiles * ds->P;
  a.dynamic = 0;
  a.mc = ds->mc;
  // items longest first, one wave each, four waves per block; waves beyond
  // 8 per SIMD stride over the rest
  const int block = 256, wpb = block / kWave;
  const int64_t grid = std::min<int64_t>((a.n_items + wpb - 1) / wpb, 8LL * ds->n_cu);
  HIPCHK(launch_filter(ds->model, a, (int)grid, block, st));
  ReduceArgs r{part, pstat, logl, status, nullptr, S, ds->P};
  HIPCHK(launch_reduce(r, st));
  return ARGUS_OK;
}
