// afqmc_reconfigure_noalloc: the comb of afqmc_reconfigure with its scratch
// in a file-scope device array instead of memory the library allocates or a
// workspace brings in, for callers that cannot allocate device memory.
//
// `scratch` below is a device symbol.  In host code its name is not a device
// address: each device's copy is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that pointer is
// passed to kernels.  Every call on one device shares that device's copy, so
// calls that overlap on one device (two streams, two threads) race.  Nothing
// in it has to start at zero: the comb writes the prefix sums, parents and
// norm factor before reading them, and every snapshot column before the
// gather reads it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "afqmc.h"

namespace afq {
afqmc_status set_error(afqmc_status s, const char* msg);
int trial_device(const afqmc_trial* tr);
afqmc_status reconfigure_scratch(afqmc_trial* tr, afqmc_walkers* wk, uint64_t seed,
                                 uint64_t pc_index, char* scratch, size_t scratch_bytes,
                                 double* norm_factor_host, hipStream_t st);
}  // namespace afq

static_assert(AFQMC_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size is a multiple of 256");

// 32 MiB per device, held until the process ends.
static __device__ __align__(256) char scratch[AFQMC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_ptr[kMaxDevices] = {};

// This device's copy of `scratch` (looked up on the first call per device).
afqmc_status scratch_ptr(int device, char** out) {
  if (device < 0 || device >= kMaxDevices)
    return afq::set_error(AFQMC_ERR_ARG, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    int prev = 0;
    hipError_t e = hipGetDevice(&prev);
    if (e == hipSuccess) e = hipSetDevice(device);
    void* p = nullptr;
    if (e == hipSuccess) e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    (void)hipSetDevice(prev);
    if (e != hipSuccess || !p)
      return afq::set_error(AFQMC_ERR_DEVICE, "hipGetSymbolAddress of the scratch array failed");
    g_ptr[device] = (char*)p;
  }
  *out = g_ptr[device];
  return AFQMC_OK;
}

}  // namespace

extern "C" afqmc_status afqmc_reconfigure_noalloc(afqmc_trial* trial, afqmc_walkers* walkers,
                                                  uint64_t seed, uint64_t pc_index,
                                                  double* norm_factor_host, void* stream) {
  if (!trial) return afq::set_error(AFQMC_ERR_ARG, "NULL trial");
  char* p = nullptr;
  afqmc_status s = scratch_ptr(afq::trial_device(trial), &p);
  if (s != AFQMC_OK) return s;
  return afq::reconfigure_scratch(trial, walkers, seed, pc_index, p, AFQMC_NOALLOC_SCRATCH_BYTES,
                                  norm_factor_host, (hipStream_t)stream);
}
