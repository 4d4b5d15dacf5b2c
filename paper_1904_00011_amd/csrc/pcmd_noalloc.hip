// Allocation-free variant of the likelihood call, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops): its block sums live in a fixed, file-scope
// device array instead of the context's grow-on-demand scratch.
#include <hip/hip_runtime.h>
#include <cmath>
#include <mutex>

#include "pcmd_ctx.h"

using namespace pcmd;

namespace {

// The largest Hess diagram the variant scores, and its block sums: one double per LL_THREADS bins.
constexpr int NOALLOC_MAX_BINS = 65536;
constexpr int SCRATCH_DOUBLES = (NOALLOC_MAX_BINS + LL_THREADS - 1) / LL_THREADS;  // 256 doubles, 2 KiB

// One copy per GPU, held until the process ends.  Host code never passes `scratch` itself to a
// kernel: on the host that name is a stand-in, not a device address.  It uses the address that
// hipGetSymbolAddress returned for the device (scratch_ptr).
static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES] = {};

}  // namespace

namespace pcmd {

// Called by pcmd_create with `device` current: looks up this device's copy of the scratch array
// once and keeps its address.
int noalloc_init(pcmd_ctx *c, int device) {
  if (device < 0 || device >= MAX_DEVICES)
    return fail(c, PCMD_E_INVAL, "device %d beyond the %d the allocation-free call supports", device, MAX_DEVICES);
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_ptr[device]) return PCMD_OK;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) return hip_fail(c, e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  scratch_ptr[device] = p;
  return PCMD_OK;
}

}  // namespace pcmd

extern "C" int pcmd_loglike_noalloc(pcmd_ctx *c, const uint32_t *hm, const uint32_t *hd, int32_t nbins,
                                    const double *mom_m, const double *mom_d, int32_t mode, double eps, double *out,
                                    pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (!hm || !hd || !out) return fail(c, PCMD_E_INVAL, "pcmd_loglike_noalloc: null argument");
  if (nbins < 1 || nbins > NOALLOC_MAX_BINS)
    return fail(c, PCMD_E_INVAL, "pcmd_loglike_noalloc: n_bins %d outside [1, %d] (the static scratch holds %d block sums)",
                nbins, NOALLOC_MAX_BINS, SCRATCH_DOUBLES);
  const bool accumulate = (mode & PCMD_LL_ACCUMULATE) != 0;
  mode &= ~PCMD_LL_ACCUMULATE;
  if (mode < 0 || mode > 2) return fail(c, PCMD_E_INVAL, "pcmd_loglike_noalloc: bad mode %d", mode);
  if (mode == PCMD_LL_POISSON && !(eps > 0.0 && std::isfinite(eps)))
    return fail(c, PCMD_E_INVAL, "pcmd_loglike_noalloc: eps must be > 0");
  if (mode != PCMD_LL_POISSON && (!mom_m || !mom_d)) return fail(c, PCMD_E_INVAL, "pcmd_loglike_noalloc: moments needed");
  void *ptr;
  {
    std::lock_guard<std::mutex> lock(scratch_mu);
    ptr = (c->device >= 0 && c->device < MAX_DEVICES) ? scratch_ptr[c->device] : nullptr;
  }
  if (!ptr) return fail(c, PCMD_E_INVAL, "pcmd_loglike_noalloc: no scratch address for device %d", c->device);
  DeviceGuard dg(c->device);
  // every block writes its own block sum before the final kernel reads it: nothing to clear
  LoglikeArgs a{hm, hd, nbins, mode, mom_m, mom_d, eps, out, (double *)ptr, accumulate ? 1 : 0, c->lnfact64};
  const hipError_t e = launch_loglike(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "k_loglike (no-alloc)");
  c->err.clear();
  return PCMD_OK;
}
