// Library context (shared by the single-call and batched entry points).
#pragma once

#include <hip/hip_runtime.h>
#include <stdarg.h>
#include <stdio.h>

#include <string>
#include <vector>

#include "pcmd_internal.h"

struct pcmd_batch_plan;  // pcmd_batch.cpp

struct Buf {
  void *p = nullptr;
  size_t n = 0;
};

struct TimerRec {
  int which;
  hipEvent_t start, stop;
  double units;
};

struct pcmd_ctx {
  int device = 0;
  int n_cu = 256;
  std::string err;
  bool timing = false;
  std::vector<TimerRec> timers;
  // timer events not in use: recycled, and created ahead when timing is switched on, because
  // creating events inside a timed loop stalled the host for tens of milliseconds now and then
  std::vector<hipEvent_t> ev_pool;
  Buf rec, thr, pc, fl64, part, F, G, mom_part, fft, ll_part, blk, alias, rdesc, alias_list;
  Buf mlp_act, mlp_pre, mlp_dza, mlp_dzb, mlp_grad, mlp_part, mlp_ws, mlp_lpart;
  float *lnfact = nullptr;     // [256]
  double *lnfact64 = nullptr;  // [LNFACT64_N] ln k! in FP64 (likelihoods)
  // [6]: status bits; the generation of the last call that thinned an entry; then two 64-bit
  // words generation << 32 | length of the list of alias parts that k_prep builds (the word of
  // generation g is g & 1, and k_prep_alias of call g prepares the other one for call g + 1)
  uint32_t *status = nullptr;
  uint32_t thin_gen = 0;       // generation of the last pcmd_simulate call
  uint32_t *counter = nullptr; // [1]
  pcmd_batch_plan *batch = nullptr;
  int tune_wg_per_cu = 4;      // persistent sampler workgroups per CU
  int tune_order = 0;          // 0 most expensive job first, 1 submission order
  // shape whose twiddles, PSF copy and spectra the FFT scratch holds (the spectra are rebuilt on
  // the device whenever the PSF's contents differ from the copy)
  const void *fft_buf = nullptr;
  int fft_B = 0, fft_N = 0, fft_K = 0, fft_R = 0;
};

namespace pcmd {

inline int fail(pcmd_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

inline int hip_fail(pcmd_ctx *c, hipError_t e, const char *what) {
  return fail(c, PCMD_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

// Grow-only device buffer.
inline int ensure(pcmd_ctx *c, Buf &b, size_t bytes, const char *what) {
  if (bytes <= b.n) return PCMD_OK;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return hip_fail(c, e, "hipFree");
    b.p = nullptr;
    b.n = 0;
  }
  size_t want = bytes + bytes / 8 + 256;
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(c, PCMD_E_NOMEM, "cannot allocate %zu bytes of scratch for %s", want, what);
  }
  b.n = want;
  return PCMD_OK;
}

inline void release(Buf &b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.n = 0;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Event pair around one launch when timing is enabled.
inline hipEvent_t take_event(pcmd_ctx *c) {
  if (!c->ev_pool.empty()) {
    const hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}
inline void give_event(pcmd_ctx *c, hipEvent_t e) {
  if (e) c->ev_pool.push_back(e);
}

struct ScopedTimer {
  pcmd_ctx *c;
  hipStream_t s;
  TimerRec r{};
  bool on;
  ScopedTimer(pcmd_ctx *c_, int which, double units, hipStream_t s_) : c(c_), s(s_), on(c_->timing) {
    if (!on) return;
    r.which = which;
    r.units = units;
    r.start = take_event(c);
    r.stop = take_event(c);
    if (!r.start || !r.stop) {
      give_event(c, r.start);
      give_event(c, r.stop);
      on = false;
      return;
    }
    (void)hipEventRecord(r.start, s);
  }
  ~ScopedTimer() {
    if (!on) return;
    (void)hipEventRecord(r.stop, s);
    c->timers.push_back(r);
  }
};

inline void clear_timers(pcmd_ctx *c) {
  for (auto &t : c->timers) {
    give_event(c, t.start);
    give_event(c, t.stop);
  }
  c->timers.clear();
}

// Observation-derived quantities shared by the single and batched paths.
inline int split_mode_of(const pcmd_obs *o) {
  const bool split = o->dust_model != PCMD_DUST_NONE && o->dust_frac > 0.0;
  if (!split) return SPLIT_NONE;
  if (o->dust_frac >= 1.0) return SPLIT_ALL;
  return o->dust_frac == 0.5 ? SPLIT_HALF : SPLIT_GENERAL;
}
inline uint32_t split_q_of(const pcmd_obs *o) {
  double q = floor(o->dust_frac * 4294967296.0);
  if (q > 4294967295.0) q = 4294967295.0;
  if (q < 0.0) q = 0.0;
  return (uint32_t)q;
}

// Validate one simulation's arguments (shapes, scalars, pointers).  Returns PCMD_OK or an error
// with the message set.
int validate_sim(pcmd_ctx *c, const pcmd_iso *iso, const pcmd_obs *o, const char *who);
// Whether a validated simulation convolves through the FFT path.
bool uses_fft(const pcmd_obs *o);
int psf_grid_of(const pcmd_obs *o);  // 1 or 4

void batch_destroy(pcmd_ctx *c);
// Looks up `device`'s copy of the allocation-free call's static scratch (pcmd_noalloc.hip).
int noalloc_init(pcmd_ctx *c, int device);

}  // namespace pcmd
