// C ABI of the pCMD forward model: context, argument validation, scratch management and the
// host-side model helpers.  Every device step runs in the gfx950 kernels of k_*.hip.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "pcmd_ctx.h"
#include "pcmd_device.h"
#include "pcmd_internal.h"

using namespace pcmd;

namespace pcmd {

int psf_grid_of(const pcmd_obs *o) { return o->psf_grid == 4 ? 4 : 1; }

// AUTO: the direct sum costs N^2 K^2 FMAs per band (15.5e12 FMA/s measured), the FFT chain
// ~7 launches and O(N^2 log N) FP64 work; measured on MI355X the direct path wins for K = 31 at
// every size tried (256^2: ~12 against 52 us; 4096^2: 3.1 against 8.7 ms) and the FFT for K = 63
// from 512^2 up, so AUTO takes the FFT from K = 48 on.
bool uses_fft(const pcmd_obs *o) {
  return o->psf_k > 1 && (o->conv_path == PCMD_CONV_FFT ||
                          (o->conv_path == PCMD_CONV_AUTO && o->psf_k >= 48 && psf_grid_of(o) == 1 &&
                           fft_supported(o->nim)));
}

int validate_sim(pcmd_ctx *c, const pcmd_iso *iso, const pcmd_obs *o, const char *who) {
  if (!iso || !o) return fail(c, PCMD_E_INVAL, "%s: null argument", who);
  const int E = iso->n_entries, B = iso->n_bands;
  if (E <= 0 || E > (1 << 26)) return fail(c, PCMD_E_INVAL, "%s: n_entries %d out of range", who, E);
  if (B < 1 || B > PCMD_MAX_BANDS) return fail(c, PCMD_E_INVAL, "%s: n_bands %d out of range", who, B);
  if (!iso->lam || !iso->flux) return fail(c, PCMD_E_INVAL, "%s: null lam/flux", who);
  const int N = o->nim;
  if (N < 1 || N > 8192) return fail(c, PCMD_E_INVAL, "%s: nim %d out of range", who, N);
  if (!isfinite(o->dmod)) return fail(c, PCMD_E_INVAL, "%s: dmod not finite", who);
  if (o->dust_model < 0 || o->dust_model > 2) return fail(c, PCMD_E_INVAL, "%s: bad dust_model", who);
  if (o->dust_model != PCMD_DUST_NONE) {
    if (!(o->dust_frac >= 0.0 && o->dust_frac <= 1.0)) return fail(c, PCMD_E_INVAL, "%s: dust_frac outside [0,1]", who);
    if (!isfinite(o->dust_mu) || !(o->dust_sigma >= 0.0) || !isfinite(o->dust_sigma))
      return fail(c, PCMD_E_INVAL, "%s: bad dust parameters", who);
    for (int b = 0; b < B; ++b)
      if (!isfinite(o->dust_R[b])) return fail(c, PCMD_E_INVAL, "%s: dust_R not finite", who);
  }
  const int K = o->psf_k;
  if (K < 1 || (K & 1) == 0 || K > N || K > PCMD_MAX_PSF_K)
    return fail(c, PCMD_E_INVAL, "%s: psf_k %d must be odd, <= nim and <= %d", who, K, PCMD_MAX_PSF_K);
  if (K > 1 && !o->psf) return fail(c, PCMD_E_INVAL, "%s: psf is NULL", who);
  if (o->psf_grid != 0 && o->psf_grid != 1 && o->psf_grid != 4)
    return fail(c, PCMD_E_INVAL, "%s: psf_grid %d must be 0, 1 or 4", who, o->psf_grid);
  if (o->conv_path < 0 || o->conv_path > 2) return fail(c, PCMD_E_INVAL, "%s: bad conv_path", who);
  if (o->noise_model < 0 || o->noise_model > 2) return fail(c, PCMD_E_INVAL, "%s: bad noise_model", who);
  if (o->sampler < PCMD_SAMPLER_POINT || o->sampler > PCMD_SAMPLER_HYBRID)
    return fail(c, PCMD_E_INVAL, "%s: bad sampler %d", who, o->sampler);
  for (int b = 0; b < B; ++b) {
    if (o->noise_model == PCMD_NOISE_GAUSS_MAG && !(o->noise_sigma_mag[b] >= 0.0 && isfinite(o->noise_sigma_mag[b])))
      return fail(c, PCMD_E_INVAL, "%s: bad noise_sigma_mag", who);
    if (o->noise_model == PCMD_NOISE_SHOT &&
        (!(o->exptime[b] > 0.0) || !isfinite(o->exptime[b]) || !isfinite(o->zp[b]) || !(o->sky[b] >= 0.0)))
      return fail(c, PCMD_E_INVAL, "%s: bad exptime/zp/sky", who);
  }
  if (uses_fft(o) && !fft_supported(N))
    return fail(c, PCMD_E_UNSUPPORTED, "%s: FFT path needs nim a power of two in [8, 4096]", who);
  if (K > 1 && !uses_fft(o) && conv_direct_lds_bytes(K) > 160 * 1024)
    return fail(c, PCMD_E_UNSUPPORTED, "%s: psf_k %d too large for the direct path; use the FFT path", who, K);
  return PCMD_OK;
}

}  // namespace pcmd

extern "C" {

const char *pcmd_version(void) { return "pcmd gfx950 HIP 1.1 (philox4x32-10, slices of up to 1024 entries)"; }

int pcmd_create(pcmd_ctx **out, int hip_device) {
  if (!out) return PCMD_E_INVAL;
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess) return PCMD_E_HIP;
  if (hip_device < 0 || hip_device >= ndev) return PCMD_E_INVAL;
  pcmd_ctx *c = new pcmd_ctx();
  c->device = hip_device;
  DeviceGuard g(hip_device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  // ln k! for k < 256: FP64 running sum of ln j, rounded to FP32.
  float tab[256];
  double acc = 0.0;
  tab[0] = tab[1] = 0.0f;
  for (int k = 2; k < 256; ++k) {
    acc = acc + log((double)k);
    tab[k] = (float)acc;
  }
  // ln k! in FP64 for the likelihoods' ln d_j! (k < LNFACT64_N; lgamma beyond)
  std::vector<double> lf(LNFACT64_N);
  for (int k = 0; k < LNFACT64_N; ++k) lf[k] = std::lgamma((double)k + 1.0);
  if (hipMalloc(&c->lnfact, sizeof tab) != hipSuccess || hipMalloc(&c->status, 32) != hipSuccess ||
      hipMalloc(&c->counter, 8) != hipSuccess || hipMalloc(&c->lnfact64, LNFACT64_N * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    pcmd_destroy(c);
    return PCMD_E_NOMEM;
  }
  uint32_t zeros[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  if (hipMemcpy(c->lnfact, tab, sizeof tab, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->lnfact64, lf.data(), LNFACT64_N * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->status, zeros, 32, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->counter, zeros, 8, hipMemcpyHostToDevice) != hipSuccess) {
    pcmd_destroy(c);
    return PCMD_E_HIP;
  }
  // this device's address of the allocation-free call's static scratch (looked up once)
  if (noalloc_init(c, hip_device) != PCMD_OK) {
    pcmd_destroy(c);
    return PCMD_E_HIP;
  }
  *out = c;
  return PCMD_OK;
}

void pcmd_destroy(pcmd_ctx *c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipDeviceSynchronize();
  clear_timers(c);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  c->ev_pool.clear();
  batch_destroy(c);
  Buf *bufs[] = {&c->rec,     &c->thr,     &c->pc,      &c->fl64,    &c->part,     &c->F,       &c->G,
                 &c->mom_part, &c->fft,    &c->mlp_act, &c->mlp_pre, &c->mlp_dza, &c->mlp_dzb, &c->mlp_grad,
                 &c->mlp_part, &c->mlp_ws, &c->mlp_lpart, &c->ll_part, &c->blk, &c->alias, &c->rdesc, &c->alias_list};
  for (Buf *b : bufs) release(*b);
  if (c->lnfact) (void)hipFree(c->lnfact);
  if (c->lnfact64) (void)hipFree(c->lnfact64);
  if (c->status) (void)hipFree(c->status);
  if (c->counter) (void)hipFree(c->counter);
  delete c;
}

const char *pcmd_last_error(const pcmd_ctx *c) { return c ? c->err.c_str() : "null context"; }

int pcmd_sync(pcmd_ctx *c, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  DeviceGuard g(c->device);
  hipStream_t s = (hipStream_t)stream;
  uint32_t st = 0;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(&st, c->status, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(c, e, "pcmd_sync");
  if (st) {
    uint32_t z = 0;
    e = hipMemcpy(c->status, &z, 4, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(c, e, "pcmd_sync");
    if (st & STATUS_BAD_LAMBDA) return fail(c, PCMD_E_INVAL, "an expected star count was negative, not finite or >= 2^22 (drawn as 0)");
    if (st & STATUS_BAD_PSF) return fail(c, PCMD_E_INVAL, "a PSF band has a negative or non-finite value or does not sum to 1 within 1e-3");
    if (st & STATUS_BAD_ROW) return fail(c, PCMD_E_INVAL, "a training row index was outside the set (row 0 was used)");
    return fail(c, PCMD_E_PTRS_RETRY, "a transformed-rejection draw exhausted its %d attempts", PTRS_MAX_ATTEMPTS);
  }
  c->err.clear();
  return PCMD_OK;
}

// ------------------------------------------------------------------------------------------
// a0 host helpers
// ------------------------------------------------------------------------------------------

// Integral of the Kroupa (2001) IMF over [lo, hi]: xi(m) = k_i m^-a_i with a = 0.3 / 1.3 / 2.3 on
// [0, 0.08) / [0.08, 0.5) / [0.5, inf) and k = 1 / 0.08 / 0.04 (continuous at the breaks).
static double kroupa_integral(double lo, double hi) {
  const double brk[4] = {0.0, 0.08, 0.5, INFINITY};
  const double a[3] = {0.3, 1.3, 2.3}, k[3] = {1.0, 0.08, 0.04};
  double s = 0.0;
  for (int j = 0; j < 3; ++j) {
    const double l = fmax(lo, brk[j]), h = fmin(hi, brk[j + 1]);
    if (h > l) s += k[j] * (pow(h, 1.0 - a[j]) - pow(l, 1.0 - a[j])) / (1.0 - a[j]);
  }
  return s;
}

int pcmd_grid_prepare(int32_t E, int32_t B, const int32_t *iso, const double *mass, const double *absmag, int32_t imf,
                      double alpha, double *imf_w, float *flux, int32_t n_iso, double *iso_imf_sum) {
  if (E <= 0 || B < 1 || B > PCMD_MAX_BANDS || !iso || !mass || !absmag || !imf_w || !flux) return PCMD_E_INVAL;
  if (imf != PCMD_IMF_POWER_LAW && imf != PCMD_IMF_KROUPA) return PCMD_E_INVAL;
  if (imf == PCMD_IMF_POWER_LAW && (!(alpha > 1.0) || !isfinite(alpha))) return PCMD_E_INVAL;
  if (iso_imf_sum) {
    if (n_iso < 1 || n_iso > PCMD_MAX_ISO) return PCMD_E_INVAL;
    for (int i = 0; i < E; ++i)
      if (iso[i] < 0 || iso[i] >= n_iso) return PCMD_E_INVAL;
  }
  int start = 0;
  while (start < E) {
    int end = start + 1;
    while (end < E && iso[end] == iso[start]) ++end;
    const int P = end - start;
    for (int i = start; i < end; ++i) {
      if (!(mass[i] > 0.0) || !isfinite(mass[i])) return PCMD_E_INVAL;
      if (i > start && !(mass[i] > mass[i - 1])) return PCMD_E_INVAL;
    }
    for (int i = start; i < end; ++i) {
      double lo, hi;
      if (P == 1) {
        lo = mass[i] * 0.99;
        hi = mass[i] * 1.01;
      } else {
        const double l = log(mass[i]);
        const double lprev = i > start ? log(mass[i - 1]) : l - (log(mass[i + 1]) - l);
        const double lnext = i + 1 < end ? log(mass[i + 1]) : l + (l - log(mass[i - 1]));
        lo = exp(0.5 * (lprev + l));
        hi = exp(0.5 * (l + lnext));
      }
      imf_w[i] = imf == PCMD_IMF_KROUPA ? kroupa_integral(lo, hi)
                                         : (pow(lo, 1.0 - alpha) - pow(hi, 1.0 - alpha)) / (alpha - 1.0);
    }
    start = end;
  }
  for (int b = 0; b < B; ++b)
    for (int i = 0; i < E; ++i) {
      const double m = absmag[(size_t)b * E + i];
      if (!isfinite(m)) return PCMD_E_INVAL;
      flux[(size_t)b * E + i] = (float)pow(10.0, -0.4 * m);
    }
  if (iso_imf_sum) {
    // the normalisation of the expected counts: the IMF weight summed over each isochrone's points
    for (int k = 0; k < n_iso; ++k) iso_imf_sum[k] = 0.0;
    for (int i = 0; i < E; ++i) iso_imf_sum[iso[i]] += imf_w[i];
  }
  return PCMD_OK;
}

int pcmd_iso_weights(const pcmd_model *m, const pcmd_isoset *set, double *w_out, double *npix_out) {
  if (!m || !set || !w_out || !npix_out) return PCMD_E_INVAL;
  const int na = set->n_age, nf = set->n_feh, ni = set->n_iso;
  if (na < 1 || nf < 1 || ni < 1 || ni > PCMD_MAX_ISO || !set->age_edges || !set->feh_grid || !set->iso_age ||
      !set->iso_feh)
    return PCMD_E_INVAL;
  std::vector<double> wa(na, 0.0), wz(nf, 0.0);
  const double T = pow(10.0, 10.2);
  double npix = pow(10.0, m->log_npix);
  switch (m->sfh) {
    case PCMD_SFH_SSP:
      if (m->ssp_age_index < 0 || m->ssp_age_index >= na) return PCMD_E_INVAL;
      wa[m->ssp_age_index] = 1.0;
      break;
    case PCMD_SFH_CONST:
      for (int a = 0; a < na; ++a) wa[a] = pow(10.0, set->age_edges[a + 1]) - pow(10.0, set->age_edges[a]);
      break;
    case PCMD_SFH_TAU:
    case PCMD_SFH_DTAU: {
      if (!(m->tau_gyr > 0.0)) return PCMD_E_INVAL;
      const double tau = m->tau_gyr * 1e9;
      for (int a = 0; a < na; ++a) {
        const double t1 = T - pow(10.0, set->age_edges[a + 1]);  // onset-relative time at the older edge
        const double t2 = T - pow(10.0, set->age_edges[a]);
        if (m->sfh == PCMD_SFH_TAU) {
          wa[a] = tau * (exp(-t1 / tau) - exp(-t2 / tau));
        } else {
          wa[a] = -tau * (t2 + tau) * exp(-t2 / tau) + tau * (t1 + tau) * exp(-t1 / tau);
        }
      }
      break;
    }
    case PCMD_SFH_NONPARAM: {
      if (!m->log_sfh) return PCMD_E_INVAL;
      npix = 0.0;
      for (int a = 0; a < na; ++a) {
        wa[a] = pow(10.0, m->log_sfh[a]);
        npix += wa[a];
      }
      break;
    }
    default:
      return PCMD_E_INVAL;
  }
  if (m->mdf == PCMD_MDF_SINGLE) {
    if (m->feh_index < 0 || m->feh_index >= nf) return PCMD_E_INVAL;
    wz[m->feh_index] = 1.0;
  } else if (m->mdf == PCMD_MDF_GAUSS) {
    if (!(m->feh_sigma > 0.0)) return PCMD_E_INVAL;
    double s = 0.0;
    for (int f = 0; f < nf; ++f) {
      const double z = (set->feh_grid[f] - m->feh_mu) / m->feh_sigma;
      wz[f] = exp(-0.5 * z * z);
      s += wz[f];
    }
    double s2 = 0.0;
    for (int f = 0; f < nf; ++f) {
      wz[f] /= s;
      if (wz[f] < m->mdf_prune) wz[f] = 0.0;
      s2 += wz[f];
    }
    if (!(s2 > 0.0)) return PCMD_E_INVAL;
    for (int f = 0; f < nf; ++f) wz[f] /= s2;
  } else {
    return PCMD_E_INVAL;
  }
  for (int k = 0; k < ni; ++k) {
    const int a = set->iso_age[k], f = set->iso_feh[k];
    if (a < 0 || a >= na || f < 0 || f >= nf) return PCMD_E_INVAL;
    w_out[k] = wa[a] * wz[f];
  }
  if (!(npix > 0.0) || !isfinite(npix)) return PCMD_E_INVAL;
  *npix_out = npix;
  return PCMD_OK;
}

int pcmd_entries(pcmd_ctx *c, const pcmd_grid *g, const double *iso_w, double npix, double *lam_out,
                 pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (!g || !iso_w || !lam_out) return fail(c, PCMD_E_INVAL, "pcmd_entries: null argument");
  if (g->n_entries <= 0 || g->n_iso <= 0 || g->n_iso > PCMD_MAX_ISO || !g->iso_of_entry || !g->imf_w ||
      !g->iso_imf_sum)
    return fail(c, PCMD_E_INVAL, "pcmd_entries: bad grid (E=%d, n_iso=%d)", g->n_entries, g->n_iso);
  if (!(npix > 0.0) || !isfinite(npix)) return fail(c, PCMD_E_INVAL, "pcmd_entries: npix must be positive");
  double norm = 0.0;
  for (int k = 0; k < g->n_iso; ++k) {
    if (!(iso_w[k] >= 0.0) || !isfinite(iso_w[k])) return fail(c, PCMD_E_INVAL, "pcmd_entries: bad iso weight %d", k);
    norm += iso_w[k] * g->iso_imf_sum[k];
  }
  if (!(norm > 0.0) || !isfinite(norm)) return fail(c, PCMD_E_INVAL, "pcmd_entries: all weights are zero");
  double scale[PCMD_MAX_ISO];
  for (int k = 0; k < g->n_iso; ++k) scale[k] = npix * iso_w[k] / norm;
  DeviceGuard dg(c->device);
  hipError_t e = launch_entries(g, scale, lam_out, c->status, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "k_entries");
  c->err.clear();
  return PCMD_OK;
}

// ------------------------------------------------------------------------------------------
// a1-a4
// ------------------------------------------------------------------------------------------

int pcmd_simulate(pcmd_ctx *c, const pcmd_iso *iso, const pcmd_obs *o, float *mags, const pcmd_debug *dbg,
                  pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (!mags) return fail(c, PCMD_E_INVAL, "pcmd_simulate: null mags_out");
  int r = validate_sim(c, iso, o, "pcmd_simulate");
  if (r) return r;
  const int E = iso->n_entries, B = iso->n_bands, N = o->nim, K = o->psf_k;
  const int64_t npx = (int64_t)N * N;
  int64_t px0 = 0, px1 = 0;
  if (dbg && (dbg->counts || dbg->reddened)) {
    px0 = dbg->px0;
    px1 = dbg->px1;
    if (!dbg->counts || px0 < 0 || px1 <= px0 || px1 > npx)
      return fail(c, PCMD_E_INVAL, "pcmd_simulate: bad debug window [%lld, %lld)", (long long)px0, (long long)px1);
  }
  const bool use_fft = uses_fft(o);
  hipStream_t s = (hipStream_t)stream;
  DeviceGuard dg(c->device);
  const int BP = B <= 2 ? 2 : 4;
  const int nchunks = sample_slices(E, npx);
  const int split_mode = split_mode_of(o);
  const int S = split_mode == SPLIT_NONE ? 1 : 2;
  const bool block = o->sampler == PCMD_SAMPLER_BLOCK, hybrid = o->sampler == PCMD_SAMPLER_HYBRID;
  const int nb = superblocks(E);
  // block-skip tables: [nb] BlockRec, [nb][THR_STRIDE] thresholds, [nb] PtrsConst, [nb][SBLK] cth
  const size_t blk_rec = (size_t)nb * sizeof(BlockRec), blk_thr = (size_t)nb * THR_STRIDE * 4,
               blk_pc = (size_t)nb * sizeof(PtrsConst), blk_cth = (size_t)nb * SBLK * 4;
  if (block || hybrid) {
    if ((r = ensure(c, c->blk, blk_rec + blk_thr + blk_pc + blk_cth, "block tables"))) return r;
  }
  if (!block) {
    if ((r = ensure(c, c->rec, rec_bytes(E), "entry records"))) return r;
    if ((r = ensure(c, c->thr, (size_t)entries_padded(E) * THR_STRIDE * 4, "thresholds"))) return r;
    if ((r = ensure(c, c->pc, (size_t)E * 2 * sizeof(PtrsConst), "rejection constants"))) return r;
    if ((r = ensure(c, c->alias, (size_t)E * 2 * ALIAS_COLS * 4, "alias columns"))) return r;
    if ((r = ensure(c, c->rdesc, (size_t)E * 4, "reddened-part descriptors"))) return r;
    if ((r = ensure(c, c->alias_list, (size_t)E * 2 * 4, "alias-part list"))) return r;
  }
  if ((r = ensure(c, c->fl64, (size_t)E * BP * 8, "fluxes"))) return r;
  if ((r = ensure(c, c->part, (size_t)nchunks * S * B * npx * 4, "partial sums"))) return r;
  if ((r = ensure(c, c->F, (size_t)B * npx * 4, "image"))) return r;
  if ((r = ensure(c, c->G, (size_t)B * npx * 4, "convolved image"))) return r;
  const int R = psf_grid_of(o) * psf_grid_of(o);
  if (K > 1 && use_fft && (r = ensure(c, c->fft, fft_scratch_bytes(B, N, K, R), "fft"))) return r;

  const uint32_t k0 = (uint32_t)(o->seed & 0xFFFFFFFFu), k1 = (uint32_t)(o->seed >> 32);
  hipError_t e = hipSuccess;
  if (dbg && dbg->counts) {
    e = launch_fill_u32(dbg->counts, 0u, (px1 - px0) * E, s);
    if (e == hipSuccess && dbg->reddened) e = launch_fill_u32(dbg->reddened, 0u, (px1 - px0) * E, s);
    if (e != hipSuccess) return hip_fail(c, e, "clearing debug counts");
  }
  // block totals, tables and cumulative thresholds (block-skip and hybrid samplers)
  BlockPrepArgs pb{};
  if (block || hybrid) {
    char *base = (char *)c->blk.p;
    pb = BlockPrepArgs{E,
                       B,
                       BP,
                       nb,
                       iso->lam,
                       iso->flux,
                       (BlockRec *)base,
                       (uint32_t *)(base + blk_rec),
                       base + blk_rec + blk_thr,
                       (uint32_t *)(base + blk_rec + blk_thr + blk_pc),
                       (double *)c->fl64.p,
                       c->status,
                       hybrid ? 1 : 0};
  }
  BlockSampleArgs ab{};
  if (block || hybrid) {
    e = launch_prep_block(pb, s);
    if (e != hipSuccess) return hip_fail(c, e, "k_prep_block");
    ab.E = E;
    ab.B = B;
    ab.BP = BP;
    ab.npx = (int)npx;
    ab.nb = nb;
    ab.nchunks = nchunks;
    ab.S = S;
    ab.k0 = k0;
    ab.k1 = k1;
    ab.split_mode = split_mode;
    ab.split_q = split_q_of(o);
    ab.brec = pb.brec;
    ab.thr = pb.thr;
    ab.pc = pb.pc;
    ab.cth = pb.cth;
    ab.fl64 = pb.fl64;
    ab.part = (float *)c->part.p;
    ab.dbg_counts = dbg ? dbg->counts : nullptr;
    ab.dbg_red = dbg ? dbg->reddened : nullptr;
    ab.px0 = px0;
    ab.px1 = px1;
    ab.status = c->status;
    ab.lnfact = c->lnfact;
    ab.accumulate = hybrid ? 1 : 0;  // hybrid: k_sample has written the partials first
  }
  if (block) {
    ScopedTimer tm(c, PCMD_TIMER_SAMPLE, (double)npx * (double)E, s);
    e = launch_sample_block(ab, s);
  } else {
    PrepArgs pa{E,
                B,
                BP,
                iso->lam,
                iso->flux,
                (EntryRec *)c->rec.p,
                (GroupRec *)((EntryRec *)c->rec.p + entries_padded(E)),
                (uint32_t *)c->thr.p,
                c->pc.p,
                (double *)c->fl64.p,
                c->status,
                (uint32_t *)c->alias.p,
                hybrid ? pb.brec : nullptr,
                thin_mode_of_split(split_mode),
                o->dust_frac,
                (uint32_t *)c->rdesc.p,
                c->status + 1,
                ++c->thin_gen,
                (uint32_t *)c->alias_list.p,
                (unsigned long long *)(c->status + 2)};
    e = launch_prep(pa, s);
    if (e == hipSuccess) e = launch_prep_alias(pa, s);
    if (e != hipSuccess) return hip_fail(c, e, "k_prep");
    SampleArgs a;
    a.E = E;
    a.B = B;
    a.BP = BP;
    a.npx = (int)npx;
    a.nchunks = nchunks;
    a.S = S;
    a.k0 = k0;
    a.k1 = k1;
    a.split_mode = split_mode;
    a.split_q = split_q_of(o);
    a.rec = pa.rec;
    a.grp = pa.grp;
    a.thr = pa.thr;
    a.pc = pa.pc;
    a.part = (float *)c->part.p;
    a.dbg_counts = dbg ? dbg->counts : nullptr;
    a.dbg_red = dbg ? dbg->reddened : nullptr;
    a.px0 = px0;
    a.px1 = px1;
    a.status = c->status;
    a.lnfact = c->lnfact;
    a.alias = pa.alias;
    a.rdesc = pa.rdesc;
    a.thin_seen = pa.thin_seen;
    a.gen = pa.gen;
    ScopedTimer tm(c, PCMD_TIMER_SAMPLE, (double)npx * (double)E, s);
    e = launch_sample(a, s);
    if (e == hipSuccess && hybrid) e = launch_sample_block(ab, s);
  }
  if (e != hipSuccess) return hip_fail(c, e, "sampler");

  ReduceArgs ra;
  ra.B = B;
  ra.npx = (int)npx;
  ra.nchunks = nchunks;
  ra.S = S;
  ra.part = (const float *)c->part.p;
  ra.F = (float *)c->F.p;
  ra.dist = pow(10.0, -0.4 * o->dmod);
  ra.dust_model = o->dust_model;
  ra.dust_mu = o->dust_mu;
  ra.dust_sigma = o->dust_sigma;
  for (int b = 0; b < PCMD_MAX_BANDS; ++b) ra.dust_R[b] = b < B ? o->dust_R[b] : 0.0;
  ra.k0 = k0;
  ra.k1 = k1;
  e = launch_reduce(ra, s);
  if (e != hipSuccess) return hip_fail(c, e, "k_reduce");
  if (dbg && dbg->flux_pre) {
    e = launch_copy_f32((const float *)c->F.p, dbg->flux_pre, (int64_t)B * npx, s);
    if (e != hipSuccess) return hip_fail(c, e, "copy flux_pre");
  }
  const float *Gp = (const float *)c->F.p;
  if (K > 1) {
    ConvArgs ca{B, N, K, (const float *)c->F.p, o->psf, (float *)c->G.p, c->status, psf_grid_of(o)};
    if (use_fft) {  // the direct convolution checks the PSF itself
      e = launch_psf_check(ca, s);
      if (e != hipSuccess) return hip_fail(c, e, "psf check");
    }
    ScopedTimer tm(c, PCMD_TIMER_CONV, 2.0 * (double)B * (double)npx, s);
    if (use_fft) {
      const bool fresh = c->fft_buf != c->fft.p || c->fft_B != B || c->fft_N != N || c->fft_K != K || c->fft_R != R;
      e = launch_conv_fft((const float *)c->F.p, o->psf, B, N, K, psf_grid_of(o), (float *)c->G.p, c->fft.p, fresh, s);
      if (e == hipSuccess) {
        c->fft_buf = c->fft.p;
        c->fft_B = B;
        c->fft_N = N;
        c->fft_K = K;
        c->fft_R = R;
      }
    } else
      e = launch_conv_direct(ca, s);
    if (e != hipSuccess) return hip_fail(c, e, "convolution");
    Gp = (const float *)c->G.p;
  }
  if (dbg && dbg->flux_psf) {
    e = launch_copy_f32(Gp, dbg->flux_psf, (int64_t)B * npx, s);
    if (e != hipSuccess) return hip_fail(c, e, "copy flux_psf");
  }
  NoiseArgs na;
  na.B = B;
  na.npx = (int)npx;
  na.G = Gp;
  na.mags = mags;
  na.noise_model = o->noise_model;
  for (int b = 0; b < PCMD_MAX_BANDS; ++b) {
    na.sigma[b] = b < B ? o->noise_sigma_mag[b] : 0.0;
    na.exptime[b] = b < B ? o->exptime[b] : 1.0;
    na.zp[b] = b < B ? o->zp[b] : 0.0;
    na.sky[b] = b < B ? o->sky[b] : 0.0;
  }
  na.k0 = k0;
  na.k1 = k1;
  e = launch_noise_mag(na, s);
  if (e != hipSuccess) return hip_fail(c, e, "k_noise_mag");
  c->err.clear();
  return PCMD_OK;
}

// ------------------------------------------------------------------------------------------
// a5, a6
// ------------------------------------------------------------------------------------------

int pcmd_hess(pcmd_ctx *c, const float *mags, int32_t B, int64_t npx, const pcmd_hess_grid *g, uint32_t *hess,
              double *moments, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (!mags || !g || !hess || !moments) return fail(c, PCMD_E_INVAL, "pcmd_hess: null argument");
  if (B < 1 || B > PCMD_MAX_BANDS) return fail(c, PCMD_E_INVAL, "pcmd_hess: n_bands %d out of range", B);
  if (npx < 1 || npx > (int64_t)1 << 31) return fail(c, PCMD_E_INVAL, "pcmd_hess: n_px out of range");
  if (g->nx < 1 || g->ny < 1 || (int64_t)g->nx * g->ny > 65536)
    return fail(c, PCMD_E_INVAL, "pcmd_hess: grid %d x %d out of range", g->nx, g->ny);
  if (!(g->dx > 0.0) || !(g->dy > 0.0) || !isfinite(g->x0) || !isfinite(g->y0) || !isfinite(g->dx) || !isfinite(g->dy))
    return fail(c, PCMD_E_INVAL, "pcmd_hess: bad grid origin or width");
  if (g->b_blue < 0 || g->b_blue >= B || g->b_red < 0 || g->b_red >= B || g->b_mag < 0 || g->b_mag >= B)
    return fail(c, PCMD_E_INVAL, "pcmd_hess: band index out of range");
  DeviceGuard dg(c->device);
  int r = ensure(c, c->mom_part, (size_t)hess_max_blocks() * 3 * 8, "moment partials");
  if (r) return r;
  HessArgs a;
  a.mags = mags;
  a.npx = npx;
  a.x0 = g->x0;
  a.dx = g->dx;
  a.y0 = g->y0;
  a.dy = g->dy;
  a.nx = g->nx;
  a.ny = g->ny;
  a.bb = g->b_blue;
  a.br = g->b_red;
  a.bm = g->b_mag;
  a.hess = hess;
  a.mom_part = (double *)c->mom_part.p;
  a.counter = c->counter;
  a.moments = moments;
  a.use_lds = hess_use_lds(g->nx * g->ny);
  hipError_t e;
  {
    ScopedTimer tm(c, PCMD_TIMER_HESS, (double)npx, (hipStream_t)stream);
    e = launch_hess(a, (hipStream_t)stream);
  }
  if (e != hipSuccess) return hip_fail(c, e, "k_hess");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_loglike(pcmd_ctx *c, const uint32_t *hm, const uint32_t *hd, int32_t nbins, const double *mom_m,
                 const double *mom_d, int32_t mode, double eps, double *out, pcmd_stream stream) {
  if (!c) return PCMD_E_INVAL;
  if (!hm || !hd || !out) return fail(c, PCMD_E_INVAL, "pcmd_loglike: null argument");
  if (nbins < 1 || nbins > 65536) return fail(c, PCMD_E_INVAL, "pcmd_loglike: n_bins %d out of range", nbins);
  const bool accumulate = (mode & PCMD_LL_ACCUMULATE) != 0;
  mode &= ~PCMD_LL_ACCUMULATE;
  if (mode < 0 || mode > 2) return fail(c, PCMD_E_INVAL, "pcmd_loglike: bad mode %d", mode);
  if (mode == PCMD_LL_POISSON && !(eps > 0.0 && isfinite(eps))) return fail(c, PCMD_E_INVAL, "pcmd_loglike: eps must be > 0");
  if (mode != PCMD_LL_POISSON && (!mom_m || !mom_d)) return fail(c, PCMD_E_INVAL, "pcmd_loglike: moments needed");
  DeviceGuard dg(c->device);
  int r;
  if ((r = ensure(c, c->ll_part, (size_t)loglike_blocks(nbins) * 8, "likelihood partials"))) return r;
  LoglikeArgs a{hm, hd, nbins, mode, mom_m, mom_d, eps, out, (double *)c->ll_part.p, accumulate ? 1 : 0, c->lnfact64};
  hipError_t e = launch_loglike(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(c, e, "k_loglike");
  c->err.clear();
  return PCMD_OK;
}

int pcmd_timer_enable(pcmd_ctx *c, int on) {
  if (!c) return PCMD_E_INVAL;
  DeviceGuard dg(c->device);
  if (on) {
    (void)hipDeviceSynchronize();
    clear_timers(c);
    // events for 512 timed launches between reads, created here rather than inside a timed loop
    while (c->ev_pool.size() < 1024) {
      hipEvent_t e = nullptr;
      if (hipEventCreate(&e) != hipSuccess) return hip_fail(c, hipErrorOutOfMemory, "pcmd_timer_enable: event");
      c->ev_pool.push_back(e);
    }
  }
  c->timing = on != 0;
  return PCMD_OK;
}

int pcmd_timer_read(pcmd_ctx *c, int which, double *total_ms, int64_t *launches, double *units) {
  if (!c) return PCMD_E_INVAL;
  if (which < 0 || which >= PCMD_TIMER_KINDS || !total_ms || !launches || !units)
    return fail(c, PCMD_E_INVAL, "pcmd_timer_read: bad argument");
  DeviceGuard dg(c->device);
  double ms = 0.0, u = 0.0;
  int64_t n = 0;
  std::vector<TimerRec> keep;
  for (auto &t : c->timers) {
    if (t.which != which) {
      keep.push_back(t);
      continue;
    }
    float dt = 0.0f;
    hipError_t e = hipEventSynchronize(t.stop);
    if (e == hipSuccess) e = hipEventElapsedTime(&dt, t.start, t.stop);
    give_event(c, t.start);
    give_event(c, t.stop);
    if (e != hipSuccess) return hip_fail(c, e, "pcmd_timer_read");
    ms += dt;
    u += t.units;
    ++n;
  }
  c->timers.swap(keep);
  *total_ms = ms;
  *launches = n;
  *units = u;
  return PCMD_OK;
}

/* ---- Appendix A: the stochastic likelihood after a nested-sampling fit (host only) ---- */

static bool any_nan(const double *x, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (std::isnan(x[i])) return true;
  return false;
}

int pcmd_lmax_ceiling(const double *logl, int64_t n, double *lmax_out) {
  if (!logl || !lmax_out || n < 1 || any_nan(logl, n)) return PCMD_E_INVAL;
  std::vector<double> v(logl, logl + n);
  const int64_t h = n / 2;
  std::nth_element(v.begin(), v.begin() + h, v.end());
  double med = v[h];
  if (n % 2 == 0) {  // even count: the mean of the two middle values
    const double lo = *std::max_element(v.begin(), v.begin() + h);
    med = (lo + med) / 2.0;
  }
  *lmax_out = med;
  return PCMD_OK;
}

int pcmd_cap_loglikes(const double *logl, int64_t n, double lmax, double *out) {
  if (!logl || !out || n < 0 || std::isnan(lmax) || any_nan(logl, n)) return PCMD_E_INVAL;
  for (int64_t i = 0; i < n; ++i) out[i] = logl[i] > lmax ? lmax : logl[i];
  return PCMD_OK;
}

/* max and log-sum-exp of a_i = logl_i + log_dx_i; false when every a_i is -inf, or one is +inf or
 * undefined (-inf + inf) */
static bool log_mass(const double *logl, const double *log_dx, int64_t n, double *amax, double *lse) {
  double m = -INFINITY;
  for (int64_t i = 0; i < n; ++i) {
    const double a = logl[i] + log_dx[i];
    if (std::isnan(a)) return false;
    m = std::fmax(m, a);
  }
  if (!(m > -INFINITY) || std::isinf(m)) return false;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += std::exp(logl[i] + log_dx[i] - m);
  *amax = m;
  *lse = m + std::log(s);
  return true;
}

int pcmd_nested_weights(const double *logl, const double *log_dx, int64_t n, double *w_out) {
  if (!logl || !log_dx || !w_out || n < 1 || any_nan(logl, n) || any_nan(log_dx, n)) return PCMD_E_INVAL;
  double m, lse;
  if (!log_mass(logl, log_dx, n, &m, &lse)) return PCMD_E_INVAL;
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += (w_out[i] = std::exp(logl[i] + log_dx[i] - m));
  for (int64_t i = 0; i < n; ++i) w_out[i] /= s;
  return PCMD_OK;
}

int pcmd_remaining_evidence(const double *logl, const double *log_dx, int64_t n, double log_x_final,
                            double logl_max_live, double *dlnz_out) {
  if (!logl || !log_dx || !dlnz_out || n < 1 || any_nan(logl, n) || any_nan(log_dx, n) ||
      std::isnan(log_x_final) || std::isnan(logl_max_live))
    return PCMD_E_INVAL;
  double m, lnz;
  if (!log_mass(logl, log_dx, n, &m, &lnz)) return PCMD_E_INVAL;
  const double r = logl_max_live + log_x_final;  // log of the evidence the live points could still add
  const double hi = std::fmax(lnz, r), lo = std::fmin(lnz, r);
  const double both = lo == -INFINITY ? hi : hi + std::log1p(std::exp(lo - hi));
  *dlnz_out = both - lnz;
  return PCMD_OK;
}

int pcmd_effective_sample_size(const double *w, int64_t n, double *ess_out) {
  if (!w || !ess_out || n < 1 || any_nan(w, n)) return PCMD_E_INVAL;
  double s2 = 0.0;
  for (int64_t i = 0; i < n; ++i) s2 += w[i] * w[i];
  if (!(s2 > 0.0)) return PCMD_E_INVAL;
  *ess_out = 1.0 / s2;
  return PCMD_OK;
}

}  // extern "C"
