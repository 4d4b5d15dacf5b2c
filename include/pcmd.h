/*
 * pcmd.h -- C ABI of the MI355X (gfx950) pixel colour-magnitude-diagram forward model.
 *
 * The library evaluates the stochastic forward model of Cook, Conroy, van Dokkum & Speagle,
 * "Measuring Star-Formation Histories, Distances, and Metallicities with Pixel Color-Magnitude
 * Diagrams I" (arXiv:1904.00011): weighted isochrone points -> per-pixel Poisson star counts ->
 * dust, distance and flux sums -> PSF -> sky and noise -> magnitudes -> Hess diagram ->
 * binned likelihood (Sec. 2.1 and 2.5, Fig. 1).
 *
 * Conventions for every call:
 *  - Pointers marked [dev] are device memory on the context's GPU, owned by the caller; the
 *    library never frees or keeps them past the call.  Pointers marked [host] are read during
 *    the call only.
 *  - All device work is queued on `stream` (a hipStream_t; NULL = the null stream) and the call
 *    returns without waiting for it.  Results are valid once the stream has reached them.
 *  - Every scalar, shape and pointer argument is validated before anything is launched; on
 *    failure the call returns a negative PCMD_E_* code, sets the message returned by
 *    pcmd_last_error(), and has no side effect.  A failed HIP launch returns PCMD_E_HIP.
 *    The contents of device arrays are checked by the kernels themselves (so that no call
 *    waits for the device): a bad value is replaced as documented and reported by pcmd_sync().
 *  - The context owns scratch buffers.  They grow on the first call that needs more and are
 *    then reused, so repeated calls with the same shapes allocate nothing.  Calls that share a
 *    context must not run concurrently on different streams.
 *  - Results are a pure function of the inputs and the seed: they do not depend on launch
 *    shapes, batching, or the stream used.
 */
#ifndef PCMD_H
#define PCMD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PCMD_MAX_BANDS 4
#define PCMD_MAX_ISO 512
#define PCMD_MAX_PSF_K 127

enum {
  PCMD_OK = 0,
  PCMD_E_INVAL = -1,        /* an argument failed validation                         */
  PCMD_E_HIP = -2,          /* a HIP runtime call or kernel launch failed            */
  PCMD_E_NOMEM = -3,        /* device scratch could not be allocated                 */
  PCMD_E_UNSUPPORTED = -4,  /* valid request the library does not implement         */
  PCMD_E_PTRS_RETRY = -5    /* a rejection draw used up its attempts (see pcmd_sync) */
};

typedef struct pcmd_ctx pcmd_ctx;
typedef void *pcmd_stream; /* hipStream_t */

/* Create a context bound to HIP device `hip_device`.  *out receives the handle. */
int pcmd_create(pcmd_ctx **out, int hip_device);
/* Free the context and its scratch.  Waits for the device to finish work that uses it. */
void pcmd_destroy(pcmd_ctx *ctx);
/* Message of the last failed call on this context ("" if none).  Valid until the next call. */
const char *pcmd_last_error(const pcmd_ctx *ctx);
/* Wait for `stream`, then report device-side findings of earlier calls and clear them:
 * PCMD_E_INVAL if an expected star count was NaN, negative or >= 2^22 or an isochrone index was
 * out of range (that point was given no stars), or if a PSF band had a negative or non-finite
 * value or did not sum to 1 within 1e-3 (the image is still convolved with it);
 * PCMD_E_PTRS_RETRY if a transformed-rejection draw exhausted its 64 attempts (probability
 * below 1e-60 per draw; that draw's count is 0). */
int pcmd_sync(pcmd_ctx *ctx, pcmd_stream stream);
/* Name of the library build, e.g. "pcmd gfx950 ...". */
const char *pcmd_version(void);

/* ---------------------------------------------------------------------------------------
 * a0: weighted isochrone entries (Sec. 2.1: age x [Fe/H] x mass points weighted by the SFH,
 * the metallicity distribution and the IMF, normalised to Npix; Sec. 2.2 and Table 1: the
 * model menu).
 * ------------------------------------------------------------------------------------- */

enum { PCMD_SFH_SSP = 0, PCMD_SFH_CONST = 1, PCMD_SFH_TAU = 2, PCMD_SFH_DTAU = 3, PCMD_SFH_NONPARAM = 4 };
enum { PCMD_MDF_SINGLE = 0, PCMD_MDF_GAUSS = 1 };

/* Shape of an isochrone set: isochrone k stands for age bin iso_age[k] (edges age_edges, log10
 * yr) and [Fe/H] grid point iso_feh[k].  All pointers [host]. */
typedef struct {
  int32_t n_iso, n_age, n_feh;
  const double *age_edges; /* [n_age + 1] log10 yr, increasing          */
  const double *feh_grid;  /* [n_feh]                                   */
  const int32_t *iso_age;  /* [n_iso] in [0, n_age)                     */
  const int32_t *iso_feh;  /* [n_iso] in [0, n_feh)                     */
} pcmd_isoset;

/* Physical model of one evaluation (Table 1).  S1 SSP uses ssp_age_index; S2 constant SFR;
 * S3 tau model SFR ~ exp(-t/tau); S4 delayed tau SFR ~ t exp(-t/tau) (t = time since onset at
 * 10^10.2 yr); S5 non-parametric with log_sfh[a] = log10 stars per pixel formed in age bin a
 * (Npix = their sum).  M1 single [Fe/H] grid point feh_index; M2/M3 Gaussian weights at the
 * grid points, weights under mdf_prune dropped and the rest renormalised. */
typedef struct {
  int32_t sfh, mdf;
  int32_t ssp_age_index, feh_index;
  double log_npix, tau_gyr;
  double feh_mu, feh_sigma, mdf_prune;
  const double *log_sfh; /* [host][n_age], S5 only */
} pcmd_model;

/* IMF forms (Sec. 2.2): a single power law m^-alpha (Salpeter, alpha = 2.35, the default) or
 * the Kroupa (2001) broken power law, slopes 0.3 / 1.3 / 2.3 with breaks at 0.08 and 0.5 Msun,
 * continuous at the breaks (alpha ignored). */
enum { PCMD_IMF_POWER_LAW = 0, PCMD_IMF_KROUPA = 1 };

/* Host helper: IMF weight of every point (the IMF integrated over the point's mass bin, edges at
 * geometric midpoints, outer edges half a log-step out; Sec. 2.2, Table 2), the star flux
 * 10^(-0.4 M) per band and, if iso_imf_sum_out is not NULL, the IMF weight summed over the points
 * of each of the n_iso isochrones (the per-isochrone normalisation that pcmd_entries needs; every
 * iso_of_entry must then lie in [0, n_iso)).  Points of one isochrone must be contiguous with
 * increasing mass.  mass [host][E]; absmag [host][B][E]; imf_w_out [host][E]; flux_out
 * [host][B][E] (FP32); iso_imf_sum_out [host][n_iso] or NULL. */
int pcmd_grid_prepare(int32_t n_entries, int32_t n_bands, const int32_t *iso_of_entry,
                      const double *mass, const double *absmag, int32_t imf, double alpha,
                      double *imf_w_out, float *flux_out, int32_t n_iso, double *iso_imf_sum_out);

/* Host helper: per-isochrone SFH x MDF weight and Npix for `model` (Sec. 2.2). w_out [host][n_iso]. */
int pcmd_iso_weights(const pcmd_model *model, const pcmd_isoset *set, double *w_out, double *npix_out);

/* ---- Stochastic likelihood after a nested-sampling fit (App. A), host only, no context ----
 * A simulated diagram is one random realisation, so a point's log-likelihood scatters from call to
 * call with a long upper tail.  App. A re-simulates the best-fit point many times, takes the median
 * as a ceiling L_max, caps every dead point's log-likelihood at L_max and recomputes the posterior
 * weights and the remaining-evidence stopping criterion.  All arrays are host FP64 owned by the
 * caller; NaN inputs, empty arrays, masses logl_i + log_dx_i that are all -inf or include +inf or
 * -inf + inf return PCMD_E_INVAL with no output written (these calls take no context, so pcmd_last_error is not set).
 *
 * pcmd_lmax_ceiling: median of logl[n] (mean of the two middle values for even n).
 * pcmd_cap_loglikes: out[i] = min(logl[i], lmax); out may alias logl; n = 0 allowed.
 * pcmd_nested_weights: w_out[i] = L_i dX_i / sum_j L_j dX_j from logl[n] and log_dx[n] (the log
 *   prior-volume width of each dead point), computed with the largest term factored out.
 * pcmd_remaining_evidence: ln(Z + L_max,live X_final) - ln Z with Z = sum_i L_i dX_i.
 * pcmd_effective_sample_size: Kish's 1 / sum w_i^2 of normalised weights w[n]. */
int pcmd_lmax_ceiling(const double *logl, int64_t n, double *lmax_out);
int pcmd_cap_loglikes(const double *logl, int64_t n, double lmax, double *out);
int pcmd_nested_weights(const double *logl, const double *log_dx, int64_t n, double *w_out);
int pcmd_remaining_evidence(const double *logl, const double *log_dx, int64_t n, double log_x_final,
                            double logl_max_live, double *dlnz_out);
int pcmd_effective_sample_size(const double *w, int64_t n, double *ess_out);

/* Device grid: per-point isochrone index and IMF weight, uploaded once per fit. */
typedef struct {
  int32_t n_entries, n_iso;
  const int32_t *iso_of_entry; /* [dev][E] */
  const double *imf_w;         /* [dev][E] */
  const double *iso_imf_sum;   /* [host][n_iso] sum of imf_w over each isochrone's points */
} pcmd_grid;

/* lambda_i = Npix * w_iso(i) * imf_w_i / sum_k w_k S_k  (expected stars per pixel; sum = Npix).
 * iso_w [host][n_iso] from pcmd_iso_weights; lam_out [dev][E] FP64. */
int pcmd_entries(pcmd_ctx *ctx, const pcmd_grid *grid, const double *iso_w, double npix,
                 double *lam_out, pcmd_stream stream);

/* ---------------------------------------------------------------------------------------
 * a1-a4: one simulated image (Sec. 2.1; dust models Sec. 2.2; noise Sec. 2.1 and Table 2).
 * ------------------------------------------------------------------------------------- */

/* Weighted points: lam [dev][E] expected stars per pixel (finite, 0 <= lam < 2^22);
 * flux [dev][B][E] star flux 10^(-0.4 M_abs) (FP32, finite, >= 0). */
typedef struct {
  int32_t n_entries, n_bands;
  const double *lam;
  const float *flux;
} pcmd_iso;

enum { PCMD_DUST_NONE = 0, PCMD_DUST_SCREEN = 1, PCMD_DUST_LOGNORMAL = 2 };
enum { PCMD_CONV_AUTO = 0, PCMD_CONV_DIRECT = 1, PCMD_CONV_FFT = 2 };
enum { PCMD_NOISE_NONE = 0, PCMD_NOISE_GAUSS_MAG = 1, PCMD_NOISE_SHOT = 2 };
enum { PCMD_SAMPLER_POINT = 0, PCMD_SAMPLER_BLOCK = 1, PCMD_SAMPLER_HYBRID = 2 };

/* Observation and nuisance model of one simulation.
 *  nim            image side (pixels = nim*nim), 1..8192
 *  seed           64-bit key of every random draw
 *  dmod           distance modulus mu_d; every flux is scaled by 10^(-0.4 mu_d)
 *  dust_model     NONE, SCREEN (E1: log10 E(B-V) = dust_mu everywhere) or LOGNORMAL
 *                 (E2/E3: log10 E(B-V) ~ N(dust_mu, dust_sigma) per pixel)
 *  dust_frac      F_dust in [0, 1]: each star is behind the screen with this probability
 *  dust_R[b]      A_b / E(B-V)
 *  psf_k, psf     odd K <= nim and <= PCMD_MAX_PSF_K; psf [dev][B][K][K] FP32, each band sums to 1
 *                 (checked to 1e-3); the convolution is periodic.  psf_k = 1 with psf NULL = no PSF
 *  psf_grid       0 or 1: one PSF per band.  4: the image is split into a 4 x 4 grid of regions,
 *                 region (ry, rx) = (floor(4 y / nim), floor(4 x / nim)), and the pixels of region
 *                 r = 4 ry + rx take the PSF psf[b][r] (psf is [dev][B][16][K][K]): the paper's
 *                 sub-pixel model, each region with a PSF shifted by a fraction of a pixel
 *                 (Sec. 2.2).  AUTO takes the direct path for the grid; the FFT path computes it
 *                 too (one forward transform, an inverse per region: several times the cost)
 *  conv_path      AUTO (direct below K = 48, FFT from 48 on where supported), DIRECT or FFT (FFT
 *                 needs nim a power of two, 8..4096; the context keeps the PSF spectra and
 *                 rebuilds them on the device whenever the PSF's contents change)
 *  noise_model    NONE, GAUSS_MAG (m += sigma_b z) or SHOT (c = G t_b 10^(0.4 zp_b) + sky_b,
 *                 c' = c + sqrt(c) z, m = -2.5 log10((c' - sky_b)/t_b) + zp_b; +inf if <= 0)
 *  sampler        POINT (0): one Poisson count per (pixel, point), the paper's rule (Sec. 2.1).
 *                 BLOCK (1): the same law by Poisson superposition (Sec. 2.1 footnote): per
 *                 pixel and block of 64 consecutive points one Poisson total, then each star's
 *                 point by its cumulative share of the block's lambda (to 2^-32) and its dust
 *                 screen by one uniform per star.  A different random stream; cheaper where most
 *                 blocks draw no star (low Npix).  Each block's lambda sum must be < 2^22
 *                 (else PCMD_E_INVAL at pcmd_sync, the block drawn as 0).
 *                 HYBRID (2): blocks whose lambda sum is below 10 by the BLOCK rule, the other
 *                 blocks' points by the POINT rule (the cheaper rule on each side; any block sum
 *                 allowed).  Batches take all three, job by job */
typedef struct {
  int32_t nim;
  int32_t dust_model;
  uint64_t seed;
  double dmod;
  double dust_mu, dust_sigma, dust_frac;
  double dust_R[PCMD_MAX_BANDS];
  int32_t psf_k, conv_path;
  const float *psf;
  int32_t noise_model, psf_grid;
  double noise_sigma_mag[PCMD_MAX_BANDS];
  double exptime[PCMD_MAX_BANDS];
  double zp[PCMD_MAX_BANDS];
  double sky[PCMD_MAX_BANDS];
  int32_t sampler, pad_;
} pcmd_obs;

/* Optional debug outputs (any pointer may be NULL):
 *  counts   [dev][px1 - px0][E] u32 star count of each pixel in [px0, px1) and point
 *  reddened [dev][px1 - px0][E] u32 how many of them sit behind the dust screen
 *  flux_pre [dev][B][nim*nim] FP32 pixel flux after dust and distance, before the PSF
 *  flux_psf [dev][B][nim*nim] FP32 pixel flux after the PSF */
typedef struct {
  uint32_t *counts;
  uint32_t *reddened;
  int64_t px0, px1;
  float *flux_pre;
  float *flux_psf;
} pcmd_debug;

/* Simulate one image: mags_out [dev][B][nim*nim] FP32 apparent magnitudes (+inf where the
 * flux or noisy count is not positive).  dbg may be NULL. */
int pcmd_simulate(pcmd_ctx *ctx, const pcmd_iso *iso, const pcmd_obs *obs, float *mags_out,
                  const pcmd_debug *dbg, pcmd_stream stream);

/* ---------------------------------------------------------------------------------------
 * a5: Hess diagram (Sec. 2.1, 2.5; 0.05 mag bins, Table 2).
 * ------------------------------------------------------------------------------------- */

/* x = m[b_blue] - m[b_red], y = m[b_mag] (computed in FP64 from the FP32 magnitudes);
 * ix = clamp(floor((x - x0)/dx), 0, nx-1) with NaN -> 0, likewise iy; H[iy][ix] += 1, so the
 * Hess total equals the pixel count.  Requires nx, ny >= 1, nx*ny <= 65536, dx, dy > 0. */
typedef struct {
  double x0, dx, y0, dy;
  int32_t nx, ny;
  int32_t b_blue, b_red, b_mag, pad_;
} pcmd_hess_grid;

/* mags [dev][n_bands][n_px] -> hess [dev][ny][nx] u32 (overwritten) and
 * moments [dev][3] FP64 = (sum x, sum y, count) over pixels whose three magnitudes are finite. */
int pcmd_hess(pcmd_ctx *ctx, const float *mags, int32_t n_bands, int64_t n_px,
              const pcmd_hess_grid *grid, uint32_t *hess, double *moments, pcmd_stream stream);

/* ---------------------------------------------------------------------------------------
 * a6: binned log-likelihood (Sec. 2.5).
 * ------------------------------------------------------------------------------------- */

enum { PCMD_LL_POISSON = 0, PCMD_LL_GAUSS_PAPER = 1, PCMD_LL_GAUSS_LITERAL = 2 };
/* OR-ed into mode: add the result to *out instead of storing it.  Summing the calls of several
 * colour-magnitude diagrams of one image (e.g. (b0 - b1, b1) and (b1 - b2, b2) for three bands)
 * gives their joint log-likelihood, the extension of the paper's two-band pCMD (Sec. 2.1). */
enum { PCMD_LL_ACCUMULATE = 0x100 };

/* POISSON: lam_j = N_d (m_j + eps) / (N_m + eps n_bins), logL = sum d_j ln lam_j - lam_j - ln d_j!
 * GAUSS_PAPER: mh_j = m_j N_d / N_m, sigma_j = max(sqrt(d_j + mh_j), 2),
 *   logL = -sum (d_j - mh_j)^2 / (2 sigma_j^2) + C
 * GAUSS_LITERAL: the printed form -sum (d_j/N_d - m_j/N_m)^2 / (2 sigma_j^2) + C with
 *   sigma_j = max(sqrt(d_j^2 + m_j^2), 2)
 * C = -(C_d - C_m)^2 / (2 0.05^2) - (M_d - M_m)^2 / (2 0.05^2) from the moments (mean colour and
 * magnitude).  hess_* [dev][n_bins] u32; mom_* [dev][3]; out [dev][1] FP64.  eps > 0 (POISSON). */
int pcmd_loglike(pcmd_ctx *ctx, const uint32_t *hess_model, const uint32_t *hess_data, int32_t n_bins,
                 const double *mom_model, const double *mom_data, int32_t mode, double eps,
                 double *out, pcmd_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): pcmd_loglike with its block sums in a static device
 * array of 256 doubles (2 KiB per GPU, held until the process ends) instead of the context's
 * scratch.  Same arguments, kernels and results as pcmd_loglike; n_bins at most 65536 (larger:
 * PCMD_E_INVAL with a message, nothing launched).  It calls no allocating routine.  Every call on
 * one GPU shares that array, so calls that overlap on one GPU (different streams, or contexts
 * used from several threads) race; calls ordered on one stream do not. */
int pcmd_loglike_noalloc(pcmd_ctx *ctx, const uint32_t *hess_model, const uint32_t *hess_data, int32_t n_bins,
                         const double *mom_model, const double *mom_data, int32_t mode, double eps, double *out,
                         pcmd_stream stream);

/* ---------------------------------------------------------------------------------------
 * a7: many parameter points in one launch (the paper's fits evaluate the stochastic likelihood
 * at many points and re-simulate the best fit 100 times, Sec. 2.5 and Appendix A).
 * ------------------------------------------------------------------------------------- */

/* One job: the weighted points and observation of one simulation. */
typedef struct {
  pcmd_iso iso;
  pcmd_obs obs;
} pcmd_job;

/* Simulate, bin and score n_jobs independent simulations, each bit-identical to pcmd_simulate +
 * pcmd_hess + pcmd_loglike on the same inputs.  The per-point sampler runs as one persistent
 * launch whose (job, 64-pixel block, entry chunk) tiles are drawn from a shared counter, so jobs of
 * uneven image size and entry count load-balance; a job with the block-skip or hybrid sampler
 * draws its block-rule stars in a launch of its own after it; the other steps run per job.  All jobs share n_bands;
 * a job's convolution must resolve to the direct path (PCMD_E_UNSUPPORTED otherwise).
 * use_graph != 0: the first call with a given shape signature (n_jobs, each job's nim, n_entries,
 * psf_k, sampler, PSF grid and how dust splits its stars: none, F = 1/2, F = 1 or another F, the
 * Hess size, the tuning) captures the launch
 * sequence into a HIP graph; later calls with that signature replay it with this call's
 * parameters, seeds and input pointers.  Scratch for all jobs stays allocated in the context.
 * jobs [host][n_jobs]; hess_data [dev][nx*ny]; mom_data [dev][3] (Gaussian modes);
 * logl_out [dev][n_jobs]; hess_out [dev][n_jobs][nx*ny] or NULL. */
int pcmd_batch_run(pcmd_ctx *ctx, int32_t n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *grid,
                   const uint32_t *hess_data, const double *mom_data, int32_t mode, double eps,
                   double *logl_out, uint32_t *hess_out, int32_t use_graph, pcmd_stream stream);

/* Schedule of the persistent sampler: workgroups per compute unit (1..8) and tile order (0: the
 * most expensive job first, 1: submission order).  It changes speed only, never results. */
typedef struct {
  int32_t wg_per_cu;
  int32_t order;
} pcmd_batch_tuning;

int pcmd_batch_set_tuning(pcmd_ctx *ctx, const pcmd_batch_tuning *tuning);
int pcmd_batch_get_tuning(pcmd_ctx *ctx, pcmd_batch_tuning *tuning);
/* Run the batch once per candidate schedule (eagerly, timed with HIP events), keep the fastest
 * as the context's schedule and return it; ms_out [host][8] (or NULL) receives each candidate's
 * time and *n_candidates their number.  Waits for the stream. */
int pcmd_batch_autotune(pcmd_ctx *ctx, int32_t n_jobs, const pcmd_job *jobs, const pcmd_hess_grid *grid,
                        const uint32_t *hess_data, const double *mom_data, int32_t mode, double eps,
                        double *logl_out, pcmd_batch_tuning *best, double *ms_out, int32_t *n_candidates,
                        pcmd_stream stream);

/* ---------------------------------------------------------------------------------------
 * a8: surrogate network of the log-Hess diagram, used to screen sampler proposals before the
 * simulator judges them.  A multilayer perceptron with GELU hidden layers whose matrix products
 * run on BF16 MFMA with FP32 accumulation:
 *   x_0 = bf16(theta); z_l = x_l W_l^T + b_l; x_{l+1} = bf16(GELU(z_l)); y = z_last.
 * Training minimises the mean squared error to log-Hess targets with Adam (beta1 0.9, beta2
 * 0.999, eps 1e-8) on FP32 master weights; BF16 copies of W and W^T feed the products.
 * ------------------------------------------------------------------------------------- */

#define PCMD_MLP_MAX_LAYERS 8

/* A network.  Parameters are packed per layer: W_l [dims[l+1]][dims[l]] then b_l [dims[l+1]]
 * (FP32).  w_bf16 / wt_bf16 hold, per layer and packed the same way without biases, W_l and
 * W_l^T ([dims[l]][dims[l+1]]) in BF16.  All pointers [dev], caller-owned. */
typedef struct {
  int32_t n_layers;
  int32_t dims[PCMD_MLP_MAX_LAYERS + 1];
  float *master;
  float *adam_m, *adam_v;
  uint16_t *w_bf16;
  uint16_t *wt_bf16;
} pcmd_mlp;

/* Number of FP32 parameters (weights and biases) and of weights. */
int64_t pcmd_mlp_param_count(const int32_t *dims, int32_t n_layers);
int64_t pcmd_mlp_weight_count(const int32_t *dims, int32_t n_layers);
/* Refresh the BF16 weight copies from the master weights (after initialisation or loading). */
int pcmd_mlp_refresh(pcmd_ctx *ctx, const pcmd_mlp *net, pcmd_stream stream);
/* Inference: x [dev][n][dims[0]] FP32 -> y [dev][n][dims[n_layers]] FP32. */
int pcmd_mlp_forward(pcmd_ctx *ctx, const pcmd_mlp *net, int32_t n, const float *x, float *y, pcmd_stream stream);
/* Forward, loss = mean((y - t)^2) over the batch and its outputs, and backward of one batch of n
 * samples: grad_out [dev][param_count] receives the packed FP32 gradient of the loss;
 * loss_out [dev][1] or NULL.  rows [dev][n] int32 or NULL: sample k of the batch is row rows[k] of
 * x [n_total][dims[0]] and of t [n_total][dims[n_layers]] (the gather runs inside the input
 * conversion and the loss kernel; a row outside [0, n_total) is read as row 0 and reported by
 * pcmd_sync as PCMD_E_INVAL); NULL: rows 0 .. n-1 (n_total ignored). */
int pcmd_mlp_backward(pcmd_ctx *ctx, const pcmd_mlp *net, int32_t n, const float *x, const float *t,
                      const int32_t *rows, int64_t n_total, float *loss_out, float *grad_out, pcmd_stream stream);
/* One Adam step number `step` (>= 1) with learning rate lr on the master weights from the packed
 * gradient grad [dev][param_count], then the BF16 copies refreshed. */
int pcmd_mlp_adam(pcmd_ctx *ctx, const pcmd_mlp *net, const float *grad, float lr, int32_t step, pcmd_stream stream);
/* pcmd_mlp_backward on rows 0 .. n-1 followed (if apply_update) by pcmd_mlp_adam.  grad_out
 * [dev][param_count] or NULL (the context then keeps the gradient). */
int pcmd_mlp_train_step(pcmd_ctx *ctx, const pcmd_mlp *net, int32_t n, const float *x, const float *t, float lr,
                        int32_t step, float *loss_out, float *grad_out, int32_t apply_update, pcmd_stream stream);
/* Mean squared error of the network over a whole set of n samples (rows as in pcmd_mlp_backward),
 * forward passes of at most 1024 samples, squared errors summed in FP64: mse_out [dev][1] FP64. */
int pcmd_mlp_loss(pcmd_ctx *ctx, const pcmd_mlp *net, int32_t n, const float *x, const float *t, const int32_t *rows,
                  int64_t n_total, double *mse_out, pcmd_stream stream);
/* Training targets of the surrogate from simulated Hess diagrams: for each of n rows of n_bins
 * counts, out[r][j] = ln((H[r][j] + 1/2) / (N_r + n_bins / 2)) with N_r the row total (computed in
 * FP64, stored FP32).  hess [dev][n][n_bins] u32; out [dev][n][n_bins] FP32. */
int pcmd_log_hess_target(pcmd_ctx *ctx, const uint32_t *hess, int32_t n, int32_t n_bins, float *out,
                         pcmd_stream stream);
/* Surrogate Poisson log-likelihood of a data Hess under predicted log-Hess diagrams:
 * lam_j = N_d exp(y_j) / sum_k exp(y_k), logL = sum_j d_j ln lam_j - lam_j - ln d_j!.
 * y [dev][n][nbins] FP32; hess_data [dev][nbins]; out [dev][n] FP64. */
int pcmd_surrogate_loglike(pcmd_ctx *ctx, const float *y, int32_t n, int32_t nbins, const uint32_t *hess_data,
                           double *out, pcmd_stream stream);
/* General BF16 product for callers that build their own layers: C[M][N] = sum_k A(m,k) B(n,k),
 * A(m,k) = a_trans ? A[k*lda + m] : A[m*lda + k], B(n,k) = b_trans ? B[k*ldb + n] : B[n*ldb + k],
 * FP32 C with leading dimension ldc.  Supported (a_trans, b_trans): any. */
int pcmd_gemm_bf16(pcmd_ctx *ctx, int32_t M, int32_t N, int32_t K, const uint16_t *A, int32_t lda, int32_t a_trans,
                   const uint16_t *B, int32_t ldb, int32_t b_trans, float *C, int32_t ldc, pcmd_stream stream);

/* ---------------------------------------------------------------------------------------
 * Kernel timing for benchmarks: HIP events recorded on the launch stream around each
 * launch of the timed kernels while enabled.
 * ------------------------------------------------------------------------------------- */

enum { PCMD_TIMER_SAMPLE = 0, PCMD_TIMER_CONV = 1, PCMD_TIMER_HESS = 2, PCMD_TIMER_BATCH = 3, PCMD_TIMER_GEMM = 4,
       PCMD_TIMER_KINDS = 5 };

/* Start (on != 0) or stop recording.  Starting discards earlier records. */
int pcmd_timer_enable(pcmd_ctx *ctx, int on);
/* Wait for the recorded launches of kernel `which` and return their summed duration (ms),
 * their number and the algorithmic units they processed (SAMPLE: pixel x entry draws;
 * CONV: image values read and written; HESS: pixels binned; BATCH: a whole pcmd_batch_run,
 * pixel x entry draws of all its jobs; GEMM: each BF16 matrix product of the surrogate,
 * 2 M N K floating-point operations).  Consumes those records. */
int pcmd_timer_read(pcmd_ctx *ctx, int which, double *total_ms, int64_t *launches, double *units);

#ifdef __cplusplus
}
#endif

#endif /* PCMD_H */
