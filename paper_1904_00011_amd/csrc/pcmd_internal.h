// Internal launch interface between the C ABI layer and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pcmd.h"

namespace pcmd {

// One entry's sampler record (16 bytes, read with scalar loads): the first three inversion
// thresholds inline (the rest in the threshold table) and K << 8 | kind.
struct EntryRec {
  uint32_t T[3];  // T_0..T_2 (valid below K)
  uint32_t kk;    // (number of thresholds K) << 8 | kind (KIND_ZERO, KIND_INV, KIND_PTRS)
};

// Device-side tables built from lambda and the star fluxes for one simulation.
struct EntryTables {
  int E = 0, B = 0, BP = 0;
  EntryRec *rec = nullptr;   // [E]
  uint32_t *thr = nullptr;   // [E][THR_STRIDE]
  void *pc = nullptr;        // [E] PtrsConst
  double *fl64 = nullptr;    // [E][BP]
};

// Device status bits, reported by pcmd_sync.
constexpr uint32_t STATUS_PTRS_RETRY = 1u, STATUS_BAD_LAMBDA = 2u, STATUS_BAD_PSF = 4u;

enum SplitMode { SPLIT_NONE = 0, SPLIT_HALF = 1, SPLIT_GENERAL = 2, SPLIT_ALL = 3 };

struct SampleArgs {
  int E, B, BP, npx, nchunks, S;
  uint32_t k0, k1;
  int split_mode;
  uint32_t split_q;
  double *part;  // [nchunks][S][B][npx]
  uint32_t *dbg_counts, *dbg_red;
  int64_t px0, px1;
  uint32_t *status;
  const float *lnfact;
};

struct ReduceArgs {
  int B, npx, nchunks, S;
  const double *part;
  float *F;  // [B][npx]
  double dist;
  int dust_model;
  double dust_mu, dust_sigma;
  double dust_R[PCMD_MAX_BANDS];
  uint32_t k0, k1;
};

struct NoiseArgs {
  int B, npx;
  const float *G;  // [B][npx]
  float *mags;     // [B][npx]
  int noise_model;
  double sigma[PCMD_MAX_BANDS], exptime[PCMD_MAX_BANDS], zp[PCMD_MAX_BANDS], sky[PCMD_MAX_BANDS];
  uint32_t k0, k1;
};

// k_sample.hip
hipError_t launch_entries(const pcmd_grid *g, const double *scale, double *lam, uint32_t *status, hipStream_t s);
hipError_t launch_prep(const double *lam, const float *flux, EntryTables &t, uint32_t *status, hipStream_t s);
hipError_t launch_sample(const EntryTables &t, const SampleArgs &a, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs &a, hipStream_t s);

// k_image.hip
hipError_t launch_psf64(const float *psf, int B, int K, double *psf64, uint32_t *status, hipStream_t s);
size_t conv_direct_lds_bytes(int K);
hipError_t launch_conv_direct(const float *F, const float *psf, int B, int N, int K, float *G, hipStream_t s);
hipError_t launch_noise_mag(const NoiseArgs &a, hipStream_t s);
hipError_t launch_copy_f32(const float *src, float *dst, int64_t n, hipStream_t s);
int fft_supported(int N);
size_t fft_scratch_bytes(int B, int N);
hipError_t launch_conv_fft(const float *F, const float *psf, int B, int N, int K, float *G, void *scratch,
                           hipStream_t s);

// k_hess.hip
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_hess(const float *mags, int B, int64_t npx, const pcmd_hess_grid &g, uint32_t *hess,
                       double *moments, double *mom_part, uint32_t *counter, hipStream_t s);
hipError_t launch_loglike(const uint32_t *hm, const uint32_t *hd, int nbins, const double *mom_m,
                          const double *mom_d, int mode, double eps, double *out, hipStream_t s);
int hess_max_blocks();

}  // namespace pcmd
