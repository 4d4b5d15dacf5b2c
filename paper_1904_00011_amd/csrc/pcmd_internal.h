// Internal launch interface between the C ABI layer and the gfx950 kernels.
//
// Every kernel's arguments form one plain struct.  A single simulation passes it by value; the
// batched path keeps one struct per job in a device table and launches the `_job` variant with
// (table, job index), so that a captured graph can be replayed with new parameters by
// rewriting the table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pcmd.h"

namespace pcmd {

// One entry's sampler record (48 bytes, read with scalar loads): the first three inversion
// thresholds inline (the first as T_0 - 1; the rest in the threshold table), K << 8 | kind, and the entry's star flux
// in each band (FP64; bands past B are zero).  The fluxes sit in the record so that the
// sampler reads them from the record address it already holds.
struct EntryHead {
  uint32_t T[3];  // T_0 - 1, T_1, T_2 (valid below K); T[0] = 0xFFFFFFFF unless drawn by inversion
  uint32_t kk;    // (number of thresholds K, or k_lo of an alias entry) << 8 | kind
};
struct EntryRec {
  uint32_t T[3];
  uint32_t kk;
  double fl[4];
};
static_assert(sizeof(EntryRec) == 48 && sizeof(EntryHead) == 16, "record layout");

// Summary of eight consecutive entries (64 bytes, scalar loads), enough to finish a group in
// which no pixel of the wave draws a star: T_0 - 1 of each entry drawn by inversion
// (0xFFFFFFFF otherwise, so u > t0m1 never holds) and the kinds present.  For inversion
// entries T_0 >= 1 (lambda < ALIAS_MIN), so u >= T_0 is exactly u > T_0 - 1.
constexpr int GRP = 8;  // entries per group record (two Philox blocks)
struct GroupRec {
  uint32_t t0m1[GRP];
  uint32_t flags;  // GRP_INV | GRP_PTRS | GRP_ALIAS (entries drawn whole) | GRP_THIN (thinned entries)
  uint32_t pad[7];
};
constexpr uint32_t GRP_INV = 1u, GRP_PTRS = 2u, GRP_ALIAS = 4u, GRP_THIN = 8u;
// The group's inversion entries are dense enough (64 sum lambda >= GRP_DENSE_LAMBDA64) that a
// 64-pixel wave almost surely draws a star from one of them: the sampler skips its no-star test.
constexpr uint32_t GRP_DENSE = 16u;
constexpr double GRP_DENSE_LAMBDA64 = 3.0;
// Sampler passes: every entry (thinned ones inline); every entry but the thinned ones; only the
// thinned ones, added to the partial sums the main pass stored.
enum SamplePass { PASS_ALL = 0, PASS_MAIN = 1, PASS_THIN = 2 };

// The record table holds E rounded up to a multiple of GRP entry records (the padding records
// have KIND_ZERO), then one group record per GRP entries and one spare group record (not read
// by the sampler, which finds its groups by index bounds; it keeps any read one group past the
// table inside the allocation).
__host__ __device__ inline int entries_padded(int E) { return (E + GRP - 1) / GRP * GRP; }
inline size_t rec_bytes(int E) {
  return (size_t)entries_padded(E) * sizeof(EntryRec) + (size_t)(entries_padded(E) / GRP + 1) * sizeof(GroupRec);
}

// Device status bits, reported by pcmd_sync.
constexpr uint32_t STATUS_PTRS_RETRY = 1u, STATUS_BAD_LAMBDA = 2u, STATUS_BAD_PSF = 4u, STATUS_BAD_ROW = 8u;

enum SplitMode { SPLIT_NONE = 0, SPLIT_HALF = 1, SPLIT_GENERAL = 2, SPLIT_ALL = 3 };
// Thinned table entries: none; every entry at lambda >= ALIAS_MIN (0 < F < 1, F != 1/2); the
// entries at lambda >= LAM_THIN_HALF (F = 1/2).
enum ThinMode { THIN_NONE = 0, THIN_TABLE = 1, THIN_HALF_HIGH = 2 };
__host__ __device__ inline int thin_mode_of_split(int split_mode) {
  return split_mode == SPLIT_GENERAL ? THIN_TABLE : split_mode == SPLIT_HALF ? THIN_HALF_HIGH : THIN_NONE;
}

struct BlockRec;  // block-skip sampler record, below

// Per-entry tables built from lambda and the star fluxes (k_prep).
struct PrepArgs {
  int E, B, BP;
  const double *lam;   // [E]
  const float *flux;   // [B][E]
  EntryRec *rec;       // [entries_padded(E)]
  GroupRec *grp;       // [entries_padded(E) / GRP + 1]
  uint32_t *thr;       // [THR_STRIDE][EP]: threshold k of entry i at k EP + i (EP = E padded to GRP)
  void *pc;            // [E][2] PtrsConst: the entry (or its unreddened part), its reddened part
  double *fl64;        // [E][BP] (block-skip sampler only; the point sampler's fluxes are in rec)
  uint32_t *status;
  uint32_t *alias;     // [E][2][ALIAS_COLS] packed alias columns of the same two parts
  const BlockRec *brec;  // hybrid sampler: entries of blocks without pad[0] set are drawn as 0
  int thin;            // THIN_* : which table entries draw two thinned parts
  double frac;         // F
  uint32_t *rdesc;     // [E] reddened part: k_lo << 12 | log2 M << 8 | KIND_ALIAS, or KIND_PTRS
  uint32_t *thin_seen;  // set to gen when an entry is thinned (null: not recorded)
  uint32_t gen;
  // k_prep appends the alias parts (i << 1 | part) to alias_list, counting them in
  // alias_n[gen & 1] = gen << 32 | count (set to gen << 32 by the previous call's k_prep_alias);
  // k_prep_alias walks that list when it is valid and short, else every entry.  Null: no list.
  uint32_t *alias_list;          // [2E]
  unsigned long long *alias_n;   // [2]
};

// Sampler over (pixel block of 256, chunk of CHUNK entries) tiles (k_sample).
struct SampleArgs {
  int E, B, BP, npx, nchunks, S;
  uint32_t k0, k1;
  int split_mode;
  uint32_t split_q;
  const EntryRec *rec;
  const GroupRec *grp;
  const uint32_t *thr;  // [THR_STRIDE][EP], k-major as in PrepArgs
  const void *pc;
  float *part;  // [nchunks][S][B][npx] slice partial sums (FP64 in registers, stored FP32)
  uint32_t *dbg_counts, *dbg_red;
  int64_t px0, px1;
  uint32_t *status;
  const float *lnfact;
  const uint32_t *alias;  // [E][2][ALIAS_COLS]
  const uint32_t *rdesc;  // [E]
  // the thinned-entry pass returns at once unless *thin_seen == gen, i.e. k_prep of this call
  // thinned an entry (null: always runs)
  const uint32_t *thin_seen;
  uint32_t gen;
};

// Block-skip sampler (Poisson superposition, Sec. 2.1 footnote): per pixel and per block of
// SBLK consecutive entries, the block's star total and then each star's entry.
constexpr int SBLK = 64;  // entries per block = lanes of a wave
inline int superblocks(int E) { return (E + SBLK - 1) / SBLK; }
// One block's record (32 bytes, scalar loads): the total's rule as in EntryRec, and istar, the
// first entry of the block whose cumulative threshold is 2^32 (the last entry with stars).
// pad[0] = 1 marks a block the hybrid sampler leaves to the per-point rule.
struct BlockRec {
  uint32_t T[3];
  uint32_t kk;
  uint32_t istar;
  uint32_t pad[3];
};
struct BlockPrepArgs {
  int E, B, BP, nb;
  const double *lam;   // [E]
  const float *flux;   // [B][E]
  BlockRec *brec;      // [nb]
  uint32_t *thr;       // [nb][THR_STRIDE]
  void *pc;            // [nb] PtrsConst
  uint32_t *cth;       // [nb][SBLK] cumulative thresholds below istar, 0xFFFFFFFF from istar on
  double *fl64;        // [E][BP]
  uint32_t *status;
  int hybrid;          // blocks with Lambda_b >= 10 go to the per-point rule (pad[0] = 1)
};
struct BlockSampleArgs {
  int E, B, BP, npx, nb, nchunks, S;
  uint32_t k0, k1;
  int split_mode;
  uint32_t split_q;
  const BlockRec *brec;
  const uint32_t *thr;  // [nb][THR_STRIDE]
  const void *pc;
  const uint32_t *cth;
  const double *fl64;
  float *part;  // [nchunks][S][B][npx], as SampleArgs
  uint32_t *dbg_counts, *dbg_red;
  int64_t px0, px1;
  uint32_t *status;
  const float *lnfact;
  int accumulate;  // add to the partial sums k_sample wrote (hybrid) instead of storing
};

// Chunk reduction and dust / distance epilogue (k_reduce).
struct ReduceArgs {
  int B, npx, nchunks, S;
  const float *part;
  float *F;  // [B][npx]
  double dist;
  int dust_model;
  double dust_mu, dust_sigma;
  double dust_R[PCMD_MAX_BANDS];
  uint32_t k0, k1;
};

// PSF check (k_psf_check) and direct periodic convolution (k_conv_direct).
struct ConvArgs {
  int B, N, K;
  const float *F;    // [B][N][N]
  const float *psf;  // [B][R][K][K], R = grid * grid
  float *G;          // [B][N][N]
  uint32_t *status;
  int grid;          // 1, or 4 for the 4 x 4 grid of sub-pixel PSFs
};

// Sky, noise and magnitudes (k_noise_mag).
struct NoiseArgs {
  int B, npx;
  const float *G;  // [B][npx]
  float *mags;     // [B][npx]
  int noise_model;
  double sigma[PCMD_MAX_BANDS], exptime[PCMD_MAX_BANDS], zp[PCMD_MAX_BANDS], sky[PCMD_MAX_BANDS];
  uint32_t k0, k1;
};

// Hess diagram (k_hess).
struct HessArgs {
  const float *mags;
  int64_t npx;
  double x0, dx, y0, dy;
  int nx, ny, bb, br, bm;
  uint32_t *hess;
  double *mom_part;  // [blocks][3]
  uint32_t *counter;
  double *moments;
  int use_lds;
};

// Log-likelihood (k_loglike).
struct LoglikeArgs {
  const uint32_t *hm, *hd;
  int nbins, mode;
  const double *mom_m, *mom_d;
  double eps;
  double *out;
  double *part;  // [loglike_blocks(nbins)] block sums
  int accumulate;  // add to *out instead of storing
  const double *lnfact64;  // ln k! for k < LNFACT64_N (host lgamma), or NULL
};
constexpr int LNFACT64_N = 4096;

// Sampler job of the persistent batched kernel: its tiles are items [item0, item0 + items).
struct BatchSampleJob {
  SampleArgs a;
  int item0, items, pblocks, pad;
};

// k_sample.hip
hipError_t launch_entries(const pcmd_grid *g, const double *scale, double *lam, uint32_t *status, hipStream_t s);
hipError_t launch_prep(const PrepArgs &a, hipStream_t s);
hipError_t launch_prep_job(const PrepArgs *table, int j, int E, hipStream_t s);
hipError_t launch_prep_alias(const PrepArgs &a, hipStream_t s);
hipError_t launch_prep_alias_job(const PrepArgs *table, int j, int E, int parts, hipStream_t s);
hipError_t launch_sample(const SampleArgs &a, hipStream_t s);
hipError_t launch_sample_persistent(const BatchSampleJob *jobs, int n_jobs, int total_items, int B, uint32_t *counter,
                                    int n_workgroups, hipStream_t s);
hipError_t launch_reset_counter(uint32_t *counter, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs &a, hipStream_t s);
hipError_t launch_reduce_job(const ReduceArgs *table, int j, int npx, int B, hipStream_t s);

// k_sample_block.hip
hipError_t launch_prep_block(const BlockPrepArgs &a, hipStream_t s);
hipError_t launch_sample_block(const BlockSampleArgs &a, hipStream_t s);
// batched: the thinned entries' pass (F = 1/2) of the job at position t of the persistent table
hipError_t launch_sample_thin_job(const BatchSampleJob *jobs, int t, int B, int npx, int nchunks, hipStream_t s);
// batched: job j of a descriptor table (nb blocks; the sampler's grid covers npx pixels x nchunks)
hipError_t launch_prep_block_job(const BlockPrepArgs *table, int j, int nb, hipStream_t s);
hipError_t launch_sample_block_job(const BlockSampleArgs *table, int j, int B, int npx, int nchunks, hipStream_t s);

// k_image.hip
hipError_t launch_psf_check(const ConvArgs &a, hipStream_t s);
size_t conv_direct_lds_bytes(int K);
hipError_t launch_conv_direct(const ConvArgs &a, hipStream_t s);
hipError_t launch_conv_direct_job(const ConvArgs *table, int j, int B, int N, int K, int grid, hipStream_t s);
hipError_t launch_noise_mag(const NoiseArgs &a, hipStream_t s);
hipError_t launch_noise_mag_job(const NoiseArgs *table, int j, int npx, hipStream_t s);
hipError_t launch_copy_f32(const float *src, float *dst, int64_t n, hipStream_t s);

// k_fft.hip
int fft_supported(int N);
size_t fft_scratch_bytes(int B, int N, int K, int R);
// fresh: the scratch's twiddles, PSF copy and spectra are not those of this (B, N, K, grid)
hipError_t launch_conv_fft(const float *F, const float *psf, int B, int N, int K, int grid, float *G, void *scratch,
                           bool fresh, hipStream_t s);

// k_hess.hip
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
int hess_max_blocks();
int hess_blocks(int64_t npx);
bool hess_use_lds(int nbins);
hipError_t launch_hess(const HessArgs &a, hipStream_t s);
hipError_t launch_hess_job(const HessArgs *table, int j, int64_t npx, int nbins, hipStream_t s);
hipError_t launch_hess_clear_job(const HessArgs *table, int j, int nbins, hipStream_t s);
constexpr int LL_THREADS = 256;  // bins per likelihood block
__host__ __device__ inline int loglike_blocks(int nbins) { return (nbins + LL_THREADS - 1) / LL_THREADS; }
hipError_t launch_loglike(const LoglikeArgs &a, hipStream_t s);
hipError_t launch_loglike_jobs(const LoglikeArgs *table, int n_jobs, int nbins, hipStream_t s);

}  // namespace pcmd
