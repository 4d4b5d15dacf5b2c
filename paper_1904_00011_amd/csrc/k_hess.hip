// Hess diagram (LDS-privatised histogram) and binned log-likelihood reduction (gfx950).
// Sec. 2.5 of the paper: pixels are binned in colour and magnitude (0.05 mag bins) and the
// model and data Hess diagrams are compared bin by bin, with a term for the difference of the
// mean colour and magnitude.
#include <math.h>

#include "pcmd_device.h"
#include "pcmd_internal.h"

namespace pcmd {

__global__ void __launch_bounds__(256) k_fill_u32(uint32_t *__restrict__ p, uint32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

constexpr int HESS_THREADS = 512;
constexpr int HESS_MAX_BLOCKS = 1024;  // four 40 KB private histograms per CU
constexpr int HESS_LDS_MAX_BINS = 40000;  // 160,000 bytes of LDS (of 163,840 per workgroup)
int hess_max_blocks() { return HESS_MAX_BLOCKS; }

__device__ __forceinline__ int bin_of(double t, int n) {
  // clamp(floor(t), 0, n-1), NaN -> 0
  if (!(t >= 0.0)) return 0;
  if (t >= (double)n) return n - 1;
  return (int)t;
}

// bin_of((d) / dx) without the division where it cannot matter: t = d * (1 / dx) is within
// 2^-51 |t| of the correctly rounded quotient (two roundings of the product, one of the
// quotient), so when t - e and t + e (e = 2^-50 |t|) fall in the same bin, that is the bin of the
// quotient (bin_of is monotone); otherwise, near a bin edge, and for infinite d, the FP64
// division decides.  NaN takes bin 0 either way.
__device__ __forceinline__ int bin_fast(double d, double inv_dx, double dx, int n) {
  const double t = d * inv_dx;
  const double e = 0x1p-50 * fabs(t);
  const int lo = bin_of(t - e, n);
  return lo == bin_of(t + e, n) ? lo : bin_of(d / dx, n);
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  // fixed-order tree: within each wave by shuffles, then over the waves in order (deterministic)
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < HESS_THREADS / 64; ++w) r += red[w];
  __syncthreads();
  return r;
}

int hess_blocks(int64_t npx) {
  // enough pixels per block to amortise clearing and merging the private histogram
  int64_t blocks = (npx + 4095) / 4096;
  if (blocks < 1) blocks = 1;
  if (blocks > HESS_MAX_BLOCKS) blocks = HESS_MAX_BLOCKS;
  return (int)blocks;
}
bool hess_use_lds(int nbins) { return nbins <= HESS_LDS_MAX_BINS; }

__device__ __forceinline__ void hess_body(const HessArgs &a) {
  extern __shared__ uint32_t lh[];
  __shared__ double red[HESS_THREADS / 64];
  __shared__ bool last;
  const int nb = a.nx * a.ny;
  if (a.use_lds) {
    for (int j = threadIdx.x; j < nb; j += HESS_THREADS) lh[j] = 0u;
    __syncthreads();
  }
  double sx = 0.0, sy = 0.0, cnt = 0.0;
  const double inv_dx = 1.0 / a.dx, inv_dy = 1.0 / a.dy;
  const float *mb = a.mags + (size_t)a.bb * a.npx;
  const float *mr = a.mags + (size_t)a.br * a.npx;
  const float *mm = a.mags + (size_t)a.bm * a.npx;
  for (int64_t p = (int64_t)blockIdx.x * HESS_THREADS + threadIdx.x; p < a.npx;
       p += (int64_t)gridDim.x * HESS_THREADS) {
    const double vb = (double)mb[p], vr = (double)mr[p], vm = (double)mm[p];
    const double x = vb - vr, y = vm;
    const int ix = bin_fast(x - a.x0, inv_dx, a.dx, a.nx);
    const int iy = bin_fast(y - a.y0, inv_dy, a.dy, a.ny);
    const int j = iy * a.nx + ix;
    if (a.use_lds)
      atomicAdd(&lh[j], 1u);
    else
      atomicAdd(&a.hess[j], 1u);
    if (isfinite(vb) && isfinite(vr) && isfinite(vm)) {
      sx += x;
      sy += y;
      cnt += 1.0;
    }
  }
  if (a.use_lds) {
    __syncthreads();
    for (int j = threadIdx.x; j < nb; j += HESS_THREADS) {
      const uint32_t v = lh[j];
      if (v) atomicAdd(&a.hess[j], v);
    }
  }
  sx = block_sum(sx, red);
  sy = block_sum(sy, red);
  cnt = block_sum(cnt, red);
  if (threadIdx.x == 0) {
    a.mom_part[blockIdx.x * 3 + 0] = sx;
    a.mom_part[blockIdx.x * 3 + 1] = sy;
    a.mom_part[blockIdx.x * 3 + 2] = cnt;
    __threadfence();
    const uint32_t prev = atomicAdd(a.counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (last) {
    // every block's partial is visible: thread t adds blocks t, t + HESS_THREADS, ... in order,
    // then the fixed-order block sum (the combination does not depend on which block is last)
    __threadfence();
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (unsigned k = threadIdx.x; k < gridDim.x; k += HESS_THREADS) {
      s0 += __builtin_nontemporal_load(&a.mom_part[k * 3 + 0]);
      s1 += __builtin_nontemporal_load(&a.mom_part[k * 3 + 1]);
      s2 += __builtin_nontemporal_load(&a.mom_part[k * 3 + 2]);
    }
    s0 = block_sum(s0, red);
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    if (threadIdx.x == 0) {
      a.moments[0] = s0;
      a.moments[1] = s1;
      a.moments[2] = s2;
      *a.counter = 0u;  // ready for the next call (also under graph replay)
    }
  }
}

__global__ void __launch_bounds__(HESS_THREADS) k_hess(HessArgs a) { hess_body(a); }
__global__ void __launch_bounds__(HESS_THREADS) k_hess_job(const HessArgs *__restrict__ t, int j) {
  const HessArgs a = t[j];
  hess_body(a);
}

hipError_t launch_hess(const HessArgs &a, hipStream_t s) {
  const int nb = a.nx * a.ny;
  hipError_t e = launch_fill_u32(a.hess, 0u, nb, s);
  if (e != hipSuccess) return e;
  const size_t lds = a.use_lds ? (size_t)nb * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL(k_hess, dim3((unsigned)hess_blocks(a.npx)), dim3(HESS_THREADS), lds, s, a);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_hess_clear_job(const HessArgs *__restrict__ t, int j, int nbins) {
  uint32_t *h = t[j].hess;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nbins; i += gridDim.x * blockDim.x) h[i] = 0u;
}

hipError_t launch_hess_clear_job(const HessArgs *table, int j, int nbins, hipStream_t s) {
  hipLaunchKernelGGL(k_hess_clear_job, dim3((nbins + 255) / 256), dim3(256), 0, s, table, j, nbins);
  return hipGetLastError();
}

// The job variant expects the histogram already cleared (k_hess_clear_job).
hipError_t launch_hess_job(const HessArgs *table, int j, int64_t npx, int nbins, hipStream_t s) {
  const size_t lds = hess_use_lds(nbins) ? (size_t)nbins * sizeof(uint32_t) : 0;
  hipLaunchKernelGGL(k_hess_job, dim3((unsigned)hess_blocks(npx)), dim3(HESS_THREADS), lds, s, table, j);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Log-likelihood: one thread per bin over ceil(nbins / LL_THREADS) blocks, each block's sum
// written to part[block]; a second one-block kernel adds the block sums in block order (fixed
// order, so the result does not depend on scheduling) and the mean-colour / mean-magnitude term.
// Every block recomputes the totals N_m, N_d itself: integer sums are exact, so they agree.
// ---------------------------------------------------------------------------------------
// Fixed-order sum over the block (tree in LDS).
template <typename T>
__device__ __forceinline__ T block_sum_ordered(T v, T *sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int s = LL_THREADS / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] = sh[t] + sh[t + s];
    __syncthreads();
  }
  const T r = sh[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void loglike_bins_body(const LoglikeArgs &a, int blk) {
  const uint32_t *__restrict__ hm = a.hm;
  const uint32_t *__restrict__ hd = a.hd;
  const int nbins = a.nbins, mode = a.mode;
  const double eps = a.eps;
  __shared__ unsigned long long shu[LL_THREADS];
  __shared__ double shd[LL_THREADS];
  const int t = threadIdx.x;
  unsigned long long sm = 0, sd = 0;
  // batches of 8 bins per thread loaded into separate registers before they are added, so the
  // 16 loads are in flight together (one register reused for every load serialised them)
  for (int j0 = t; j0 < nbins; j0 += 8 * LL_THREADS) {
    uint32_t vm[8], vd[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int j = j0 + u * LL_THREADS;
      vm[u] = j < nbins ? hm[j] : 0u;
      vd[u] = j < nbins ? hd[j] : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sm += vm[u];
      sd += vd[u];
    }
  }
  const double Nm = (double)block_sum_ordered(sm, shu);
  const double Nd = (double)block_sum_ordered(sd, shu);
  double acc = 0.0;
  const int j = blk * LL_THREADS + t;
  if (j < nbins) {
    const double m = (double)hm[j], d = (double)hd[j];
    if (mode == PCMD_LL_POISSON) {
      const double lam = Nd * (m + eps) / (Nm + eps * (double)nbins);
      const double lf = (a.lnfact64 && d < (double)LNFACT64_N) ? a.lnfact64[(int)d] : lgamma(d + 1.0);
      acc = d * log(lam) - lam - lf;
    } else if (mode == PCMD_LL_GAUSS_PAPER) {
      const double mh = m * Nd / Nm;
      const double sig = fmax(sqrt(d + mh), 2.0);
      const double df = d - mh;
      acc = -df * df / (2.0 * sig * sig);
    } else {
      const double sig = fmax(sqrt(d * d + m * m), 2.0);
      const double df = d / Nd - m / Nm;
      acc = -df * df / (2.0 * sig * sig);
    }
  }
  const double bsum = block_sum_ordered(acc, shd);
  if (t == 0) a.part[blk] = bsum;
}

__device__ __forceinline__ void loglike_final_body(const LoglikeArgs &a) {
  // the 64 lanes fetch the block sums together; lane 0 adds them in block order
  __shared__ double ps[256];
  const int nb = loglike_blocks(a.nbins);
  double r = 0.0;
  for (int b0 = 0; b0 < nb; b0 += 256) {
    const int n = min(256, nb - b0);
    for (int k = threadIdx.x; k < n; k += 64) ps[k] = a.part[b0 + k];
    __syncthreads();
    if (threadIdx.x == 0)
      for (int k = 0; k < n; ++k) r += ps[k];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  if (a.mode != PCMD_LL_POISSON) {
    const double Cm = a.mom_m[0] / a.mom_m[2], Mm = a.mom_m[1] / a.mom_m[2];
    const double Cd = a.mom_d[0] / a.mom_d[2], Md = a.mom_d[1] / a.mom_d[2];
    r += -(Cd - Cm) * (Cd - Cm) / (2.0 * 0.05 * 0.05) - (Md - Mm) * (Md - Mm) / (2.0 * 0.05 * 0.05);
  }
  a.out[0] = a.accumulate ? a.out[0] + r : r;
}

__global__ void __launch_bounds__(LL_THREADS) k_loglike_bins(LoglikeArgs a) { loglike_bins_body(a, blockIdx.x); }
__global__ void __launch_bounds__(64) k_loglike_final(LoglikeArgs a) { loglike_final_body(a); }
// batched: grid.y (bins) / grid.x (final) runs over the jobs of a descriptor table
__global__ void __launch_bounds__(LL_THREADS) k_loglike_bins_jobs(const LoglikeArgs *__restrict__ t) {
  const LoglikeArgs a = t[blockIdx.y];
  loglike_bins_body(a, blockIdx.x);
}
__global__ void __launch_bounds__(64) k_loglike_final_jobs(const LoglikeArgs *__restrict__ t) {
  const LoglikeArgs a = t[blockIdx.x];
  loglike_final_body(a);
}

hipError_t launch_loglike(const LoglikeArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_loglike_bins, dim3((unsigned)loglike_blocks(a.nbins)), dim3(LL_THREADS), 0, s, a);
  hipLaunchKernelGGL(k_loglike_final, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_loglike_jobs(const LoglikeArgs *table, int n_jobs, int nbins, hipStream_t s) {
  hipLaunchKernelGGL(k_loglike_bins_jobs, dim3((unsigned)loglike_blocks(nbins), (unsigned)n_jobs), dim3(LL_THREADS), 0,
                     s, table);
  hipLaunchKernelGGL(k_loglike_final_jobs, dim3((unsigned)n_jobs), dim3(64), 0, s, table);
  return hipGetLastError();
}

}  // namespace pcmd
