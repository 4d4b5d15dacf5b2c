// Image-plane kernels (gfx950): periodic PSF convolution (LDS-tiled direct sum), sky / noise /
// flux -> magnitude.  Sec. 2.1 of the paper: each band's image is convolved with its PSF, sky and
// shot noise are added and pixel counts become magnitudes.
#include <math.h>

#include "pcmd_device.h"
#include "pcmd_internal.h"

namespace pcmd {

// One block per PSF (band, and region of the sub-pixel grid): check that it is finite,
// non-negative and sums to one within 1e-3 (a failure sets a status bit reported by pcmd_sync).
// The FFT path runs this kernel; the direct convolution makes the same check in its first tile of
// each PSF (psf_check_wave).
__device__ __forceinline__ void psf_check_body(const ConvArgs &a) {
  __shared__ double red[256];
  __shared__ int bad;
  const int b = blockIdx.x;  // PSF index b_band * grid^2 + region
  const int KK = a.K * a.K;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  double s = 0.0;
  for (int i = threadIdx.x; i < KK; i += 256) {
    const float v = a.psf[(size_t)b * KK + i];
    if (!(v >= 0.0f) || !isfinite(v)) bad = 1;
    s += (double)v;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0 && (bad || !(fabs(red[0] - 1.0) <= 1e-3))) atomicOr(a.status, STATUS_BAD_PSF);
}

__global__ void __launch_bounds__(256) k_psf_check(ConvArgs a) { psf_check_body(a); }

hipError_t launch_psf_check(const ConvArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_psf_check, dim3(a.B * a.grid * a.grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_copy_f32(const float *__restrict__ src, float *__restrict__ dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

hipError_t launch_copy_f32(const float *src, float *dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Direct periodic convolution.  G[y][x] = sum_{u,v} P[u][v] F[(y-u+h) mod N][(x-v+h) mod N].
// A 64 x 16 output tile per 256-thread block; each thread owns four neighbouring outputs of one
// row.  The input tile with its K-1 halo (wrapped periodically) and the flipped PSF (rows
// zero-padded to a multiple of 4) are staged in LDS as FP32 and read 16 bytes at a time: tile
// values into a sliding register window, PSF values as broadcasts.  For every PSF row the thread
// forms the four K-term dot products in FP32 (all terms positive, ascending column; the zero
// padding adds exact zeros) and adds them to FP64 accumulators in ascending row order.
// ---------------------------------------------------------------------------------------
constexpr int CT_X = 64, CT_Y = 16;

__host__ __device__ inline int conv_kp(int K) { return (K + 3) & ~3; }
__host__ __device__ inline int conv_tile_w(int K) { return CT_X + conv_kp(K) + 4; }

size_t conv_direct_lds_bytes(int K) {
  return ((size_t)(CT_Y + K - 1) * conv_tile_w(K) + (size_t)K * conv_kp(K)) * sizeof(float);
}
// Row splits RS > 1: RS groups of 256 threads share one output tile, group g taking PSF rows
// [g K / RS, (g + 1) K / RS); groups 1.. leave their FP64 sums in LDS and group 0 adds them in
// group order.  Used when the image is too small for one-group blocks to fill the chip.
constexpr int CONV_RS = 4;
static size_t conv_split_lds_bytes(int K) {
  return conv_direct_lds_bytes(K) + (size_t)(CONV_RS - 1) * 256 * 4 * sizeof(double);
}

// The PSF check of psf_check_body done by one wave (the direct convolution's first tile of each
// PSF runs it beside its own work, which saves the check's launch): per-lane FP64 sums, then a
// shuffle reduction.
__device__ __forceinline__ void psf_check_wave(const ConvArgs &a, int b) {
  const int KK = a.K * a.K, lane = (int)(threadIdx.x & 63u);
  double s = 0.0;
  bool bad = false;
  for (int i = lane; i < KK; i += 64) {
    const float v = a.psf[(size_t)b * KK + i];
    if (!(v >= 0.0f) || !isfinite(v)) bad = true;
    s += (double)v;
  }
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
  if (lane == 0 && (__ballot(bad) != 0ull || !(fabs(s - 1.0) <= 1e-3))) atomicOr(a.status, STATUS_BAD_PSF);
}

template <int RS>
__device__ __forceinline__ void conv_direct_body(const ConvArgs &ca) {
  extern __shared__ float4 lds4[];
  float *tile = reinterpret_cast<float *>(lds4);
  const float *__restrict__ F = ca.F;
  float *__restrict__ G = ca.G;
  const int N = ca.N, K = ca.K, Kp = conv_kp(K);
  // blockIdx.z = band * grid^2 + region; region (ry, rx) holds the pixels with
  // floor(grid y / N) = ry and floor(grid x / N) = rx, i.e. y in [ceil(ry N / grid), ceil((ry+1) N / grid))
  const int R = ca.grid * ca.grid;
  const int b = blockIdx.z / R, r = blockIdx.z - b * R;
  const int ry = r / ca.grid, rx = r - ry * ca.grid;
  const int y0r = (ry * N + ca.grid - 1) / ca.grid, y1r = ((ry + 1) * N + ca.grid - 1) / ca.grid;
  const int x0r = (rx * N + ca.grid - 1) / ca.grid, x1r = ((rx + 1) * N + ca.grid - 1) / ca.grid;
  const int ox = x0r + blockIdx.x * CT_X, oy = y0r + blockIdx.y * CT_Y;
  if (ox >= x1r || oy >= y1r) return;  // the grid is sized for the largest region
  if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 64) psf_check_wave(ca, (int)blockIdx.z);
  const int h = (K - 1) >> 1;
  const int TW = conv_tile_w(K), TH = CT_Y + K - 1;
  float *Pf = tile + TW * TH;  // Pf[a][c] = P[K-1-a][K-1-c], 0 for c >= K
  const float *Fb = F + (size_t)b * N * N;
  const float *psf = ca.psf + (size_t)blockIdx.z * K * K;
  // tile[ty][tx] = F[(oy - h + ty) mod N][(ox - h + tx) mod N]; columns past the halo are padding
  for (int idx = threadIdx.x; idx < TW * TH; idx += 256 * RS) {
    const int ty = idx / TW, tx = idx - ty * TW;
    int gy = (oy - h + ty) % N;
    if (gy < 0) gy += N;
    int gx = (ox - h + tx) % N;
    if (gx < 0) gx += N;
    tile[idx] = Fb[(size_t)gy * N + gx];
  }
  for (int idx = threadIdx.x; idx < K * Kp; idx += 256 * RS) {
    const int a = idx / Kp, c = idx - a * Kp;
    Pf[idx] = c < K ? psf[(size_t)(K - 1 - a) * K + (K - 1 - c)] : 0.0f;
  }
  __syncthreads();
  const int grp = threadIdx.x >> 8, lt = threadIdx.x & 255;
  const int tx4 = lt & 15, ty = lt >> 4;
  // output (oy + ty, ox + 4 tx4 + i) = sum_{a,c} Pf[a][c] tile[ty + a][4 tx4 + i + c]
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int a0 = grp * K / RS, a1 = (grp + 1) * K / RS;
  for (int a = a0; a < a1; ++a) {
    const float *row = tile + (ty + a) * TW + 4 * tx4;
    const float *prow = Pf + a * Kp;
    float d0 = 0.0f, d1 = 0.0f, d2 = 0.0f, d3 = 0.0f;
    float4 lo = *reinterpret_cast<const float4 *>(row);
    for (int c = 0; c < Kp; c += 4) {
      const float4 hi = *reinterpret_cast<const float4 *>(row + c + 4);
      const float4 p4 = *reinterpret_cast<const float4 *>(prow + c);
      const float w[8] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
      const float pk[4] = {p4.x, p4.y, p4.z, p4.w};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        d0 = fmaf(pk[k], w[k], d0);
        d1 = fmaf(pk[k], w[k + 1], d1);
        d2 = fmaf(pk[k], w[k + 2], d2);
        d3 = fmaf(pk[k], w[k + 3], d3);
      }
      lo = hi;
    }
    acc[0] += (double)d0;
    acc[1] += (double)d1;
    acc[2] += (double)d2;
    acc[3] += (double)d3;
  }
  if (RS > 1) {
    double *part = reinterpret_cast<double *>(Pf + K * Kp);  // [RS - 1][256][4]
    if (grp > 0) {
#pragma unroll
      for (int i = 0; i < 4; ++i) part[((grp - 1) * 256 + lt) * 4 + i] = acc[i];
    }
    __syncthreads();
    if (grp > 0) return;
#pragma unroll
    for (int g = 1; g < RS; ++g)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += part[((g - 1) * 256 + lt) * 4 + i];
  }
  const int y = oy + ty;
  if (y < y1r) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int x = ox + 4 * tx4 + i;
      if (x < x1r) G[(size_t)b * N * N + (size_t)y * N + x] = (float)acc[i];
    }
  }
}

template <int RS>
__global__ void __launch_bounds__(256 * RS) k_conv_direct(ConvArgs a) { conv_direct_body<RS>(a); }
template <int RS>
__global__ void __launch_bounds__(256 * RS) k_conv_direct_job(const ConvArgs *__restrict__ t, int j) {
  const ConvArgs a = t[j];
  conv_direct_body<RS>(a);
}

// Blocks per region side: the largest region of a grid x grid split is ceil(N / grid) wide.
static dim3 conv_grid(int B, int N, int grid) {
  const int side = (N + grid - 1) / grid;
  return dim3((side + CT_X - 1) / CT_X, (side + CT_Y - 1) / CT_Y, B * grid * grid);
}

// Row splits when one-group blocks would leave most SIMDs with a single wave (fewer than 2048
// blocks) and the split's LDS fits.
static bool conv_use_split(dim3 g, int K) {
  return (int64_t)g.x * g.y * g.z < 2048 && conv_split_lds_bytes(K) <= 160 * 1024;
}

hipError_t launch_conv_direct(const ConvArgs &a, hipStream_t s) {
  const size_t lds = conv_direct_lds_bytes(a.K);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const dim3 g = conv_grid(a.B, a.N, a.grid);
  if (conv_use_split(g, a.K))
    hipLaunchKernelGGL(k_conv_direct<CONV_RS>, g, dim3(256 * CONV_RS), conv_split_lds_bytes(a.K), s, a);
  else
    hipLaunchKernelGGL(k_conv_direct<1>, g, dim3(256), lds, s, a);
  return hipGetLastError();
}
hipError_t launch_conv_direct_job(const ConvArgs *table, int j, int B, int N, int K, int grid, hipStream_t s) {
  const size_t lds = conv_direct_lds_bytes(K);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const dim3 g = conv_grid(B, N, grid);
  if (conv_use_split(g, K))
    hipLaunchKernelGGL(k_conv_direct_job<CONV_RS>, g, dim3(256 * CONV_RS), conv_split_lds_bytes(K), s, table, j);
  else
    hipLaunchKernelGGL(k_conv_direct_job<1>, g, dim3(256), lds, s, table, j);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Noise and magnitudes (FP64 arithmetic per pixel, FP32 storage).
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void noise_mag_body(const NoiseArgs &a, int p) {
  if (p >= a.npx) return;
  for (int b = 0; b < a.B; ++b) {
    const double G = (double)a.G[(size_t)b * a.npx + p];
    double m;
    if (a.noise_model == PCMD_NOISE_NONE) {
      m = G > 0.0 ? -2.5 * log10(G) : INFINITY;
    } else {
      const u4 w = philox10((uint32_t)p, (uint32_t)b, TAG_NOISE, 0u, a.k0, a.k1);
      const double z = box_muller(w.x, w.y);
      if (a.noise_model == PCMD_NOISE_GAUSS_MAG) {
        m = G > 0.0 ? -2.5 * log10(G) + a.sigma[b] * z : INFINITY;
      } else {
        const double t = a.exptime[b];
        const double c = G * t * exp10(0.4 * a.zp[b]) + a.sky[b];
        const double c2 = c + sqrt(c > 0.0 ? c : 0.0) * z - a.sky[b];
        m = c2 > 0.0 ? -2.5 * log10(c2 / t) + a.zp[b] : INFINITY;
      }
    }
    a.mags[(size_t)b * a.npx + p] = (float)m;
  }
}

__global__ void __launch_bounds__(256) k_noise_mag(NoiseArgs a) { noise_mag_body(a, blockIdx.x * blockDim.x + threadIdx.x); }
__global__ void __launch_bounds__(256) k_noise_mag_job(const NoiseArgs *__restrict__ t, int j) {
  const NoiseArgs a = t[j];
  noise_mag_body(a, blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_noise_mag_job(const NoiseArgs *table, int j, int npx, hipStream_t s) {
  hipLaunchKernelGGL(k_noise_mag_job, dim3((npx + 255) / 256), dim3(256), 0, s, table, j);
  return hipGetLastError();
}

hipError_t launch_noise_mag(const NoiseArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_noise_mag, dim3((a.npx + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pcmd
