// FFT path of the periodic PSF convolution (gfx950), for power-of-two image sides.
//
// G_b = IFFT2( FFT2(F_b) * FFT2(P~_b) ) / N^2, where P~_b is the K x K PSF wrapped onto the N x N
// torus with its centre at the origin; this is the same periodic convolution as the direct sum
// (Sec. 2.1 of the paper convolves each band with its PSF).  Transforms run in LDS, two
// radix-2 stages per pass, one row (or a few columns) per workgroup, in FP64 complex arithmetic
// (full rate on MI355X), so the result agrees with the direct sum to ~1e-15 relative to the
// image's RMS.
//
// The PSF spectra and twiddles are kept between calls: a one-workgroup kernel compares the
// caller's PSF with the copy the spectra were built from (and takes the new one), and the
// spectrum kernels return at once unless something changed, so repeated evaluations with one
// PSF transform only the image.  With the 4 x 4 sub-pixel grid (Sec. 2.2) each of the 16 regions
// has its own spectrum: the image is transformed forward once, and per region the product is
// transformed back (all columns, then the rows of the region's band of rows) and only the
// region's pixels are kept.
#include <math.h>

#include <algorithm>

#include "pcmd_device.h"
#include "pcmd_internal.h"

namespace pcmd {

struct cplx {
  double x, y;
};

__device__ __forceinline__ cplx cmul(cplx a, cplx b) { return cplx{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

int fft_supported(int N) { return N >= 8 && N <= 4096 && (N & (N - 1)) == 0; }

static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Scratch layout (complex doubles unless noted): [twiddles N/2][image spectrum B N^2]
// [per-region inverse B N^2, sub-pixel grid only][PSF spectra R B N^2][PSF copy R B K K floats]
// [change flag u32]
static size_t fft_psf_copy_offset(int B, int N, int R) {
  return sizeof(cplx) * ((size_t)N / 2 + (size_t)(R > 1 ? 2 : 1) * B * N * N + (size_t)R * B * N * N);
}
size_t fft_scratch_bytes(int B, int N, int K, int R) {
  return fft_psf_copy_offset(B, N, R) + sizeof(float) * (size_t)R * B * K * K + 256;
}

// flag = force or (any element of psf differs from copy); copy = psf.  One workgroup: each
// thread compares its elements with their old copies before overwriting them.
__global__ void __launch_bounds__(1024) k_psf_update(const float *__restrict__ psf, float *__restrict__ copy, int64_t n,
                                                      int force, uint32_t *__restrict__ flag) {
  __shared__ int any;
  if (threadIdx.x == 0) any = force;
  __syncthreads();
  int d = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const float v = psf[i];
    if (__float_as_uint(v) != __float_as_uint(copy[i])) d = 1;
    copy[i] = v;
  }
  if (d) any = 1;
  __syncthreads();
  if (threadIdx.x == 0) *flag = (uint32_t)any;
}

__global__ void k_twiddles(cplx *tw, int N) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < N / 2) {
    double s, c;
    sincospi(-2.0 * (double)m / (double)N, &s, &c);  // exp(-2 pi i m / N)
    tw[m] = cplx{c, s};
  }
}

// In-LDS decimation-in-time transform of n = 2^logn points a[0], a[1], ... (input already in
// bit-reversed order), by threads t = 0 .. per-1 of the block (active ones; every thread of the
// block reaches the barriers).  inv = conjugate twiddles.  Stages go two at a time (radix 2^2):
// from blocks of length L, one thread takes x0..x3 = a[base + {0, L, 2L, 3L}] and applies both
// radix-2 stages, y0,1 = x0 +- w1 x1, y2,3 = x2 +- w1 x3 (w1 = W_2L^pos), then
// a[base], a[base + 2L] = y0 +- w2 y2 and a[base + L], a[base + 3L] = y1 -+ i w2 y3 (w2 = W_4L^pos;
// +i for the inverse), so each element goes through LDS once per two stages and there is one
// barrier per two stages.  An odd logn starts with one radix-2 stage.
__device__ __forceinline__ void fft_stages(cplx *a, int logn, int N, const cplx *__restrict__ tw, bool inv, int t,
                                           int per, bool active) {
  const int n = 1 << logn;
  int s = 1;
  if (logn & 1) {
    if (active)
      for (int k = t; k < n / 2; k += per) {
        const int i = 2 * k;
        const cplx u = a[i], v = a[i + 1];  // first stage: twiddle 1
        a[i] = cplx{u.x + v.x, u.y + v.y};
        a[i + 1] = cplx{u.x - v.x, u.y - v.y};
      }
    __syncthreads();
    s = 2;
  }
  for (; s < logn; s += 2) {
    const int L = 1 << (s - 1);
    const int ts1 = N >> s, ts2 = N >> (s + 1);  // W_2L^pos = tw[pos N / 2L], W_4L^pos = tw[pos N / 4L]
    if (active)
      for (int k = t; k < n / 4; k += per) {
        const int pos = k & (L - 1);
        const int base = (k >> (s - 1)) * 4 * L + pos;
        cplx w1 = tw[pos * ts1], w2 = tw[pos * ts2];
        if (inv) {
          w1.y = -w1.y;
          w2.y = -w2.y;
        }
        const cplx x0 = a[base], x1 = a[base + L], x2 = a[base + 2 * L], x3 = a[base + 3 * L];
        const cplx t1 = cmul(w1, x1), t3 = cmul(w1, x3);
        const cplx y0{x0.x + t1.x, x0.y + t1.y}, y1{x0.x - t1.x, x0.y - t1.y};
        const cplx y2{x2.x + t3.x, x2.y + t3.y}, y3{x2.x - t3.x, x2.y - t3.y};
        const cplx u2 = cmul(w2, y2), u3 = cmul(w2, y3);
        const cplx v3 = inv ? cplx{-u3.y, u3.x} : cplx{u3.y, -u3.x};  // (+i or -i) u3
        a[base] = cplx{y0.x + u2.x, y0.y + u2.y};
        a[base + 2 * L] = cplx{y0.x - u2.x, y0.y - u2.y};
        a[base + L] = cplx{y1.x + v3.x, y1.y + v3.y};
        a[base + 3 * L] = cplx{y1.x - v3.x, y1.y - v3.y};
      }
    __syncthreads();
  }
}

__device__ __forceinline__ int bitrev(int i, int logn) { return (int)(__brev((unsigned)i) >> (32 - logn)); }

// Row transforms.  mode 0: real FP32 input rows -> forward -> complex out.
//                  mode 1: complex in -> inverse -> real FP32 out scaled by 1/N^2.
//                  mode 2: complex in -> forward, times the row of S (cin2), inverse -> complex out.
//                  mode 3: complex in -> forward -> complex out.
// Block x transforms row y0 + x of band y; mode 1 writes only the columns [xa, xb) of it.  With
// `skip` given, the kernel does nothing unless *skip is non-zero (PSF spectra that are current).
// Modes 2 and 3 read their whole row before writing it, so cout may be cin.
template <int MODE>
__global__ void __launch_bounds__(1024) k_fft_rows(const float *__restrict__ rin, const cplx *cin, cplx *cout,
                                                  float *__restrict__ rout, int N, int logN,
                                                  const cplx *__restrict__ tw, int y0, int xa, int xb,
                                                  const uint32_t *__restrict__ skip, const cplx *__restrict__ cin2) {
  extern __shared__ cplx row[];
  if (skip && *skip == 0u) return;
  const int y = y0 + blockIdx.x, b = blockIdx.y;
  const size_t base = ((size_t)b * N + y) * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    const int r = bitrev(i, logN);
    if (MODE == 0)
      row[i] = cplx{(double)rin[base + r], 0.0};
    else
      row[i] = cin[base + r];
  }
  __syncthreads();
  fft_stages(row, logN, N, tw, MODE == 1, threadIdx.x, blockDim.x, true);
  if (MODE == 2) {
    // times the spectrum, in-place bit reversal (the thread of the smaller index of each pair
    // swaps it), inverse
    for (int i = threadIdx.x; i < N; i += blockDim.x) row[i] = cmul(row[i], cin2[base + i]);
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += blockDim.x) {
      const int r = bitrev(i, logN);
      if (i < r) {
        const cplx u = row[i];
        row[i] = row[r];
        row[r] = u;
      }
    }
    __syncthreads();
    fft_stages(row, logN, N, tw, true, threadIdx.x, blockDim.x, true);
  }
  const double scale = 1.0 / ((double)N * (double)N);
  if (MODE != 1) {
    for (int i = threadIdx.x; i < N; i += blockDim.x) cout[base + i] = row[i];
  } else {
    for (int i = xa + threadIdx.x; i < xb; i += blockDim.x) rout[base + i] = (float)(row[i].x * scale);
  }
}

// In-place transpose of each band's N x N complex matrix: the block at (i, j), i < j, swaps
// the 32 x 32 tiles (i, j) and (j, i) through LDS (rows of 32 elements, 512 contiguous bytes per
// access); a diagonal block transposes its tile; blocks below the diagonal return.  It turns the
// column transform into a row transform over contiguous memory: the column pass over 4096-point
// columns held two columns per workgroup and read 32 bytes of every 64 KB row.
constexpr int TT = 32;
__global__ void __launch_bounds__(256) k_transpose_c(cplx *X, int N, const uint32_t *__restrict__ skip) {
  __shared__ cplx ta[TT][TT + 1], tb[TT][TT + 1];
  if (skip && *skip == 0u) return;
  const int i = blockIdx.y, j = blockIdx.x;
  if (i > j) return;
  cplx *M = X + (size_t)blockIdx.z * N * N;
  const int tx = threadIdx.x & (TT - 1), ty = threadIdx.x >> 5;  // 32 x 8 threads
  for (int r = ty; r < TT; r += 8) {
    ta[r][tx] = M[(size_t)(i * TT + r) * N + j * TT + tx];
    if (i != j) tb[r][tx] = M[(size_t)(j * TT + r) * N + i * TT + tx];
  }
  __syncthreads();
  for (int r = ty; r < TT; r += 8) {
    M[(size_t)(j * TT + r) * N + i * TT + tx] = ta[tx][r];
    if (i != j) M[(size_t)(i * TT + r) * N + j * TT + tx] = tb[tx][r];
  }
}

// Column transforms over CB adjacent columns.  mode 0: forward only (PSF spectrum; with `skip`
// given, only when *skip is non-zero).  mode 1: forward, multiply by the PSF spectrum, inverse.
// mode 2: multiply the forward-transformed columns by the spectrum and inverse, into Y.
template <int MODE>
__global__ void __launch_bounds__(1024) k_fft_cols(cplx *__restrict__ X, const cplx *__restrict__ S, int N, int logN,
                                                  int CB, const cplx *__restrict__ tw, cplx *__restrict__ Y,
                                                  const uint32_t *__restrict__ skip) {
  extern __shared__ cplx col[];  // [CB][N]
  if (MODE == 0 && skip && *skip == 0u) return;
  const int x0 = blockIdx.x * CB, b = blockIdx.y;
  const size_t base = (size_t)b * N * N;
  for (int idx = threadIdx.x; idx < N * CB; idx += blockDim.x) {
    const int y = idx / CB, c = idx - y * CB;  // consecutive threads read consecutive columns of a row
    col[c * N + (MODE == 2 ? y : bitrev(y, logN))] = X[base + (size_t)y * N + x0 + c];
  }
  __syncthreads();
  // each column's transform is done by blockDim / CB threads
  const int per = blockDim.x / CB;
  const int c = threadIdx.x / per, t = threadIdx.x - c * per;
  if (MODE != 2) fft_stages(col + (c < CB ? c : 0) * N, logN, N, tw, false, t, per, c < CB);
  if (MODE >= 1) {
    // multiply by the PSF spectrum in place, bit-reverse in place (the thread of the smaller
    // index of each pair swaps it), then the inverse transform
    for (int idx = threadIdx.x; idx < N * CB; idx += blockDim.x) {
      const int cc = idx / N, y = idx - cc * N;
      col[cc * N + y] = cmul(col[cc * N + y], S[base + (size_t)y * N + x0 + cc]);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < N * CB; idx += blockDim.x) {
      const int cc = idx / N, y = idx - cc * N, r = bitrev(y, logN);
      if (y < r) {
        const cplx u = col[cc * N + y];
        col[cc * N + y] = col[cc * N + r];
        col[cc * N + r] = u;
      }
    }
    __syncthreads();
    fft_stages(col + (c < CB ? c : 0) * N, logN, N, tw, true, t, per, c < CB);
  }
  cplx *out = MODE == 2 ? Y : X;
  for (int idx = threadIdx.x; idx < N * CB; idx += blockDim.x) {
    const int y = idx / CB, cc = idx - y * CB;
    out[base + (size_t)y * N + x0 + cc] = col[cc * N + y];
  }
}

// PSF wrapped onto the N x N torus: Pw[(u - h) mod N][(v - h) mod N] = P[u][v], zero elsewhere.
// Band b's PSF at psf + b pstride.  Only when *skip is non-zero.
__global__ void k_psf_wrap(const float *__restrict__ psf, int K, int N, float *__restrict__ out, int64_t pstride,
                           const uint32_t *__restrict__ skip) {
  if (*skip == 0u) return;
  const int b = blockIdx.y;
  const size_t NN = (size_t)N * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < NN; i += (size_t)gridDim.x * blockDim.x) {
    const int y = (int)(i / N), x = (int)(i - (size_t)y * N);
    const int h = (K - 1) / 2;
    const int u = (y + h) % N, v = (x + h) % N;  // inverse of the wrap
    float val = 0.0f;
    if (u < K && v < K) val = psf[(size_t)b * pstride + (size_t)u * K + v];
    out[(size_t)b * NN + i] = val;
  }
}

static int cols_per_block(int N) {
  int cb = 8;
  while (cb > 1 && (size_t)cb * N * sizeof(cplx) > 160 * 1024) cb >>= 1;
  return cb;
}

hipError_t launch_conv_fft(const float *F, const float *psf, int B, int N, int K, int grid, float *G, void *scratch,
                           bool fresh, hipStream_t s) {
  if (!fft_supported(N) || (grid != 1 && grid != 4)) return hipErrorInvalidValue;
  const int R = grid * grid;
  const int logN = ilog2(N);
  const size_t NN = (size_t)N * N;
  cplx *tw = (cplx *)scratch;
  cplx *X = tw + N / 2;
  cplx *Y = X + (size_t)B * NN;                      // sub-pixel grid only
  cplx *Sp = R > 1 ? Y + (size_t)B * NN : Y;         // [R][B][N][N]
  float *copy = (float *)((char *)scratch + fft_psf_copy_offset(B, N, R));
  uint32_t *flag = (uint32_t *)(copy + (size_t)R * B * K * K);
  const int CB = cols_per_block(N);
  if ((size_t)CB * N * sizeof(cplx) > 160 * 1024) return hipErrorInvalidValue;
  // one thread per radix-2^2 butterfly (N / 4 per transform) up to 1024: a 4096-point row holds
  // 64 KB of LDS, so two blocks fit a CU, and 256 threads left two waves per SIMD to hide the
  // LDS and barrier latency of the stages
  const int rthreads = std::min(std::max(N / 4, 64), 1024);
  const int cthreads = std::min(std::max(CB * N / 4, 64), 1024);
  const size_t rl = N * sizeof(cplx), cl = CB * N * sizeof(cplx);
  if (fresh) hipLaunchKernelGGL(k_twiddles, dim3((N / 2 + 255) / 256), dim3(256), 0, s, tw, N);
  // PSF spectra, rebuilt only when the PSF (or the layout: fresh) changed.  psf is
  // [B][K][K] (grid 1) or [B][16][K][K]: region r of band b at psf + (b R + r) K K.
  hipLaunchKernelGGL(k_psf_update, dim3(1), dim3(1024), 0, s, psf, copy, (int64_t)R * B * K * K, fresh ? 1 : 0, flag);
  // One PSF and N >= 1024: the column transforms run as row transforms of the transposed matrix
  // (its spectrum is kept transposed); the sub-pixel grid and smaller N keep the column kernels
  // (at 512 the two transposes cost more than the strided column reads they save).
  const bool tr = R == 1 && N >= 1024;
  const dim3 tgrid((unsigned)(N / TT), (unsigned)(N / TT), (unsigned)B);
  for (int r = 0; r < R; ++r) {
    cplx *Sr = Sp + (size_t)r * B * NN;
    // wrap into G (free at this point), transform rows and columns
    hipLaunchKernelGGL(k_psf_wrap, dim3(256, B), dim3(256), 0, s, psf + (size_t)r * K * K, K, N, G, (int64_t)R * K * K,
                       flag);
    hipLaunchKernelGGL(k_fft_rows<0>, dim3(N, B), dim3(rthreads), rl, s, G, nullptr, Sr, nullptr, N, logN, tw, 0, 0, N,
                       flag, nullptr);
    if (tr) {
      hipLaunchKernelGGL(k_transpose_c, tgrid, dim3(256), 0, s, Sr, N, flag);
      hipLaunchKernelGGL(k_fft_rows<3>, dim3(N, B), dim3(rthreads), rl, s, nullptr, Sr, Sr, nullptr, N, logN, tw, 0, 0,
                         N, flag, nullptr);
    } else {
      hipLaunchKernelGGL(k_fft_cols<0>, dim3(N / CB, B), dim3(cthreads), cl, s, Sr, nullptr, N, logN, CB, tw, nullptr,
                         flag);
    }
  }
  // image: rows forward
  hipLaunchKernelGGL(k_fft_rows<0>, dim3(N, B), dim3(rthreads), rl, s, F, nullptr, X, nullptr, N, logN, tw, 0, 0, N,
                     nullptr, nullptr);
  if (tr) {
    // transpose, columns forward x spectrum inverse as rows, transpose back, rows inverse
    hipLaunchKernelGGL(k_transpose_c, tgrid, dim3(256), 0, s, X, N, nullptr);
    hipLaunchKernelGGL(k_fft_rows<2>, dim3(N, B), dim3(rthreads), rl, s, nullptr, X, X, nullptr, N, logN, tw, 0, 0, N,
                       nullptr, Sp);
    hipLaunchKernelGGL(k_transpose_c, tgrid, dim3(256), 0, s, X, N, nullptr);
    hipLaunchKernelGGL(k_fft_rows<1>, dim3(N, B), dim3(rthreads), rl, s, nullptr, X, nullptr, G, N, logN, tw, 0, 0, N,
                       nullptr, nullptr);
    return hipGetLastError();
  }
  if (R == 1) {
    // columns forward x spectrum inverse, rows inverse
    hipLaunchKernelGGL(k_fft_cols<1>, dim3(N / CB, B), dim3(cthreads), cl, s, X, Sp, N, logN, CB, tw, nullptr, nullptr);
    hipLaunchKernelGGL(k_fft_rows<1>, dim3(N, B), dim3(rthreads), rl, s, nullptr, X, nullptr, G, N, logN, tw, 0, 0, N,
                       nullptr, nullptr);
    return hipGetLastError();
  }
  // sub-pixel grid: columns forward once; per region the product transformed back, the rows of
  // the region's band of rows, only its columns written
  hipLaunchKernelGGL(k_fft_cols<0>, dim3(N / CB, B), dim3(cthreads), cl, s, X, nullptr, N, logN, CB, tw, nullptr, nullptr);
  const int side = N / grid;
  for (int r = 0; r < R; ++r) {
    const int ry = r / grid, rx = r - ry * grid;
    hipLaunchKernelGGL(k_fft_cols<2>, dim3(N / CB, B), dim3(cthreads), cl, s, X, Sp + (size_t)r * B * NN, N, logN, CB, tw,
                       Y, nullptr);
    hipLaunchKernelGGL(k_fft_rows<1>, dim3(side, B), dim3(rthreads), rl, s, nullptr, Y, nullptr, G, N, logN, tw,
                       ry * side, rx * side, (rx + 1) * side, nullptr, nullptr);
  }
  return hipGetLastError();
}

}  // namespace pcmd
