// Block-skip sampler: the per-pixel star counts by Poisson superposition (Sec. 2.1 footnote).
//
// A sum of independent Poisson counts is Poisson with the summed mean, and given that sum the
// individual counts are multinomial.  Per pixel and per block b of SBLK = 64 consecutive entries:
//   * the block total N ~ Poisson(Lambda_b), Lambda_b = sum of the block's lambda_i (FP64, left
//     to right): below 10 by inversion of word 0 of Philox(p, b, TAG_BLOCK, 0), from 10 on by
//     transformed rejection on Philox(p, b, TAG_BLOCK_PTRS, j) (the per-entry routines);
//   * star s of the block takes word s mod 4 of Philox(p, b, TAG_STAR, s / 4) and lands on the
//     first entry i whose cumulative threshold C_i = floor(2^32 cum_i / Lambda_b) exceeds it
//     (entry i with probability lambda_i / Lambda_b to 2^-32);
//   * star s is behind the dust screen iff word s mod 4 of Philox(p, b, TAG_STAR_SPLIT, s / 4)
//     is below floor(F 2^32) (F = 1: every star; no dust: none).
// The law of the counts is that of the per-entry rule; the random stream is a different one.
// At low stellar density most blocks draw nothing in every pixel of a wave and cost one Philox
// block and one compare, instead of the per-entry rule's sixteen Philox blocks.
//
// Layout: one lane per pixel as in k_sample; a wave's 64 lanes also hold one block's 64
// cumulative thresholds and entry fluxes in registers, so each star's binary search and flux
// gather are cross-lane reads (ds_bpermute) with no LDS allocation.  Slices interleave blocks
// like k_sample's interleaved 16-entry blocks and write the same partial-sum layout, which
// k_reduce then sums in the same order.
#include "pcmd_device.h"
#include "pcmd_internal.h"

namespace pcmd {

// One wave per block: lane l takes entry SBLK b + l.
__device__ __forceinline__ void prep_block_body(const BlockPrepArgs &a) {
  __shared__ double lam_s[4][SBLK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int b = blockIdx.x * 4 + w;
  if (b >= a.nb) return;  // whole waves only: nothing below synchronises across waves
  const int i = b * SBLK + lane;
  double l = 0.0;
  if (i < a.E) {
    double fv[4];  // every load before the first store
#pragma unroll
    for (int k = 0; k < 4; ++k) {  // band min(k, B - 1) is always in range: no branch around the load
      const float v = a.flux[(size_t)min(k, a.B - 1) * a.E + i];
      fv[k] = k < a.B ? (double)v : 0.0;
    }
    l = a.lam[i];
    for (int k = 0; k < a.BP; ++k) a.fl64[(size_t)i * a.BP + k] = fv[k];
    if (!(l >= 0.0 && l < 4194304.0)) {  // NaN, negative or too large: drawn as zero, reported
      atomicOr(a.status, STATUS_BAD_LAMBDA);
      l = 0.0;
    }
  }
  lam_s[w][lane] = l;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // cum_l: every lane sums the entries 0..l of its block left to right, the order of Lambda_b
  double cum = 0.0;
  for (int k = 0; k <= lane; ++k) cum += lam_s[w][k];
  const double L = __shfl(cum, SBLK - 1, 64);  // Lambda_b = cum_63
  BlockRec r{{0u, 0u, 0u}, KIND_ZERO, (uint32_t)SBLK - 1u, {0u, 0u, 0u}};
  if (a.hybrid && L >= 10.0) {  // hybrid: this block's entries go to the per-point rule
    r.pad[0] = 1u;
  } else if (!(L < 4194304.0)) {  // the block total must stay in the per-entry rule's range
    if (lane == 0) atomicOr(a.status, STATUS_BAD_LAMBDA);
  } else if (L > 0.0) {
    // C_l = floor(2^32 cum_l / Lambda_b); the last entry with stars reaches cum = Lambda_b
    // exactly (same additions), so C = 2^32 from there on
    const double C = floor(cum / L * 4294967296.0);
    const uint64_t full = __ballot(C >= 4294967296.0);  // lane 63 always
    const uint32_t istar = (uint32_t)__builtin_ctzll(full);
    a.cth[(size_t)b * SBLK + lane] = (uint32_t)lane < istar ? (uint32_t)C : 0xFFFFFFFFu;
    r.istar = istar;
    if (lane == 0) {
      if (L >= 10.0) {
        ((PtrsConst *)a.pc)[b] = ptrs_constants(L);
        r.kk = KIND_PTRS;
      } else {
        uint32_t first[3] = {0u, 0u, 0u};
        const uint32_t K = inversion_table(L, a.thr + (size_t)b * THR_STRIDE, 1, first);
        if (K > 0) {
          for (uint32_t k = 0; k < 3 && k < K; ++k) r.T[k] = first[k];
          r.kk = (K << 8) | KIND_INV;
        }
      }
    }
  }
  if (lane == 0) a.brec[b] = r;
}

__global__ void __launch_bounds__(256) k_prep_block(BlockPrepArgs a) { prep_block_body(a); }
// batched: the arguments of job j of a descriptor table
__global__ void __launch_bounds__(256) k_prep_block_job(const BlockPrepArgs *__restrict__ t, int j) {
  const BlockPrepArgs a = t[j];
  prep_block_body(a);
}

hipError_t launch_prep_block(const BlockPrepArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_block, dim3((unsigned)((a.nb + 3) / 4)), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_prep_block_job(const BlockPrepArgs *table, int j, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_block_job, dim3((unsigned)((nb + 3) / 4)), dim3(256), 0, s, table, j);
  return hipGetLastError();
}

template <int B, int S, bool DBG>
__device__ __forceinline__ void sample_block_body(const BlockSampleArgs &a) {
  constexpr int BP = B <= 2 ? 2 : 4;
  const int nblk_px = (a.npx + 255) >> 8;
  const int chunk = blockIdx.x / nblk_px;
  const uint32_t p = (uint32_t)((blockIdx.x - chunk * nblk_px) * 256 + threadIdx.x);
  const uint32_t lane = threadIdx.x & 63u;
  const PCMD_CONST BlockRec *brec = (const PCMD_CONST BlockRec *)a.brec;
  const PCMD_CONST uint32_t *thr = (const PCMD_CONST uint32_t *)a.thr;
  const PCMD_CONST PtrsConst *pc = (const PCMD_CONST PtrsConst *)a.pc;
  const bool live = p < (uint32_t)a.npx;
  const bool dbg = DBG && live && (int64_t)p >= a.px0 && (int64_t)p < a.px1;
  const bool draw_split = S == 2 && (a.split_mode == SPLIT_HALF || a.split_mode == SPLIT_GENERAL);

  double acc_c[B], acc_r[B];
#pragma unroll
  for (int k = 0; k < B; ++k) {
    acc_c[k] = 0.0;
    acc_r[k] = 0.0;
  }
  uint32_t ptrs_failed = 0u;
  // every lane runs every step below (lanes past the image included), so the cross-lane reads
  // always find their source lane active; branches on N go through wave-wide votes
  for (int b = chunk; b < a.nb; b += a.nchunks) {
    const BlockRec r = ld_const(brec + b);
    const uint32_t kind = r.kk & KIND_MASK;
    if (kind == KIND_ZERO) continue;
    uint32_t n = 0u;
    if (kind == KIND_INV) {
      // N = #{k < K : T_k <= u}, walking up while any lane of the wave is still above
      const uint32_t u = philox10(p, (uint32_t)b, TAG_BLOCK, 0u, a.k0, a.k1).x;
      const uint32_t K = r.kk >> 8;
      n = u >= r.T[0] ? 1u : 0u;
      if (!wave_any(n != 0u)) continue;
      for (uint32_t k = 1; k < K; ++k) {
        const uint32_t t = k < 3 ? r.T[k] : thr[(size_t)b * THR_STRIDE + k];
        const uint32_t c = u >= t ? 1u : 0u;
        if (!wave_any(c != 0u)) break;
        n += c;
      }
    } else {
      n = ptrs_draw(ld_const(pc + b), p, (uint32_t)b, TAG_BLOCK_PTRS, a.k0, a.k1, a.lnfact, ptrs_failed);
      if (!wave_any(n != 0u)) continue;
    }
    // the block's thresholds and fluxes, one entry per lane
    const int e = b * SBLK + (int)lane;
    const uint32_t cl = a.cth[(size_t)b * SBLK + lane];
    double fl[B];
#pragma unroll
    for (int k = 0; k < B; ++k) fl[k] = e < a.E ? a.fl64[(size_t)e * BP + k] : 0.0;
    const uint32_t istar = r.istar;
    u4 ws{0u, 0u, 0u, 0u}, wr{0u, 0u, 0u, 0u};
    for (uint32_t s = 0; wave_any(s < n); ++s) {
      if ((s & 3u) == 0u) {
        ws = philox10(p, (uint32_t)b, TAG_STAR, s >> 2, a.k0, a.k1);
        if (draw_split) wr = philox10(p, (uint32_t)b, TAG_STAR_SPLIT, s >> 2, a.k0, a.k1);
      }
      const uint32_t u = word_of(ws, (int)(s & 3u));
      // number of thresholds <= u among the 64 (sorted; the count stops at 63), then capped at
      // istar: the first entry whose threshold exceeds u
      uint32_t pos = 0u;
#pragma unroll
      for (uint32_t st = 32u; st != 0u; st >>= 1) {
        const uint32_t v = (uint32_t)__shfl((int)cl, (int)(pos + st - 1u), 64);
        pos += v <= u ? st : 0u;
      }
      const uint32_t cat = min(pos, istar);
      double f[B];
#pragma unroll
      for (int k = 0; k < B; ++k) f[k] = __shfl(fl[k], (int)cat, 64);
      const bool red = S == 2 && (a.split_mode == SPLIT_ALL || (draw_split && word_of(wr, (int)(s & 3u)) < a.split_q));
      if (s < n) {
        if (red) {
#pragma unroll
          for (int k = 0; k < B; ++k) acc_r[k] += f[k];
        } else {
#pragma unroll
          for (int k = 0; k < B; ++k) acc_c[k] += f[k];
        }
        if (DBG && dbg && b * SBLK + (int)cat < a.E) {  // always true: cat <= istar, an entry with stars
          const size_t o = (size_t)((int64_t)p - a.px0) * (size_t)a.E + (size_t)b * SBLK + cat;
          a.dbg_counts[o] += 1u;
          if (red && a.dbg_red) a.dbg_red[o] += 1u;
        }
      }
    }
  }
  if (wave_any(ptrs_failed != 0u) && lane == 0u) atomicOr(a.status, STATUS_PTRS_RETRY);
  if (!live) return;
  const size_t plane = (size_t)a.npx;
#pragma unroll
  for (int k = 0; k < B; ++k) {
    float *pc = a.part + ((size_t)(chunk * S + 0) * B + k) * plane + p;
    *pc = (float)(a.accumulate ? (double)*pc + acc_c[k] : acc_c[k]);
    if (S == 2) {
      float *pr = a.part + ((size_t)(chunk * S + 1) * B + k) * plane + p;
      *pr = (float)(a.accumulate ? (double)*pr + acc_r[k] : acc_r[k]);
    }
  }
}

template <int B, int S, bool DBG>
__global__ void __launch_bounds__(256) k_sample_block(BlockSampleArgs a) {
  sample_block_body<B, S, DBG>(a);
}
// batched: job j of a descriptor table, both partial streams (as every batch job)
template <int B>
__global__ void __launch_bounds__(256) k_sample_block_job(const BlockSampleArgs *__restrict__ t, int j) {
  const BlockSampleArgs a = t[j];
  sample_block_body<B, 2, false>(a);
}

template <int B>
static hipError_t launch_sample_block_b(const BlockSampleArgs &a, hipStream_t s) {
  const int nblk_px = (a.npx + 255) / 256;
  dim3 grid((unsigned)(nblk_px * a.nchunks));
  const bool dbg = a.dbg_counts != nullptr;
  if (a.S == 2 && dbg)
    hipLaunchKernelGGL((k_sample_block<B, 2, true>), grid, dim3(256), 0, s, a);
  else if (a.S == 2)
    hipLaunchKernelGGL((k_sample_block<B, 2, false>), grid, dim3(256), 0, s, a);
  else if (dbg)
    hipLaunchKernelGGL((k_sample_block<B, 1, true>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_sample_block<B, 1, false>), grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sample_block(const BlockSampleArgs &a, hipStream_t s) {
  switch (a.B) {
    case 1: return launch_sample_block_b<1>(a, s);
    case 2: return launch_sample_block_b<2>(a, s);
    case 3: return launch_sample_block_b<3>(a, s);
    case 4: return launch_sample_block_b<4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_sample_block_job(const BlockSampleArgs *table, int j, int B, int npx, int nchunks, hipStream_t s) {
  const dim3 grid((unsigned)((npx + 255) / 256 * nchunks));
  switch (B) {
    case 1: hipLaunchKernelGGL(k_sample_block_job<1>, grid, dim3(256), 0, s, table, j); break;
    case 2: hipLaunchKernelGGL(k_sample_block_job<2>, grid, dim3(256), 0, s, table, j); break;
    case 3: hipLaunchKernelGGL(k_sample_block_job<3>, grid, dim3(256), 0, s, table, j); break;
    case 4: hipLaunchKernelGGL(k_sample_block_job<4>, grid, dim3(256), 0, s, table, j); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pcmd
