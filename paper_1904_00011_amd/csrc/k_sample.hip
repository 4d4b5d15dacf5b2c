// Weighted entries, per-entry sampler tables, the pixel x entry Poisson sampler with fused
// flux accumulation, and the chunk reduction with the dust / distance epilogue (gfx950).
//
// Sec. 2.1 of the paper: every pixel draws an independent Poisson count for every weighted
// isochrone point, the stars' fluxes are reddened by dust, dimmed by the distance modulus and
// summed into the pixel.  One lane owns one pixel; the entry table is wave-uniform, so it is
// read through the scalar cache.  A wave handles 64 pixels x one chunk of CHUNK entries and
// keeps the per-band sums in FP64 registers; chunk partials are written once, rounded to FP32
// (a relative error of at most 2^-24 per partial, and the partials are non-negative, so the
// pixel sum keeps that bound), and combined in FP64 in ascending chunk order by the reduction
// kernel, which fixes the summation order independently of the launch shape.
#include <math.h>

#include <algorithm>

#include "pcmd_device.h"
#include "pcmd_internal.h"

namespace pcmd {

// ---------------------------------------------------------------------------------------
// a0: lambda_i = scale[iso(i)] * imf_w_i   (scale_k = Npix w_k / sum_k w_k S_k)
// ---------------------------------------------------------------------------------------
struct IsoScale {
  double v[PCMD_MAX_ISO];
};

__global__ void __launch_bounds__(256) k_entries(int E, int n_iso, const int32_t *__restrict__ iso,
                                                 const double *__restrict__ imf_w, IsoScale scale,
                                                 double *__restrict__ lam, uint32_t *__restrict__ status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= E) return;
  const int k = iso[i];
  if (k < 0 || k >= n_iso) {  // malformed grid: no stars, reported by pcmd_sync
    atomicOr(status, STATUS_BAD_LAMBDA);
    lam[i] = 0.0;
    return;
  }
  lam[i] = scale.v[k] * imf_w[i];
}

hipError_t launch_entries(const pcmd_grid *g, const double *scale, double *lam, uint32_t *status, hipStream_t s) {
  IsoScale sc;
  for (int k = 0; k < PCMD_MAX_ISO; ++k) sc.v[k] = k < g->n_iso ? scale[k] : 0.0;
  const int E = g->n_entries;
  hipLaunchKernelGGL(k_entries, dim3((E + 255) / 256), dim3(256), 0, s, E, g->n_iso, g->iso_of_entry, g->imf_w, sc,
                     lam, status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Per-entry tables: inversion thresholds (lambda < ALIAS_MIN), an alias marker (the columns come
// from k_prep_alias) or rejection constants (lambda >= ALIAS_MAX)
// and the FP64 star fluxes, in each entry's record.
// ---------------------------------------------------------------------------------------
__device__ __forceinline__ void prep_body(const PrepArgs &a, int i) {
  // every lane of the block takes part in the group summary below (no early return)
  const int E = a.E, B = a.B;
  EntryRec r{{0xFFFFFFFFu, 0u, 0u}, KIND_ZERO, {0.0, 0.0, 0.0, 0.0}};
  bool red_alias = false;  // the entry is thinned and its reddened part is on the alias rule
  double lam_inv = 0.0;    // lambda of an entry drawn by inversion (the group's density flag)
  if (i < E) {
    // every load before the first store (the output could alias the inputs for the compiler,
    // which otherwise waits for each load in turn)
    double fv[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {  // band min(b, B - 1) is always in range: no branch around the load
      const float v = a.flux[(size_t)min(b, B - 1) * E + i];
      fv[b] = b < B ? (double)v : 0.0;
    }
    double l = a.lam[i];
    const bool block_rule = a.brec && a.brec[i / SBLK].pad[0] == 0u;  // hybrid: the block rule draws it
#pragma unroll
    for (int b = 0; b < 4; ++b) r.fl[b] = fv[b];
    if (!(l >= 0.0 && l < 4194304.0)) {  // NaN, negative or too large: drawn as zero, reported
      atomicOr(a.status, STATUS_BAD_LAMBDA);
      l = 0.0;
    }
    if (block_rule) l = 0.0;
    // thinned: the unreddened and reddened counts are two independent parts
    const bool thin = l >= ALIAS_MIN && (a.thin == THIN_TABLE || (a.thin == THIN_HALF_HIGH && l >= LAM_THIN_HALF));
    if (a.thin != THIN_NONE) a.rdesc[i] = KIND_ZERO;  // overwritten below for a thinned entry
    if (l >= ALIAS_MIN) {
      // table entry: the count (or, thinned, the unreddened part) in slot 0, the reddened part in
      // slot 1; alias parts are built by k_prep_alias, which completes their descriptors
      const double l0 = thin ? l * (1.0 - a.frac) : l;
      if (l0 >= ALIAS_MAX) {
        ((PtrsConst *)a.pc)[2 * (size_t)i] = ptrs_constants(l0);
        r.kk = KIND_PTRS;
      } else {
        r.kk = KIND_ALIAS;
      }
      if (thin) {
        r.kk |= FLAG_THIN;
        if (a.thin_seen) *a.thin_seen = a.gen;  // every writer stores the same value
        const double l1 = l * a.frac;
        if (l1 >= ALIAS_MAX) {
          ((PtrsConst *)a.pc)[2 * (size_t)i + 1] = ptrs_constants(l1);
          a.rdesc[i] = KIND_PTRS;
        } else {
          a.rdesc[i] = KIND_ALIAS;
          // F = 1/2: both halves have the same lambda and so the same table, which k_prep_alias
          // builds once, with the unreddened half, and writes to both slots
          red_alias = a.thin != THIN_HALF_HIGH;
        }
      }
    } else if (l > 0.0) {
      // k-major: threshold k of entry i at thr[k EP + i], so that a wave's stores coalesce
      uint32_t first[3] = {0u, 0u, 0u};
      const uint32_t K = inversion_table(l, a.thr + i, (size_t)entries_padded(E), first);
      if (K > 0) {
        // T_0 >= 1 below ALIAS_MIN, so u >= T_0 is exactly u > T_0 - 1
        r.T[0] = first[0] - 1u;
        for (uint32_t k = 1; k < 3 && k < K; ++k) r.T[k] = first[k];
        r.kk = (K << 8) | KIND_INV;
        lam_inv = l;
      }
    }
  }
  const int EP = entries_padded(E);
  if (i < EP) a.rec[i] = r;
  if (a.alias_list) {
    // the alias parts (i << 1 | part) to the call's list, one reservation per wave; a count word
    // not prepared for this generation (the previous call stopped early) is left alone, and
    // k_prep_alias then walks every entry
    const bool al0 = i < E && (r.kk & KIND_MASK) == KIND_ALIAS, al1 = i < E && red_alias;
    const uint64_t b0 = __ballot(al0), b1 = __ballot(al1);
    const uint32_t cnt = (uint32_t)(__popcll(b0) + __popcll(b1));
    if (cnt != 0u) {
      unsigned long long old = 0ull;
      if ((threadIdx.x & 63u) == 0u) old = atomicAdd(a.alias_n + (a.gen & 1u), (unsigned long long)cnt);
      const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(old >> 32), 0, 64);
      const uint32_t base = (uint32_t)__shfl((int)(uint32_t)old, 0, 64);
      if (hi == a.gen && (uint64_t)base + cnt <= 2ull * (uint64_t)E) {
        const uint64_t below = (1ull << (threadIdx.x & 63u)) - 1ull;
        if (al0) a.alias_list[base + (uint32_t)__popcll(b0 & below)] = (uint32_t)i << 1;
        if (al1) a.alias_list[base + (uint32_t)__popcll(b0) + (uint32_t)__popcll(b1 & below)] = ((uint32_t)i << 1) | 1u;
      }
    }
  }

  // group of entries GRP g .. GRP g + GRP - 1 = neighbouring lanes of one wave (256-thread blocks)
  const uint32_t kind = r.kk & KIND_MASK;
  const uint32_t t0m1 = r.T[0];  // 0xFFFFFFFF unless drawn by inversion
  const uint32_t fl = (r.kk & FLAG_THIN) ? GRP_THIN
                      : kind == KIND_INV ? GRP_INV : kind == KIND_PTRS ? GRP_PTRS : kind == KIND_ALIAS ? GRP_ALIAS : 0u;
  const int first = (int)(threadIdx.x & 63u) & ~(GRP - 1);
  GroupRec gr;
  gr.flags = 0u;
  double gsum = 0.0;
#pragma unroll
  for (int q = 0; q < GRP; ++q) {
    gr.t0m1[q] = (uint32_t)__shfl((int)t0m1, first + q, 64);
    gr.flags |= (uint32_t)__shfl((int)fl, first + q, 64);
    gsum += __shfl(lam_inv, first + q, 64);
  }
  if (64.0 * gsum >= GRP_DENSE_LAMBDA64) gr.flags |= GRP_DENSE;
#pragma unroll
  for (int q = 0; q < 7; ++q) gr.pad[q] = 0u;
  if ((i & (GRP - 1)) == 0 && i < EP) a.grp[i / GRP] = gr;
}

__global__ void __launch_bounds__(256) k_prep(PrepArgs a) { prep_body(a, blockIdx.x * blockDim.x + threadIdx.x); }
__global__ void __launch_bounds__(256) k_prep_job(const PrepArgs *__restrict__ t, int j) {
  const PrepArgs a = t[j];
  prep_body(a, blockIdx.x * blockDim.x + threadIdx.x);
}

// Alias columns of the entries with ALIAS_MIN <= lambda < ALIAS_MAX (rule C1b), one wave per
// entry at a time.  The wave runs the inversion rule's FP64 recurrence without its cap until T_k
// reaches 2^32 - 1 (that threshold then counts as 2^32: the FP64 sum can stall just below 1); with
// k_lo = #{k : T_k = 0}, outcome k_lo + j has mass m_j = T_{k_lo+j} - T_{k_lo+j-1}
// (T_{k_lo-1} = 0).  M = the smallest power of two >= the number of outcomes, at least 16.
// Vose's construction then splits the masses over M columns of 2^32 / M words: "small"
// (m < 2^32 / M) and "large" column stacks, both filled in ascending order; pop s from small and
// l from large, column s keeps height m_s and alias l, m_l -= 2^32 / M - m_s, and l goes back on
// the stack its mass now selects; columns left on the large stack are full (the wave computes the
// same table from prefix sums, below).  All integer: the table selects every outcome on exactly
// m_j of the 2^32 words.  A part so small (below about
// 2^-32) that T_0 already reaches 2^32 - 1 has the single outcome 0: every column then holds
// height 0 and alias 0.  The record keeps k_lo << 12 | log2 M << 8 | KIND_ALIAS.
// Each wave walks entries w, w + W, w + 2W, ... (W = waves in the grid), reusing its LDS: a grid
// of one launch per entry held most of its blocks' LDS for waves without an alias part and
// dispatched tens of thousands of blocks that had nothing to do.
constexpr int ALIAS_WAVES = 4;      // waves per 256-thread block
constexpr int ALIAS_BLOCKS = 1024;  // blocks over both parts: 4 per CU (bound by LDS) on 256 CUs

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sums, in pop order (list position n - 1 - k for pop index k), of the deficits
// cap - m (small) or excesses m - cap (large) of the n listed columns: dst[k] for k < n (every
// partial sum is below 2^32).  Each
// lane sums a run of consecutive pop indices, then a wave scan of the run totals offsets them.
__device__ __forceinline__ void scan_pop_order(const uint16_t *list, int n, const uint32_t *m, uint32_t cap,
                                               bool small, uint32_t *dst, int lane) {
  const int per = (n + 63) >> 6;
  const int k0 = min(n, lane * per), k1 = min(n, k0 + per);
  uint32_t tot = 0u;
  for (int k = k0; k < k1; ++k) {
    const uint32_t c = m[list[n - 1 - k]];
    tot += small ? cap - c : c - cap;
  }
  uint32_t x = tot;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)x, (unsigned)d, 64);
    if (lane >= d) x += y;
  }
  uint32_t run = x - tot;
  for (int k = k0; k < k1; ++k) {
    const uint32_t c = m[list[n - 1 - k]];
    run += small ? cap - c : c - cap;
    dst[k] = run;
  }
}

__device__ __forceinline__ void prep_alias_body(const PrepArgs &a, int i, int part) {
  __shared__ uint32_t m_s[ALIAS_WAVES][ALIAS_COLS];
  __shared__ uint16_t small_s[ALIAS_WAVES][ALIAS_COLS], large_s[ALIAS_WAVES][ALIAS_COLS];
  __shared__ uint32_t D_s[ALIAS_WAVES][ALIAS_COLS + 1], E_s[ALIAS_WAVES][ALIAS_COLS];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (i >= a.E) return;  // whole waves: i is wave-uniform
  // part 0: the entry's count (or its unreddened part); part 1: the reddened part (thinned)
  // (rdesc holds KIND_ZERO for every entry that is not thinned whenever thinning is on)
  // (at F = 1/2 the reddened half's table is the unreddened half's, written with it)
  if (part == 0 ? (a.rec[i].kk & KIND_MASK) != KIND_ALIAS
                : a.thin != THIN_TABLE || (a.rdesc[i] & KIND_MASK) != KIND_ALIAS)
    return;
  uint32_t *m = m_s[wv];
  uint16_t *sm = small_s[wv], *lg = large_s[wv];
  for (int j = lane; j < ALIAS_COLS; j += 64) m[j] = 0u;
  wave_lds_sync();
  // Every lane runs the recurrence on the same values (a wave issues the same instructions for
  // one lane as for 64) and the loop's decisions are read from lane 0 into scalar registers, so
  // its branches are uniform; lane 0 stores the masses.
  const double lam = a.lam[i];
  // part 1 exists only for a thinned entry; part 0 of one is its unreddened share
  const bool thin = part == 1 || (a.rec[i].kk & FLAG_THIN) != 0u;
  // F = 1/2, thinned, and the reddened half also on the alias rule (it has the same lambda): the
  // table goes to both slots and the descriptor to both records
  const bool twin = part == 0 && thin && a.thin == THIN_HALF_HIGH && (a.rdesc[i] & KIND_MASK) == KIND_ALIAS;
  const double l = !thin ? lam : part == 0 ? lam * (1.0 - a.frac) : lam * a.frac;
  double pk = exp(-l);
  double F = pk;
  int klo = -1, J = 0;
  bool single = false;
  uint32_t prev = 0u;
  for (int k = 0;; ++k) {
    // the loop's integers are the same in every lane: said so, they stay in scalar registers
    klo = __builtin_amdgcn_readfirstlane(klo);
    J = __builtin_amdgcn_readfirstlane(J);
    prev = (uint32_t)__builtin_amdgcn_readfirstlane((int)prev);
    if (k > 0) {
      pk = pk * l / (double)k;
      F = F + pk;
    }
    const double t = floor(F * 4294967296.0);
    if (__builtin_amdgcn_readfirstlane(t >= 4294967295.0 ? 1 : 0)) {
      // the last word or more: the rest of the mass goes to outcome k
      if (klo < 0) {  // all of it (a part below about 2^-32): every word draws k
        klo = k;
        single = true;
      } else {
        if (lane == 0) m[J] = 0u - prev;  // 2^32 - T_{k-1}; prev >= 1 here (T_{klo} > 0)
        ++J;
      }
      break;
    }
    // converted before the read (the empty asm keeps the compiler from reading the double and
    // converting in a vector register), so T and everything computed from it stay scalar
    uint32_t Tv = (uint32_t)t;
    asm volatile("" : "+v"(Tv));
    const uint32_t T = (uint32_t)__builtin_amdgcn_readfirstlane((int)Tv);
    if (klo < 0 && T > 0u) klo = k;
    if (klo >= 0) {
      if (lane == 0) m[J] = T - prev;
      ++J;
      prev = T;
      if (J == ALIAS_COLS) {  // wider than the table (not reached below ALIAS_MAX)
        if (lane == 0) atomicOr(a.status, STATUS_BAD_LAMBDA);
        break;
      }
    }
  }
  int bits = 4;
  while ((1 << bits) < J) ++bits;
  if (lane == 0) {
    const uint32_t desc = ((uint32_t)klo << 12) | ((uint32_t)bits << 8) | KIND_ALIAS;
    if (part == 0)
      a.rec[i].kk = desc | (a.rec[i].kk & FLAG_THIN);
    if (part == 1 || twin) a.rdesc[i] = desc;
  }
  wave_lds_sync();
  const int M = 1 << bits;
  const uint32_t cap = 1u << (32 - bits);
  uint32_t *out = a.alias + ((size_t)i * 2 + part) * ALIAS_COLS;
  // column j's word to this part's slot and, for a twin, to the reddened half's slot after it
  auto put = [&](int j, uint32_t word) {
    out[j] = word;
    if (twin) out[ALIAS_COLS + j] = word;
  };
  if (single) {  // one outcome: height 0 and alias 0 in every column, n = k_lo always
    for (int j = lane; j < M; j += 64) put(j, 0u);
    return;
  }
  // stacks in ascending column order: each lane takes one column of every 64, ballots give the
  // positions
  int ns = 0, nl = 0;
  const uint64_t below = (1ull << lane) - 1ull;
  for (int c0 = 0; c0 < M; c0 += 64) {
    const int j = c0 + lane;
    const bool in = j < M;
    const bool is_small = in && m[j] < cap;
    const bool is_large = in && !(m[j] < cap);
    const uint64_t bs = __ballot(is_small), bl = __ballot(is_large);
    if (is_small) sm[ns + __popcll(bs & below)] = (uint16_t)j;
    if (is_large) lg[nl + __popcll(bl & below)] = (uint16_t)j;
    ns += __popcll(bs);
    nl += __popcll(bl);
  }
  wave_lds_sync();
  // Vose's loop pops both lists from the top (highest column first): a large column takes the
  // small columns in pop order until its excess m - cap is used up, then is itself the next small
  // column, taken by the next large one.  With D(i) the deficits cap - m of the first i smalls
  // popped and E(j) the excesses of the first j larges, the i-th small gets the first large j with
  // E(j) >= D(i - 1); the j-th large turns small after the first small a with D(a) > E(j), keeping
  // height cap + E(j) - D(a) and the alias large j + 1; larges that never turn small are full.
  // The sums are exact integers below 2^32 (the total deficit equals the total excess, and that
  // is below M cap = 2^32), so prefix sums and searches give the loop's table exactly, every lane
  // working instead of one walking the loop through LDS.
  uint32_t *Dp = D_s[wv], *Ep = E_s[wv];
  if (lane == 0) Dp[0] = 0u;
  scan_pop_order(sm, ns, m, cap, true, Dp + 1, lane);  // Dp[k] = D(k)
  scan_pop_order(lg, nl, m, cap, false, Ep, lane);     // Ep[j] = E(j + 1)
  wave_lds_sync();
  for (int i = lane; i < ns; i += 64) {  // pop index i: small number i + 1
    const int col = sm[ns - 1 - i];
    const uint32_t need = Dp[i];
    int lo = 0, hi = nl - 1;  // first j with Ep[j] >= need
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Ep[mid] >= need)
        hi = mid;
      else
        lo = mid + 1;
    }
    const uint32_t al = nl > 0 ? (uint32_t)lg[nl - 1 - lo] : (uint32_t)col;  // nl = 0 only for malformed masses
    put(col, (m[col] << bits) | al);
  }
  for (int j = lane; j < nl; j += 64) {  // pop index j: large number j + 1
    const int col = lg[nl - 1 - j];
    const uint32_t ex = Ep[j];
    int lo = 1, hi = ns + 1;  // first k in [1, ns] with Dp[k] > ex (ns + 1: none)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Dp[mid] > ex)
        hi = mid;
      else
        lo = mid + 1;
    }
    // a column whose alias is itself is full (2^32 / M words, stored as 2^32 / M - 1: the last
    // word then falls to the alias, the column itself)
    uint32_t word = ((cap - 1u) << bits) | (uint32_t)col;
    if (lo <= ns && j + 1 < nl) word = ((cap - (Dp[lo] - ex)) << bits) | (uint32_t)lg[nl - 2 - j];  // Dp[lo] - ex <= cap
    put(col, word);
  }
}

__device__ __forceinline__ void prep_alias_walk(const PrepArgs &a) {
  const int w = (int)blockIdx.x * ALIAS_WAVES + (int)(threadIdx.x >> 6), stride = (int)gridDim.x * ALIAS_WAVES;
  if (a.alias_list) {
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0)  // the next call's count word
      a.alias_n[(a.gen + 1u) & 1u] = (unsigned long long)(a.gen + 1u) << 32;
    const unsigned long long v = a.alias_n[a.gen & 1u];
    const uint32_t n = (uint32_t)v;
    // the list, when k_prep filled it in this call and it has at most one part per wave of the
    // first grid row (a longer one, spread by arrival order, balanced worse than the entry walk)
    if ((uint32_t)(v >> 32) == a.gen && n <= (uint32_t)stride && n <= 2u * (uint32_t)a.E) {
      if (blockIdx.y == 0 && w < (int)n) {
        const uint32_t it = a.alias_list[w];
        prep_alias_body(a, (int)(it >> 1), (int)(it & 1u));
      }
      return;
    }
  }
  for (int i = w; i < a.E; i += stride) prep_alias_body(a, i, (int)blockIdx.y);  // grid.y: the part
}
__global__ void __launch_bounds__(64 * ALIAS_WAVES) k_prep_alias(PrepArgs a) { prep_alias_walk(a); }
__global__ void __launch_bounds__(64 * ALIAS_WAVES) k_prep_alias_job(const PrepArgs *__restrict__ t, int j) {
  const PrepArgs a = t[j];
  prep_alias_walk(a);
}

static dim3 prep_alias_grid(int E, int parts) {
  const int per_part = ALIAS_BLOCKS / parts;
  return dim3((unsigned)std::min((E + ALIAS_WAVES - 1) / ALIAS_WAVES, per_part), (unsigned)parts);
}
hipError_t launch_prep_alias(const PrepArgs &a, hipStream_t s) {
  // grid.y: part 1 (the reddened part of a thinned entry) has a table of its own only when
  // 0 < F < 1 and F != 1/2
  hipLaunchKernelGGL(k_prep_alias, prep_alias_grid(a.E, a.thin == THIN_TABLE ? 2 : 1), dim3(64 * ALIAS_WAVES), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_prep_alias_job(const PrepArgs *table, int j, int E, int parts, hipStream_t s) {
  if (parts != 1 && parts != 2) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_prep_alias_job, prep_alias_grid(E, parts), dim3(64 * ALIAS_WAVES), 0, s, table, j);
  return hipGetLastError();
}

hipError_t launch_prep(const PrepArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_prep, dim3((a.E + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_prep_job(const PrepArgs *table, int j, int E, hipStream_t s) {
  hipLaunchKernelGGL(k_prep_job, dim3((E + 255) / 256), dim3(256), 0, s, table, j);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Sampler.
// ---------------------------------------------------------------------------------------

__device__ __forceinline__ uint32_t low_mask(uint32_t cnt) { return cnt >= 32u ? 0xFFFFFFFFu : ((1u << cnt) - 1u); }

// Reddened stars among n (dust split).  F = 1/2: one bit per star, the first 8 from the
// entry's byte of its 16-entry split block, the rest from (p, i, TAG_SPLIT_X, j) blocks.
// Other fractions: star s compares word s mod 4 of (p, i, TAG_SPLIT_X, s / 4) with fq.
constexpr uint32_t SPLIT_FIRST_BITS = 8;

__device__ __forceinline__ uint32_t split_count(uint32_t n, uint32_t word, uint32_t shift, int mode, uint32_t fq,
                                                uint32_t p, uint32_t i, uint32_t k0, uint32_t k1) {
  if (mode == SPLIT_ALL) return n;
  if (mode == SPLIT_NONE) return 0u;
  uint32_t red = 0;
  if (mode == SPLIT_HALF) {
    // no lane with more than one star (most entries of a sparse field): the byte's first bit
    if (!wave_any(n > 1u)) return n & __builtin_amdgcn_ubfe(word, shift, 1u);
    // no lane with more stars than the byte has bits
    if (!wave_any(n > SPLIT_FIRST_BITS)) return __popc(__builtin_amdgcn_ubfe(word, shift, n));
    // the entry's byte sits at bit `shift` of `word`; its low min(n, 8) bits decide the first stars
    red = __popc(__builtin_amdgcn_ubfe(word, shift, min(n, SPLIT_FIRST_BITS)));
    const uint32_t extra = n > SPLIT_FIRST_BITS ? n - SPLIT_FIRST_BITS : 0u;
    for (uint32_t j = 0; wave_any(extra > 128u * j); ++j) {
      const u4 x = philox10(p, i, TAG_SPLIT_X, j, k0, k1);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint32_t base = 128u * j + 32u * (uint32_t)q;
        const uint32_t cnt = extra > base ? min(extra - base, 32u) : 0u;
        red += __popc(word_of(x, q) & low_mask(cnt));
      }
    }
    return red;
  }
  for (uint32_t j = 0; wave_any(n > 4u * j); ++j) {
    const u4 x = philox10(p, i, TAG_SPLIT_X, j, k0, k1);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t st = 4u * j + (uint32_t)q;
      red += (n > st && word_of(x, q) < fq) ? 1u : 0u;
    }
  }
  return red;
}

// Poisson count of one table part: desc = k_lo << 12 | log2 M << 8 | KIND_ALIAS (one column of
// the alias table: n = k_lo + (c if r < height_c else alias_c), u = c << (32 - b) | r) or
// KIND_PTRS (transformed rejection on (p, i, tag, j) with the part's constants).
__device__ __forceinline__ uint32_t alias_column_of(uint32_t desc, uint32_t u) { return u >> (32u - ((desc >> 8) & 0xFu)); }
// the count from column word x of the column that u selects
__device__ __forceinline__ uint32_t alias_count(uint32_t desc, uint32_t u, uint32_t x) {
  const uint32_t b = (desc >> 8) & 0xFu;
  const uint32_t c = u >> (32u - b);
  return (desc >> 12) + ((u & (0xFFFFFFFFu >> b)) < (x >> b) ? c : (x & ((1u << b) - 1u)));
}

__device__ __forceinline__ uint32_t table_draw(uint32_t desc, uint32_t u, const uint32_t *__restrict__ tab,
                                               const PCMD_CONST PtrsConst *pcp, uint32_t p, uint32_t i, uint32_t tag,
                                               uint32_t k0, uint32_t k1, const float *__restrict__ lnfact,
                                               uint32_t &failed) {
  if ((desc & KIND_MASK) == KIND_ALIAS) return alias_count(desc, u, tab[alias_column_of(desc, u)]);
  const PtrsConst cst = ld_const(pcp);
  return ptrs_draw(cst, p, i, tag, k0, k1, lnfact, failed);
}

// The thinned entries of quad q0 .. q0 + 3 in the thinned-entry pass (F = 1/2), with the quad's
// inversion words w: the same counts and sums as the entry-by-entry path, but the column reads of
// every alias part of the quad (up to eight) are issued before the first is used, so that their
// latencies overlap instead of adding up.
template <int B, bool DBG>
__device__ __forceinline__ void thin_quad(const SampleArgs &a, uint32_t q0, const u4 &w, uint32_t p, bool dbg,
                                          double (&acc_c)[B], double (&acc_r)[B], uint32_t &ptrs_failed) {
  const PCMD_CONST EntryRec *rec = (const PCMD_CONST EntryRec *)a.rec;
  const PCMD_CONST PtrsConst *pc = (const PCMD_CONST PtrsConst *)a.pc;
  const PCMD_CONST uint32_t *rdesc = (const PCMD_CONST uint32_t *)a.rdesc;
  uint32_t kk[4], d[4];
  bool any = false;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    kk[q] = rec[q0 + q].kk;  // q0 + 3 < EP: the table is padded to whole groups
    d[q] = (kk[q] & FLAG_THIN) ? rdesc[q0 + q] : 0u;
    any = any || (kk[q] & FLAG_THIN);
  }
  if (!any) return;
  // the quad's reddened-part words: counters (p, i / 4, TAG_RED, 0)
  const u4 wr = philox10(p, q0 >> 2, TAG_RED, 0u, a.k0, a.k1);
  uint32_t x0[4], x1[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const size_t i = q0 + (uint32_t)q;
    x0[q] = 0u;
    x1[q] = 0u;
    if (!(kk[q] & FLAG_THIN)) continue;
    if ((kk[q] & KIND_MASK) == KIND_ALIAS) x0[q] = a.alias[i * 2 * ALIAS_COLS + alias_column_of(kk[q], word_of(w, q))];
    if ((d[q] & KIND_MASK) == KIND_ALIAS)
      x1[q] = a.alias[(i * 2 + 1) * ALIAS_COLS + alias_column_of(d[q], word_of(wr, q))];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (!(kk[q] & FLAG_THIN)) continue;
    const uint32_t i = q0 + (uint32_t)q;
    const uint32_t nc = (kk[q] & KIND_MASK) == KIND_ALIAS
                            ? alias_count(kk[q], word_of(w, q), x0[q])
                            : ptrs_draw(ld_const(pc + 2 * (size_t)i), p, i, TAG_PTRS, a.k0, a.k1, a.lnfact, ptrs_failed);
    const uint32_t red = (d[q] & KIND_MASK) == KIND_ALIAS
                             ? alias_count(d[q], word_of(wr, q), x1[q])
                             : ptrs_draw(ld_const(pc + 2 * (size_t)i + 1), p, i, TAG_PTRS_RED, a.k0, a.k1, a.lnfact,
                                         ptrs_failed);
    if (DBG && dbg) {
      const size_t o = (size_t)((int64_t)p - a.px0) * (size_t)a.E + i;
      a.dbg_counts[o] = nc + red;
      if (a.dbg_red) a.dbg_red[o] = red;
    }
    if (!wave_any(nc + red != 0u)) continue;
    const PCMD_CONST double *f = rec[i].fl;
    double fv[B];
#pragma unroll
    for (int b = 0; b < B; ++b) fv[b] = f[b];
    {
      const double dc = (double)nc;
#pragma unroll
      for (int b = 0; b < B; ++b) acc_c[b] = fma(dc, fv[b], acc_c[b]);
    }
    if (wave_any(red != 0u)) {
      const double dr = (double)red;
#pragma unroll
      for (int b = 0; b < B; ++b) acc_r[b] = fma(dr, fv[b], acc_r[b]);
    }
  }
}

// PASS (SamplePass): PASS_ALL draws every entry, the thinned ones (FLAG_THIN: two independent
// parts, k_prep's choice under a split 0 < F < 1) inline; PASS_MAIN leaves the thinned ones out,
// and PASS_THIN then draws only those and adds them to the partial sums PASS_MAIN stored, so the
// thinning code (live state that slows the common path) is not in the main pass.
template <int B, int S, bool DBG, int PASS>
__device__ __forceinline__ void sample_tile(const SampleArgs &a, uint32_t p, int chunk) {
  const PCMD_CONST EntryRec *rec = (const PCMD_CONST EntryRec *)a.rec;
  const PCMD_CONST uint32_t *thr = (const PCMD_CONST uint32_t *)a.thr;
  const PCMD_CONST PtrsConst *pc = (const PCMD_CONST PtrsConst *)a.pc;
  const PCMD_CONST uint32_t *rdesc = (const PCMD_CONST uint32_t *)a.rdesc;
  const bool live = p < (uint32_t)a.npx;
  const bool dbg = DBG && live && (int64_t)p >= a.px0 && (int64_t)p < a.px1;

  double acc_c[B], acc_r[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    acc_c[b] = 0.0;
    acc_r[b] = 0.0;
  }

  u4 sw{0u, 0u, 0u, 0u};
  int split_blk = -1;         // the 16-entry block whose split bits sw holds
  uint32_t ptrs_failed = 0u;  // per lane, kept in a vector register
  const PCMD_CONST GroupRec *grp = (const PCMD_CONST GroupRec *)a.grp;
  // Slice `chunk` of nchunks takes the 16-entry blocks chunk, chunk + nchunks, chunk + 2 nchunks,
  // ...: every slice then spans all isochrones and masses, so slices cost about the same (runs
  // of consecutive entries differ in cost several-fold: high-lambda low-mass stars cluster at the
  // start of each isochrone).  The j-th group of GRP entries of the slice is group
  // slice_group(j) of the table.
  const int ngrp = entries_padded(a.E) / GRP;
  const int stride = a.nchunks * (16 / GRP);
  auto slice_group = [&](int j) { return chunk * (16 / GRP) + (j >> 1) * stride + (j & 1); };
  static_assert(GRP == 8, "two groups per 16-entry block");
  const int lane = (int)(threadIdx.x & 63u);
  for (int jb = 0; slice_group(jb) < ngrp; jb += 64) {
    // lane l reads the flags of the slice's group jb + l: one vector load finds the groups with
    // entries to draw among the next 64, where one dependent scalar load per group kept a wave
    // waiting through runs of groups with nothing to draw (pruned isochrones; the hybrid
    // sampler's block-rule entries)
    const int gl = slice_group(jb + lane);
    const uint32_t fl = gl < ngrp ? grp[gl].flags : 0u;
    const uint32_t want = PASS == PASS_ALL ? 0xFFu : PASS == PASS_MAIN ? (GRP_INV | GRP_PTRS | GRP_ALIAS) : GRP_THIN;
    for (uint64_t pend = __ballot((fl & want) != 0u); pend != 0ull; pend &= pend - 1ull) {
      const int lsel = (int)__builtin_ctzll(pend);  // wave-uniform
      // slice_group(jb + lsel), read from lane lsel: one vector instruction instead of seven scalar
      const int gi = __builtin_amdgcn_readlane(gl, lsel);
      const int g0 = gi * GRP;
      const PCMD_CONST GroupRec *gr = grp + gi;
      // at small lambda most groups end after two Philox blocks and eight compares, without
      // touching the entry records
      const uint32_t flags = (uint32_t)__builtin_amdgcn_readlane((int)fl, lsel);
      // inversion words of the group's two quads: counters (p, i / 4, TAG_MAIN, 0)
      const u4 wa = philox10(p, (uint32_t)(2 * gi), TAG_MAIN, 0u, a.k0, a.k1);
      const u4 wb = philox10(p, (uint32_t)(2 * gi + 1), TAG_MAIN, 0u, a.k0, a.k1);
      // the first thresholds are loaded only now: held across the Philox rounds they pushed the
      // scalar register file into spilling inside this loop
      __builtin_amdgcn_sched_barrier(0);
      if (PASS != PASS_THIN && !(flags & (GRP_PTRS | GRP_ALIAS | GRP_DENSE | (PASS == PASS_ALL ? GRP_THIN : 0u))) &&
          (__ballot(wa.x > gr->t0m1[0]) | __ballot(wa.y > gr->t0m1[1]) | __ballot(wa.z > gr->t0m1[2]) |
           __ballot(wa.w > gr->t0m1[3]) | __ballot(wb.x > gr->t0m1[4]) | __ballot(wb.y > gr->t0m1[5]) |
           __ballot(wb.z > gr->t0m1[6]) | __ballot(wb.w > gr->t0m1[7])) == 0ull)
        continue;
      if (PASS == PASS_THIN) {
#pragma unroll
        for (int h = 0; h < 2; ++h) thin_quad<B, DBG>(a, (uint32_t)(g0 + 4 * h), h ? wb : wa, p, dbg, acc_c, acc_r, ptrs_failed);
        continue;
      }
      // the split bits of the group's 16-entry block: a slow group almost always has a star to
      // split, and the two groups of a block share them
      if (S == 2 && PASS != PASS_THIN && a.split_mode == SPLIT_HALF && split_blk != (gi >> 1)) {
        sw = philox10(p, (uint32_t)(gi >> 1), TAG_SPLIT, 0u, a.k0, a.k1);
        split_blk = gi >> 1;
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int q0 = g0 + 4 * h;  // first entry of the quad
        const u4 &w = h ? wb : wa;
        const uint32_t sq = word_of(sw, 2 * (gi & 1) + h);  // the quad's word of the split block
        u4 wr{0u, 0u, 0u, 0u};  // thinned entries: the quad's reddened-part words
        bool wr_ok = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint32_t i = (uint32_t)(q0 + q);
          // one record at a time keeps the scalar registers of the loop below the spill point
          const EntryHead rq = ld_const((const PCMD_CONST EntryHead *)(rec + i));  // padded to a multiple of GRP
          uint32_t n = 0, red_thin = 0u;
          bool thinned = false;
          // a pass leaves out the entries of the other pass (wave-uniform: the record is)
          if (PASS == PASS_MAIN && (rq.kk & FLAG_THIN)) continue;
          if (PASS == PASS_THIN && !(rq.kk & FLAG_THIN)) continue;
          const uint32_t kind = rq.kk & KIND_MASK;
          if (kind <= KIND_INV) {  // inversion; a KIND_ZERO entry never passes its first threshold
            // n = #{k < K : T_k <= u}, walking up while any lane of the wave is still above
            const uint32_t u = word_of(w, q);
            const uint32_t K = rq.kk >> 8;
            n = u > rq.T[0] ? 1u : 0u;
            if (!wave_any(n != 0u)) continue;
            if (K > 1) {
              uint32_t c = u >= rq.T[1] ? 1u : 0u;
              if (wave_any(c != 0u)) {
                n += c;
                if (K > 2) {
                  c = u >= rq.T[2] ? 1u : 0u;
                  if (wave_any(c != 0u)) {
                    n += c;
                    const PCMD_CONST uint32_t *t = thr + i;  // threshold k at t[k EP]
                    const size_t ep = (size_t)entries_padded(a.E);
                    for (uint32_t k = 3; k < K; ++k) {
                      c = u >= t[k * ep] ? 1u : 0u;
                      if (!wave_any(c != 0u)) break;
                      n += c;
                    }
                  }
                }
              }
            }
          } else {
            // table entry: slot 0 holds the count (or, thinned, the unreddened part), slot 1 the
            // reddened part, each an alias column read or a rejection draw
            n = table_draw(rq.kk, word_of(w, q), a.alias + (size_t)i * 2 * ALIAS_COLS, pc + 2 * (size_t)i, p, i,
                           TAG_PTRS, a.k0, a.k1, a.lnfact, ptrs_failed);
            if (S == 2 && PASS != PASS_MAIN && (rq.kk & FLAG_THIN)) {
              if (!wr_ok) {  // the quad's reddened-part words, drawn once
                wr = philox10(p, i >> 2, TAG_RED, 0u, a.k0, a.k1);
                wr_ok = true;
              }
              const uint32_t d = ld_const(rdesc + i);
              red_thin = table_draw(d, word_of(wr, q), a.alias + ((size_t)i * 2 + 1) * ALIAS_COLS, pc + 2 * (size_t)i + 1,
                                    p, i, TAG_PTRS_RED, a.k0, a.k1, a.lnfact, ptrs_failed);
              n += red_thin;
              thinned = true;
            }
          }
          if (!wave_any(n != 0u)) continue;
          uint32_t red = 0u;
          if (S == 2) {
            red = PASS != PASS_MAIN && thinned ? red_thin
                                                : split_count(n, sq, 8u * q, a.split_mode, a.split_q, p, i, a.k0, a.k1);
          }
          // the entry's fluxes, loaded once for both streams
          const PCMD_CONST double *f = rec[i].fl;
          double fv[B];
#pragma unroll
          for (int b = 0; b < B; ++b) fv[b] = f[b];
          // the unreddened stream has a star whenever the entry has one, nearly always: added
          // without a test (zero counts add exact zeros); the reddened stream is skipped when no
          // lane has a reddened star
          const uint32_t nc = n - red;
          {
            const double dc = (double)nc;
#pragma unroll
            for (int b = 0; b < B; ++b) acc_c[b] = fma(dc, fv[b], acc_c[b]);
          }
          if (S == 2 && wave_any(red != 0u)) {
            const double dr = (double)red;
#pragma unroll
            for (int b = 0; b < B; ++b) acc_r[b] = fma(dr, fv[b], acc_r[b]);
          }
          if (DBG && dbg) {
            const size_t o = (size_t)((int64_t)p - a.px0) * (size_t)a.E + i;
            a.dbg_counts[o] = n;
            if (a.dbg_red) a.dbg_red[o] = red;
          }
        }
      }
    }
  }
  if (wave_any(ptrs_failed != 0u) && (threadIdx.x & 63) == 0) atomicOr(a.status, STATUS_PTRS_RETRY);
  if (!live) return;
  const size_t plane = (size_t)a.npx;
#pragma unroll
  for (int b = 0; b < B; ++b) {
    float *pc = a.part + ((size_t)(chunk * S + 0) * B + b) * plane + p;
    float *pr = a.part + ((size_t)(chunk * S + 1) * B + b) * plane + p;
    if (PASS == PASS_THIN) {  // exact zeros change nothing: a slice without thinned stars skips
      if (acc_c[b] != 0.0) *pc = (float)((double)*pc + acc_c[b]);
      if (S == 2 && acc_r[b] != 0.0) *pr = (float)((double)*pr + acc_r[b]);
    } else {
      *pc = (float)acc_c[b];
      if (S == 2) *pr = (float)acc_r[b];
    }
  }
}

// The scalar unit issues about as many instructions as the vector unit here, so scalar-load
// latency is hidden by other waves: the sampler kernels are held to the 80 scalar registers that
// allow 8 waves per SIMD (the compiler moves the rest into vector-register lanes), which measured
// faster than 7 waves without those moves.
template <int B, int S, bool DBG, int PASS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_sample(SampleArgs a) {
  if (PASS == PASS_THIN && a.thin_seen && *(const PCMD_CONST uint32_t *)a.thin_seen != a.gen) return;  // nothing thinned
  const int nblk_px = (a.npx + 255) >> 8;
  const int chunk = blockIdx.x / nblk_px;
  sample_tile<B, S, DBG, PASS>(a, (uint32_t)((blockIdx.x - chunk * nblk_px) * 256 + threadIdx.x), chunk);
}

template <int B, int PASS>
static void launch_sample_pass(const SampleArgs &a, dim3 grid, hipStream_t s) {
  const bool dbg = a.dbg_counts != nullptr;
  if (a.S == 2 && dbg)
    hipLaunchKernelGGL((k_sample<B, 2, true, PASS>), grid, dim3(256), 0, s, a);
  else if (a.S == 2)
    hipLaunchKernelGGL((k_sample<B, 2, false, PASS>), grid, dim3(256), 0, s, a);
  else if (dbg)
    hipLaunchKernelGGL((k_sample<B, 1, true, PASS_MAIN>), grid, dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_sample<B, 1, false, PASS_MAIN>), grid, dim3(256), 0, s, a);
}

// Thinning of every table entry (0 < F < 1, F != 1/2): one pass with the thinned entries inline.
// F = 1/2 (only entries at lambda >= LAM_THIN_HALF thinned): the main pass, then the thinned
// entries' pass.  Otherwise nothing is thinned: the main pass alone.
template <int B>
static hipError_t launch_sample_b(const SampleArgs &a, hipStream_t s) {
  const int nblk_px = (a.npx + 255) / 256;
  dim3 grid((unsigned)(nblk_px * a.nchunks));
  const int tm = a.S == 2 ? thin_mode_of_split(a.split_mode) : THIN_NONE;
  if (tm == THIN_TABLE) {
    launch_sample_pass<B, PASS_ALL>(a, grid, s);
  } else {
    launch_sample_pass<B, PASS_MAIN>(a, grid, s);
    if (tm == THIN_HALF_HIGH) {
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      launch_sample_pass<B, PASS_THIN>(a, grid, s);
    }
  }
  return hipGetLastError();
}

hipError_t launch_sample(const SampleArgs &a, hipStream_t s) {
  switch (a.B) {
    case 1: return launch_sample_b<1>(a, s);
    case 2: return launch_sample_b<2>(a, s);
    case 3: return launch_sample_b<3>(a, s);
    case 4: return launch_sample_b<4>(a, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------------------
// Persistent batched sampler.  Workgroups take tiles (job, pixel block, chunk) from one atomic
// counter until none is left; jobs appear in the table in execution order (the host puts the
// most expensive first) and each job's tiles are contiguous items, pixel block fastest.  Every
// tile is computed exactly as by k_sample, so the schedule never changes a result.
// ---------------------------------------------------------------------------------------
__global__ void k_reset_counter(uint32_t *c) { *c = 0u; }

hipError_t launch_reset_counter(uint32_t *counter, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_counter, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

// Persistent batched sampler: every wave takes (job, 64-pixel block, slice) items from one
// atomic counter until none is left, so no wave waits for another (items of one job are
// consecutive; jobs come in the host's order).
template <int B>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8))) k_sample_persistent(const BatchSampleJob *__restrict__ jobs, int n_jobs,
                                                           int total_items, uint32_t *__restrict__ counter) {
  const PCMD_CONST BatchSampleJob *cj = (const PCMD_CONST BatchSampleJob *)jobs;
  const uint32_t lane = threadIdx.x & 63u;
  for (;;) {
    uint32_t got = 0u;
    if (lane == 0) got = atomicAdd(counter, 1u);
    const int item = (int)__builtin_amdgcn_readfirstlane(got);
    if (item >= total_items) break;
    // job owning the item: last job with item0 <= item (binary search over the table)
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (cj[mid].item0 <= item)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int j = __builtin_amdgcn_readfirstlane(lo);
    const int local = item - cj[j].item0;
    const int pblocks = cj[j].pblocks;  // 64-pixel blocks of the job
    const int chunk = local / pblocks;
    const int pblk = local - chunk * pblocks;
    const SampleArgs a = ld_const(&cj[j].a);
    // batch jobs always carry two streams; F = 1/2 jobs draw their thinned entries afterwards in
    // a launch of their own (k_sample_thin_job), as pcmd_simulate does
    if (thin_mode_of_split(a.split_mode) == THIN_TABLE)
      sample_tile<B, 2, false, PASS_ALL>(a, (uint32_t)(pblk * 64) + lane, chunk);
    else
      sample_tile<B, 2, false, PASS_MAIN>(a, (uint32_t)(pblk * 64) + lane, chunk);
  }
}

// The thinned entries' pass of one batch job (position t of the persistent sampler's table); a
// job whose k_prep thinned nothing returns on one scalar load.  Held to 8 waves per SIMD like the
// other sampler kernels (the compiler's own choice, 7 with 106 scalar registers, ran the uneven
// batch 2.5% slower).  One persistent launch over the items of all listed jobs, as for the main
// pass, measured 8% slower than these launches.
template <int B>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_sample_thin_job(const BatchSampleJob *__restrict__ jobs, int t) {
  const SampleArgs a = jobs[t].a;
  if (a.thin_seen && *(const PCMD_CONST uint32_t *)a.thin_seen != a.gen) return;  // nothing thinned
  const int nblk_px = (a.npx + 255) >> 8;
  const int chunk = blockIdx.x / nblk_px;
  sample_tile<B, 2, false, PASS_THIN>(a, (uint32_t)((blockIdx.x - chunk * nblk_px) * 256 + threadIdx.x), chunk);
}

hipError_t launch_sample_thin_job(const BatchSampleJob *jobs, int t, int B, int npx, int nchunks, hipStream_t s) {
  const dim3 grid((unsigned)((npx + 255) / 256 * nchunks));
  switch (B) {
    case 1: hipLaunchKernelGGL(k_sample_thin_job<1>, grid, dim3(256), 0, s, jobs, t); break;
    case 2: hipLaunchKernelGGL(k_sample_thin_job<2>, grid, dim3(256), 0, s, jobs, t); break;
    case 3: hipLaunchKernelGGL(k_sample_thin_job<3>, grid, dim3(256), 0, s, jobs, t); break;
    case 4: hipLaunchKernelGGL(k_sample_thin_job<4>, grid, dim3(256), 0, s, jobs, t); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sample_persistent(const BatchSampleJob *jobs, int n_jobs, int total_items, int B, uint32_t *counter,
                                    int n_workgroups, hipStream_t s) {
  dim3 grid((unsigned)n_workgroups);
  switch (B) {
    case 1: hipLaunchKernelGGL(k_sample_persistent<1>, grid, dim3(256), 0, s, jobs, n_jobs, total_items, counter); break;
    case 2: hipLaunchKernelGGL(k_sample_persistent<2>, grid, dim3(256), 0, s, jobs, n_jobs, total_items, counter); break;
    case 3: hipLaunchKernelGGL(k_sample_persistent<3>, grid, dim3(256), 0, s, jobs, n_jobs, total_items, counter); break;
    case 4: hipLaunchKernelGGL(k_sample_persistent<4>, grid, dim3(256), 0, s, jobs, n_jobs, total_items, counter); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Slice reduction + epilogue: F_b = 10^(-0.4 mu_d) (F_clr_b + F_red_b 10^(-0.4 R_b E_p)).
// One thread per (band, pixel); the partials of all slices are loaded in batches of eight
// before they are added, in ascending slice order (the order fixes the rounding).
// ---------------------------------------------------------------------------------------
constexpr int RED_BATCH = 8;

__device__ __forceinline__ void reduce_body(const ReduceArgs &a, int idx) {
  const int npx = a.npx;
  if (idx >= a.B * npx) return;
  const int b = idx / npx, p = idx - b * npx;
  const size_t plane = (size_t)npx;
  const size_t step = (size_t)a.S * a.B * plane;  // from one slice to the next
  const float *pc = a.part + (size_t)b * plane + p;
  const float *pr = pc + (size_t)a.B * plane;  // reddened stream (S == 2)
  double c = 0.0, r = 0.0;
  int ch = 0;
  for (; ch + RED_BATCH <= a.nchunks; ch += RED_BATCH) {
    double xc[RED_BATCH], xr[RED_BATCH];
#pragma unroll
    for (int k = 0; k < RED_BATCH; ++k) {
      xc[k] = (double)pc[(size_t)(ch + k) * step];
      xr[k] = a.S == 2 ? (double)pr[(size_t)(ch + k) * step] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < RED_BATCH; ++k) {
      c += xc[k];
      r += xr[k];
    }
  }
  for (; ch < a.nchunks; ++ch) {
    c += (double)pc[(size_t)ch * step];
    if (a.S == 2) r += (double)pr[(size_t)ch * step];
  }
  double F;
  if (a.dust_model == PCMD_DUST_NONE) {
    F = a.dist * (c + r);
  } else {
    double ebv;
    if (a.dust_model == PCMD_DUST_SCREEN) {
      ebv = exp10(a.dust_mu);
    } else {
      const u4 w = philox10((uint32_t)p, 0u, TAG_DUST, 0u, a.k0, a.k1);
      ebv = exp10(a.dust_mu + a.dust_sigma * box_muller(w.x, w.y));
    }
    F = a.dist * (c + r * exp10(-0.4 * a.dust_R[b] * ebv));
  }
  a.F[(size_t)b * plane + p] = (float)F;
}

__global__ void __launch_bounds__(256) k_reduce(ReduceArgs a) { reduce_body(a, blockIdx.x * blockDim.x + threadIdx.x); }
__global__ void __launch_bounds__(256) k_reduce_job(const ReduceArgs *__restrict__ t, int j) {
  const ReduceArgs a = t[j];
  reduce_body(a, blockIdx.x * blockDim.x + threadIdx.x);
}

hipError_t launch_reduce(const ReduceArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3((a.B * a.npx + 255) / 256), dim3(256), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_reduce_job(const ReduceArgs *table, int j, int npx, int B, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_job, dim3((B * npx + 255) / 256), dim3(256), 0, s, table, j);
  return hipGetLastError();
}

}  // namespace pcmd
