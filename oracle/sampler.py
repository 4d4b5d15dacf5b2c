"""Per-pixel Poisson star counts and pixel fluxes (oracle side).

Sec. 2.1: for every pixel of an Nim x Nim image the number of stars at each
weighted isochrone point is an independent Poisson draw with the point's weight
as its mean; the stars' fluxes are reddened by dust, dimmed by the distance
modulus and summed into the pixel.  Sec. 2.2 (dust models E1-E3): a thin dust
screen with log E(B-V) fixed (E1) or log-normal per pixel (E2/E3), covering a
fraction F_dust of the stars; distance enters as the distance modulus mu_d.

How a Poisson count is drawn is not fixed by the paper.  The rule here:

* C1, lambda < 2 -- inversion in the integer domain.  p_0 = exp(-lambda),
  p_k = p_{k-1} * lambda / k, F_k = F_{k-1} + p_k (FP64, in that order);
  T_k = floor(F_k * 2^32).  K is the first k with T_k >= 2^32 - 1, or 63; that
  threshold counts as 2^32, so outcome K takes the last word too (the FP64 sum can
  stall just below 1, where floor(F 2^32) = 2^32 - 1: ending there keeps the
  largest word from reaching a count the Poisson law gives less than 2^-32).  With
  u a 32-bit word, n = #{k < K : T_k <= u}, i.e. the least k with u < T_k (T_K =
  2^32).  Exact to 2^-32 per outcome; a point with lambda below about 2^-32 has
  K = 0 and never draws a star (the rule's 2^-32 floor).  (The block-skip
  sampler's block totals use this rule below lambda = 10.)
* C1b, 2 <= lambda < 512 -- the same quantised law by an integer alias table
  (Walker 1977; construction of Vose 1991).  The C1 recurrence, uncapped, runs
  until T_k >= 2^32 - 1; that last threshold is taken as 2^32 (so the outcome
  takes the last word too: the FP64 sum can stall just below 1).  With k_lo = #{k : T_k = 0}, outcome k_lo + j has
  mass m_j = T_{k_lo+j} - T_{k_lo+j-1} (T_{k_lo-1} = 0).  M = the smallest power
  of two >= the number of outcomes, at least 16; column j of M holds height
  h_j <= 2^32/M and alias a_j; with u the entry's inversion word, column
  c = u >> (32 - log2 M) and r = u mod 2^(32 - log2 M), n = k_lo + (c if r < h_c
  else a_c).  Vose's construction in integers: columns with m_j < 2^32/M on a
  "small" stack, the rest on a "large" stack, both pushed in ascending j;
  repeatedly pop s from small and l from large, set h_s = m_s, a_s = l,
  m_l -= 2^32/M - m_s and push l on the stack its new mass selects; columns left
  on large get h = 2^32/M, a = j.  Every outcome then has exactly mass m_j over
  the 2^32 words (exact to 2^-32, like C1), at one table read per draw.
* C2, lambda >= 512 -- transformed rejection with squeeze (Hormann 1993, "The
  transformed rejection method for generating Poisson random variables"),
  decisions taken in IEEE FP32 operation by operation, with a logarithm written
  here from the atanh series and ln k! from an FP64-built table (k < 256) or a
  Stirling series.  Both sides of the parity test take the same FP32 steps.
* C3b, thinning -- for an entry drawn by C1b or C2 under a split 0 < F < 1 --
  every such entry (lambda >= 2) when F is not 1/2; at F = 1/2 the entries with
  lambda >= 4, the lowest lambda whose halves still take the alias rule (below
  that nearly all stars take bits of a block shared by 16 entries; from about
  there on most entries have more stars than those 8 bits, and the rest would
  each need a bit of a block of their own) -- the unreddened and reddened counts
  are drawn directly as independent
  Poisson((1 - F) lambda) and Poisson(F lambda) counts (the two products in
  FP64): the first with the entry's inversion word, the second with word
  (entry mod 4) of Philox(pixel, entry // 4, TAG_RED, 0), each part by the alias
  rule below 512 and by transformed rejection above (attempts on
  (pixel, entry, TAG_PTRS, j) and (pixel, entry, TAG_PTRS_RED, j)).  Independent
  thinning of a Poisson count gives exactly this law; it costs two draws however
  many stars the entry has, where C3 needs a random bit or word per star.
* C3, dust split -- each of the n stars is reddened independently with
  probability F_dust (reading of "fraction of stars that are reddened").  For
  F_dust = 1/2 one random bit per star: the first 8 stars of entry i use byte
  (i mod 16) of Philox(pixel, i // 16, TAG_SPLIT, 0) (word (i mod 16) // 4, bits
  8 (i mod 4) upward), star 8 + t uses bit t mod 32 of word (t mod 128) // 32 of
  Philox(pixel, i, TAG_SPLIT_X, t // 128).  For any other fraction star s uses
  word s mod 4 of Philox(pixel, i, TAG_SPLIT_X, s // 4), reddened iff the word is
  below floor(F * 2^32).

Random words come from Philox4x32-10 keyed by the seed with counters
(pixel, entry // 4, TAG_MAIN, 0) word entry % 4 (inversion and alias),
(pixel, entry, TAG_PTRS, j) (rejection attempts 2j and 2j+1),
(pixel, entry // 16, TAG_SPLIT, 0) and (pixel, entry, TAG_SPLIT_X, j) (dust split),
and (pixel, 0, TAG_DUST, 0) (per-pixel dust).

Pins: threshold tables against the Poisson pmf to 2^-32; the PTRS sampler by
chi-square and moment tests; the project logarithm against np.log; the split
by exact enumeration; pixel flux mean sum(lambda f) and variance
sum(lambda f^2) (the surface-brightness-fluctuation signal); distance and dust
invariants (tests/test_oracle_sampler.py).
"""
from __future__ import annotations

import math

import numpy as np

from .rng import (TAG_DUST, TAG_MAIN, TAG_PTRS, TAG_PTRS_RED, TAG_RED, TAG_SPLIT, TAG_SPLIT_X, box_muller_f64,
                  philox4x32_10, u01_open_f32)

LAM_SWITCH = 10.0
LAM_THIN_HALF = 4.0      # F = 1/2: entries at or above this lambda are thinned (C3b)
KMAX = 63
TWO32 = 2 ** 32
F32 = np.float32


# ---------------------------------------------------------------------------
# C1: inversion thresholds
# ---------------------------------------------------------------------------


def inversion_thresholds(lam: float) -> list[int]:
    """Thresholds T_0..T_{K-1} (all < 2^32 - 1) of the integer inversion rule; outcome K takes
    the words from T_{K-1} to 2^32 - 1."""
    lam = float(lam)
    p = math.exp(-lam)
    F = p
    out = []
    for k in range(KMAX):
        if k > 0:
            p = p * lam / k
            F = F + p
        t = math.floor(F * 4294967296.0)
        if t >= TWO32 - 1:             # the last word or more: outcome k takes the rest
            break
        out.append(int(t))
    return out


ALIAS_MIN = 2.0
ALIAS_MAX = 512.0
ALIAS_MIN_COLS = 16
ALIAS_MAX_COLS = 512


def alias_masses(lam: float, p0: float | None = None):
    """(k_lo, m): the C1b outcome masses (integers summing to 2^32) of outcomes k_lo, k_lo + 1, ...
    p0 replaces exp(-lambda) (for checking how a last-bit difference of exp would move them)."""
    lam = float(lam)
    p = math.exp(-lam) if p0 is None else float(p0)
    F = p
    T = []                      # T_0, T_1, ... with the last one set to 2^32
    k = 0
    while True:
        if k > 0:
            p = p * lam / k
            F = F + p
        t = math.floor(F * 4294967296.0)
        if t >= TWO32 - 1:             # the last word or more: the rest of the mass goes here
            T.append(TWO32)
            break
        T.append(int(t))
        k += 1
    k_lo = next(kk for kk, t in enumerate(T) if t > 0)
    m = [T[k_lo]] + [T[kk] - T[kk - 1] for kk in range(k_lo + 1, len(T))]
    return k_lo, m


def alias_columns(n_outcomes: int) -> int:
    """M: the smallest power of two >= the number of outcomes, at least 16."""
    M = ALIAS_MIN_COLS
    while M < n_outcomes:
        M *= 2
    return M


def alias_table(lam: float, p0: float | None = None):
    """(k_lo, log2 M, packed[M] uint32): column j's height h_j (stored as min(h_j, 2^32/M - 1);
    alias = j when h_j = 2^32/M) in the top 32 - log2 M bits, its alias a_j in the low log2 M."""
    k_lo, m = alias_masses(lam, p0)
    M = alias_columns(len(m))
    assert M <= ALIAS_MAX_COLS, "support too wide for the alias rule"
    bits = M.bit_length() - 1
    cap = TWO32 // M
    w = list(m) + [0] * (M - len(m))
    small = [j for j in range(M) if w[j] < cap]
    large = [j for j in range(M) if w[j] >= cap]
    h = [0] * M
    a = [0] * M
    while small and large:
        sj = small.pop()
        lj = large.pop()
        h[sj] = w[sj]
        a[sj] = lj
        w[lj] -= cap - w[sj]
        (small if w[lj] < cap else large).append(lj)
    for j in large:
        h[j] = cap
        a[j] = j
    assert not small, "masses do not sum to 2^32"
    packed = np.array([(min(h[j], cap - 1) << bits) | a[j] for j in range(M)], dtype=np.uint32)
    return k_lo, bits, packed


def count_from_alias(u: np.ndarray, k_lo: int, bits: int, packed: np.ndarray) -> np.ndarray:
    """n = k_lo + (c if u mod 2^(32-b) < h_c else a_c), c = u >> (32 - b), M = 2^b columns."""
    u = np.asarray(u, dtype=np.uint64)
    sh = np.uint64(32 - bits)
    c = (u >> sh).astype(np.int64)
    r = u & np.uint64((1 << (32 - bits)) - 1)
    x = packed[c].astype(np.uint64)
    j = np.where(r < (x >> np.uint64(bits)), c, (x & np.uint64((1 << bits) - 1)).astype(np.int64))
    return (k_lo + j).astype(np.int64)


def draw_part(mu: float, u: np.ndarray, seed: int, px: np.ndarray, entry: int, tag_ptrs: int) -> np.ndarray:
    """Poisson(mu) counts for one entry: the alias rule (C1b) with words u below ALIAS_MAX,
    transformed rejection (C2) on (pixel, entry, tag_ptrs, j) above."""
    if mu < ALIAS_MAX:
        return count_from_alias(u, *alias_table(mu))
    n, _ = ptrs_draw(ptrs_constants(mu), seed, px, entry, tag=tag_ptrs)
    return n


def count_from_thresholds(u: np.ndarray, thr: list[int]) -> np.ndarray:
    """n = #{k : T_k <= u}."""
    u = np.asarray(u, dtype=np.uint64)
    n = np.zeros(u.shape, dtype=np.uint32)
    for t in thr:
        n += (u >= np.uint64(t)).astype(np.uint32)
    return n


# ---------------------------------------------------------------------------
# C2: transformed rejection in FP32
# ---------------------------------------------------------------------------

LN2_HI = F32(0.693145751953125)
LN2_LO = F32(1.428606765330187e-06)
SQRT2_F32 = F32(1.41421353816986083984375)
LN_COEF = [F32(2.0 / (2 * j + 1)) for j in range(6)]   # 2, 2/3, 2/5, 2/7, 2/9, 2/11


def ln32(x):
    """Natural log in FP32 from frexp and the series ln m = 2 atanh((m-1)/(m+1)).

    x must be positive, finite and normal.  Every step is one IEEE FP32 operation."""
    x = np.asarray(x, dtype=np.float32)
    bits = x.view(np.uint32)
    e = ((bits >> np.uint32(23)) & np.uint32(0xFF)).astype(np.int32) - 127
    m = ((bits & np.uint32(0x007FFFFF)) | np.uint32(0x3F800000)).view(np.float32)
    big = m > SQRT2_F32
    m = np.where(big, m * F32(0.5), m).astype(np.float32)
    e = e + big.astype(np.int32)
    s = (m - F32(1.0)) / (m + F32(1.0))
    z = s * s
    P = LN_COEF[5]
    for c in (LN_COEF[4], LN_COEF[3], LN_COEF[2], LN_COEF[1], LN_COEF[0]):
        P = P * z + c
    ef = e.astype(np.float32)
    return ef * LN2_HI + (ef * LN2_LO + s * P)


def lnfact_table() -> np.ndarray:
    """ln k! for k < 256: FP64 running sum of ln j, rounded to FP32."""
    t = np.zeros(256, dtype=np.float64)
    acc = 0.0
    for k in range(2, 256):
        acc = acc + math.log(k)
        t[k] = acc
    return t.astype(np.float32)


_LNFACT = lnfact_table()
HALF_LN_2PI = F32(0.9189385332046727)
INV12 = F32(1.0 / 12.0)
INV360 = F32(1.0 / 360.0)


def lnfact32(kf: np.ndarray) -> np.ndarray:
    """ln k! in FP32: table below 256, Stirling series with x = k + 1 above."""
    kf = np.asarray(kf, dtype=np.float32)
    small = kf < F32(256.0)
    ki = np.clip(kf, 0, 255).astype(np.int64)
    x = kf + F32(1.0)
    xs = np.where(small, F32(300.0), x).astype(np.float32)   # keep ln32 away from the table range
    lx = ln32(xs)
    t = (xs - F32(0.5)) * lx
    t = t - xs
    t = t + HALF_LN_2PI
    r = F32(1.0) / xs
    t = t + r * INV12
    r3 = (r * r) * r
    t = t - r3 * INV360
    return np.where(small, _LNFACT[ki], t).astype(np.float32)


def ptrs_constants(lam: float) -> dict:
    """Per-entry constants, computed in FP64 and rounded to FP32."""
    lam = float(lam)
    slam = math.sqrt(lam)
    b = 0.931 + 2.53 * slam
    a = -0.059 + 0.02483 * b
    inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
    vr = 0.9277 - 3.6224 / (b - 2.0)
    return dict(mu=F32(lam), lnmu=F32(math.log(lam)), b=F32(b), a=F32(a), twoa=F32(2.0 * a),
                lninva=F32(math.log(inv_alpha)), vr=F32(vr))


def ptrs_draw(c: dict, seed: int, px: np.ndarray, entry: int, max_attempts: int = 64, tag: int = TAG_PTRS):
    """Transformed-rejection Poisson draw for each pixel in `px` (entry fixed).

    Attempt j uses words (2(j%2), 2(j%2)+1) of Philox(pixel, entry, tag, j//2) (tag TAG_PTRS for
    the per-point rule).  Returns (counts, attempts_used)."""
    npx = px.shape[0]
    out = np.zeros(npx, dtype=np.int64)
    done = np.zeros(npx, dtype=bool)
    used = np.zeros(npx, dtype=np.int32)
    words = None
    for j in range(max_attempts):
        if j % 2 == 0:
            words = philox4x32_10(px, entry, tag, j // 2, seed)
        u = u01_open_f32(words[2 * (j % 2)])
        V = u01_open_f32(words[2 * (j % 2) + 1])
        U = u - F32(0.5)
        us = F32(0.5) - np.abs(U)
        t = c["twoa"] / us
        t = t + c["b"]
        t = t * U
        t = t + c["mu"]
        t = t + F32(0.43)
        kf = np.floor(t).astype(np.float32)
        fast = (us >= F32(0.07)) & (V <= c["vr"])
        rej = (kf < F32(0.0)) | ((us < F32(0.013)) & (V > us))
        q = c["a"] / (us * us)
        q = q + c["b"]
        lhs = (ln32(V) + c["lninva"]) - ln32(q)
        kpos = np.maximum(kf, F32(0.0)).astype(np.float32)
        rhs = ((-c["mu"]) + kpos * c["lnmu"]) - lnfact32(kpos)
        acc = fast | (~rej & (lhs <= rhs))
        new = acc & ~done
        out[new] = kf[new].astype(np.int64)
        used[new] = j + 1
        done |= acc
        if done.all():
            return out, used
    raise RuntimeError("transformed rejection exceeded its attempt limit")


# ---------------------------------------------------------------------------
# C3: dust split
# ---------------------------------------------------------------------------


def popcount32(w: np.ndarray) -> np.ndarray:
    return np.bitwise_count(np.asarray(w, dtype=np.uint64)).astype(np.int64)


SPLIT_FIRST_BITS = 8     # stars covered by the entry's byte of the 16-entry split block


def split_first_byte(px: np.ndarray, entry: int, seed: int) -> np.ndarray:
    """Byte (entry mod 16) of Philox(pixel, entry // 16, TAG_SPLIT, 0), as uint32."""
    w = philox4x32_10(px, entry // 16, TAG_SPLIT, 0, seed)[(entry % 16) // 4]
    return (np.asarray(w, dtype=np.uint32) >> np.uint32(8 * (entry % 4))) & np.uint32(0xFF)


def split_reddened(n: np.ndarray, first_byte: np.ndarray, frac: float, seed: int,
                   px: np.ndarray, entry: int) -> np.ndarray:
    """Number of the n stars that sit behind the dust screen (C3), one entry."""
    r = split_block(np.asarray(n, dtype=np.int64)[:, None], np.asarray(first_byte, dtype=np.uint64)[:, None],
                    frac, seed, np.asarray(px, dtype=np.int64), np.array([entry]))
    return r[:, 0]


# ---------------------------------------------------------------------------
# counts and fluxes over a pixel window
# ---------------------------------------------------------------------------


def _popcount_masked(w: np.ndarray, cnt: np.ndarray) -> np.ndarray:
    """popcount of the low `cnt` bits (cnt in [0, 32]) of uint32 words."""
    w = np.asarray(w, dtype=np.uint64)
    cnt = np.asarray(cnt, dtype=np.int64)
    mask = np.where(cnt >= 32, np.uint64(0xFFFFFFFF),
                    (np.uint64(1) << np.clip(cnt, 0, 31).astype(np.uint64)) - np.uint64(1))
    return popcount32(w & mask)


def sample_window(lam: np.ndarray, flux32: np.ndarray, seed: int, px0: int, px1: int,
                  dust_model: int = 0, dust_frac: float = 0.5, want_counts: bool = False,
                  block: int = 1024):
    """Star counts and flux sums for the pixel window [px0, px1) (see sample_pixels)."""
    return sample_pixels(lam, flux32, seed, np.arange(px0, px1, dtype=np.int64), dust_model, dust_frac,
                         want_counts, block)


def sample_pixels(lam: np.ndarray, flux32: np.ndarray, seed: int, px: np.ndarray,
                  dust_model: int = 0, dust_frac: float = 0.5, want_counts: bool = False,
                  block: int = 1024):
    """Star counts and unreddened / reddened flux sums for the pixels listed in `px`.

    Entries are handled a block at a time, vectorised over (pixel, entry); each count follows
    the C1 / C1b / C2 rule of its entry and each split the C3 rule.  Returns dict with F_clr, F_red
    ([B][npx] FP64) and, if asked, counts n and reddened counts r ([npx][E] int64)."""
    lam = np.asarray(lam, dtype=np.float64)
    E = lam.shape[0]
    B = flux32.shape[0]
    f = np.asarray(flux32, dtype=np.float32).astype(np.float64)
    px = np.asarray(px, dtype=np.int64)
    npx = px.shape[0]
    split = dust_model != 0
    frac = float(dust_frac) if split else 0.0
    F_clr = np.zeros((B, npx))
    F_red = np.zeros((B, npx))
    counts = np.zeros((npx, E), dtype=np.int64) if want_counts else None
    red = np.zeros((npx, E), dtype=np.int64) if want_counts else None
    block = max(4, block - block % 4)
    for e0 in range(0, E, block):
        e1 = min(E, e0 + block)
        ents = np.arange(e0, e1)
        g = np.arange(e0 // 4, (e1 + 3) // 4)
        w = philox4x32_10(px[:, None], g[None, :], TAG_MAIN, 0, seed)
        U = np.stack(w, axis=-1).reshape(npx, 4 * len(g))[:, : e1 - e0].astype(np.uint64)
        n = np.zeros((npx, e1 - e0), dtype=np.int64)
        lb = lam[e0:e1]
        inv = np.nonzero(lb < ALIAS_MIN)[0]
        tables = [inversion_thresholds(lb[j]) for j in inv]
        K = np.array([len(t) for t in tables], dtype=np.int64)
        # n = #{k : T_k <= u}; entries bucketed by table length, tables padded with 2^32
        for lo, hi in ((1, 4), (5, 8), (9, 16), (17, 32), (33, KMAX)):
            sel = np.nonzero((K >= lo) & (K <= hi))[0]
            if len(sel) == 0:
                continue
            T = np.full((len(sel), hi), TWO32, dtype=np.uint64)
            for r_, j in enumerate(sel):
                T[r_, : K[j]] = tables[j]
            cols = inv[sel]
            n[:, cols] = (U[:, cols, None] >= T[None, :, :]).sum(axis=-1)
        tab = np.nonzero(lb >= ALIAS_MIN)[0]          # entries drawn by C1b or C2
        # C3b: the thinned entries (all of tab when F != 1/2; those at lambda >= 4 when F = 1/2)
        if split and 0.0 < frac < 1.0:
            thin = tab if frac != 0.5 else np.nonzero(lb >= LAM_THIN_HALF)[0]
        else:
            thin = tab[:0]
        n_red_thin = None
        if len(thin):
            # two independent Poisson parts, (1 - F) lambda and F lambda
            wr = philox4x32_10(px[:, None], g[None, :], TAG_RED, 0, seed)
            UR = np.stack(wr, axis=-1).reshape(npx, 4 * len(g))[:, : e1 - e0].astype(np.uint64)
            n_red_thin = np.zeros((npx, len(thin)), dtype=np.int64)
            for c_, j in enumerate(thin):
                lc = float(lb[j]) * (1.0 - frac)
                lr = float(lb[j]) * frac
                nc = draw_part(lc, U[:, j], seed, px, e0 + j, TAG_PTRS)
                nr = draw_part(lr, UR[:, j], seed, px, e0 + j, TAG_PTRS_RED)
                n[:, j] = nc + nr
                n_red_thin[:, c_] = nr
        for j in np.setdiff1d(tab, thin):
            n[:, j] = draw_part(float(lb[j]), U[:, j], seed, px, e0 + j, TAG_PTRS)
        if split and 0.0 < frac < 1.0:
            W = None
            if frac == 0.5:
                g16 = np.arange(e0 // 16, (e1 + 15) // 16)
                sw = philox4x32_10(px[:, None], g16[None, :], TAG_SPLIT, 0, seed)
                words = np.stack(sw, axis=-1).reshape(npx, 4 * len(g16)).astype(np.uint64)
                q = ents - 16 * g16[0]                       # entry's position from the first block
                W = (words[:, q // 4] >> (np.uint64(8) * (q % 4).astype(np.uint64))) & np.uint64(0xFF)
            n_split = n.copy()
            if n_red_thin is not None:
                n_split[:, thin] = 0                     # thinned entries are already split
            r = split_block(n_split, W, frac, seed, px, ents)
            if n_red_thin is not None:
                r[:, thin] = n_red_thin
        elif split and frac >= 1.0:
            r = n.copy()
        else:
            r = np.zeros_like(n)
        fb = f[:, e0:e1]
        F_clr += fb @ (n - r).T.astype(np.float64)
        F_red += fb @ r.T.astype(np.float64)
        if want_counts:
            counts[:, e0:e1] = n
            red[:, e0:e1] = r
    return dict(F_clr=F_clr, F_red=F_red, counts=counts, red=red)


def split_block(n: np.ndarray, W, frac: float, seed: int, px: np.ndarray, ents: np.ndarray):
    """C3 for a block: n [npx][nent] counts; W [npx][nent] the entries' split bytes (F = 1/2)."""
    n = np.asarray(n, dtype=np.int64)
    r = np.zeros_like(n)
    if frac <= 0.0:
        return r
    if frac >= 1.0:
        return n.copy()
    if frac == 0.5:
        r += _popcount_masked(W, np.minimum(n, SPLIT_FIRST_BITS))
        extra = n - SPLIT_FIRST_BITS
        j = 0
        while np.any(extra > 128 * j):
            cols = np.nonzero(np.any(extra > 128 * j, axis=0))[0]
            x = philox4x32_10(px[:, None], ents[cols][None, :], TAG_SPLIT_X, j, seed)
            for q in range(4):
                cnt = np.clip(extra[:, cols] - (128 * j + 32 * q), 0, 32)
                r[:, cols] += _popcount_masked(x[q], cnt)
            j += 1
        return r
    fq = np.uint64(int(math.floor(frac * 4294967296.0)))
    j = 0
    while np.any(n > 4 * j):
        cols = np.nonzero(np.any(n > 4 * j, axis=0))[0]
        x = philox4x32_10(px[:, None], ents[cols][None, :], TAG_SPLIT_X, j, seed)
        for q in range(4):
            s_ = 4 * j + q
            r[:, cols] += ((n[:, cols] > s_) & (np.asarray(x[q], dtype=np.uint64) < fq)).astype(np.int64)
        j += 1
    return r


def dust_ebv(px: np.ndarray, seed: int, dust_model: int, mu: float, sigma: float) -> np.ndarray:
    """E(B-V) per pixel: 10^mu (E1) or 10^(mu + sigma z_p) (E2/E3)."""
    px = np.asarray(px, dtype=np.int64)
    if dust_model == 1:
        return np.full(px.shape, 10.0 ** mu)
    w = philox4x32_10(px, 0, TAG_DUST, 0, seed)
    z = box_muller_f64(w[0], w[1])
    return 10.0 ** (mu + sigma * z)


def pixel_flux(F_clr, F_red, px, seed, dmod, dust_model=0, dust_mu=-0.5, dust_sigma=0.2,
               dust_R=(3.6, 1.9, 1.3)):
    """F_b = 10^(-0.4 mu_d) (F_clr_b + F_red_b 10^(-0.4 R_b E_p))  (FP64)."""
    B = F_clr.shape[0]
    dist = 10.0 ** (-0.4 * dmod)
    if dust_model == 0:
        return dist * (F_clr + F_red)
    ebv = dust_ebv(px, seed, dust_model, dust_mu, dust_sigma)
    out = np.empty_like(F_clr)
    for b in range(B):
        out[b] = dist * (F_clr[b] + F_red[b] * 10.0 ** (-0.4 * dust_R[b] * ebv))
    return out


def simulate_flux(lam, flux32, obs, px0=0, px1=None, want_counts=False, px=None):
    """Pre-PSF pixel fluxes [B][npx] (FP64) for pixels [px0, px1) or the list `px`."""
    npx_all = obs.nim * obs.nim
    px1 = npx_all if px1 is None else px1
    if px is None:
        px = np.arange(px0, px1, dtype=np.int64)
    px = np.asarray(px, dtype=np.int64)
    if getattr(obs, "sampler", 0) == 1:
        from .sampler_block import sample_pixels_block
        s = sample_pixels_block(lam, flux32, obs.seed, px, obs.dust_model, obs.dust_frac, want_counts)
    elif getattr(obs, "sampler", 0) == 2:
        from .sampler_block import sample_pixels_hybrid
        s = sample_pixels_hybrid(lam, flux32, obs.seed, px, obs.dust_model, obs.dust_frac, want_counts)
    else:
        s = sample_pixels(lam, flux32, obs.seed, px, obs.dust_model, obs.dust_frac, want_counts)
    F = pixel_flux(s["F_clr"], s["F_red"], px, obs.seed, obs.dmod, obs.dust_model, obs.dust_mu,
                   obs.dust_sigma, obs.dust_R[:flux32.shape[0]])
    return F, s
