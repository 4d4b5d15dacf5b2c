"""Block-skip sampler (oracle side): the star counts by Poisson superposition.

The footnote of Sec. 2.1 recalls that a sum of independent Poisson counts is Poisson with the
summed mean.  The plain rule draws one count per (pixel, point); this rule draws per pixel and per
block of BLOCK = 64 consecutive points

* the block total N ~ Poisson(Lambda_b), Lambda_b = sum of the block's lambda_i (FP64, left to
  right): below 10 by C1 inversion with word 0 of Philox(pixel, b, TAG_BLOCK, 0), from 10 on by
  C2 transformed rejection with Philox(pixel, b, TAG_BLOCK_PTRS, j);
* the point of each of its N stars: star s takes word s mod 4 of Philox(pixel, b, TAG_STAR, s // 4)
  and lands on the first point i of the block whose cumulative threshold
  C_i = floor(2^32 sum_{k <= i} lambda_k / Lambda_b) (FP64, left to right; C_63 = 2^32) exceeds the
  word, i.e. on point i with probability lambda_i / Lambda_b to 2^-32;
* its dust screen: star s is reddened iff word s mod 4 of Philox(pixel, b, TAG_STAR_SPLIT, s // 4)
  is below floor(F 2^32) (F = 1: every star; F = 0 or no dust: none).

Given N the points are multinomial with probabilities lambda_i / Lambda_b, so the per-point
counts are again independent Poisson(lambda_i): the same law as the plain rule with fewer random
numbers where most blocks are empty (Lambda_b << 1), but a different stream.

The hybrid rule draws the blocks with Lambda_b < 10 by the block rule and the entries of the
other blocks one by one with the per-point rule: the cheaper rule on each side of the crossover.

Pins (tests/test_oracle_block.py): per-point means and variances against lambda_i, block totals
against the Poisson pmf by chi-square, independence of two points of one block (correlation), the
cumulative thresholds against the block's probabilities, and the split fraction.
"""
from __future__ import annotations

import numpy as np

from .rng import TAG_BLOCK, TAG_BLOCK_PTRS, TAG_STAR, TAG_STAR_SPLIT, philox4x32_10
from .sampler import LAM_SWITCH, TWO32, count_from_thresholds, inversion_thresholds, ptrs_constants, ptrs_draw

BLOCK = 64
STAR_CHUNK = 1024


def block_sums(lam: np.ndarray) -> np.ndarray:
    """Lambda_b of every block (points past E count as lambda = 0), summed left to right."""
    lam = np.asarray(lam, dtype=np.float64)
    nb = (len(lam) + BLOCK - 1) // BLOCK
    out = np.zeros(nb)
    for b in range(nb):
        s = 0.0
        for v in lam[b * BLOCK: (b + 1) * BLOCK]:
            s += float(v)
        out[b] = s
    return out


def category_thresholds(lam_block: np.ndarray, total: float) -> np.ndarray:
    """C_i = floor(2^32 cum_i / Lambda_b) for the BLOCK points (padded with lambda = 0); uint64."""
    C = np.empty(BLOCK, dtype=np.uint64)
    cum = 0.0
    for i in range(BLOCK):
        if i < len(lam_block):
            cum += float(lam_block[i])
        C[i] = np.uint64(int(np.floor(cum / total * 4294967296.0)))
    C[BLOCK - 1] = np.uint64(TWO32)
    return C


def sample_pixels_block(lam: np.ndarray, flux32: np.ndarray, seed: int, px: np.ndarray, dust_model: int = 0,
                        dust_frac: float = 0.5, want_counts: bool = False):
    """Counts and unreddened / reddened flux sums for the pixels `px` by the block-skip rule.
    Returns dict like sampler.sample_pixels (F_clr, F_red [B][npx] FP64; counts, red [npx][E])."""
    lam = np.asarray(lam, dtype=np.float64)
    E = len(lam)
    B = flux32.shape[0]
    f = np.asarray(flux32, dtype=np.float32).astype(np.float64)
    px = np.asarray(px, dtype=np.int64)
    npx = len(px)
    split = dust_model != 0
    frac = float(dust_frac) if split else 0.0
    fq = np.uint64(int(np.floor(frac * 4294967296.0)))
    counts = np.zeros((npx, E), dtype=np.int64)
    red = np.zeros((npx, E), dtype=np.int64)
    tot = block_sums(lam)
    for b, L in enumerate(tot):
        if L <= 0.0:
            continue
        e0 = b * BLOCK
        lb = lam[e0: e0 + BLOCK]
        if L < LAM_SWITCH:
            u = philox4x32_10(px, b, TAG_BLOCK, 0, seed)[0]
            N = count_from_thresholds(u, inversion_thresholds(L)).astype(np.int64)
        else:
            N, _ = ptrs_draw(ptrs_constants(L), seed, px, b, tag=TAG_BLOCK_PTRS)
        nmax = int(N.max()) if npx else 0
        if nmax == 0:
            continue
        C = category_thresholds(lb, L)
        # stars s = 0 .. nmax - 1 of every pixel, STAR_CHUNK at a time (a multiple of 4)
        for s0 in range(0, nmax, STAR_CHUNK):
            s1 = min(nmax, s0 + STAR_CHUNK)
            g = np.arange(s0 // 4, (s1 + 3) // 4)
            W = np.stack(philox4x32_10(px[:, None], b, TAG_STAR, g[None, :], seed), axis=-1)
            w = W.reshape(npx, 4 * len(g))[:, : s1 - s0].astype(np.uint64)
            live = np.arange(s0, s1)[None, :] < N[:, None]
            cat = np.searchsorted(C, w, side="right")         # first i with C_i > w
            if split and frac >= 1.0:
                r = np.ones_like(live)
            elif split and frac > 0.0:
                R = np.stack(philox4x32_10(px[:, None], b, TAG_STAR_SPLIT, g[None, :], seed), axis=-1)
                r = R.reshape(npx, 4 * len(g))[:, : s1 - s0].astype(np.uint64) < fq
            else:
                r = np.zeros_like(live)
            rows = np.broadcast_to(np.arange(npx)[:, None], live.shape)
            np.add.at(counts, (rows[live], e0 + cat[live]), 1)
            np.add.at(red, (rows[live & r], e0 + cat[live & r]), 1)
    F_clr = f @ (counts - red).T.astype(np.float64)
    F_red = f @ red.T.astype(np.float64)
    return dict(F_clr=F_clr, F_red=F_red, counts=counts if want_counts else None, red=red if want_counts else None)


def hybrid_split(lam: np.ndarray):
    """The hybrid rule's partition: (lambda of the blocks drawn by the block rule, lambda of the
    blocks drawn entry by entry), each with the other blocks' entries set to zero.  A block takes
    the block rule when Lambda_b < 10 (its total is then drawn by inversion)."""
    lam = np.asarray(lam, dtype=np.float64)
    tot = block_sums(lam)
    lam_blk = lam.copy()
    lam_pt = lam.copy()
    for b, L in enumerate(tot):
        sl = slice(b * BLOCK, (b + 1) * BLOCK)
        if L < LAM_SWITCH:
            lam_pt[sl] = 0.0
        else:
            lam_blk[sl] = 0.0
    return lam_blk, lam_pt


def sample_pixels_hybrid(lam: np.ndarray, flux32: np.ndarray, seed: int, px: np.ndarray, dust_model: int = 0,
                         dust_frac: float = 0.5, want_counts: bool = False):
    """Hybrid rule: blocks with Lambda_b < 10 by the block rule (this module's stream), the other
    blocks' entries by the per-point rule (sampler.sample_pixels' stream).  Same law as both."""
    from .sampler import sample_pixels
    lam_blk, lam_pt = hybrid_split(lam)
    a = sample_pixels_block(lam_blk, flux32, seed, px, dust_model, dust_frac, want_counts)
    c = sample_pixels(lam_pt, flux32, seed, px, dust_model, dust_frac, want_counts)
    out = dict(F_clr=a["F_clr"] + c["F_clr"], F_red=a["F_red"] + c["F_red"], counts=None, red=None)
    if want_counts:
        out["counts"] = a["counts"] + c["counts"]
        out["red"] = a["red"] + c["red"]
    return out
