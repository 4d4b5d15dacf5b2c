"""Process-parallel driver of the oracle (test infrastructure, like the rest of this package).

The oracle's cost is exactly linear in pixels for the sampler (Sec. 2.1: every pixel draws its own
counts) and in bands for the convolution, so the whole-image oracle can run on every host core by
handing the oracle's own functions independent pieces: pixel slabs of `sampler.simulate_flux`
(each pixel's counts and sums do not depend on which slab holds it) and single bands of
`psf.convolve_periodic`.  This module holds no arithmetic of the method; it splits, runs and
joins.

Worker processes are started with the "spawn" method (fresh interpreters that import only numpy
and this package) and each uses one BLAS thread.

Star counts of a whole image do not fit in memory (65,536 pixels x 52,500 points), so a worker
can also return a digest of each pixel's count vector, d_p = sum_i n_{p,i} r_i mod 2^64 with fixed
odd 64-bit multipliers r_i (`count_digest`): two count vectors that differ in one entry by d with
0 < |d| < 2^32 always have different digests, so comparing digests compares the counts.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

from . import noise, psf, sampler

_G = {}


def default_workers() -> int:
    """Host cores this process may use (its CPU affinity), at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover - not Linux
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def digest_multipliers(n_entries: int, seed: int = 20190401) -> np.ndarray:
    """r_i: fixed odd 64-bit multipliers of the count digest."""
    r = np.random.default_rng(seed).integers(0, 2 ** 63, size=n_entries, dtype=np.uint64)
    return (r << np.uint64(1)) | np.uint64(1)


def count_digest(counts: np.ndarray, mult: np.ndarray) -> np.ndarray:
    """d_p = sum_i counts[p, i] * r_i mod 2^64 for counts [npx][E] (any integer dtype)."""
    c = np.asarray(counts).astype(np.uint64)
    with np.errstate(over="ignore"):
        return (c * mult[None, :]).sum(axis=1, dtype=np.uint64)


def _init(lam, flux32, obs, with_digest):
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:  # pragma: no cover
        pass
    _G["lam"] = lam
    _G["f32"] = flux32
    _G["obs"] = obs
    _G["mult"] = digest_multipliers(len(lam)) if with_digest else None


def _slab(task):
    px0, px1 = task
    F, s = sampler.simulate_flux(_G["lam"], _G["f32"], _G["obs"], px0, px1, want_counts=_G["mult"] is not None)
    if _G["mult"] is None:
        return px0, F, None, None
    return px0, F, count_digest(s["counts"], _G["mult"]), count_digest(s["red"], _G["mult"])


def _band(task):
    Fb, Pb = task
    return psf.convolve_periodic(Fb[None], Pb[None])[0]


def _ctx():
    return mp.get_context("spawn")


def simulate_flux(lam, flux32, obs, windows, with_digest: bool = False, workers: int | None = None,
                  slab: int = 128):
    """Pre-PSF fluxes (FP64, the oracle's `sampler.simulate_flux`) of the pixel windows
    [(px0, px1), ...], computed in slabs on `workers` processes.  Returns (F [B][npx] in window
    order, digests of the counts [npx] or None, digests of the reddened counts or None)."""
    lam = np.ascontiguousarray(lam, np.float64)
    flux32 = np.ascontiguousarray(flux32, np.float32)
    tasks = []
    for a, b in windows:
        tasks += [(p, min(b, p + slab)) for p in range(a, b, slab)]
    n = sum(b - a for a, b in windows)
    B = flux32.shape[0]
    F = np.empty((B, n))
    dc = np.empty(n, np.uint64) if with_digest else None
    dr = np.empty(n, np.uint64) if with_digest else None
    # position of each pixel in the output
    offs = {}
    o = 0
    for a, b in windows:
        for p in range(a, b, slab):
            offs[p] = o + (p - a)
        o += b - a
    with _ctx().Pool(workers or default_workers(), initializer=_init,
                     initargs=(lam, flux32, obs, with_digest)) as pool:
        for px0, Fs, c, r in pool.imap_unordered(_slab, tasks):
            k = offs[px0]
            F[:, k:k + Fs.shape[1]] = Fs
            if with_digest:
                dc[k:k + len(c)] = c
                dr[k:k + len(r)] = r
    return F, dc, dr


def convolve(F, psf_stack, workers: int | None = None):
    """The oracle's periodic convolution (`psf.convolve_periodic`), one band per process.
    F [B][N][N], psf_stack [B][K][K] -> G [B][N][N] (FP64)."""
    F = np.asarray(F, np.float64)
    P = np.asarray(psf_stack, np.float32)
    B = F.shape[0]
    with _ctx().Pool(min(B, workers or default_workers())) as pool:
        G = pool.map(_band, [(F[b], P[b]) for b in range(B)])
    return np.stack(G)


def simulate(lam, flux32, obs, with_digest: bool = False, workers: int | None = None):
    """The oracle's whole-image forward model (`pipeline.simulate`) on all host cores:
    dict(F, G, mags64, mags (FP32), digest_counts, digest_red)."""
    N = obs.nim
    B = flux32.shape[0]
    F, dc, dr = simulate_flux(lam, flux32, obs, [(0, N * N)], with_digest, workers)
    if obs.psf is not None:
        assert np.asarray(obs.psf).ndim == 3, "the sub-pixel PSF grid runs through pipeline.simulate"
        G = convolve(F.reshape(B, N, N), np.asarray(obs.psf)[:B], workers).reshape(B, N * N)
    else:
        G = F.copy()
    mags = noise.magnitudes(G, obs)
    return dict(F=F, G=G, mags64=mags, mags=mags.astype(np.float32), digest_counts=dc, digest_red=dr)
