"""The block-skip sampler's oracle (Poisson superposition, Sec. 2.1 footnote): a different stream
with the same law as the per-point rule."""
import numpy as np
import pytest
from scipy import stats

from oracle import sampler_block as sb


def _lam():
    r = np.random.default_rng(11)
    a = r.uniform(0.0, 0.08, 64)          # a sparse block (most pixels draw nothing)
    a[[3, 17, 40]] = 0.0                  # points without stars
    b = r.uniform(0.05, 0.35, 64)         # Lambda_b ~ 13: totals by transformed rejection
    c = np.full(20, 0.4)                  # a ragged last block
    return np.concatenate([a, b, c])


def test_per_point_counts_are_poisson_lambda():
    lam = _lam()
    f = np.ones((1, len(lam)), np.float32)
    npx = 20000
    out = sb.sample_pixels_block(lam, f, 12345, np.arange(npx), want_counts=True)
    n = out["counts"]
    m, v = n.mean(axis=0), n.var(axis=0)
    se = np.sqrt(np.maximum(lam, 1e-12) / npx)
    assert np.all(np.abs(m - lam) <= 5 * se + 1e-12)
    nz = lam > 0.02
    assert np.all(np.abs(v[nz] / lam[nz] - 1) <= 5 * np.sqrt(2.0 / npx) + 5 * se[nz] / lam[nz])
    assert np.all(n[:, lam == 0] == 0)
    # block totals against the Poisson pmf (chi-square over the well-filled outcomes)
    for b, L in enumerate(sb.block_sums(lam)):
        N = n[:, b * 64:(b + 1) * 64].sum(axis=1)
        ks = np.arange(max(0, int(L - 4 * np.sqrt(L))), int(L + 4 * np.sqrt(L) + 2))
        exp_ = npx * stats.poisson.pmf(ks, L)
        keep = exp_ > 20
        obs = np.array([(N == k).sum() for k in ks[keep]])
        e = exp_[keep] * obs.sum() / exp_[keep].sum()
        chi2 = ((obs - e) ** 2 / e).sum()
        assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4, (b, chi2)
    # two points of one block: unconditionally independent (correlation ~ 0)
    x, y = n[:, 70], n[:, 90]
    assert abs(np.corrcoef(x, y)[0, 1]) < 5 / np.sqrt(npx)


def test_category_thresholds_and_split_fraction():
    lam = _lam()
    L = sb.block_sums(lam)[1]
    C = sb.category_thresholds(lam[64:128], L).astype(np.float64)
    widths = np.diff(np.concatenate([[0.0], C]))
    assert np.all(np.abs(widths - lam[64:128] / L * 2.0 ** 32) <= 1.0)
    assert C[-1] == 2.0 ** 32
    f = np.ones((1, len(lam)), np.float32)
    out = sb.sample_pixels_block(lam, f, 777, np.arange(5000), dust_model=2, dust_frac=0.3, want_counts=True)
    tot, red = out["counts"].sum(), out["red"].sum()
    assert abs(red / tot - 0.3) <= 5 * np.sqrt(0.3 * 0.7 / tot)
    all_red = sb.sample_pixels_block(lam, f, 777, np.arange(200), dust_model=2, dust_frac=1.0, want_counts=True)
    assert np.array_equal(all_red["red"], all_red["counts"])
    none = sb.sample_pixels_block(lam, f, 777, np.arange(200), dust_model=0, want_counts=True)
    assert none["red"].sum() == 0 and np.array_equal(none["counts"], all_red["counts"])
    # fluxes are the counts weighted by the point fluxes
    assert np.allclose(out["F_clr"][0] + out["F_red"][0], out["counts"].sum(axis=1))


def test_hybrid_partition_and_law():
    """The hybrid rule splits the entries by block total (the two parts add up to the input, no
    block in both), draws each part with its own rule (so each part equals that rule on the part
    alone), and keeps the Poisson law per entry."""
    from oracle import sampler as sp
    lam = _lam()
    blk, pt = sb.hybrid_split(lam)
    assert np.array_equal(blk + pt, lam) and not np.any((blk > 0) & (pt > 0))
    tot = sb.block_sums(lam)
    assert all((tot[b] < 10) == (pt[64 * b:64 * (b + 1)].sum() == 0) for b in range(len(tot)))
    f = np.ones((1, len(lam)), np.float32)
    px = np.arange(20000)
    h = sb.sample_pixels_hybrid(lam, f, 99, px, dust_model=2, dust_frac=0.3, want_counts=True)
    a = sb.sample_pixels_block(blk, f, 99, px[:500], dust_model=2, dust_frac=0.3, want_counts=True)
    c = sp.sample_pixels(pt, f, 99, px[:500], dust_model=2, dust_frac=0.3, want_counts=True)
    assert np.array_equal(h["counts"][:500], a["counts"] + c["counts"])
    assert np.array_equal(h["red"][:500], a["red"] + c["red"])
    n = h["counts"]
    se = np.sqrt(np.maximum(lam, 1e-12) / len(px))
    assert np.all(np.abs(n.mean(axis=0) - lam) <= 5 * se + 1e-12)
