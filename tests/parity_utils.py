"""Helpers shared by the GPU parity tests: run one case through the C ABI and through the
oracle on the same seeded inputs, and compare them to the stated bars.

Bars:
* star counts and reddened counts: bit-exact;
* per-pixel fluxes (before and after the PSF): within 1e-5 relative of the FP64 oracle;
* magnitudes: within 1e-4 mag;
* Hess: every pixel in the same bin, except pixels whose oracle position lies within 1e-4 mag of
  a bin edge (checked pixel by pixel);
* log-likelihood: within 1e-3 absolute.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import hess as oh
from oracle import rng as orng
from oracle import sampler as osamp

FLUX_RTOL = 1e-5
MAG_ATOL = 1e-4
LOGL_ATOL = 1e-3


def gpu_simulate(ctx, lam, f32, obs, conv_path=0, window=None, want_flux=True, stream=None):
    import torch
    dev = torch.device("cuda")
    B, E = f32.shape
    npx = obs.nim * obs.nim
    lam_d = torch.from_numpy(np.ascontiguousarray(lam, np.float64)).to(dev)
    flux_d = torch.from_numpy(np.ascontiguousarray(f32, np.float32)).to(dev)
    psf_d = None if obs.psf is None else torch.from_numpy(np.ascontiguousarray(obs.psf[:B], np.float32)).to(dev)
    mags = torch.full((B, npx), float("nan"), dtype=torch.float32, device=dev)
    counts = red = None
    px0 = px1 = 0
    if window is not None:
        px0, px1 = window
        counts = torch.full(((px1 - px0) * E,), 7, dtype=torch.int32, device=dev)
        red = torch.full(((px1 - px0) * E,), 7, dtype=torch.int32, device=dev)
    fpre = torch.empty((B, npx), dtype=torch.float32, device=dev) if want_flux else None
    fpsf = torch.empty((B, npx), dtype=torch.float32, device=dev) if want_flux else None
    ctx.simulate(lam_d, flux_d, obs, mags, psf=psf_d, conv_path=conv_path, counts=counts, reddened=red,
                 px0=px0, px1=px1, flux_pre=fpre, flux_psf=fpsf, stream=stream)
    ctx.sync(stream)
    out = dict(mags=mags.cpu().numpy())
    if window is not None:
        out["counts"] = counts.cpu().numpy().view(np.uint32).reshape(px1 - px0, E).astype(np.int64)
        out["red"] = red.cpu().numpy().view(np.uint32).reshape(px1 - px0, E).astype(np.int64)
    if want_flux:
        out["flux_pre"] = fpre.cpu().numpy()
        out["flux_psf"] = fpsf.cpu().numpy()
    return out


def gpu_hess(ctx, mags_np, grid, bands=(0, 1, 1)):
    import torch
    dev = torch.device("cuda")
    m = torch.from_numpy(np.ascontiguousarray(mags_np, np.float32)).to(dev)
    h = torch.full((grid["nx"] * grid["ny"],), 12345, dtype=torch.int32, device=dev)
    mom = torch.empty(3, dtype=torch.float64, device=dev)
    ctx.hess(m, m.shape[0], m.shape[1], grid, h, mom, bands)
    ctx.sync()
    return h.cpu().numpy().reshape(grid["ny"], grid["nx"]).astype(np.int64), mom.cpu().numpy()


def gpu_loglike(ctx, hm, hd, mom_m, mom_d, mode, eps=0.01):
    import torch
    dev = torch.device("cuda")
    a = torch.from_numpy(np.ascontiguousarray(hm.ravel(), np.int32)).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(hd.ravel(), np.int32)).to(dev)
    mm = torch.from_numpy(np.asarray(mom_m, np.float64)).to(dev)
    md = torch.from_numpy(np.asarray(mom_d, np.float64)).to(dev)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    ctx.loglike(a, b, mm, md, out, mode, eps)
    ctx.sync()
    return float(out.cpu().numpy()[0])


def explain_count_mismatches(lam, seed, px0, got, want):
    """Sort the (pixel, entry) pairs whose counts differ into (unexplained, on_threshold): a pair is
    on a threshold when its 32-bit word lies within 1 of an inversion threshold, or when its alias
    table would move under a one-ulp change of exp(-lambda) (where two FP64 exp implementations may
    legitimately differ).  Diagnostic only: the tests require both lists empty."""
    bad = np.argwhere(got != want)
    unexplained, on_threshold = [], []
    for r, i in bad:
        p = px0 + int(r)
        li = float(lam[i])
        if osamp.ALIAS_MIN <= li < osamp.ALIAS_MAX:
            e = math.exp(-li)
            ref = osamp.alias_table(li)
            moved = False
            for d in (0.0, 1.0):
                alt = osamp.alias_table(li, np.nextafter(e, d))
                moved |= alt[:2] != ref[:2] or not np.array_equal(alt[2], ref[2])
            (on_threshold if moved else unexplained).append((p, int(i)))
            continue
        if li >= osamp.ALIAS_MAX:
            unexplained.append((p, int(i)))
            continue
        w = orng.philox4x32_10(p, i // 4, orng.TAG_MAIN, 0, seed)[i % 4]
        u = int(w)
        near = any(abs(u - t) <= 1 for t in osamp.inversion_thresholds(li))
        (on_threshold if near else unexplained).append((p, int(i)))
    return unexplained, on_threshold


def assert_counts_exact(lam, seed, px0, got, want, what="counts"):
    """Star counts bit-exact: every (pixel, entry) equal.  Prints the number compared and, on a
    failure, how many mismatches sit on a threshold (see explain_count_mismatches)."""
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    n_bad = int((got != want).sum())
    print(f"[bit-exact] {what}: {got.size} compared, {n_bad} differ", flush=True)
    if n_bad:
        unexplained, on_thr = explain_count_mismatches(lam, seed, px0, got, want)
        raise AssertionError(f"{what}: {n_bad} of {got.size} differ ({len(on_thr)} on a threshold, "
                             f"{len(unexplained)} not); first {(unexplained or on_thr)[:5]}")


def explain_block_mismatches(lam, seed, px0, got, want):
    """Block-skip sampler: the (pixel, block) pairs whose counts differ, sorted into (unexplained,
    on_threshold) like explain_count_mismatches (the block total's word within 1 of an inversion
    threshold of Lambda_b).  Diagnostic only."""
    from oracle import sampler_block as sb
    tot = sb.block_sums(lam)
    unexplained, on_threshold = [], []
    for r, b in sorted({(int(r), int(i) // sb.BLOCK) for r, i in np.argwhere(got != want)}):
        p = px0 + r
        L = float(tot[b])
        if L >= osamp.LAM_SWITCH:
            unexplained.append((p, b))
            continue
        u = int(orng.philox4x32_10(p, b, orng.TAG_BLOCK, 0, seed)[0])
        near = any(abs(u - t) <= 1 for t in osamp.inversion_thresholds(L))
        (on_threshold if near else unexplained).append((p, b))
    return unexplained, on_threshold


def assert_block_counts_exact(lam, seed, px0, got, want, what="block-rule counts"):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (got.shape, want.shape)
    n_bad = int((got != want).sum())
    print(f"[bit-exact] {what}: {got.size} compared, {n_bad} differ", flush=True)
    if n_bad:
        unexplained, on_thr = explain_block_mismatches(lam, seed, px0, got, want)
        raise AssertionError(f"{what}: {n_bad} of {got.size} differ ({len(on_thr)} blocks on a threshold, "
                             f"{len(unexplained)} not); first {(unexplained or on_thr)[:5]}")


def rel_err(a, b, floor=1e-300):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def mags_close(gpu, ora64, atol=MAG_ATOL):
    g = np.asarray(gpu, np.float64)
    o = np.asarray(ora64, np.float64)
    same_inf = np.isinf(g) & np.isinf(o) & (np.sign(g) == np.sign(o))
    fin = np.isfinite(g) & np.isfinite(o)
    ok = same_inf | (fin & (np.abs(g - o) <= atol))
    return ok


def near_edge_pixels(mags64, grid, bands=(0, 1, 1), tol=MAG_ATOL):
    """Pixels whose oracle colour or magnitude lies within `tol` mag of a bin edge."""
    m = np.asarray(mags64, np.float64)
    with np.errstate(invalid="ignore"):
        x = m[bands[0]] - m[bands[1]]
        y = m[bands[2]]
        tx = (x - grid["x0"]) / grid["dx"]
        ty = (y - grid["y0"]) / grid["dy"]
        dxe = np.abs(tx - np.round(tx)) * grid["dx"]
        dye = np.abs(ty - np.round(ty)) * grid["dy"]
    near = (np.isfinite(dxe) & (dxe <= tol)) | (np.isfinite(dye) & (dye <= tol))
    return near


def assert_hess_per_pixel(gpu_mags, ora_mags64, grid, bands=(0, 1, 1), tol=MAG_ATOL, what="Hess"):
    """Per pixel: the bin of the GPU magnitudes and the bin of the oracle's (both by the oracle's
    rule) are identical for every pixel whose oracle colour and magnitude lie more than `tol` mag
    from a bin edge.  Returns (pixels compared, pixels near an edge, near-edge pixels that moved)."""
    ixg, iyg, _, _ = oh.pixel_bins(np.asarray(gpu_mags, np.float32), grid, *bands)
    ixo, iyo, _, _ = oh.pixel_bins(np.asarray(ora_mags64, np.float32), grid, *bands)
    near = near_edge_pixels(ora_mags64, grid, bands, tol)
    moved = (ixg != ixo) | (iyg != iyo)
    far_moved = int((moved & ~near).sum())
    print(f"[bit-exact] {what}: {moved.size} pixels binned, {int(near.sum())} within {tol} mag of an edge, "
          f"{int((moved & near).sum())} of those moved, {far_moved} others moved", flush=True)
    assert far_moved == 0, (f"{what}: {far_moved} pixels away from a bin edge land in another bin",
                            np.nonzero(moved & ~near)[0][:5])
    return moved.size, int(near.sum()), int((moved & near).sum())
