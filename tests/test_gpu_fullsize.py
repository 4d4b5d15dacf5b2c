"""GPU parity at the benchmarked sizes, against the oracle run on every host core.

256 x 256, 52,500 points, 3 bands, log-normal dust with F = 1/2, 31 x 31 PSF, shot noise, 100 x 100
Hess (the headline evaluation): the oracle simulates the whole image; the star counts and
reddened counts of 8 windows of 4,096 pixels are compared (through per-pixel digests of the
52,500-long count vectors), the fluxes before and after the PSF and the magnitudes of every
pixel, the Hess pixel by pixel, and the three log-likelihoods.

512 x 512 at Npix = 1e6 (points above the rejection threshold), 63 x 63 PSF on the FFT path,
200 x 200 Hess: the oracle would need ~80 CPU-minutes for the whole image, so the counts and
pre-PSF fluxes are compared on 8 windows of 1,024 pixels, one pixel end to end from its oracle
neighbourhood, and the FFT convolution, noise, magnitudes, Hess and likelihoods over the whole
image against the oracle's own steps applied to the GPU's pre-PSF image.
"""
import dataclasses
import time

import numpy as np
import pytest

import synth_inputs as si
from oracle import entries as oe
from oracle import hess as oh
from oracle import loglike as ol
from oracle import noise as on
from oracle import parallel as opar
from oracle import sampler as osamp
from tests import parity_utils as pu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1904_00011_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _log(msg):
    print(f"[fullsize] {msg}", flush=True)


def _gpu_image(ctx, lam, f32, obs, conv_path=0):
    """Whole image through pcmd_simulate: pre-PSF and post-PSF fluxes and magnitudes."""
    return pu.gpu_simulate(ctx, lam, f32, obs, conv_path, window=None, want_flux=True)


def _gpu_count_digests(ctx, lam, f32, obs, windows, conv_path=0):
    """Digests of the GPU's count and reddened-count vectors of every pixel of `windows`
    (one pcmd_simulate per window with the debug count outputs)."""
    import torch
    dev = torch.device("cuda")
    B, E = f32.shape
    mult = opar.digest_multipliers(E)
    lam_d = torch.from_numpy(np.ascontiguousarray(lam, np.float64)).to(dev)
    flux_d = torch.from_numpy(np.ascontiguousarray(f32, np.float32)).to(dev)
    psf_d = torch.from_numpy(np.ascontiguousarray(obs.psf[:B], np.float32)).to(dev)
    mags = torch.empty((B, obs.nim * obs.nim), dtype=torch.float32, device=dev)
    dc, dr = [], []
    for px0, px1 in windows:
        n = px1 - px0
        counts = torch.full((n * E,), 7, dtype=torch.int32, device=dev)
        red = torch.full((n * E,), 7, dtype=torch.int32, device=dev)
        ctx.simulate(lam_d, flux_d, obs, mags, psf=psf_d, conv_path=conv_path, counts=counts, reddened=red,
                     px0=px0, px1=px1)
        ctx.sync()
        c = counts.cpu().numpy().view(np.uint32).reshape(n, E)
        r = red.cpu().numpy().view(np.uint32).reshape(n, E)
        del counts, red
        for a in range(0, n, 512):
            dc.append(opar.count_digest(c[a:a + 512], mult))
            dr.append(opar.count_digest(r[a:a + 512], mult))
    return np.concatenate(dc), np.concatenate(dr)


def _count_check(lam, obs, windows, dig_g, dig_o, what):
    """Counts bit-exact: the digests agree for every pixel; on a mismatch the pixel's counts are
    recomputed by the oracle to name the entries."""
    bad = np.nonzero(dig_g != dig_o)[0]
    n = len(dig_g)
    _log(f"{what}: {n} pixels x {len(lam)} points compared by digest, {len(bad)} pixels differ")
    assert len(bad) == 0, f"{what}: {len(bad)} pixels with a differing count vector, first {bad[:5]}"


def _windows(npx, n_win, size):
    step = npx // n_win
    return [(k * step, k * step + size) for k in range(n_win)]


def _likelihoods(ctx, hm_g, mom_g, hm_o, mom_o, hd, md, moved, what):
    for mode in (ol.POISSON, ol.GAUSS_PAPER, ol.GAUSS_LITERAL):
        lg = pu.gpu_loglike(ctx, hm_g, hd, mom_g, md, mode)
        # the GPU's likelihood of its own Hess, by the oracle's formula
        assert abs(lg - ol.loglike(hm_g, hd, mom_g, md, mode)) <= max(1e-9 * abs(lg), 1e-9), (what, mode)
        lo = ol.loglike(hm_o, hd, mom_o, md, mode)
        _log(f"{what}: mode {mode} logL GPU {lg:.6f} oracle {lo:.6f} |d| {abs(lg - lo):.2e} "
             f"(near-edge pixels moved: {moved})")
        if moved == 0:
            assert abs(lg - lo) <= pu.LOGL_ATOL, (what, mode, lg, lo)


def test_headline_whole_image_against_the_oracle(ctx):
    """The headline evaluation (256 x 256, 52,500 points) against the oracle's whole image."""
    G = si.headline_grid()
    model, obs = si.draw_headline_params(1011)
    lam, _, f32 = oe.build_entries(model, G)
    N = obs.nim
    npx = N * N
    _log(f"headline: nim={N} E={len(lam)} log_npix={model.log_npix:.3f} alias={(lam >= 2).sum()} "
         f"workers={opar.default_workers()}")
    t = time.time()
    ora = opar.simulate(lam, f32, obs, with_digest=True)
    _log(f"headline: oracle whole image {time.time() - t:.1f} s")
    g = _gpu_image(ctx, lam, f32, obs)
    # every pixel: fluxes before and after the 31 x 31 PSF, magnitudes
    e_pre = np.max(pu.rel_err(g["flux_pre"], ora["F"]))
    e_psf = np.max(pu.rel_err(g["flux_psf"], ora["G"]))
    ok = pu.mags_close(g["mags"], ora["mags64"])
    _log(f"headline: {3 * npx} fluxes, max rel err pre-PSF {e_pre:.2e} post-PSF {e_psf:.2e}; "
         f"{int((~ok).sum())} magnitudes off by > 1e-4")
    assert e_pre <= pu.FLUX_RTOL and e_psf <= pu.FLUX_RTOL
    assert ok.all()
    # counts on 8 windows of 4,096 pixels
    wins = _windows(npx, 8, 4096)
    t = time.time()
    dg_c, dg_r = _gpu_count_digests(ctx, lam, f32, obs, wins)
    _log(f"headline: GPU count digests {time.time() - t:.1f} s")
    idx = np.concatenate([np.arange(a, b) for a, b in wins])
    _count_check(lam, obs, wins, dg_c, ora["digest_counts"][idx], "headline counts")
    _count_check(lam, obs, wins, dg_r, ora["digest_red"][idx], "headline reddened counts")
    # Hess pixel by pixel and the likelihoods against a seeded data Hess
    m64 = ora["mags64"]
    fin = np.isfinite(m64).all(axis=0)
    hgrid = si.hess_grid_from_median(float(np.median((m64[0] - m64[1])[fin])), float(np.median(m64[1][fin])), 100, 100)
    hm_g, mom_g = pu.gpu_hess(ctx, g["mags"], hgrid)
    assert hm_g.sum() == npx
    assert np.array_equal(hm_g, oh.hess(g["mags"], hgrid)[0])
    _, _, moved = pu.assert_hess_per_pixel(g["mags"], m64, hgrid, what="headline Hess")
    hm_o, mom_o = oh.hess(ora["mags"], hgrid)
    if moved == 0:
        assert np.array_equal(hm_g, hm_o)
    hd = np.random.default_rng(2).poisson(hm_o.astype(np.float64) * 1.02)
    md = mom_o * np.array([1.001, 0.999, 1.0])
    _likelihoods(ctx, hm_g, mom_g, hm_o, mom_o, hd, md, moved, "headline")


def test_large_config_against_the_oracle(ctx):
    """512 x 512, Npix = 1e6, 63 x 63 PSF (FFT), 200 x 200 Hess."""
    G = si.headline_grid()
    model, obs = si.draw_large_params(3000)
    lam, _, f32 = oe.build_entries(model, G)
    N = obs.nim
    npx = N * N
    K = obs.psf.shape[-1]
    _log(f"large: nim={N} E={len(lam)} alias={((lam >= 2) & (lam < 512)).sum()} rejection={(lam >= 512).sum()} "
         f"K={K} workers={opar.default_workers()}")
    g = _gpu_image(ctx, lam, f32, obs, conv_path=2)
    # counts and pre-PSF fluxes on 8 windows of 1,024 pixels
    wins = _windows(npx, 8, 1024)
    t = time.time()
    Fo, dc_o, dr_o = opar.simulate_flux(lam, f32, obs, wins, with_digest=True)
    _log(f"large: oracle on {sum(b - a for a, b in wins)} pixels {time.time() - t:.1f} s")
    idx = np.concatenate([np.arange(a, b) for a, b in wins])
    e_pre = np.max(pu.rel_err(g["flux_pre"][:, idx], Fo))
    _log(f"large: pre-PSF fluxes on the windows, max rel err {e_pre:.2e}")
    assert e_pre <= pu.FLUX_RTOL
    dg_c, dg_r = _gpu_count_digests(ctx, lam, f32, obs, wins, conv_path=2)
    _count_check(lam, obs, wins, dg_c, dc_o, "large counts")
    _count_check(lam, obs, wins, dg_r, dr_o, "large reddened counts")
    # one pixel end to end: its 63 x 63 neighbourhood simulated by the oracle
    y0, x0, h = 300, 77, (K - 1) // 2
    nb = [(((y0 + dy) % N) * N + (x0 + dx) % N) for dy in range(-h, h + 1) for dx in range(-h, h + 1)]
    # contiguous runs of the neighbourhood as windows
    runs = []
    for dy in range(-h, h + 1):
        row = ((y0 + dy) % N) * N
        a, b = x0 - h, x0 + h + 1
        assert 0 <= a and b <= N
        runs.append((row + a, row + b))
    t = time.time()
    Fn, _, _ = opar.simulate_flux(lam, f32, obs, runs)
    _log(f"large: oracle neighbourhood of one pixel ({len(nb)} pixels) {time.time() - t:.1f} s")
    Gp = np.einsum("buv,buv->b", obs.psf.astype(np.float32).astype(np.float64)[:, ::-1, ::-1], Fn.reshape(3, K, K))
    p = y0 * N + x0
    assert np.max(pu.rel_err(g["flux_psf"][:, p], Gp)) <= pu.FLUX_RTOL
    assert pu.mags_close(g["mags"][:, p:p + 1], on.magnitudes(Gp[:, None], obs, px=np.array([p]))).all()
    # the whole image from the GPU's pre-PSF fluxes on: the oracle's direct periodic sum (the FFT
    # path computes the same operator), noise and magnitudes, Hess, likelihoods
    t = time.time()
    Go = opar.convolve(g["flux_pre"].astype(np.float64).reshape(3, N, N), obs.psf).reshape(3, npx)
    _log(f"large: oracle direct 63x63 convolution of the whole image {time.time() - t:.1f} s")
    e_psf = np.max(pu.rel_err(g["flux_psf"], Go))
    mo = on.magnitudes(Go, obs)
    ok = pu.mags_close(g["mags"], mo)
    _log(f"large: post-PSF fluxes max rel err {e_psf:.2e}; {int((~ok).sum())} magnitudes off by > 1e-4")
    assert e_psf <= pu.FLUX_RTOL and ok.all()
    fin = np.isfinite(mo).all(axis=0)
    hgrid = si.hess_grid_from_median(float(np.median((mo[0] - mo[1])[fin])), float(np.median(mo[1][fin])), 200, 200)
    hm_g, mom_g = pu.gpu_hess(ctx, g["mags"], hgrid)
    assert hm_g.sum() == npx
    assert np.array_equal(hm_g, oh.hess(g["mags"], hgrid)[0])
    _, _, moved = pu.assert_hess_per_pixel(g["mags"], mo, hgrid, what="large Hess")
    hm_o, mom_o = oh.hess(mo.astype(np.float32), hgrid)
    hd = np.random.default_rng(3).poisson(hm_o.astype(np.float64) * 0.98)
    md = mom_o * np.array([0.999, 1.001, 1.0])
    _likelihoods(ctx, hm_g, mom_g, hm_o, mom_o, hd, md, moved, "large")
