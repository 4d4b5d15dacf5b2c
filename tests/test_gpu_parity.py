"""GPU parity: the HIP path through the C ABI against the oracle on the same seeded inputs."""
import dataclasses
import math

import numpy as np
import pytest

import synth_inputs as si
from oracle import entries as oe
from oracle import hess as oh
from oracle import loglike as ol
from oracle import noise as on
from oracle import pipeline as op
from oracle import psf as ops
from oracle import sampler as osamp
from tests import parity_utils as pu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1904_00011_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def _full_compare(ctx, lam, f32, obs, conv_path=0, hgrid=None, bands=(0, 1, 1)):
    """Whole image on both sides: counts, fluxes, magnitudes, Hess."""
    npx = obs.nim * obs.nim
    g = pu.gpu_simulate(ctx, lam, f32, obs, conv_path, window=(0, npx))
    ora = op.simulate(lam, f32, obs, want_counts=True)
    pu.assert_counts_exact(lam, obs.seed, 0, g["counts"], ora["counts"])
    pu.assert_counts_exact(lam, obs.seed, 0, g["red"], ora["red"], "reddened counts")
    assert np.max(pu.rel_err(g["flux_pre"], ora["F"])) <= pu.FLUX_RTOL
    assert np.max(pu.rel_err(g["flux_psf"], ora["G"])) <= pu.FLUX_RTOL
    ok = pu.mags_close(g["mags"], ora["mags64"])
    assert ok.all(), f"{(~ok).sum()} magnitudes differ by more than 1e-4"
    if hgrid is not None:
        hg, mg = pu.gpu_hess(ctx, g["mags"], hgrid, bands)
        assert hg.sum() == npx
        assert np.array_equal(hg, oh.hess(g["mags"], hgrid, *bands)[0])
        pu.assert_hess_per_pixel(g["mags"], ora["mags64"], hgrid, bands)
    return g, ora


def test_small_case_end_to_end(ctx):
    """64x64, 2 bands, 500 Salpeter points at Npix=100, 5x5 PSF, 0.02 mag noise: all 2.05M counts."""
    grid, model, obs = si.small_case()
    lam, _, f32 = oe.build_entries(model, grid)
    _print_case("small_case_end_to_end", nim=obs.nim, E=len(lam))
    g, ora = _full_compare(ctx, lam, f32, obs)
    x = np.median(ora["mags64"][0] - ora["mags64"][1])
    y = np.median(ora["mags64"][1])
    hgrid = si.hess_grid_from_median(x, y, 100, 100)
    # data Hess from a second seed, likelihood on both sides
    _, _, obs2 = si.small_case(seed=2)
    g2 = pu.gpu_simulate(ctx, lam, f32, obs2, want_flux=False)
    ora2 = op.simulate(lam, f32, obs2)
    hm_g, mm_g = pu.gpu_hess(ctx, g["mags"], hgrid)
    hd_g, md_g = pu.gpu_hess(ctx, g2["mags"], hgrid)
    hm_o, mm_o = oh.hess(ora["mags64"], hgrid)
    hd_o, md_o = oh.hess(ora2["mags64"], hgrid)
    for mode in (ol.POISSON, ol.GAUSS_PAPER, ol.GAUSS_LITERAL):
        lg = pu.gpu_loglike(ctx, hm_g, hd_g, mm_g, md_g, mode)
        lo = ol.loglike(hm_o, hd_o, mm_o, md_o, mode)
        assert abs(lg - lo) <= pu.LOGL_ATOL, (mode, lg, lo)


def test_hess_bit_exact_on_identical_magnitudes(ctx):
    """Given the same FP32 magnitudes both sides bin in FP64: Hess and counts are identical."""
    r = np.random.default_rng(3)
    n = 70001
    mags = np.stack([r.normal(21, 0.7, n), r.normal(20.5, 0.6, n), r.normal(20, 0.6, n)]).astype(np.float32)
    mags[0, :50] = np.inf
    mags[1, 25:75] = np.inf
    mags[2, 100:110] = -np.inf
    mags[0, 200:210] = np.nan
    # magnitudes on a 0.25 lattice and their FP32 neighbours: with the 0.25-wide grid below, the
    # bin quotients are integers or straddle them, where the kernel takes the exact division
    lat = (18.0 + 0.25 * r.integers(0, 40, (3, 3000))).astype(np.float32)
    lat[:, 1000:2000] = np.nextafter(lat[:, 1000:2000], np.float32(np.inf))
    lat[:, 2000:3000] = np.nextafter(lat[:, 2000:3000], np.float32(-np.inf))
    mags[:, 1000:4000] = lat
    for grid, bands in ((dict(x0=-1.0, dx=0.05, nx=60, y0=19.0, dy=0.05, ny=50), (0, 1, 1)),
                        (dict(x0=-5.0, dx=0.25, nx=40, y0=17.0, dy=0.25, ny=24), (0, 1, 1)),
                        (dict(x0=-0.5, dx=0.02, nx=200, y0=18.5, dy=0.02, ny=200), (1, 2, 2)),
                        (dict(x0=-3.0, dx=0.05, nx=256, y0=15.0, dy=0.05, ny=256), (0, 2, 1))):
        _print_case("hess_identical", nx=grid["nx"], ny=grid["ny"], bands=bands)
        hg, mg = pu.gpu_hess(ctx, mags, grid, bands)
        ho, mo = oh.hess(mags, grid, *bands)
        assert np.array_equal(hg, ho)
        assert mg[2] == mo[2] and mg[0] == pytest.approx(mo[0], rel=1e-12) and mg[1] == pytest.approx(mo[1], rel=1e-12)


def test_hess_hand_example(ctx):
    from tests.test_oracle_pipeline import load_hess_example
    rows, Hx = load_hess_example()
    mags = np.array([[r[0] for r in rows], [r[1] for r in rows]], dtype=np.float32)
    hg, _ = pu.gpu_hess(ctx, mags, dict(x0=0.0, dx=0.05, nx=4, y0=20.0, dy=0.05, ny=3))
    assert np.array_equal(hg, Hx)


def test_loglike_modes_against_oracle(ctx):
    r = np.random.default_rng(4)
    for nb in (1, 7, 10000, 40000):
        hm = r.poisson(3.0, nb)
        hd = r.poisson(3.0, nb)
        if nb > 1:
            hm[:: max(nb // 5, 1)] = 0        # empty model bins
        hm[-1] += 1                           # a non-empty model Hess
        mom_m = np.array([40.0 * hm.sum(), 2e3 * hm.sum(), float(hm.sum())])
        mom_d = np.array([41.0 * hd.sum(), 2.01e3 * hd.sum(), float(hd.sum())])
        for mode in (0, 1, 2):
            _print_case("loglike", nbins=nb, mode=mode)
            lg = pu.gpu_loglike(ctx, hm, hd, mom_m, mom_d, mode)
            lo = ol.loglike(hm, hd, mom_m, mom_d, mode)
            assert abs(lg - lo) <= max(1e-9 * abs(lo), 1e-9)
    # an empty model Hess stays finite under the Poisson pseudo-count
    hm = np.zeros(100, np.int64)
    hd = r.poisson(2.0, 100)
    lg = pu.gpu_loglike(ctx, hm, hd, [0, 0, 0], [1, 1, 1], ol.POISSON)
    assert np.isfinite(lg) and abs(lg - ol.loglike(hm, hd, None, None, ol.POISSON)) <= 1e-9 * abs(lg)


def test_entries_against_oracle(ctx):
    import torch
    import paper_1904_00011_amd as P
    G = si.headline_grid()
    for seed in (1000, 1001, 7):
        model, obs = si.draw_headline_params(seed)
        ev = P.Evaluator(ctx, G, 64, None, dict(x0=0, dx=0.05, y0=0, dy=0.05, nx=10, ny=10))
        lam_g = ev.entries(model).cpu().numpy()
        lam_o, _, f32 = oe.build_entries(model, G)
        _print_case("entries", seed=seed)
        assert np.max(pu.rel_err(lam_g, lam_o, 1e-300)[lam_o > 0]) <= 1e-12
        assert np.all(lam_g[lam_o == 0] == 0)
        assert np.array_equal(ev.flux_d.cpu().numpy(), f32)
    for sfh in ("ssp", "const", "dtau", "nonparam"):
        m = si.Model(sfh=sfh, log_npix=3.0, tau_gyr=1.5, ssp_age_index=3, mdf="single", feh_index=2,
                     log_sfh=(1.0, 0.3, 0.5, 1.5, 2.0, 2.2, 1.0))
        ev = P.Evaluator(ctx, G, 64, None, dict(x0=0, dx=0.05, y0=0, dy=0.05, nx=10, ny=10))
        lam_g = ev.entries(m).cpu().numpy()
        lam_o, _, _ = oe.build_entries(m, G)
        _print_case("entries", sfh=sfh)
        assert np.max(pu.rel_err(lam_g, lam_o)[lam_o > 0]) <= 1e-12
        assert lam_g.sum() == pytest.approx(oe.npix_of(m), rel=1e-12)


def _headline_lam(log_npix, seed=1000, stride=1):
    G = si.headline_grid()
    if stride > 1:
        G = G.subsample(stride)
    model, obs = si.draw_headline_params(seed, log_npix=log_npix)
    lam, _, f32 = oe.build_entries(model, G)
    return G, lam, f32, obs


def test_headline_grid_dust_ptrs_fft_sized_psf(ctx):
    """Headline grid (52,500 entries, 52 slices, ragged last block) at Npix=1e5 (PTRS entries), log-normal dust
    with F=1/2, shot noise, 31x31 PSF, on a 40x40 image (ragged pixel blocks)."""
    G, lam, f32, obs = _headline_lam(5.0)
    obs.nim = 40
    _print_case("headline_dust_ptrs", nim=40, E=len(lam), ptrs=int((lam >= 10).sum()))
    assert (lam >= 10).sum() > 100
    npx = 40 * 40
    g = pu.gpu_simulate(ctx, lam, f32, obs, window=(0, npx))
    Fo, s = osamp.simulate_flux(lam, f32, obs, 0, npx, want_counts=True)
    pu.assert_counts_exact(lam, obs.seed, 0, g["counts"], s["counts"])
    pu.assert_counts_exact(lam, obs.seed, 0, g["red"], s["red"], "reddened counts")
    assert np.max(pu.rel_err(g["flux_pre"], Fo)) <= pu.FLUX_RTOL
    Go = ops.convolve_periodic(Fo.reshape(3, 40, 40), obs.psf).reshape(3, npx)
    assert np.max(pu.rel_err(g["flux_psf"], Go)) <= pu.FLUX_RTOL
    mo = on.magnitudes(Go, obs)
    assert pu.mags_close(g["mags"], mo).all()


@pytest.mark.parametrize("log_npix,dust_model,frac,noise,K,sky", [
    (5.0, 1, 0.3, 1, 5, 0.0),      # fixed screen, general split fraction (one word per star)
    (6.0, 2, 0.5, 1, 5, 0.0),      # rejection-heavy (mean lambda ~190), log-normal screen
    (4.0, 2, 1.0, 0, 1, 0.0),      # all stars reddened, no PSF, no noise
    (3.0, 2, 0.0, 2, 3, 0.0),      # dust with F = 0 (no star reddened)
    (2.0, 0, 0.5, 1, 7, 0.0),      # no dust at all
    (3.5, 2, 0.5, 2, 5, 1e5),      # shot noise over a sky as bright as the pixels (1e5 electrons)
])
def test_dust_and_noise_variants(ctx, log_npix, dust_model, frac, noise, K, sky):
    G, lam, f32, obs = _headline_lam(log_npix, seed=1003, stride=10)
    obs.nim = 24
    obs.dust_model = dust_model
    obs.dust_frac = frac
    obs.noise_model = noise
    obs.noise_sigma_mag = (0.02, 0.03, 0.04)
    obs.sky = (sky, 0.5 * sky, 2.0 * sky)
    obs.psf = None if K == 1 else si.psf_stack(K, (1.0, 1.2, 1.4))
    _print_case("variant", log_npix=log_npix, dust=dust_model, frac=frac, noise=noise, K=K, sky=sky, E=len(lam))
    _full_compare(ctx, lam, f32, obs)


def test_edge_cases(ctx):
    # one entry, one pixel, no PSF
    obs = si.Obs(nim=1, seed=5, dmod=20.0, psf=None, noise_model=0)
    lam = np.array([3.0])
    f32 = np.array([[1.0], [0.5]], dtype=np.float32)
    _print_case("edge_one_entry_one_pixel")
    _full_compare(ctx, lam, f32, obs)
    # ragged group of entries, odd image, PSF as wide as the image, zero-lambda entries
    r = np.random.default_rng(6)
    lam = r.uniform(0, 2, 7)
    lam[2] = 0.0
    lam[5] = 12.5
    f32 = r.uniform(0.1, 1, (2, 7)).astype(np.float32)
    obs = si.Obs(nim=17, seed=9, dmod=22.0, psf=si.psf_stack(17, (3.0, 4.0)), noise_model=1,
                 noise_sigma_mag=(0.02, 0.02), dust_model=2, dust_frac=0.5, dust_R=(3.0, 2.0))
    _print_case("edge_ragged", nim=17, E=7)
    _full_compare(ctx, lam, f32, obs)
    # all entries zero: every pixel empty -> +inf magnitudes, NaN colours in bin 0
    lam0 = np.zeros(9)
    obs0 = si.Obs(nim=8, seed=1, dmod=25.0, psf=si.psf_stack(3, (1.0, 1.0)), noise_model=1, noise_sigma_mag=(0.02, 0.02))
    _print_case("edge_empty_pixels")
    g = pu.gpu_simulate(ctx, lam0, f32[:, :1].repeat(9, axis=1), obs0, window=(0, 64))
    assert (g["counts"] == 0).all() and np.isinf(g["mags"]).all()
    hg, mg = pu.gpu_hess(ctx, g["mags"], dict(x0=0.0, dx=0.05, nx=5, y0=20.0, dy=0.05, ny=4))
    assert hg[3, 0] == 64 and mg[2] == 0
    # one band
    lam1 = np.array([0.5, 2.0, 11.0])
    f1 = np.array([[1.0, 0.2, 0.05]], dtype=np.float32)
    obs1 = si.Obs(nim=9, seed=2, dmod=24.0, psf=si.psf_stack(3, (1.0,)), noise_model=1, noise_sigma_mag=(0.05,))
    _print_case("edge_one_band")
    _full_compare(ctx, lam1, f1, obs1)


def test_rule_boundaries(ctx):
    """Entries on both sides of every switch of the count rule (inversion / alias at lambda = 2,
    alias / rejection at 512), the widest alias tables (M = 512) and the narrowest, without dust,
    with the F = 1/2 bit split and with thinning (F = 0.3, 0.8): every count against the oracle."""
    lam = np.array([1.9999999, 2.0, 2.0000001, 3.7, 9.99, 10.0, 63.5, 255.0, 300.0, 511.9, 511.999999,
                    512.0, 512.5, 700.0, 0.0, 0.7, 1000.0, 1500.0, 1e-11, 3e-10, 1e-7, 63.99999999, 64.0,
                    1023.9, 1024.0, 5000.0, 3.99999999, 4.0, 4.0000001])
    E = len(lam)
    f32 = np.linspace(0.2, 1.0, 2 * E).reshape(2, E).astype(np.float32) * 1e-3
    # F = 0.3 and 0.8 thin the entries at lambda >= 2 into two parts, whose own lambdas fall on
    # both sides of 512 (700 x 0.8, 1000 x 0.3, 1500 x 0.3) and below 2 (2.0 x 0.3); F = 1/2 thins
    # the entries from lambda = 4 on (halves on both sides of 512: 1023.9, 1024, 5000) and splits
    # the others one bit per star (3.99999999 on the edge)
    # F = 1e-12 and 1 - 1e-12: one thinned part of every table entry is below 2^-32 per pixel, so
    # its table has the single outcome 0
    for dust, frac in ((0, 0.5), (2, 0.5), (2, 0.3), (1, 0.8), (2, 1e-12), (1, 1.0 - 1e-12)):
        obs = si.Obs(nim=20, seed=4242 + dust, dmod=24.0, psf=None, noise_model=0, dust_model=dust, dust_frac=frac,
                     dust_R=(3.0, 2.0))
        _print_case("rule_boundaries", E=E, dust=dust, frac=frac)
        _full_compare(ctx, lam, f32, obs)


def test_determinism_and_streams(ctx):
    import torch
    G, lam, f32, obs = _headline_lam(4.0, seed=1004, stride=5)
    obs.nim = 48
    a = pu.gpu_simulate(ctx, lam, f32, obs, window=(100, 300))
    b = pu.gpu_simulate(ctx, lam, f32, obs, window=(100, 300))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        c = pu.gpu_simulate(ctx, lam, f32, obs, window=(100, 300), stream=s)
    for k in ("counts", "red", "flux_pre", "flux_psf", "mags"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
    # the counts do not depend on the debug window
    d = pu.gpu_simulate(ctx, lam, f32, obs, window=(200, 260))
    assert np.array_equal(d["counts"], a["counts"][100:160])


def test_device_side_validation(ctx):
    import paper_1904_00011_amd as P
    obs = si.Obs(nim=8, seed=1, dmod=25.0, psf=None, noise_model=0)
    f32 = np.ones((2, 3), np.float32)
    for bad in (np.array([1.0, np.nan, 0.1]), np.array([1.0, -0.5, 0.1]), np.array([1.0, 5e6, 0.1])):
        with pytest.raises(P.PcmdError) as ei:
            pu.gpu_simulate(ctx, bad, f32, obs, want_flux=False)
        assert ei.value.code == P._lib.E_INVAL
    good = si.psf_stack(3, (1.0, 1.0)).astype(np.float32)
    neg = good.copy()   # a negative weight, the sum kept at one
    neg[1, 2, 2] += good[1, 0, 0] + 0.02
    neg[1, 0, 0] = -0.02
    nan = good.copy()
    nan[0, 1, 1] = np.nan
    # the direct path checks the PSF inside the convolution, the FFT path in its own kernel
    for path in (P._lib.CONV_DIRECT, P._lib.CONV_FFT):
        for psf in ((good * 1.1).astype(np.float32), neg, nan):
            obs.psf = psf
            with pytest.raises(P.PcmdError) as ei:
                pu.gpu_simulate(ctx, np.array([1.0, 0.5, 0.1]), f32, obs, conv_path=path, want_flux=False)
            assert ei.value.code == P._lib.E_INVAL
        obs.psf = good
        pu.gpu_simulate(ctx, np.array([1.0, 0.5, 0.1]), f32, obs, conv_path=path, want_flux=False)
    ctx.sync()


def test_host_side_validation(ctx):
    import torch
    import paper_1904_00011_amd as P
    dev = torch.device("cuda")
    lam = torch.ones(3, dtype=torch.float64, device=dev)
    flux = torch.ones((2, 3), dtype=torch.float32, device=dev)
    mags = torch.empty((2, 64), dtype=torch.float32, device=dev)
    for kw in (dict(nim=0), dict(nim=8, psf_k=4), dict(nim=8, dust_frac=1.5, dust_model=2), dict(nim=8, noise_model=5)):
        o = si.Obs(nim=kw.get("nim", 8), seed=1, dmod=25.0, psf=None, noise_model=kw.get("noise_model", 0),
                   dust_model=kw.get("dust_model", 0), dust_frac=kw.get("dust_frac", 0.5))
        psf = None
        if "psf_k" in kw:
            psf = torch.ones((2, 4, 4), dtype=torch.float32, device=dev) / 16
        with pytest.raises(P.PcmdError) as ei:
            ctx.simulate(lam, flux, o, mags, psf=psf)
        assert ei.value.code == P._lib.E_INVAL
    h = torch.empty(10, dtype=torch.int32, device=dev)
    mom = torch.empty(3, dtype=torch.float64, device=dev)
    with pytest.raises(P.PcmdError):
        ctx.hess(mags, 2, 64, dict(x0=0, dx=0.0, y0=0, dy=0.05, nx=5, ny=2), h, mom)
    with pytest.raises(P.PcmdError):
        ctx.hess(mags, 2, 64, dict(x0=0, dx=0.05, y0=0, dy=0.05, nx=5, ny=2), h, mom, bands=(0, 2, 1))
    out = torch.empty(1, dtype=torch.float64, device=dev)
    with pytest.raises(P.PcmdError):
        ctx.loglike(h, h, mom, mom, out, mode=0, eps=0.0)


def test_headline_full_size_sampled(ctx):
    """256x256 image with the full 52,500-entry grid, in the benchmark's configuration: counts and fluxes
    on sampled pixels, post-PSF flux and magnitude of one pixel from its oracle-computed neighbourhood,
    flux conservation and the Hess total over the whole image."""
    import torch
    import paper_1904_00011_amd as P
    G = si.headline_grid()
    model, obs = si.draw_headline_params(1000)
    lam, _, f32 = oe.build_entries(model, G)
    N = obs.nim
    npx = N * N
    _print_case("headline_full_size", nim=N, E=len(lam), log_npix=round(model.log_npix, 3))
    for px0 in (0, 33333):
        g = pu.gpu_simulate(ctx, lam, f32, obs, window=(px0, px0 + 48))
        Fo, s = osamp.simulate_flux(lam, f32, obs, px0, px0 + 48, want_counts=True)
        pu.assert_counts_exact(lam, obs.seed, px0, g["counts"], s["counts"])
        pu.assert_counts_exact(lam, obs.seed, px0, g["red"], s["red"], "reddened counts")
        assert np.max(pu.rel_err(g["flux_pre"][:, px0:px0 + 48], Fo)) <= pu.FLUX_RTOL
    # total flux is conserved by the normalised periodic PSF
    for b in range(3):
        assert g["flux_psf"][b].astype(np.float64).sum() == pytest.approx(g["flux_pre"][b].astype(np.float64).sum(), rel=1e-5)
    # one pixel after the PSF: the oracle builds its 31x31 neighbourhood
    y0, x0 = 100, 200
    K, h = 31, 15
    nb = np.array([((y0 + dy) % N) * N + (x0 + dx) % N for dy in range(-h, h + 1) for dx in range(-h, h + 1)])
    Fr, _ = osamp.simulate_flux(lam, f32, obs, px=nb)
    Fn = Fr.reshape(3, K, K)
    Gp = np.einsum("buv,buv->b", obs.psf.astype(np.float64)[:, ::-1, ::-1], Fn)
    p = y0 * N + x0
    assert np.max(pu.rel_err(g["flux_psf"][:, p], Gp)) <= pu.FLUX_RTOL
    mo = on.magnitudes(Gp[:, None], obs, px=np.array([p]))
    assert pu.mags_close(g["mags"][:, p:p + 1], mo).all()
    hg, mg = pu.gpu_hess(ctx, g["mags"], si.hess_grid_from_median(0.5, 30.0, 100, 100))
    assert hg.sum() == npx


def test_large_config_sampled(ctx):
    """512x512 image, 52,500 entries at Npix = 1e6 (one entry in eight above the rejection
    threshold), 63x63 PSF on the FFT path, 200x200 Hess: counts, splits and fluxes on sampled
    pixels against the oracle, the FFT and direct paths against each other over the whole image,
    flux conservation and the Hess total."""
    G = si.headline_grid()
    model, obs = si.draw_large_params(3000)
    lam, _, f32 = oe.build_entries(model, G)
    N = obs.nim
    npx = N * N
    _print_case("large_full_size", nim=N, E=len(lam), ptrs=int((lam >= 10).sum()), K=obs.psf.shape[-1])
    assert (lam >= 10).sum() > 5000
    for px0 in (0, 200000):
        g = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=2, window=(px0, px0 + 12))
        Fo, s = osamp.simulate_flux(lam, f32, obs, px0, px0 + 12, want_counts=True)
        pu.assert_counts_exact(lam, obs.seed, px0, g["counts"], s["counts"])
        pu.assert_counts_exact(lam, obs.seed, px0, g["red"], s["red"], "reddened counts")
        assert np.max(pu.rel_err(g["flux_pre"][:, px0:px0 + 12], Fo)) <= pu.FLUX_RTOL
    for b in range(3):
        assert g["flux_psf"][b].astype(np.float64).sum() == pytest.approx(g["flux_pre"][b].astype(np.float64).sum(), rel=1e-5)
    d = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1)
    assert np.array_equal(d["flux_pre"], g["flux_pre"])
    assert np.max(pu.rel_err(d["flux_psf"], g["flux_psf"])) <= 1e-6
    m = g["mags"].astype(np.float64)
    fin = np.isfinite(m).all(axis=0)
    hgrid = si.hess_grid_from_median(float(np.median((m[0] - m[1])[fin])), float(np.median(m[1][fin])), 200, 200)
    hg, mg = pu.gpu_hess(ctx, g["mags"], hgrid)
    assert hg.sum() == npx
    ho, mo = oh.hess(m, hgrid)
    assert np.array_equal(hg, ho)  # identical magnitudes bin identically


@pytest.mark.parametrize("N,K", [(64, 5), (64, 31), (64, 63), (128, 31), (32, 1), (32, 7), (16, 5)])
def test_fft_path_against_oracle(ctx, N, K):
    """FFT convolution (power-of-two sides) against the oracle's direct periodic sum."""
    G, lam, f32, obs = _headline_lam(3.5, seed=1005, stride=25)
    obs.nim = N
    obs.psf = None if K == 1 else si.psf_stack(K, (1.6, 1.8, 2.0))
    _print_case("fft_path", N=N, K=K)
    g = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=2 if K > 1 else 0)
    Fo, _ = osamp.simulate_flux(lam, f32, obs)
    assert np.max(pu.rel_err(g["flux_pre"], Fo)) <= pu.FLUX_RTOL
    Go = Fo if K == 1 else ops.convolve_periodic(Fo.reshape(3, N, N), obs.psf).reshape(3, N * N)
    assert np.max(pu.rel_err(g["flux_psf"], Go)) <= pu.FLUX_RTOL
    assert pu.mags_close(g["mags"], on.magnitudes(Go, obs)).all()


def test_fft_and_direct_agree_full_size(ctx):
    G, lam, f32, obs = _headline_lam(3.0, seed=1006, stride=5)
    a = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1)
    b = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=2)
    _print_case("fft_vs_direct", N=obs.nim, K=obs.psf.shape[-1])
    assert np.array_equal(a["flux_pre"], b["flux_pre"])
    assert np.max(pu.rel_err(a["flux_psf"], b["flux_psf"])) <= 1e-6
    assert np.max(np.abs(a["mags"] - b["mags"])) <= 1e-5


def test_fft_transposed_path_agrees_with_direct(ctx):
    """1024 x 1024: the FFT path's column transforms run as row transforms between two in-place
    transposes, with the PSF spectrum kept transposed; against the direct sum (itself checked
    against the oracle at this size), for two PSFs in a row so that the kept spectra are rebuilt."""
    G, lam, f32, obs = _headline_lam(3.0, seed=1007, stride=50)
    obs.nim = 1024
    for sig in ((1.6, 1.8, 2.0), (2.4, 1.2, 3.0)):
        obs.psf = si.psf_stack(31, sig)
        _print_case("fft_transposed", N=1024, K=31, sigma=sig)
        a = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1)
        b = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=2)
        assert np.array_equal(a["flux_pre"], b["flux_pre"])
        assert np.max(pu.rel_err(a["flux_psf"], b["flux_psf"])) <= 1e-6
        assert np.max(np.abs(a["mags"] - b["mags"])) <= 1e-5


def test_fft_needs_power_of_two(ctx):
    import paper_1904_00011_amd as P
    G, lam, f32, obs = _headline_lam(2.0, seed=1, stride=50)
    obs.nim = 48
    with pytest.raises(P.PcmdError) as ei:
        pu.gpu_simulate(ctx, lam, f32, obs, conv_path=2, want_flux=False)
    assert ei.value.code == P._lib.E_UNSUPPORTED


def test_multi_cmd_loglike(ctx):
    """Three bands scored on two colour-magnitude diagrams, (b0 - b1, b1) and (b1 - b2, b2), their
    log-likelihoods added on the device (PCMD_LL_ACCUMULATE): against the oracle's sum on the same
    magnitudes, and the oracle's own simulation of the same image."""
    import torch
    import paper_1904_00011_amd as P
    G, lam, f32, obs = _headline_lam(3.0, seed=1007, stride=25)
    obs.nim = 48
    obs.psf = si.psf_stack(5, (1.0, 1.2, 1.4))
    dev = torch.device("cuda")
    _print_case("multi_cmd", nim=48, E=len(lam))
    ora = op.simulate(lam, f32, obs)
    m64 = ora["mags64"]
    cmd_bands = [(0, 1, 1), (1, 2, 2)]
    grids = []
    for bb, br, bm in cmd_bands:
        fin = np.isfinite(m64).all(axis=0)
        grids.append(si.hess_grid_from_median(float(np.median((m64[bb] - m64[br])[fin])),
                                              float(np.median(m64[bm][fin])), 60, 60))
    # data diagrams from a second seed (oracle side)
    obs_d = dataclasses.replace(obs, seed=obs.seed + 1)
    md = op.simulate(lam, f32, obs_d)["mags64"]
    cmds_o, cmds_g = [], []
    for bands, hg in zip(cmd_bands, grids):
        hd, mom_d = oh.hess(md, hg, *bands)
        cmds_o.append((bands, hg, hd, mom_d))
        cmds_g.append((bands, hg, torch.from_numpy(hd.ravel().astype(np.int32)).to(dev),
                       torch.from_numpy(mom_d.astype(np.float64)).to(dev)))
    model = si.Model(sfh="tau", log_npix=3.0, tau_gyr=1.0, mdf="gauss", feh_mu=0.0, feh_sigma=0.2)
    ev = P.Evaluator(ctx, G, obs.nim, obs.psf, grids[0])
    ev.lam.copy_(torch.from_numpy(lam).to(dev))
    for mode in (ol.POISSON, ol.GAUSS_PAPER):
        # the simulation from the given lambda (the model only fixes the shapes here)
        ctx.simulate(ev.lam, ev.flux_d, obs, ev.mags, psf=ev.psf_d)
        for k, (bands, hg, hd, mom_d) in enumerate(cmds_g):
            h = torch.empty(hg["nx"] * hg["ny"], dtype=torch.int32, device=dev)
            ctx.hess(ev.mags, 3, obs.nim ** 2, hg, h, ev.mom, bands)
            ctx.loglike(h, hd, ev.mom, mom_d, ev.out, mode | (P.LL_ACCUMULATE if k else 0))
        ctx.sync()
        lg = float(ev.out.item())
        mg = ev.mags.cpu().numpy().astype(np.float64)
        lo_same = op.loglike_multi_cmd(mg, cmds_o, mode)
        assert abs(lg - lo_same) <= 1e-9 * abs(lo_same), (mode, lg, lo_same)
        # end to end: each diagram of the GPU image equals the oracle's except for pixels within
        # 1e-4 mag of a bin edge; with none of those the likelihoods agree to 1e-3
        moved = 0
        for b, hg in zip(cmd_bands, grids):
            _, _, nmoved = pu.assert_hess_per_pixel(mg, m64, hg, b, what=f"Hess {b}")
            moved += nmoved
        _print_case("multi_cmd_e2e", mode=mode, near_edge_pixels_moved=moved)
        if moved == 0:
            lo_e2e = op.loglike_multi_cmd(m64, cmds_o, mode)
            assert abs(lg - lo_e2e) <= pu.LOGL_ATOL, (mode, lg, lo_e2e)
    # the Evaluator's own path: one simulation, then both diagrams
    ll = ev.loglike_multi(model, obs, cmds_g)
    ctx.sync()
    assert np.isfinite(float(ll.item()))


@pytest.mark.parametrize("N", [48, 50])
def test_subpixel_psf_grid(ctx, N):
    """The 4 x 4 grid of sub-pixel PSFs (Sec. 2.2) on the direct path: the whole pipeline against
    the oracle (N = 50: regions of 13 and 12 pixels); sixteen copies of one PSF reproduce the
    single-PSF image bit for bit."""
    G, lam, f32, obs = _headline_lam(3.0, seed=1008, stride=25)
    obs.nim = N
    obs.psf = si.psf_subpixel_stack(7, (1.0, 1.2, 1.4))
    _print_case("subpixel_psf", N=N, E=len(lam))
    _full_compare(ctx, lam, f32, obs, conv_path=1)
    one = si.psf_stack(7, (1.0, 1.2, 1.4))
    obs.psf = one
    a = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1)
    obs.psf = np.ascontiguousarray(np.repeat(one[:, None], 16, axis=1))
    b = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1)
    assert np.array_equal(a["flux_psf"], b["flux_psf"])


@pytest.mark.parametrize("N,K", [(64, 7), (128, 31)])
def test_subpixel_psf_grid_fft(ctx, N, K):
    """The 4 x 4 sub-pixel grid on the FFT path (one forward transform, an inverse per region)
    against the oracle's region-by-region periodic sum of the GPU's own pre-PSF image."""
    G, lam, f32, obs = _headline_lam(3.0, seed=1009, stride=25)
    obs.nim = N
    obs.psf = si.psf_subpixel_stack(K, (1.0, 1.2, 1.4))
    _print_case("subpixel_psf_fft", N=N, K=K)
    g = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=2)
    Go = ops.convolve_periodic_subpixel(g["flux_pre"].astype(np.float64).reshape(3, N, N), obs.psf).reshape(3, N * N)
    assert np.max(pu.rel_err(g["flux_psf"], Go)) <= pu.FLUX_RTOL
    assert pu.mags_close(g["mags"], on.magnitudes(Go, obs)).all()
    d = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1)
    assert np.max(pu.rel_err(g["flux_psf"], d["flux_psf"])) <= 1e-6


def test_fft_psf_spectra_follow_the_psf(ctx):
    """The FFT path keeps its PSF spectra between calls: a new PSF in the same buffer, a PSF
    in another buffer and back, and a change of image size each give the oracle's convolution."""
    import torch
    G, lam, f32, obs = _headline_lam(3.0, seed=1010, stride=25)
    dev = torch.device("cuda")
    lam_d = torch.from_numpy(lam).to(dev)
    flux_d = torch.from_numpy(f32).to(dev)
    pa = si.psf_stack(9, (1.0, 1.2, 1.4))
    pb = si.psf_stack(9, (2.0, 1.5, 1.1))
    buf = torch.from_numpy(pa).to(dev)
    other = torch.from_numpy(pb).to(dev)
    # (side, PSF, buffer): `buf` is first given the PSF's contents, `other` always holds pb
    for N, psf_np, psf_d in ((64, pa, buf), (64, pa, buf), (64, pb, buf), (64, pb, other), (64, pa, buf),
                             (128, pa, buf), (128, pa, buf)):
        if psf_d is buf:
            buf.copy_(torch.from_numpy(psf_np))
        o = dataclasses.replace(obs, nim=N, psf=psf_np)
        mags = torch.empty((3, N * N), dtype=torch.float32, device=dev)
        pre = torch.empty_like(mags)
        post = torch.empty_like(mags)
        ctx.simulate(lam_d, flux_d, o, mags, psf=psf_d, conv_path=2, flux_pre=pre, flux_psf=post)
        ctx.sync()
        Fo = pre.cpu().numpy().astype(np.float64).reshape(3, N, N)
        Go = ops.convolve_periodic(Fo, psf_np).reshape(3, N * N)
        _print_case("fft_psf_cache", N=N)
        assert np.max(pu.rel_err(post.cpu().numpy(), Go)) <= pu.FLUX_RTOL


def test_evaluator_writes_into_a_result_slot(ctx):
    """Evaluator.loglike(out=...) writes into one slot of a results vector: the value of the
    default output, the neighbouring slots untouched; an output of the wrong shape is refused."""
    import torch
    import paper_1904_00011_amd as P
    grid, model, obs = si.small_case(nim=32, seed=3)
    dev = torch.device("cuda")
    _print_case("evaluator_out_slot", nim=32)
    ev = P.Evaluator(ctx, grid, obs.nim, obs.psf, dict(x0=0.0, dx=0.05, y0=0.0, dy=0.05, nx=60, ny=60))
    m = ev.simulate(model, obs).cpu().numpy().astype(np.float64)
    fin = np.isfinite(m).all(axis=0)
    ev.hess_grid = si.hess_grid_from_median(float(np.median((m[0] - m[1])[fin])), float(np.median(m[1][fin])), 60, 60)
    dh = torch.empty(3600, dtype=torch.int32, device=dev)
    dm = torch.empty(3, dtype=torch.float64, device=dev)
    ev.hess_of(ev.simulate(model, dataclasses.replace(obs, seed=obs.seed + 1)).clone(), dh, dm)
    ref = float(ev.loglike(model, obs, dh, dm).item())
    res = torch.full((4,), -7.0, dtype=torch.float64, device=dev)
    got = ev.loglike(model, obs, dh, dm, out=res[2:3])
    ctx.sync()
    r = res.cpu().numpy()
    assert got.data_ptr() == res[2:3].data_ptr()
    assert np.isfinite(ref) and r[2] == ref and np.all(r[[0, 1, 3]] == -7.0)
    with pytest.raises(ValueError):
        ev.loglike(model, obs, dh, dm, out=res[0:2])


@pytest.mark.parametrize("K,sub", [(5, False), (9, False), (7, True)])
def test_direct_conv_one_group_blocks_against_oracle(ctx, K, sub):
    """1024 x 1024 x 2 bands: enough 64 x 16 tiles (2,048) that the direct convolution runs its
    one-group blocks (no row split).  The GPU's post-PSF image against the oracle's FP64 periodic
    sum of the GPU's own pre-PSF image, every pixel; with the 4 x 4 sub-pixel grid too."""
    from oracle import parallel as opar
    grid, model, obs = si.small_case(nim=1024, seed=11)
    lam, _, f32 = oe.build_entries(model, grid)
    obs.psf = si.psf_subpixel_stack(K, (1.0, 1.3)) if sub else si.psf_stack(K, (1.0, 1.3))
    _print_case("direct_conv_one_group", N=1024, K=K, subpixel=sub)
    g = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1)
    F = g["flux_pre"].astype(np.float64).reshape(2, 1024, 1024)
    if sub:
        Go = ops.convolve_periodic_subpixel(F, obs.psf)
    else:
        Go = opar.convolve(F, obs.psf)
    e = np.max(pu.rel_err(g["flux_psf"], Go.reshape(2, -1)))
    print(f"[case] direct_conv_one_group K={K} sub={sub}: max rel err {e:.2e}", flush=True)
    assert e <= pu.FLUX_RTOL
