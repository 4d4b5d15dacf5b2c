"""GPU parity of the block-skip sampler (Poisson superposition, Sec. 2.1 footnote) against its
oracle, and its law against the per-point rule's."""
import dataclasses

import numpy as np
import pytest

import synth_inputs as si
from oracle import entries as oe
from oracle import pipeline as op
from oracle import sampler as osamp
from oracle import sampler_block as sb
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


def _block(obs):
    return dataclasses.replace(obs, sampler=1)


def _compare_window(ctx, lam, f32, obs, px0, px1, conv_path=0):
    g = pu.gpu_simulate(ctx, lam, f32, obs, conv_path, window=(px0, px1))
    Fo, s = osamp.simulate_flux(lam, f32, obs, px0, px1, want_counts=True)
    pu.assert_block_counts_exact(lam, obs.seed, px0, g["counts"], s["counts"])
    assert np.array_equal(g["red"], s["red"])
    assert np.max(pu.rel_err(g["flux_pre"][:, px0:px1], Fo)) <= pu.FLUX_RTOL
    return g, s


def test_small_case_end_to_end(ctx):
    """64x64, 500 Salpeter points at Npix = 100, 5x5 PSF, noise: every count, flux, magnitude."""
    grid, model, obs = si.small_case()
    obs = _block(obs)
    lam, _, f32 = oe.build_entries(model, grid)
    _print_case("block_small_case", nim=obs.nim, E=len(lam), blocks=len(sb.block_sums(lam)))
    npx = obs.nim * obs.nim
    g = pu.gpu_simulate(ctx, lam, f32, obs, window=(0, npx))
    ora = op.simulate(lam, f32, obs, want_counts=True)
    pu.assert_block_counts_exact(lam, obs.seed, 0, g["counts"], ora["counts"])
    assert np.array_equal(g["red"], ora["red"])
    assert np.max(pu.rel_err(g["flux_pre"], ora["F"])) <= pu.FLUX_RTOL
    assert np.max(pu.rel_err(g["flux_psf"], ora["G"])) <= pu.FLUX_RTOL
    assert pu.mags_close(g["mags"], ora["mags64"]).all()
    # a different stream from the per-point rule, with the same total star count to a few sigma
    p = pu.gpu_simulate(ctx, lam, f32, dataclasses.replace(obs, sampler=0), window=(0, npx))
    assert not np.array_equal(p["counts"], g["counts"])
    tot = lam.sum() * npx
    assert abs(g["counts"].sum() - tot) < 6 * np.sqrt(tot) and abs(p["counts"].sum() - tot) < 6 * np.sqrt(tot)


@pytest.mark.parametrize("log_npix,dust_model,frac,K", [
    (1.0, 2, 0.5, 5),     # sparse: most blocks draw no star
    (3.0, 1, 0.3, 3),     # general split fraction (one word per star)
    (4.5, 2, 1.0, 1),     # block totals by transformed rejection, every star reddened
    (2.0, 2, 0.0, 5),     # dust with F = 0
    (2.5, 0, 0.5, 7),     # no dust at all
])
def test_variants(ctx, log_npix, dust_model, frac, K):
    """Headline grid (every 10th point: 5,250 points, 83 blocks, a ragged last block) on a 24x24
    image: counts, reddened counts and fluxes of every pixel."""
    G = si.headline_grid().subsample(10)
    model, obs = si.draw_headline_params(1003, log_npix=log_npix)
    lam, _, f32 = oe.build_entries(model, G)
    obs = dataclasses.replace(obs, nim=24, dust_model=dust_model, dust_frac=frac, sampler=1,
                              psf=None if K == 1 else si.psf_stack(K, (1.0, 1.2, 1.4)))
    tot = sb.block_sums(lam)
    _print_case("block_variant", log_npix=log_npix, dust=dust_model, frac=frac, K=K, E=len(lam),
                ptrs_blocks=int((tot >= 10).sum()))
    if log_npix >= 4.5:
        assert (tot >= 10).sum() >= 10
    _compare_window(ctx, lam, f32, obs, 0, 24 * 24)


def test_headline_full_size_sampled(ctx):
    """256x256 image, all 52,500 points (821 blocks, 52 slices) at Npix = 100 and at Npix = 1e4:
    two sampled pixel windows each, against the oracle."""
    G = si.headline_grid()
    for log_npix in (2.0, 4.0):
        model, obs = si.draw_headline_params(1000, log_npix=log_npix)
        obs = _block(obs)
        lam, _, f32 = oe.build_entries(model, G)
        _print_case("block_headline_full_size", nim=obs.nim, E=len(lam), log_npix=log_npix)
        for px0 in (0, 40001):
            _compare_window(ctx, lam, f32, obs, px0, px0 + 40)


def test_edge_cases(ctx):
    # one point, one pixel
    obs = si.Obs(nim=1, seed=5, dmod=20.0, psf=None, noise_model=0, sampler=1)
    _print_case("block_edge_one_point")
    _compare_window(ctx, np.array([3.0]), np.array([[1.0], [0.5]], np.float32), obs, 0, 1)
    # zero points inside blocks, a block of zeros, a block whose stars all sit on its first point,
    # a point whose share rounds to nothing, and a ragged last block
    r = np.random.default_rng(8)
    lam = r.uniform(0.0, 0.3, 64 * 4 + 9)
    lam[64:128] = 0.0
    lam[128:192] = 0.0
    lam[128] = 2.5
    lam[200] = 1e-12
    lam[10:20] = 0.0
    f32 = r.uniform(0.1, 1.0, (2, len(lam))).astype(np.float32)
    obs = si.Obs(nim=19, seed=11, dmod=23.0, psf=si.psf_stack(5, (1.0, 1.3)), noise_model=1,
                 noise_sigma_mag=(0.02, 0.02), dust_model=2, dust_frac=0.5, dust_R=(3.0, 2.0), sampler=1)
    _print_case("block_edge_ragged", nim=19, E=len(lam))
    g, s = _compare_window(ctx, lam, f32, obs, 0, 19 * 19)
    assert (g["counts"][:, lam == 0] == 0).all()
    assert (g["counts"][:, 129:192] == 0).all() and g["counts"][:, 128].sum() > 0
    # every point empty
    lam0 = np.zeros(70)
    _print_case("block_edge_empty")
    g0 = pu.gpu_simulate(ctx, lam0, np.ones((2, 70), np.float32), si.Obs(nim=8, seed=1, dmod=25.0, psf=None,
                                                                          noise_model=0, sampler=1), window=(0, 64))
    assert (g0["counts"] == 0).all() and np.isinf(g0["mags"]).all()


def test_law_matches_per_point_rule(ctx):
    """Same law as the per-point rule (no oracle involved): over 65,536 pixels the per-point star
    totals of the three samplers are Poisson(65,536 lambda_i) to a few sigma, and the total of
    each block has the Poisson variance."""
    r = np.random.default_rng(21)
    lam = np.concatenate([r.uniform(0.0, 0.02, 128), r.uniform(0.05, 0.4, 64), np.full(40, 0.25)])
    E = len(lam)
    f32 = np.ones((2, E), np.float32)
    npx = 256 * 256
    obs = si.Obs(nim=256, seed=77, dmod=25.0, psf=None, noise_model=0, dust_model=2, dust_frac=0.3,
                 dust_R=(3.0, 2.0), sampler=1)
    _print_case("block_law", E=E, npx=npx)
    for sampler in (1, 0, 2):
        g = pu.gpu_simulate(ctx, lam, f32, dataclasses.replace(obs, sampler=sampler), window=(0, npx),
                            want_flux=False)
        n = g["counts"]
        z = (n.sum(axis=0) - npx * lam) / np.sqrt(np.maximum(npx * lam, 1e-9))
        assert np.all(np.abs(z) < 5.5), (sampler, np.abs(z).max())
        red = g["red"].sum() / n.sum()
        assert abs(red - 0.3) < 5 * np.sqrt(0.21 / n.sum())
        for b in range(3):
            Nb = n[:, 64 * b: 64 * (b + 1)].sum(axis=1)
            L = lam[64 * b: 64 * (b + 1)].sum()
            assert abs(Nb.var() / L - 1.0) < 6 * np.sqrt(2.0 / npx) + 0.02, (sampler, b, Nb.var(), L)


def _compare_window_hybrid(ctx, lam, f32, obs, px0, px1):
    g = pu.gpu_simulate(ctx, lam, f32, obs, window=(px0, px1))
    Fo, s = osamp.simulate_flux(lam, f32, obs, px0, px1, want_counts=True)
    lam_blk, lam_pt = sb.hybrid_split(lam)
    on_blk = lam_blk > 0
    gb, ob = np.where(on_blk, g["counts"], 0), np.where(on_blk, s["counts"], 0)
    gp, op_ = np.where(on_blk, 0, g["counts"]), np.where(on_blk, 0, s["counts"])
    pu.assert_block_counts_exact(lam_blk, obs.seed, px0, gb, ob, "hybrid: block-rule counts")
    pu.assert_counts_exact(lam_pt, obs.seed, px0, gp, op_, "hybrid: per-point counts")
    assert np.array_equal(g["red"], s["red"])
    assert np.max(pu.rel_err(g["flux_pre"][:, px0:px1], Fo)) <= pu.FLUX_RTOL
    return g, s


@pytest.mark.parametrize("log_npix,dust_model,frac", [(1.0, 2, 0.5), (3.5, 1, 0.3), (4.5, 2, 1.0), (5.0, 0, 0.5)])
def test_hybrid_variants(ctx, log_npix, dust_model, frac):
    """Hybrid sampler (blocks with Lambda_b < 10 by the block rule, the others per point) on the
    headline grid's every 10th point, 24x24: every count and flux against the oracle."""
    G = si.headline_grid().subsample(10)
    model, obs = si.draw_headline_params(1003, log_npix=log_npix)
    lam, _, f32 = oe.build_entries(model, G)
    obs = dataclasses.replace(obs, nim=24, dust_model=dust_model, dust_frac=frac, sampler=2,
                              psf=si.psf_stack(5, (1.0, 1.2, 1.4)))
    tot = sb.block_sums(lam)
    _print_case("hybrid_variant", log_npix=log_npix, dust=dust_model, frac=frac,
                block_rule=int(((tot > 0) & (tot < 10)).sum()), point_rule=int((tot >= 10).sum()))
    _compare_window_hybrid(ctx, lam, f32, obs, 0, 24 * 24)


def test_hybrid_full_size_sampled(ctx):
    """256x256, all 52,500 points at Npix = 1e4 (both rules in use): two sampled windows."""
    model, obs = si.draw_headline_params(1000, log_npix=4.0)
    obs = dataclasses.replace(obs, sampler=2)
    lam, _, f32 = oe.build_entries(model, si.headline_grid())
    tot = sb.block_sums(lam)
    _print_case("hybrid_full_size", E=len(lam), block_rule=int(((tot > 0) & (tot < 10)).sum()),
                point_rule=int((tot >= 10).sum()))
    assert ((tot > 0) & (tot < 10)).sum() > 50 and (tot >= 10).sum() > 50
    for px0 in (0, 40001):
        _compare_window_hybrid(ctx, lam, f32, obs, px0, px0 + 40)


def test_validation(ctx):
    import paper_1904_00011_amd as P
    f32 = np.ones((2, 64), np.float32)
    # block sums at or above 2^22 are reported (each point alone is in range)
    obs = si.Obs(nim=8, seed=1, dmod=25.0, psf=None, noise_model=0, sampler=1)
    with pytest.raises(P.PcmdError) as ei:
        pu.gpu_simulate(ctx, np.full(64, 1e5), f32, obs, want_flux=False)
    assert ei.value.code == P._lib.E_INVAL
    ctx.sync()
    with pytest.raises(P.PcmdError) as ei:
        pu.gpu_simulate(ctx, np.full(64, 0.1), f32, dataclasses.replace(obs, sampler=3), want_flux=False)
    assert ei.value.code == P._lib.E_INVAL
    # the hybrid rule leaves such a block to the per-point rule: no error
    pu.gpu_simulate(ctx, np.full(64, 1e5), f32, dataclasses.replace(obs, sampler=2), want_flux=False)
    # a batch job with the block rule reports the same block-sum finding at pcmd_sync
    import torch
    dev = torch.device("cuda")
    lam = torch.full((64,), 1e5, dtype=torch.float64, device=dev)
    flux = torch.ones((2, 64), dtype=torch.float32, device=dev)
    hd = torch.zeros(16, dtype=torch.int32, device=dev)
    md = torch.zeros(3, dtype=torch.float64, device=dev)
    ll = torch.empty(1, dtype=torch.float64, device=dev)
    hg = dict(x0=0.0, dx=0.5, nx=4, y0=20.0, dy=0.5, ny=4)
    ctx.batch_run([dict(lam=lam, flux=flux, obs=obs, psf=None, conv_path=P._lib.CONV_DIRECT)], hg, hd, md, ll)
    with pytest.raises(P.PcmdError) as ei:
        ctx.sync()
    assert ei.value.code == P._lib.E_INVAL
    ctx.sync()
