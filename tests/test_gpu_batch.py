"""Batched persistent launch: bit-identical to sequential single calls, under every schedule and
under graph replay with new parameters."""
import dataclasses

import numpy as np
import pytest

import synth_inputs as si
from oracle import entries as oe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1904_00011_amd as P
    c = P.Context(0)
    yield c
    c.close()


def _jobs(n, seed0, psf_k=7, nim_log2=(4.0, 5.6), entries=(400, 2500)):
    import torch
    dev = torch.device("cuda")
    out = []
    for grid, model, obs in si.batch_workload(n, seed0, nim_log2=nim_log2, entries=entries, psf_k=psf_k):
        lam, _, f32 = oe.build_entries(model, grid)
        if seed0 % 2 == 0 and len(out) % 3 == 1:
            obs.dust_model = 1          # some jobs with a fixed screen and a general fraction
            obs.dust_frac = 0.3
        if len(out) % 4 == 3:
            obs.dust_model = 0          # some without dust (no split)
        if len(out) % 5 == 2 and psf_k > 1:
            obs.psf = si.psf_subpixel_stack(psf_k, (1.0, 1.2, 1.4))   # some with the 4 x 4 sub-pixel grid
        out.append(dict(lam=torch.from_numpy(lam).to(dev), flux=torch.from_numpy(f32).to(dev), obs=obs,
                        psf=torch.from_numpy(obs.psf).to(dev), conv_path=1))
    return out


def _data(ctx):
    import torch
    dev = torch.device("cuda")
    r = np.random.default_rng(0)
    hess = torch.from_numpy(r.poisson(2.0, 100 * 100).astype(np.int32)).to(dev)
    mom = torch.tensor([0.4 * 1e4, 30.0 * 1e4, 1e4], dtype=torch.float64, device=dev)
    grid = dict(x0=-2.0, dx=0.05, y0=26.0, dy=0.05, nx=100, ny=100)
    return hess, mom, grid


def _sequential(ctx, jobs, grid, hess_d, mom_d, mode):
    import torch
    dev = torch.device("cuda")
    ll, hs = [], []
    for j in jobs:
        N = j["obs"].nim
        mags = torch.empty((3, N * N), dtype=torch.float32, device=dev)
        ctx.simulate(j["lam"], j["flux"], j["obs"], mags, psf=j["psf"], conv_path=j["conv_path"])
        h = torch.empty(100 * 100, dtype=torch.int32, device=dev)
        mom = torch.empty(3, dtype=torch.float64, device=dev)
        ctx.hess(mags, 3, N * N, grid, h, mom)
        out = torch.empty(1, dtype=torch.float64, device=dev)
        ctx.loglike(h, hess_d, mom, mom_d, out, mode, 0.01)
        ll.append(out.clone())
        hs.append(h.clone())
    ctx.sync()
    return torch.cat(ll).cpu().numpy(), torch.stack(hs).cpu().numpy()


@pytest.mark.parametrize("mode", [0, 1])
def test_batch_equals_sequential(ctx, mode):
    import torch
    dev = torch.device("cuda")
    jobs = _jobs(12, 10)
    hess_d, mom_d, grid = _data(ctx)
    print(f"[case] batch_equals_sequential mode={mode} sizes={[j['obs'].nim for j in jobs]}", flush=True)
    ll_s, h_s = _sequential(ctx, jobs, grid, hess_d, mom_d, mode)
    ll_b = torch.empty(len(jobs), dtype=torch.float64, device=dev)
    h_b = torch.empty((len(jobs), 100 * 100), dtype=torch.int32, device=dev)
    ctx.batch_run(jobs, grid, hess_d, mom_d, ll_b, mode=mode, hess_out=h_b)
    ctx.sync()
    assert np.array_equal(h_b.cpu().numpy(), h_s)
    assert np.array_equal(ll_b.cpu().numpy(), ll_s)


def test_batch_schedules_do_not_change_results(ctx):
    import torch
    dev = torch.device("cuda")
    jobs = _jobs(9, 21)
    hess_d, mom_d, grid = _data(ctx)
    ref = None
    for wg, order in ((1, 0), (2, 1), (4, 0), (8, 1)):
        print(f"[case] schedule wg={wg} order={order}", flush=True)
        ctx.batch_set_tuning(wg, order)
        ll = torch.empty(len(jobs), dtype=torch.float64, device=dev)
        ctx.batch_run(jobs, grid, hess_d, mom_d, ll)
        ctx.sync()
        v = ll.cpu().numpy()
        if ref is None:
            ref = v
        assert np.array_equal(v, ref)
    ctx.batch_set_tuning(4, 0)


def test_batch_graph_replay_with_new_parameters(ctx):
    import torch
    dev = torch.device("cuda")
    hess_d, mom_d, grid = _data(ctx)
    base = _jobs(8, 30)
    for rep in range(4):
        # same shapes, new seeds and parameters on every replay
        jobs = []
        for k, j in enumerate(base):
            _, model, obs = si.batch_workload(8, 30, nim_log2=(4.0, 5.6), entries=(400, 2500), psf_k=7)[k]
            o = j["obs"]
            obs.nim = o.nim
            obs.dust_model, obs.dust_frac = o.dust_model, o.dust_frac
            obs.seed = 1000 * rep + k
            obs.dmod = 24.0 + rep
            jobs.append(dict(j, obs=obs))
        print(f"[case] graph replay {rep}", flush=True)
        ll_s, _ = _sequential(ctx, jobs, grid, hess_d, mom_d, 0)
        ll_g = torch.empty(len(jobs), dtype=torch.float64, device=dev)
        ctx.batch_run(jobs, grid, hess_d, mom_d, ll_g, use_graph=True)
        x = torch.ones(1000, device=dev).sum()          # eager work between replays
        ctx.sync()
        assert np.array_equal(ll_g.cpu().numpy(), ll_s), rep
        assert float(x) == 1000.0


def test_batch_draws_the_thinned_entries_of_the_jobs_that_have_them(ctx):
    """F = 1/2 jobs with many entries at lambda >= 4 (log Npix 4.5, thinned) among jobs with none
    (log Npix 1): the thinned-entry pass runs for the jobs whose preparation of this call thinned
    an entry (the others' launches return at once), bit-identical to sequential calls; then the
    two kinds swap places under the replayed graph."""
    import torch
    dev = torch.device("cuda")
    hess_d, mom_d, grid = _data(ctx)
    for rep in range(2):
        jobs, n_thin = [], []
        for k, (g, model, obs) in enumerate(si.batch_workload(10, 80, nim_log2=(4.0, 5.6), entries=(400, 2500),
                                                              psf_k=7)):
            model.log_npix = 4.5 if (k + rep) % 2 == 0 else 1.0
            obs.dust_model, obs.dust_frac, obs.seed = 2, 0.5, 900 + 10 * rep + k
            lam, _, f32 = oe.build_entries(model, g)
            n_thin.append(int((lam >= 4.0).sum()))
            jobs.append(dict(lam=torch.from_numpy(lam).to(dev), flux=torch.from_numpy(f32).to(dev), obs=obs,
                             psf=torch.from_numpy(obs.psf).to(dev), conv_path=1))
        assert min(n_thin) == 0 and min(n_thin[(rep % 2)::2]) > 50, n_thin
        print(f"[case] batch thinned jobs rep={rep} thinned entries per job={n_thin}", flush=True)
        ll_s, h_s = _sequential(ctx, jobs, grid, hess_d, mom_d, 0)
        ll_b = torch.empty(len(jobs), dtype=torch.float64, device=dev)
        h_b = torch.empty((len(jobs), 100 * 100), dtype=torch.int32, device=dev)
        ctx.batch_run(jobs, grid, hess_d, mom_d, ll_b, mode=0, hess_out=h_b, use_graph=True)
        ctx.sync()
        assert np.array_equal(h_b.cpu().numpy(), h_s)
        assert np.array_equal(ll_b.cpu().numpy(), ll_s)


def test_batch_autotune_and_validation(ctx):
    import torch
    import paper_1904_00011_amd as P
    dev = torch.device("cuda")
    jobs = _jobs(6, 40)
    hess_d, mom_d, grid = _data(ctx)
    ll = torch.empty(len(jobs), dtype=torch.float64, device=dev)
    best, ms = ctx.batch_autotune(jobs, grid, hess_d, mom_d, ll)
    print(f"[case] autotune best={best} ms={ms}", flush=True)
    assert len(ms) == 8 and all(m > 0 for m in ms)
    assert ctx.batch_get_tuning() == best
    ll_s, _ = _sequential(ctx, jobs, grid, hess_d, mom_d, 0)
    ctx.batch_run(jobs, grid, hess_d, mom_d, ll)
    ctx.sync()
    assert np.array_equal(ll.cpu().numpy(), ll_s)
    # a job whose convolution resolves to the FFT path is refused
    bad = [dict(jobs[0], conv_path=2)]
    with pytest.raises(P.PcmdError) as ei:
        ctx.batch_run(bad, grid, hess_d, mom_d, ll)
    assert ei.value.code in (P._lib.E_UNSUPPORTED, P._lib.E_INVAL)
    two = [jobs[0], dict(jobs[1], flux=jobs[1]["flux"][:2].contiguous())]
    with pytest.raises(P.PcmdError):
        ctx.batch_run(two, grid, hess_d, mom_d, ll)
    ctx.batch_set_tuning(4, 0)


def test_batch_graph_replay_when_the_split_mode_changes(ctx):
    """Same shapes, but the jobs' dust fraction moves from 1/2 (one bit per star) to 0.3 (entries
    at lambda >= 2 thinned into two parts, each with its own alias table) and back: every replay
    equals the sequential calls.  A plan keyed on the shapes alone would keep the 1/2 plan, whose
    launches build no tables for the reddened parts."""
    import torch
    dev = torch.device("cuda")
    hess_d, mom_d, grid = _data(ctx)
    base = si.batch_workload(6, 50, nim_log2=(4.0, 5.0), entries=(1000, 2500), psf_k=7)
    jobs0 = []
    for k, (g, model, obs) in enumerate(base):
        model.log_npix = 4.5                     # entries above lambda = 2, drawn by alias tables
        lam, _, f32 = oe.build_entries(model, g)
        assert (lam >= 2.0).sum() > 10
        obs.dust_model = 2
        jobs0.append(dict(lam=torch.from_numpy(lam).to(dev), flux=torch.from_numpy(f32).to(dev), obs=obs,
                          psf=torch.from_numpy(obs.psf).to(dev), conv_path=1))
    for rep, frac in enumerate((0.5, 0.3, 0.5, 0.8)):
        jobs = []
        for k, j in enumerate(jobs0):
            o = dataclasses.replace(j["obs"], dust_frac=frac, seed=700 + 10 * rep + k)
            jobs.append(dict(j, obs=o))
        print(f"[case] split mode replay {rep} frac={frac}", flush=True)
        ll_s, h_s = _sequential(ctx, jobs, grid, hess_d, mom_d, 0)
        ll_g = torch.empty(len(jobs), dtype=torch.float64, device=dev)
        h_g = torch.empty((len(jobs), 100 * 100), dtype=torch.int32, device=dev)
        ctx.batch_run(jobs, grid, hess_d, mom_d, ll_g, hess_out=h_g, use_graph=True)
        ctx.sync()
        assert np.array_equal(h_g.cpu().numpy(), h_s), rep
        assert np.array_equal(ll_g.cpu().numpy(), ll_s), rep


def test_batch_at_uneven_full_shapes_against_the_oracle(ctx):
    """Jobs of the uneven-batch workload's own shapes (sides 64 to 512, 5,000 to 52,500 points,
    31 x 31 PSF, log-normal dust with F = 1/2, shot noise) through pcmd_batch_run, each against the
    oracle's whole image run on every host core: the counts and reddened counts of a 1,024-pixel
    window bit-exact (digests), the Hess pixel by pixel (the GPU magnitudes are those of the
    sequential call, whose Hess equals the batch's), and the log-likelihood (Appendix A
    re-simulations go through this call)."""
    import torch
    from oracle import hess as oh
    from oracle import loglike as ol
    from oracle import parallel as opar
    from tests import parity_utils as pu
    dev = torch.device("cuda")
    base = si.headline_grid()
    specs = [(64, 5000), (128, 20000), (256, 52500), (512, 12000), (208, 30000)]
    jobs, host = [], []
    for k, (N, E) in enumerate(specs):
        G = base.subsample(max(1, int(round(base.n_entries / E))))
        model, obs = si.draw_headline_params(600 + k)
        obs.nim = N
        lam, _, f32 = oe.build_entries(model, G)
        host.append((lam, f32, obs))
        jobs.append(dict(lam=torch.from_numpy(lam).to(dev), flux=torch.from_numpy(f32).to(dev), obs=obs,
                         psf=torch.from_numpy(obs.psf).to(dev), conv_path=1))
    # data: the 256 x 256 job at seed 2, Hess grid from its medians
    lam2, f2, o2 = host[2]
    d = pu.gpu_simulate(ctx, lam2, f2, dataclasses.replace(o2, seed=2), conv_path=1, want_flux=False)
    md = d["mags"].astype(np.float64)
    fin = np.isfinite(md).all(axis=0)
    hgrid = si.hess_grid_from_median(float(np.median((md[0] - md[1])[fin])), float(np.median(md[1][fin])), 100, 100)
    hd, momd = pu.gpu_hess(ctx, d["mags"], hgrid)
    hd_d = torch.from_numpy(hd.astype(np.int32)).to(dev)
    md_d = torch.from_numpy(momd).to(dev)
    ll_b = torch.empty(len(jobs), dtype=torch.float64, device=dev)
    h_b = torch.empty((len(jobs), 100 * 100), dtype=torch.int32, device=dev)
    ctx.batch_run(jobs, hgrid, hd_d, md_d, ll_b, mode=0, hess_out=h_b)
    ctx.sync()
    ll_b, h_b = ll_b.cpu().numpy(), h_b.cpu().numpy()
    for k, (lam, f32, obs) in enumerate(host):
        N = obs.nim
        npx = N * N
        w0 = (npx // 3) & ~63
        w1 = min(npx, w0 + 1024)
        print(f"[case] batch job {k}: nim={N} E={len(lam)} log_npix={si.draw_headline_params(600 + k)[0].log_npix:.2f} "
              f"window=({w0}, {w1})", flush=True)
        g = pu.gpu_simulate(ctx, lam, f32, obs, conv_path=1, window=(w0, w1), want_flux=False)
        hg, momg = pu.gpu_hess(ctx, g["mags"], hgrid)
        assert np.array_equal(hg.ravel(), h_b[k]), k            # batch == sequential
        assert h_b[k].sum() == npx
        ora = opar.simulate(lam, f32, obs, with_digest=True)
        mult = opar.digest_multipliers(len(lam))
        assert np.array_equal(opar.count_digest(g["counts"], mult), ora["digest_counts"][w0:w1]), k
        assert np.array_equal(opar.count_digest(g["red"], mult), ora["digest_red"][w0:w1]), k
        _, _, moved = pu.assert_hess_per_pixel(g["mags"], ora["mags64"], hgrid, what=f"batch job {k} Hess")
        ho, momo = oh.hess(ora["mags"], hgrid)
        lo = ol.loglike(ho, hd, momo, momd, ol.POISSON, 0.01)
        print(f"[case] batch job {k}: logL batch {ll_b[k]:.6f} oracle {lo:.6f} |d| {abs(ll_b[k] - lo):.2e} "
              f"(near-edge pixels moved: {moved})", flush=True)
        assert abs(ll_b[k] - ol.loglike(h_b[k], hd.ravel(), momg, momd, ol.POISSON, 0.01)) <= 1e-9 * abs(ll_b[k])
        if moved == 0:
            assert np.array_equal(h_b[k], ho.ravel())
            assert abs(ll_b[k] - lo) <= pu.LOGL_ATOL


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_with_block_and_hybrid_samplers(ctx, use_graph):
    """Jobs with the per-point, block-skip and hybrid samplers in one batch: every job's Hess and
    log-likelihood bit-identical to its sequential call (the hybrid's block-rule stars are added
    to the per-point partials in the same order), also under graph replay with new seeds; the
    hybrid job's counts on a window against the hybrid oracle."""
    import torch
    from oracle import sampler_block as sb
    from tests import parity_utils as pu
    dev = torch.device("cuda")
    hess_d, mom_d, grid = _data(ctx)
    base = _jobs(9, 50)
    for rep in range(3 if use_graph else 1):
        jobs = []
        for k, j in enumerate(base):
            obs = dataclasses.replace(j["obs"], sampler=k % 3, seed=7000 + 100 * rep + k)
            jobs.append(dict(j, obs=obs))
        print(f"[case] mixed samplers graph={use_graph} rep={rep} samplers={[j['obs'].sampler for j in jobs]}",
              flush=True)
        ll_s, h_s = _sequential(ctx, jobs, grid, hess_d, mom_d, 0)
        ll_b = torch.empty(len(jobs), dtype=torch.float64, device=dev)
        h_b = torch.empty((len(jobs), 100 * 100), dtype=torch.int32, device=dev)
        ctx.batch_run(jobs, grid, hess_d, mom_d, ll_b, hess_out=h_b, use_graph=use_graph)
        x = torch.ones(1000, device=dev).sum()          # eager work between replays
        ctx.sync()
        assert np.array_equal(h_b.cpu().numpy(), h_s), rep
        assert np.array_equal(ll_b.cpu().numpy(), ll_s), rep
        assert float(x) == 1000.0
    # the hybrid job (sampler 2) against the hybrid oracle on its first 64 pixels
    j = jobs[2]
    lam = j["lam"].cpu().numpy()
    f32 = j["flux"].cpu().numpy()
    o = j["obs"]
    g = pu.gpu_simulate(ctx, lam, f32, o, conv_path=1, window=(0, 64), want_flux=False)
    s = sb.sample_pixels_hybrid(lam, f32, o.seed, np.arange(64), o.dust_model, o.dust_frac, want_counts=True)
    assert np.array_equal(g["counts"], s["counts"])
    assert np.array_equal(g["red"], s["red"])
