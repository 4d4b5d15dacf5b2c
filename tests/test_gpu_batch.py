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
