"""Benchmark: pCMD likelihood evaluations per second on one MI355X.

One step = one full likelihood evaluation of the 256x256, 3-band, 52,500-entry workload
(7 log-age bins x 5 [Fe/H] x 1500 masses, tau-model SFH, Gaussian MDF, log-normal dust with
F_dust = 1/2, 31x31 PSF, shot noise, 100x100 Hess, Poisson likelihood against a data Hess):
weighted entries -> Poisson sampler with flux sums -> dust / distance -> PSF -> noise ->
magnitudes -> Hess -> log-likelihood.  Parameters are drawn per step from the mock-test priors
(log Npix ~ U[2, 5], tau ~ U[0.1, 8] Gyr, mu_[Fe/H] ~ U[-0.5, 0.25], mu_dust ~ U[-1, 0],
mu_d ~ U[24, 30]) with seeds 1000, 1001, ...; the data Hess comes from seed 2.  All inputs are
synthetic and resident on the GPU before the timed region starts.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import contextlib
import dataclasses
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


@contextlib.contextmanager
def collector_paused():
    """Python's cyclic garbage collector paused over a timed loop, as timeit does: a full
    collection with torch loaded takes tens of milliseconds, which a loop whose GPU work is
    shorter than its host work (the 64x64 workload) would otherwise count as evaluation time."""
    was = gc.isenabled()
    gc.disable()
    try:
        yield
    finally:
        if was:
            gc.enable()


HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
# MI355X published figures: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 39.3e12 VALU lane-instructions/s.
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9
# Minimum VALU lane-instructions of one pixel x entry draw on gfx950: a quarter of one
# Philox4x32-10 evaluation (10 rounds x (2 v_mad_u64_u32, each giving both halves of a 32x32
# product, + 2 three-input XORs) = 40 for 4 words) plus the threshold compare.  Only entries
# with lambda > 0 draw; data-dependent work (accumulation, further thresholds, rejection, dust
# split) is not counted, so the fraction is a lower bound.
OPS_PER_DRAW = 40 / 4 + 1
# HBM bytes of the sampler (both k_sample passes) of the first headline step, from FETCH_SIZE
# and WRITE_SIZE calibrated against a copy of known size
# (profiles/k_sample_headline_256x256_52500_counters.md).  Set to None whenever k_sample changes
# until the counters are taken again.
SAMPLE_TRAFFIC_BYTES = 111.2e6
# The same for the first 512x512, Npix = 1e6 step (profiles/k_sample_large_512x512_52500_counters.md).
LARGE_SAMPLE_TRAFFIC_BYTES = 1076.2e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pixels", type=int, default=None,
                    help="pixels of the oracle's timed sampler sample (default 32768 headline, 8192 large)")
    ap.add_argument("--conv", type=int, default=0, help="0 auto, 1 direct, 2 fft")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "large", "small", "batch", "counters", "surrogate", "scatter", "ablation", "gemm"],
                    help="headline: 256x256 single evaluations; large: 512x512 at Npix = 1e6 with a 63x63 PSF and "
                         "200x200 Hess; small: 64x64, 500 points, the oracle timed on whole evaluations; "
                         "batch: 256 uneven jobs per step; counters: one headline simulation plus a "
                         "copy of known size, for hardware-counter runs; surrogate: the learned screen; scatter: "
                         "log-likelihood scatter against image size and the L_max ceiling")
    ap.add_argument("--counters-of", default="headline", choices=["headline", "large"],
                    help="counters workload: the simulation it runs")
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--train-pairs", type=int, default=16384)
    ap.add_argument("--train-steps", type=int, default=3000)
    ap.add_argument("--train-nim", type=int, default=128, help="image side of the surrogate's training simulations")
    ap.add_argument("--refine-pairs", type=int, default=8192)
    ap.add_argument("--refine-steps", type=int, default=2000)
    ap.add_argument("--mcmc-steps", type=int, default=300)
    ap.add_argument("--seeds", type=int, default=64, help="re-simulations per image side (scatter workload)")
    return ap.parse_args()


def run_batch(args):
    """256 uneven parameter points per step (image sides 2^U[6,9] rounded to 16, 5k-52.5k entries,
    parameters from the mock-test priors, 31x31 PSF on the direct path) through the persistent
    batched launch replayed from a HIP graph, against the same jobs as sequential single calls."""
    import torch

    import paper_1904_00011_amd as P
    import synth_inputs as si

    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    work = si.batch_workload(args.jobs, 0)
    evs = {}
    jobs = []
    for grid, model, obs in work:
        key = id(grid)
        if key not in evs:
            evs[key] = P.Evaluator(ctx, grid, 64, None, dict(x0=0, dx=0.05, y0=0, dy=0.05, nx=100, ny=100))
        ev = evs[key]
        lam = torch.empty(grid.n_entries, dtype=torch.float64, device=dev)
        jobs.append(dict(ev=ev, model=model, lam=lam, flux=ev.flux_d, obs=obs,
                         psf=torch.from_numpy(obs.psf).to(dev), conv_path=P.CONV_DIRECT))
    # data Hess: the 256x256 headline data image (seed 2), direct convolution
    model_d, obs_d = si.draw_headline_params(2)
    hd = P.Evaluator(ctx, si.headline_grid(), obs_d.nim, obs_d.psf, dict(x0=0.0, dx=0.05, y0=0.0, dy=0.05, nx=100, ny=100))
    mags_d = hd.simulate(model_d, obs_d, P.CONV_DIRECT).clone()
    ctx.sync()
    md = mags_d.cpu().numpy().astype(np.float64)
    fin = np.isfinite(md).all(axis=0)
    hgrid = si.hess_grid_from_median(float(np.median((md[0] - md[1])[fin])), float(np.median(md[1][fin])), 100, 100)
    hd.hess_grid = hgrid
    data_hess = torch.empty(10000, dtype=torch.int32, device=dev)
    data_mom = torch.empty(3, dtype=torch.float64, device=dev)
    hd.hess_of(mags_d, data_hess, data_mom)
    n = len(jobs)
    ll = torch.empty(n, dtype=torch.float64, device=dev)

    def entries_all():
        for j in jobs:
            w, npix = P.iso_weights(j["model"], j["ev"].grid)
            ctx.entries(j["ev"].E, j["ev"].iso_d, j["ev"].imf_d, j["ev"].iso_imf_sum, w, npix, j["lam"])

    entries_all()
    best, cand_ms = ctx.batch_autotune(jobs, hgrid, data_hess, data_mom, ll)
    use_graph = not args.no_graph
    for _ in range(max(args.warmup, 1)):
        entries_all()
        ctx.batch_run(jobs, hgrid, data_hess, data_mom, ll, use_graph=use_graph)
    torch.cuda.synchronize()
    ctx.timer_enable(True)
    with collector_paused():
        t0 = time.perf_counter()
        for _ in range(args.steps):
            entries_all()
            ctx.batch_run(jobs, hgrid, data_hess, data_mom, ll, use_graph=use_graph)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    b_ms, b_n, b_units = ctx.timer_read(P._lib.TIMER_BATCH)
    ctx.timer_enable(False)
    ll_batch = ll.cpu().numpy().copy()
    # the same jobs as sequential single calls
    ll_seq = torch.empty(n, dtype=torch.float64, device=dev)
    mags = {}
    hs = torch.empty(10000, dtype=torch.int32, device=dev)
    mom = torch.empty(3, dtype=torch.float64, device=dev)

    def sequential():
        for k, j in enumerate(jobs):
            N = j["obs"].nim
            if N not in mags:
                mags[N] = torch.empty((3, N * N), dtype=torch.float32, device=dev)
            w, npix = P.iso_weights(j["model"], j["ev"].grid)
            ctx.entries(j["ev"].E, j["ev"].iso_d, j["ev"].imf_d, j["ev"].iso_imf_sum, w, npix, j["lam"])
            ctx.simulate(j["lam"], j["flux"], j["obs"], mags[N], psf=j["psf"], conv_path=P.CONV_DIRECT)
            ctx.hess(mags[N], 3, N * N, hgrid, hs, mom)
            ctx.loglike(hs, data_hess, mom, data_mom, ll_seq[k:k + 1])

    sequential()
    torch.cuda.synchronize()
    ctx.timer_enable(True)
    with collector_paused():
        s0 = time.perf_counter()
        sequential()
        torch.cuda.synchronize()
        s1 = time.perf_counter()
    seq_sample_ms, _, seq_draws = ctx.timer_read(P._lib.TIMER_SAMPLE)
    ctx.timer_enable(False)
    identical = bool(np.array_equal(ll_seq.cpu().numpy(), ll_batch))
    elapsed = t1 - t0
    res = {
        "metric": "batched likelihood evals/sec (256 uneven parameter points per launch)",
        "value": n * args.steps / elapsed,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 counts / f64 sums / f32 images",
        "data": "synthetic",
        "config": {"workload": f"{n} jobs: sides 2^U[6,9] rounded to 16, 5k-52.5k entries, mock-test priors, "
                               "31x31 PSF (direct), shot noise, 100x100 Hess, Poisson logL",
                   "graph": use_graph, "tuning": {"wg_per_cu": best[0], "order": best[1]},
                   "autotune_ms": cand_ms, "draws_per_step": b_units / max(b_n, 1)},
        "sequential_evals_per_s": n / (s1 - s0),
        "speedup_vs_sequential": (n * args.steps / elapsed) / (n / (s1 - s0)),
        # GPU time of one batched run (prep, persistent sampler, reduction, PSF, noise, Hess and
        # likelihood of all jobs) and the sampler kernels alone of the sequential calls
        "batch_gpu_ms_per_step": b_ms / max(b_n, 1),
        "sequential_sampler_ms_per_step": seq_sample_ms,
        "identical_to_sequential": identical,
    }
    ctx.close()
    print(json.dumps(res), flush=True)


def run_surrogate(args):
    """The log-Hess surrogate: simulator-generated training pairs (batched launches), BF16 MFMA
    training, its likelihood error against the simulator, and delayed-acceptance MCMC with the
    surrogate as a screen against plain Metropolis-Hastings (both on the likelihood tempered to
    its own stochastic scatter)."""
    import torch
    from scipy import stats

    import paper_1904_00011_amd as P
    import synth_inputs as si
    from paper_1904_00011_amd.surrogate_pipeline import SurrogateWorkflow

    dims = (12, 512, 512, 512, 512, 10000)
    ctx = P.Context(0)
    dev = torch.device("cuda:0")
    G = si.headline_grid()
    th_true, box = si.surrogate_truth(), si.surrogate_box()
    model, obs = si.theta_to_model(th_true, seed=2, nim=256)
    ev = P.Evaluator(ctx, G, 256, obs.psf, dict(x0=0, dx=0.05, y0=0, dy=0.05, nx=100, ny=100))
    md = ev.simulate(model, obs).cpu().numpy().astype(np.float64)
    fin = np.isfinite(md).all(axis=0)
    hg = si.hess_grid_from_median(float(np.median((md[0] - md[1])[fin])), float(np.median(md[1][fin])), 100, 100)
    ev.hess_grid = hg
    dh = torch.empty(10000, dtype=torch.int32, device=dev)
    dm = torch.empty(3, dtype=torch.float64, device=dev)
    ev.hess_of(ev.mags, dh, dm)
    ctx.sync()
    wf = SurrogateWorkflow(ctx, G, si.theta_to_model, hg, dh, dm, box, train_nim=args.train_nim, dims=dims,
                           init_master=si.mlp_init(dims, 0))
    th = si.surrogate_theta_draws(args.train_pairs, seed=1)
    last = [time.perf_counter()]

    def progress(done, n):
        if time.perf_counter() - last[0] > 30.0 or done == n:
            print(f"[surrogate] simulated {done}/{n} training pairs", file=sys.stderr, flush=True)
            last[0] = time.perf_counter()

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = wf.simulate_hess(th, seed0=10 ** 6, progress=progress)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    X, T = wf.inputs(th), wf.targets(H)
    del H
    thv = si.surrogate_theta_draws(512, seed=2)
    Xv, Tv = wf.inputs(thv), wf.targets(wf.simulate_hess(thv, seed0=2 * 10 ** 6))
    mse0 = wf.mse(Xv, Tv)
    ctx.timer_enable(True)
    t0 = time.perf_counter()
    wf.fit(X, T, args.train_steps, batch=1024)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    g_ms, g_n, g_flops = ctx.timer_read(P._lib.TIMER_GEMM)
    ctx.timer_enable(False)
    mse1 = wf.mse(Xv, Tv)
    # sequential design: pairs around the chain's start, training continued on the union
    t0 = time.perf_counter()
    wf.refine(X, T, th_true, 0.15, args.refine_pairs, args.refine_steps, seed0=3 * 10 ** 6)
    torch.cuda.synchronize()
    t_refine = time.perf_counter() - t0
    mse2 = wf.mse(Xv, Tv)
    # likelihood error on held-out points and the simulator's own seed-to-seed scatter
    ths = si.surrogate_theta_draws(128, seed=3)
    L1 = np.array([wf.simulator_loglike(t, 5000 + k) for k, t in enumerate(ths)])
    L2 = np.array([wf.simulator_loglike(t, 9000 + k) for k, t in enumerate(ths)])
    S = wf.surrogate_loglike_batch(ths)
    # throughput: surrogate likelihoods (4096 points per call) vs one simulator likelihood at a time
    xs = si.surrogate_theta_draws(4096, seed=4)
    wf.surrogate_loglike_batch(xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        wf.surrogate_loglike_batch(xs)
    torch.cuda.synchronize()
    sur_rate = 5 * 4096 / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    for k in range(20):
        wf.simulator_loglike(ths[k], 7000 + k)
    sim_rate = 20 / (time.perf_counter() - t0)
    # the dominant product of training and inference alone: 8192 x 10000 x 512
    A = torch.randn((8192, 512), device=dev).to(torch.bfloat16)
    Bw = torch.randn((10000, 512), device=dev).to(torch.bfloat16)
    Cm = torch.empty((8192, 10000), dtype=torch.float32, device=dev)
    ctx.gemm_bf16(A, Bw, Cm)
    ctx.timer_enable(True)
    for _ in range(10):
        ctx.gemm_bf16(A, Bw, Cm)
    torch.cuda.synchronize()
    b_ms, b_n, b_flops = ctx.timer_read(P._lib.TIMER_GEMM)
    ctx.timer_enable(False)
    mc = {}
    for frac in (0.06, 0.1):
        scale = frac * (box[1] - box[0])
        for screen in (False, True):
            _, _, info = wf.run_mcmc(th_true, args.mcmc_steps, scale, np.random.default_rng(1), screen=screen,
                                     temperature=3000.0)
            info["accepted_per_simulator_call"] = info["accepted"] / info["simulator_calls"]
            info["accepted_per_s"] = info["accepted"] / info["seconds"]
            mc[f"step{frac}_{'screened' if screen else 'plain'}"] = info
    res = {
        "metric": "accepted MCMC moves/sec with the surrogate screen (256^2 simulator judge, 12 parameters)",
        "value": mc["step0.1_screened"]["accepted_per_s"],
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.mcmc_steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16 MFMA, fp32 accumulate",
        "data": "synthetic",
        "config": {"workload": f"MLP {dims}, {args.train_pairs} simulator pairs at {args.train_nim}x{args.train_nim} over the prior box + "
                               f"{args.refine_pairs} within 15% of its width around the start, {args.train_steps}+"
                               f"{args.refine_steps} Adam steps of 1024, data Hess 256x256 at the fiducial parameters",
                   "temperature": 3000.0, "step": "10% of the prior box"},
        "plain_accepted_per_s": mc["step0.1_plain"]["accepted_per_s"],
        "mcmc": mc,
        "train_pairs_per_s": args.train_pairs / t_gen,
        "train_seconds": t_fit,
        "refine_seconds": t_refine,
        "gemm_tflops": g_flops / (g_ms / 1e3) / 1e12 if g_ms > 0 else None,
        "gemm_frac_of_bf16_peak": (g_flops / (g_ms / 1e3)) / 2.5e15 if g_ms > 0 else None,
        "roofline": {"bound": "mfma", "kernel": "k_gemm 8192x10000x512 bf16", "achieved": b_flops / (b_ms / 1e3) / 1e12,
                     "peak": 2500.0, "unit": "TFLOP/s", "frac": b_flops / (b_ms / 1e3) / 2.5e15, "traffic": None},
        "val_mse": [mse0, mse1, mse2],
        "spearman_surrogate_simulator": float(stats.spearmanr(S, L1)[0]),
        "median_abs_logL_error": float(np.median(np.abs(S - L1))),
        "median_abs_simulator_seed_scatter": float(np.median(np.abs(L1 - L2))),
        "surrogate_loglikes_per_s": sur_rate,
        "simulator_loglikes_per_s": sim_rate,
    }
    ctx.close()
    print(json.dumps(res), flush=True)


def run_gemm(args):
    """The surrogate's dominant matrix product alone, C[8192][10000] = A[8192][512] B[10000][512]^T
    in BF16 with FP32 output (10 timed launches), and one training step of the configured network
    (12 -> 4 x 512 -> 10,000) at a batch of 1,024, its products timed by HIP events."""
    import torch

    import paper_1904_00011_amd as P
    import synth_inputs as si
    from paper_1904_00011_amd.surrogate import SurrogateNet

    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    g = torch.Generator(device="cpu").manual_seed(5)
    A = torch.randn((8192, 512), generator=g).to(dev).to(torch.bfloat16)
    Bw = torch.randn((10000, 512), generator=g).to(dev).to(torch.bfloat16)
    Cm = torch.empty((8192, 10000), dtype=torch.float32, device=dev)
    ctx.gemm_bf16(A, Bw, Cm)
    torch.cuda.synchronize()
    ctx.timer_enable(True)
    for _ in range(10):
        ctx.gemm_bf16(A, Bw, Cm)
    torch.cuda.synchronize()
    b_ms, b_n, b_flops = ctx.timer_read(P._lib.TIMER_GEMM)
    ctx.timer_enable(False)
    dims = (12, 512, 512, 512, 512, 10000)
    net = SurrogateNet(ctx, dims, si.mlp_init(dims, 1))
    x = torch.rand((1024, 12), generator=g).to(dev) * 2 - 1
    t = torch.randn((1024, 10000), generator=g).to(dev)
    net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    ctx.timer_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s_ms, s_n, s_flops = ctx.timer_read(P._lib.TIMER_GEMM)
    ctx.timer_enable(False)
    ctx.close()
    avg = b_ms / max(b_n, 1)
    out_bytes = 8192 * 10000 * 4
    res = {
        "metric": "BF16 product 8192x10000x512 (FP32 out), TFLOP/s",
        "value": b_flops / (b_ms / 1e3) / 1e12, "unit": "TFLOP/s", "n_gpus": 1, "steps": 10, "warmup": 1,
        "ms_per_step": avg, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 MFMA, fp32 accumulate", "data": "synthetic",
        "config": {"workload": "8192x10000x512 product; training step of 12-512-512-512-512-10000 at batch 1024"},
        "roofline": {"bound": "mfma", "kernel": "k_gemm 8192x10000x512 bf16", "achieved": b_flops / (b_ms / 1e3) / 1e12,
                     "peak": 2500.0, "unit": "TFLOP/s", "frac": b_flops / (b_ms / 1e3) / 2.5e15, "traffic": None,
                     "avg_launch_ms": avg,
                     # the FP32 output alone is 328 MB: at 8 TB/s a 41 us floor
                     "output_write_floor_ms": out_bytes / 8e12 * 1e3},
        "train_step_ms": 1e3 * (t1 - t0) / args.steps,
        "train_step_gemm_ms": s_ms / args.steps,
        "train_step_gemm_tflops": s_flops / (s_ms / 1e3) / 1e12 if s_ms > 0 else None,
    }
    print(json.dumps(res), flush=True)


def run_scatter(args):
    """Stochastic likelihoods (Appendix A): the fiducial-tau-like point re-simulated with 64 seeds
    at image sides 64..512 against a data image of the same side; the scatter, its skew and the
    median (the paper's ceiling L_max for a best fit), each side's seeds in one batched launch."""
    import paper_1904_00011_amd as P
    import synth_inputs as si
    from paper_1904_00011_amd import stochastic as st

    ctx = P.Context(0)
    model, obs = si.theta_to_model(si.surrogate_truth(), seed=0, nim=256)
    t0 = time.perf_counter()
    rows = st.scatter_vs_image_size(ctx, si.headline_grid(), model, obs, (64, 128, 256, 512), args.seeds)
    elapsed = time.perf_counter() - t0
    sims = args.seeds * 4
    ctx.close()
    print(json.dumps({
        "metric": "log-likelihood scatter vs image size (fiducial point, seeds re-simulated in batched launches)",
        "value": sims / elapsed, "unit": "re-simulations/s (all sides)", "n_gpus": 1, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32 counts / f64 sums / f32 images", "data": "synthetic",
        "config": {"workload": f"{args.seeds} seeds per side, sides 64-512, 52,500 entries, 31x31 PSF (direct), "
                               "100x100 Hess, Poisson logL"},
        "rows": rows}), flush=True)


def run_ablation(args):
    """Block-skip sampler (Poisson superposition over 64-point blocks) and the hybrid (block rule
    below a block sum of 10, per-point rule above) against the per-point rule on the headline
    workload at fixed log Npix = 1 .. 5: sampler time (the hybrid's two kernels together) and
    whole likelihood evaluations per second of each, the same parameters and seeds for all."""
    import torch

    import paper_1904_00011_amd as P
    import synth_inputs as si

    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    grid = si.headline_grid()
    model_d, obs_d = si.draw_headline_params(2)
    ev = P.Evaluator(ctx, grid, obs_d.nim, obs_d.psf, dict(x0=0.0, dx=0.05, y0=0.0, dy=0.05, nx=100, ny=100))
    mags_d = ev.simulate(model_d, obs_d).clone()
    ctx.sync()
    md = mags_d.cpu().numpy().astype(np.float64)
    fin = np.isfinite(md).all(axis=0)
    ev.hess_grid = si.hess_grid_from_median(float(np.median((md[0] - md[1])[fin])), float(np.median(md[1][fin])),
                                            100, 100)
    data_hess = torch.empty(100 * 100, dtype=torch.int32, device=dev)
    data_mom = torch.empty(3, dtype=torch.float64, device=dev)
    ev.hess_of(mags_d, data_hess, data_mom)
    out = torch.empty(1, dtype=torch.float64, device=dev)
    rows = []
    for lnp in (1.0, 2.0, 3.0, 4.0, 5.0):
        params = [si.draw_headline_params(1000 + k, log_npix=lnp) for k in range(args.steps + args.warmup)]
        row = {"log_npix": lnp}
        for name, sampler in (("point", P.SAMPLER_POINT), ("block", P.SAMPLER_BLOCK), ("hybrid", P.SAMPLER_HYBRID)):
            runs = [(m, dataclasses.replace(o, sampler=sampler)) for m, o in params]
            for m, o in runs[:args.warmup]:
                out.copy_(ev.loglike(m, o, data_hess, data_mom))
            torch.cuda.synchronize()
            ctx.timer_enable(True)
            t0 = time.perf_counter()
            for m, o in runs[args.warmup:]:
                out.copy_(ev.loglike(m, o, data_hess, data_mom))
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx.sync()
            s_ms, s_n, _ = ctx.timer_read(P._lib.TIMER_SAMPLE)
            ctx.timer_enable(False)
            row[name] = {"sample_ms": s_ms / max(s_n, 1), "evals_per_s": args.steps / (t1 - t0)}
        row["sampler_speedup"] = row["point"]["sample_ms"] / row["block"]["sample_ms"]
        row["eval_speedup"] = row["block"]["evals_per_s"] / row["point"]["evals_per_s"]
        row["hybrid_sampler_speedup"] = row["point"]["sample_ms"] / row["hybrid"]["sample_ms"]
        rows.append(row)
        print(f"[ablation] log Npix {lnp}: k_sample {row['point']['sample_ms']:.3f} ms, k_sample_block "
              f"{row['block']['sample_ms']:.3f} ms, hybrid {row['hybrid']['sample_ms']:.3f} ms", file=sys.stderr,
              flush=True)
    ctx.close()
    at2 = next(r for r in rows if r["log_npix"] == 2.0)
    print(json.dumps({
        "metric": "block-skip sampler speed-up over the per-point rule (sampler kernel time, 256^2, 52,500 points, "
                  "log Npix = 2)",
        "value": at2["sampler_speedup"], "unit": "x", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 counts / f64 sums / f32 images", "data": "synthetic",
        "config": {"workload": "headline workload (256x256, 3 bands, 52,500 entries, log-normal dust F=0.5, 31x31 "
                               "PSF, shot noise, 100x100 Hess) at fixed log Npix 1-5, both samplers on the same "
                               "parameters and seeds"},
        "rows": rows}), flush=True)


def run_counters(args):
    """One simulation (the headline benchmark's first step, or with --counters-of large the first
    512x512 step) and a 2048x2048x3 FP32 image copy of known size (50,331,648 bytes read and
    written) that calibrates FETCH_SIZE / WRITE_SIZE."""
    import torch

    import paper_1904_00011_amd as P
    import synth_inputs as si

    ctx = P.Context(0)
    grid = si.headline_grid()
    model, obs = si.draw_large_params(1000) if args.counters_of == "large" else si.draw_headline_params(1000)
    ev = P.Evaluator(ctx, grid, obs.nim, obs.psf, dict(x0=0.0, dx=0.05, y0=0.0, dy=0.05, nx=100, ny=100))
    ev.simulate(model, obs)
    ctx.sync()
    dev = torch.device("cuda:0")
    o2 = si.Obs(nim=2048, seed=1, dmod=25.0, psf=None, noise_model=0)
    lam = torch.tensor([0.5], dtype=torch.float64, device=dev)
    flux = torch.ones((3, 1), dtype=torch.float32, device=dev)
    mags = torch.empty((3, 2048 * 2048), dtype=torch.float32, device=dev)
    pre = torch.empty_like(mags)
    ctx.simulate(lam, flux, o2, mags, flux_pre=pre)
    ctx.sync()
    ctx.close()
    print(json.dumps({"counters_run": "done", "copy_bytes_each_way": 3 * 2048 * 2048 * 4}), flush=True)


def image_plane_at_scale(ctx, P, si, hgrid, N: int = 4096, reps: int = 3) -> dict:
    """PSF convolution (both paths) and Hess binning of a 4096x4096x3 image: at the benchmark's
    256x256 the image-plane kernels are bound by launch latency, here by the memory system.  The
    stars come from the headline grid thinned to 1,050 entries so that sampling stays short."""
    import torch

    G = si.headline_grid().subsample(50)
    model, obs = si.draw_headline_params(1000)
    obs.nim = N
    ev = P.Evaluator(ctx, G, N, obs.psf, hgrid)
    out = {"image": f"{N}x{N}x3, 31x31 PSF, {hgrid['nx']}x{hgrid['ny']} Hess"}
    for path, name in ((P.CONV_FFT, "conv_fft"), (P.CONV_DIRECT, "conv_direct")):
        ev.simulate(model, obs, path)
        ctx.sync()
        ctx.timer_enable(True)
        for _ in range(reps):
            ev.simulate(model, obs, path)
        ctx.sync()
        c_ms, c_n, _ = ctx.timer_read(P._lib.TIMER_CONV)
        ctx.timer_enable(False)
        out[name] = hbm_roofline(8.0 * 3 * N * N, c_ms / max(c_n, 1), name)
    h = torch.empty(hgrid["nx"] * hgrid["ny"], dtype=torch.int32, device=ev.mags.device)
    mom = torch.empty(3, dtype=torch.float64, device=ev.mags.device)
    ev.hess_of(ev.mags, h, mom)
    ctx.sync()
    ctx.timer_enable(True)
    for _ in range(reps):
        ev.hess_of(ev.mags, h, mom)
    ctx.sync()
    h_ms, h_n, _ = ctx.timer_read(P._lib.TIMER_HESS)
    ctx.timer_enable(False)
    out["hess"] = hbm_roofline(8.0 * N * N + 4.0 * hgrid["nx"] * hgrid["ny"], h_ms / max(h_n, 1), "k_hess")
    del ev
    torch.cuda.empty_cache()
    return out


def hbm_roofline(nbytes: float, ms: float, kernel: str) -> dict:
    gbs = nbytes / (ms / 1e3) / 1e9 if ms > 0 else None
    return {"bound": "hbm", "kernel": kernel, "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS if gbs else None, "bytes": nbytes, "avg_launch_ms": ms}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(grid, model, obs, hgrid, n_px_sample, min_seconds: float = 0.0):
    """Time the oracle on every host core this process may use (pixel slabs of the sampler and
    one band per process of the convolution, as `oracle.parallel` splits them) on a bounded
    sample of one evaluation: entries, the sampler on n_px_sample pixels (its cost is linear in
    pixels, so the time is scaled to the image), then PSF, noise, Hess and logL at full size on an
    image tiled from the sampled pixels.  n_px_sample = 0 runs the sampler on the whole image.
    The evaluation is repeated until min_seconds have passed and the mean time is reported."""
    from oracle import entries as oe
    from oracle import hess as oh
    from oracle import loglike as ol
    from oracle import noise as on
    from oracle import parallel as opar

    N = obs.nim
    npx = N * N
    n_s = npx if not n_px_sample else min(npx, n_px_sample)
    workers = opar.default_workers()
    # the sample: up to 64 windows spread over the image
    n_win = min(max(1, n_s // 128), 64)
    step = npx // n_win
    wins = [(k * step, k * step + n_s // n_win) for k in range(n_win)]
    n_s = sum(b - a for a, b in wins)
    t_evals, t_samp, t_all = [], [], 0.0
    while True:
        t0 = time.perf_counter()
        lam, _, f32 = oe.build_entries(model, grid)
        t1 = time.perf_counter()
        F, _, _ = opar.simulate_flux(lam, f32, obs, wins, workers=workers)
        t2 = time.perf_counter()
        reps = int(np.ceil(npx / n_s))
        Ffull = np.tile(F, (1, reps))[:, :npx].reshape(F.shape[0], N, N)
        G = opar.convolve(Ffull, obs.psf, workers=workers) if obs.psf is not None else Ffull
        m = on.magnitudes(G.reshape(F.shape[0], npx), obs)
        H, mom = oh.hess(m, hgrid)
        ol.loglike(H, H, mom, mom, ol.POISSON, 0.01)
        t3 = time.perf_counter()
        t_evals.append((t1 - t0) + (t2 - t1) * (npx / n_s) + (t3 - t2))
        t_samp.append(t2 - t1)
        t_all += t3 - t0
        if t_all >= min_seconds:
            break
    t_eval = float(np.mean(t_evals))
    what = (f"the whole image" if n_s == npx else
            f"{n_s} of {npx} pixels ({n_win} windows; time scaled x{npx / n_s:.2f})")
    return dict(value=1.0 / t_eval, unit="evals/s", cores=workers, kind="oracle",
                cpu=cpu_model(), host_cpu_count=os.cpu_count(),
                sample=(f"oracle on {workers} processes: entries + sampler on {what} + PSF, noise, Hess and logL at "
                        f"full size; log Npix = {model.log_npix:.3f}; {len(t_evals)} evaluation(s), measured "
                        f"{t_all:.1f} s"),
                sampler_draws_per_s=n_s * len(lam) / float(np.mean(t_samp)))


def run_small(args):
    """The small configuration: 64x64 px, 2 bands, one isochrone of 500 masses (Salpeter, Npix =
    100), no dust, 5x5 PSF, Gaussian magnitude noise 0.02, 100x100 Hess.  Each step is one whole
    evaluation with a new seed (1000, 1001, ...) against the data Hess of seed 2; far too little
    work to fill the GPU, so the value is a latency figure.  The oracle is timed on the whole
    evaluation (no sampling)."""
    import torch

    import paper_1904_00011_amd as P
    import synth_inputs as si

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    grid, model, obs = si.small_case(64, seed=2)
    nh = 100
    ev = P.Evaluator(ctx, grid, obs.nim, obs.psf, dict(x0=0.0, dx=0.05, y0=0.0, dy=0.05, nx=nh, ny=nh))
    mags_d = ev.simulate(model, obs).clone()
    ctx.sync()
    md = mags_d.cpu().numpy().astype(np.float64)
    fin = np.isfinite(md).all(axis=0)
    hgrid = si.hess_grid_from_median(float(np.median((md[0] - md[1])[fin])), float(np.median(md[1][fin])), nh, nh)
    ev.hess_grid = hgrid
    data_hess = torch.empty(nh * nh, dtype=torch.int32, device=dev)
    data_mom = torch.empty(3, dtype=torch.float64, device=dev)
    ev.hess_of(mags_d, data_hess, data_mom)
    obss = [dataclasses.replace(obs, seed=1000 + k) for k in range(args.steps + args.warmup)]
    logls = torch.empty(args.steps + args.warmup, dtype=torch.float64, device=dev)
    for k in range(args.warmup):
        ev.loglike(model, obss[k], data_hess, data_mom, P.LL_POISSON, 0.01, out=logls[k:k + 1])
    torch.cuda.synchronize()
    ctx.timer_enable(True)
    torch.cuda.synchronize()
    with collector_paused():
        t0 = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            ev.loglike(model, obss[k], data_hess, data_mom, P.LL_POISSON, 0.01, out=logls[k:k + 1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ctx.sync()
    s_ms, s_n, s_units = ctx.timer_read(P._lib.TIMER_SAMPLE)
    c_ms, c_n, _ = ctx.timer_read(P._lib.TIMER_CONV)
    h_ms, h_n, _ = ctx.timer_read(P._lib.TIMER_HESS)
    ctx.timer_enable(False)
    ll = logls.cpu().numpy()[args.warmup:]
    assert np.all(np.isfinite(ll)), "non-finite log-likelihood"
    elapsed = t1 - t0
    draws = s_units / max(s_n, 1)
    avg_sample_s = s_ms / max(s_n, 1) / 1e3
    achieved = OPS_PER_DRAW * draws / avg_sample_s
    res = {
        "metric": "likelihood evals/sec (64^2 image, 500 isochrone points)",
        "value": args.steps / elapsed, "unit": "evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32 counts / f64 sums / f32 images", "data": "synthetic",
        "config": {"workload": "64x64 px, 2 bands, 500 masses of one isochrone (Salpeter, Npix = 100), no dust, "
                               "5x5 PSF, Gaussian magnitude noise 0.02, 100x100 Hess, Poisson logL",
                   "nim": 64, "entries": grid.n_entries, "bands": 2, "psf_k": 5, "hess": [nh, nh],
                   "parallelism": "1 GPU"},
        "poisson_draws_per_s": s_units / (s_ms / 1e3) if s_ms > 0 else None,
        "draws_per_eval": draws,
        "kernel_ms_per_eval": {"sample": s_ms / max(s_n, 1), "conv": c_ms / max(c_n, 1), "hess": h_ms / max(h_n, 1)},
        "roofline": {"bound": "alu", "kernel": "k_sample", "achieved": achieved / 1e12,
                     "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "T lane-instr/s (VALU)",
                     "frac": achieved / VALU_LANE_OPS_PEAK, "traffic": None, "ops_per_draw": OPS_PER_DRAW,
                     "avg_launch_ms": avg_sample_s * 1e3,
                     "note": "2.05e6 draws per launch fill 4,096 lanes only: launch- and latency-bound"},
        "mean_logL": float(ll.mean()),
    }
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(grid, model, obss[args.warmup], hgrid, 0, min_seconds=10.0)
    ctx.close()
    print(json.dumps(res), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): sharding the image across GPUs "
              "is not built", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "counters":
        run_counters(args)
        return
    if args.workload == "surrogate":
        run_surrogate(args)
        return
    if args.workload == "scatter":
        run_scatter(args)
        return
    if args.workload == "ablation":
        run_ablation(args)
        return
    if args.workload == "small":
        run_small(args)
        return
    if args.workload == "gemm":
        run_gemm(args)
        return
    import torch

    import paper_1904_00011_amd as P
    import synth_inputs as si

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    ctx = P.Context(0)
    grid = si.headline_grid()
    large = args.workload == "large"
    draw = si.draw_large_params if large else si.draw_headline_params
    nh = 200 if large else 100
    cpu_pixels = args.cpu_pixels if args.cpu_pixels else (8192 if large else 32768)
    model_d, obs_d = draw(2)
    # data image and Hess grid (untimed set-up)
    ev = P.Evaluator(ctx, grid, obs_d.nim, obs_d.psf, dict(x0=0.0, dx=0.05, y0=0.0, dy=0.05, nx=nh, ny=nh))
    mags_d = ev.simulate(model_d, obs_d, args.conv).clone()
    ctx.sync()
    md = mags_d.cpu().numpy().astype(np.float64)
    fin = np.isfinite(md).all(axis=0)
    hgrid = si.hess_grid_from_median(float(np.median((md[0] - md[1])[fin])), float(np.median(md[1][fin])), nh, nh)
    ev.hess_grid = hgrid
    data_hess = torch.empty(nh * nh, dtype=torch.int32, device=dev)
    data_mom = torch.empty(3, dtype=torch.float64, device=dev)
    ev.hess_of(mags_d, data_hess, data_mom)
    params = [draw(1000 + k) for k in range(args.steps + args.warmup)]
    # share of entries with lambda > 0 (the rest, e.g. pruned metallicities, draw nothing)
    active = [float(np.mean(P.iso_weights(m, grid)[0][grid.iso_of_entry] > 0.0)) for m, _ in params[args.warmup:]]
    logls = torch.empty(args.steps + args.warmup, dtype=torch.float64, device=dev)
    for k in range(args.warmup):
        m, o = params[k]
        ev.loglike(m, o, data_hess, data_mom, P.LL_POISSON, 0.01, args.conv, out=logls[k:k + 1])
    torch.cuda.synchronize()
    ctx.timer_enable(True)
    torch.cuda.synchronize()
    with collector_paused():
        t0 = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            m, o = params[k]
            ev.loglike(m, o, data_hess, data_mom, P.LL_POISSON, 0.01, args.conv, out=logls[k:k + 1])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    ctx.sync()
    s_ms, s_n, s_units = ctx.timer_read(P._lib.TIMER_SAMPLE)
    c_ms, c_n, _ = ctx.timer_read(P._lib.TIMER_CONV)
    h_ms, h_n, _ = ctx.timer_read(P._lib.TIMER_HESS)
    ctx.timer_enable(False)
    ll = logls.cpu().numpy()[args.warmup:]
    # the same evaluations with the PSF convolution forced onto the FFT path (AUTO takes the
    # direct path below 48x48: faster at 31x31), reported beside the headline value
    fft = None
    n_im = obs_d.nim
    if not large and args.conv == P.CONV_AUTO and (n_im & (n_im - 1)) == 0 and 8 <= n_im <= 4096:
        m, o = params[0]
        ev.loglike(m, o, data_hess, data_mom, P.LL_POISSON, 0.01, P.CONV_FFT)  # untimed first use
        torch.cuda.synchronize()
        ctx.timer_enable(True)
        torch.cuda.synchronize()
        t0f = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            m, o = params[k]
            ev.loglike(m, o, data_hess, data_mom, P.LL_POISSON, 0.01, P.CONV_FFT, out=logls[k:k + 1])
        torch.cuda.synchronize()
        t1f = time.perf_counter()
        ctx.sync()
        cf_ms, cf_n, _ = ctx.timer_read(P._lib.TIMER_CONV)
        ctx.timer_enable(False)
        fft = {"evals_per_s": args.steps / (t1f - t0f), "conv_ms_per_eval": cf_ms / max(cf_n, 1)}
    # the same evaluations with the hybrid sampler (block rule where a 64-point block's expected
    # star count is below 10, per-point rule elsewhere): the same Poisson law from another random
    # stream, reported beside the headline value, which uses the per-point rule
    hyb = None
    if not large:
        m, o = params[0]
        ev.loglike(m, dataclasses.replace(o, sampler=P.SAMPLER_HYBRID), data_hess, data_mom, P.LL_POISSON, 0.01,
                   args.conv)  # untimed first use
        torch.cuda.synchronize()
        ctx.timer_enable(True)
        torch.cuda.synchronize()
        t0h = time.perf_counter()
        for k in range(args.warmup, args.warmup + args.steps):
            m, o = params[k]
            ev.loglike(m, dataclasses.replace(o, sampler=P.SAMPLER_HYBRID), data_hess, data_mom, P.LL_POISSON, 0.01,
                       args.conv, out=logls[k:k + 1])
        torch.cuda.synchronize()
        t1h = time.perf_counter()
        ctx.sync()
        hs_ms, hs_n, _ = ctx.timer_read(P._lib.TIMER_SAMPLE)
        ctx.timer_enable(False)
        llh = logls.cpu().numpy()[args.warmup:]
        assert np.all(np.isfinite(llh)), "non-finite log-likelihood (hybrid sampler)"
        hyb = {"evals_per_s": args.steps / (t1h - t0h), "sample_ms_per_eval": hs_ms / max(hs_n, 1),
               "mean_logL": float(llh.mean())}
    assert np.all(np.isfinite(ll)), "non-finite log-likelihood"
    elapsed = t1 - t0
    evals_per_s = args.steps / elapsed
    draws_per_launch = s_units / max(s_n, 1) * float(np.mean(active))
    avg_sample_s = s_ms / max(s_n, 1) / 1e3
    achieved = OPS_PER_DRAW * draws_per_launch / avg_sample_s
    if large:
        metric = "likelihood evals/sec (512^2 image, 52,500 isochrone points, Npix = 1e6)"
        workload = ("512x512 px, 3 bands, 52,500 entries (7 ages x 5 [Fe/H] x 1500 masses), Npix = 1e6 (1 entry in 8 "
                    "above the rejection threshold), log-normal dust F=0.5, 63x63 PSF (FFT), shot noise, 200x200 Hess, "
                    "Poisson logL")
    else:
        metric = "likelihood evals/sec (256^2 image, 52,500 isochrone points)"
        workload = ("256x256 px, 3 bands, 52,500 entries (7 ages x 5 [Fe/H] x 1500 masses), log Npix ~ U[2,5], "
                    "log-normal dust F=0.5, 31x31 PSF, shot noise, 100x100 Hess, Poisson logL")
    res = {
        "metric": metric,
        "value": evals_per_s,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 counts / f64 sums / f32 images",
        "data": "synthetic",
        "config": {"workload": workload, "nim": obs_d.nim, "entries": grid.n_entries, "bands": 3,
                   "psf_k": int(obs_d.psf.shape[-1]), "hess": [nh, nh], "parallelism": "1 GPU"},
        "poisson_draws_per_s": s_units / (s_ms / 1e3) if s_ms > 0 else None,
        "draws_per_eval": draws_per_launch,
        "kernel_ms_per_eval": {"sample": s_ms / max(s_n, 1), "conv": c_ms / max(c_n, 1), "hess": h_ms / max(h_n, 1)},
        # HBM view of the image-plane steps: algorithmic bytes (convolution: read F, write G, 4 B
        # each per pixel and band; Hess: read the two magnitude planes it bins, 4 B each per
        # pixel, write the bins) over the timed launches' average duration, against 8 TB/s
        "conv_roofline": hbm_roofline(8.0 * 3 * obs_d.nim ** 2, c_ms / max(c_n, 1),
                                      "PSF convolution (FFT chain)" if obs_d.psf.shape[-1] >= 48 else "PSF convolution (direct)"),
        "hess_roofline": hbm_roofline(8.0 * obs_d.nim ** 2 + 4.0 * nh * nh, h_ms / max(h_n, 1), "k_hess"),
        "roofline": {"bound": "alu", "kernel": "k_sample", "achieved": achieved / 1e12,
                     "peak": VALU_LANE_OPS_PEAK / 1e12, "unit": "T lane-instr/s (VALU)",
                     "frac": achieved / VALU_LANE_OPS_PEAK,
                     "traffic": (LARGE_SAMPLE_TRAFFIC_BYTES if large else SAMPLE_TRAFFIC_BYTES),
                     "ops_per_draw": OPS_PER_DRAW, "avg_launch_ms": avg_sample_s * 1e3,
                     # the same lane-instruction rate against the published FP32 peaks (one
                     # lane-instruction counted as one operation): an integer random-number
                     # generator issues no packed FP32 FMAs, so 157.3 TFLOP/s is out of its reach
                     "frac_of_fp32_78_6_tflops": achieved / 78.6e12,
                     "frac_of_fp32_packed_157_3_tflops": achieved / 157.3e12},
        "mean_logL": float(ll.mean()),
        "fft_conv_path": fft,
        "hybrid_sampler": hyb,
    }
    if not large:
        res["image_plane_at_scale"] = image_plane_at_scale(ctx, P, si, hgrid)
    if not args.no_cpu_baseline:
        m, o = params[args.warmup]
        res["cpu_baseline"] = cpu_baseline(grid, m, o, hgrid, cpu_pixels)
    ctx.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
