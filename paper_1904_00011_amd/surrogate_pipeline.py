"""Training data, training and evaluation of the log-Hess surrogate, all through the C ABI.

Training pairs (theta, log-Hess) come from the batched simulator (one persistent launch per 256
parameter points, replayed from a HIP graph); the network trains on the library's BF16 MFMA
kernels; the surrogate log-likelihood screens proposals in delayed-acceptance MCMC with the
simulator's log-likelihood taking the final accept/reject decision.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from . import _lib
from .pipeline import Evaluator
from .surrogate import Standardizer, SurrogateNet, delayed_acceptance_mcmc, log_hess_target

class SurrogateWorkflow:
    def __init__(self, ctx: _lib.Context, grid, theta_to_model, hess_grid: dict, data_hess: torch.Tensor,
                 data_mom: torch.Tensor, box, train_nim: int = 128, dims=(12, 512, 512, 512, 512, 10000),
                 init_master=None):
        """box = (lo, hi): the flat prior of the 12 parameters, also the training domain."""
        self.ctx = ctx
        self.grid = grid
        self.theta_to_model = theta_to_model
        self.hess_grid = dict(hess_grid)
        self.nbins = hess_grid["nx"] * hess_grid["ny"]
        self.data_hess = data_hess
        self.data_mom = data_mom
        self.train_nim = train_nim
        self.dev = data_hess.device
        self.lo = np.asarray(box[0], np.float64)
        self.hi = np.asarray(box[1], np.float64)
        self.std = Standardizer(self.lo, self.hi)
        self.ev = Evaluator(ctx, grid, train_nim, None, hess_grid)
        self.net = SurrogateNet(ctx, dims, init_master)
        self.eval_256 = None
        self._x1 = torch.empty((1, 12), dtype=torch.float32, device=self.dev)
        self._y1 = torch.empty((1, dims[-1]), dtype=torch.float32, device=self.dev)
        self._ll1 = torch.empty(1, dtype=torch.float64, device=self.dev)

    # ---------------------------------------------------------------- data generation
    def simulate_hess(self, thetas: np.ndarray, seed0: int, nim: int | None = None, batch: int | None = None,
                      progress=None):
        """Hess diagrams [n][nbins] (int32, device) of the parameter vectors, one batched launch
        per `batch` points (default: 256 at 128x128 and below, fewer for larger images so that the
        batch's partial sums stay within a few tens of GB).  `progress(done, n)` is called after
        every launch."""
        nim = self.train_nim if nim is None else nim
        if batch is None:
            batch = max(16, min(256, 256 * 128 * 128 // (nim * nim)))
        n = len(thetas)
        out = torch.empty((n, self.nbins), dtype=torch.int32, device=self.dev)
        lams = [torch.empty(self.ev.E, dtype=torch.float64, device=self.dev) for _ in range(min(batch, n))]
        psf = None
        ll = torch.empty(min(batch, n), dtype=torch.float64, device=self.dev)
        for b0 in range(0, n, batch):
            b1 = min(n, b0 + batch)
            jobs = []
            for k in range(b0, b1):
                model, obs = self.theta_to_model(thetas[k], seed=seed0 + k, nim=nim)
                if psf is None:
                    psf = torch.from_numpy(obs.psf).to(self.dev)
                w, npix = _lib.iso_weights(model, self.grid)
                lam = lams[k - b0]
                self.ctx.entries(self.ev.E, self.ev.iso_d, self.ev.imf_d, self.ev.iso_imf_sum, w, npix, lam)
                jobs.append(dict(lam=lam, flux=self.ev.flux_d, obs=obs, psf=psf, conv_path=_lib.CONV_DIRECT))
            self.ctx.batch_run(jobs, self.hess_grid, self.data_hess, self.data_mom, ll[: b1 - b0],
                               hess_out=out[b0:b1], use_graph=True)
            if progress is not None:
                progress(b1, n)
        return out

    def targets(self, hess: torch.Tensor) -> torch.Tensor:
        return log_hess_target(self.ctx, hess)

    def inputs(self, thetas: np.ndarray) -> torch.Tensor:
        return torch.from_numpy(self.std(thetas)).to(self.dev)

    # ---------------------------------------------------------------- training
    def fit(self, x: torch.Tensor, t: torch.Tensor, steps: int, batch: int = 256, lr: float = 1e-3,
            lr_final: float = 1e-4, seed: int = 0, log_every: int = 0):
        """Adam with a geometric learning-rate decay from lr to lr_final; returns the loss history."""
        g = torch.Generator(device="cpu").manual_seed(seed)
        n = x.shape[0]
        loss = torch.empty(1, dtype=torch.float32, device=self.dev)
        grad = torch.empty(self.net.n_params, dtype=torch.float32, device=self.dev)
        hist = []
        # every step's batch rows in one copy: a host-to-device copy per step would wait for the
        # previous step's kernels and leave the GPU idle while the next step is launched; the
        # library reads the batch's rows of x and t itself
        all_idx = torch.randint(0, n, (steps, batch), generator=g, dtype=torch.int32).to(self.dev)
        for s in range(steps):
            cur = lr * (lr_final / lr) ** (s / max(steps - 1, 1))
            self.net.train_step_rows(x, t, all_idx[s], cur, grad, loss_out=loss)
            if log_every and (s % log_every == 0 or s == steps - 1):
                hist.append((s, float(loss.item())))
        return hist

    def local_draws(self, center, frac: float, n: int, seed: int) -> np.ndarray:
        """n parameter vectors uniform in center +- frac x (prior width), clipped to the prior box."""
        r = np.random.default_rng(np.random.SeedSequence([31337, seed]))
        w = self.hi - self.lo
        u = r.uniform(-1.0, 1.0, size=(n, len(self.lo)))
        return np.clip(np.asarray(center, np.float64) + u * frac * w, self.lo, self.hi)

    def refine(self, x: torch.Tensor, t: torch.Tensor, center, frac: float, n: int, steps: int, seed0: int,
               batch: int = 1024, lr: float = 3e-4, lr_final: float = 3e-5, seed: int = 1):
        """Sequential design: simulate n extra pairs around `center` (e.g. the chain's start),
        then continue training on the union of the old and new pairs.  Returns the union."""
        th = self.local_draws(center, frac, n, seed)
        xl = self.inputs(th)
        tl = self.targets(self.simulate_hess(th, seed0=seed0))
        xu, tu = torch.cat([x, xl]), torch.cat([t, tl])
        self.fit(xu, tu, steps, batch=batch, lr=lr, lr_final=lr_final, seed=seed)
        return xu, tu

    def mse(self, x: torch.Tensor, t: torch.Tensor) -> float:
        """Mean squared error of the network over the set (computed by the library)."""
        out = torch.empty(1, dtype=torch.float64, device=self.dev)
        self.net.loss(x.contiguous(), t.contiguous(), out)
        return float(out.item())

    # ---------------------------------------------------------------- likelihoods
    def surrogate_loglike_batch(self, thetas: np.ndarray) -> np.ndarray:
        x = self.inputs(thetas)
        y = self.net.forward(x)
        out = torch.empty(len(thetas), dtype=torch.float64, device=self.dev)
        self.ctx.surrogate_loglike(y, self.data_hess, out)
        return out.cpu().numpy()

    def surrogate_loglike(self, theta: np.ndarray) -> float:
        self._x1.copy_(torch.from_numpy(self.std(np.asarray(theta)[None, :])))
        self.net.forward(self._x1, self._y1)
        self.ctx.surrogate_loglike(self._y1, self.data_hess, self._ll1)
        return float(self._ll1.item())

    def simulator_loglike(self, theta: np.ndarray, seed: int, nim: int = 256, data_nim: int | None = None) -> float:
        """Simulator Poisson log-likelihood of the data Hess at theta (one simulation)."""
        if self.eval_256 is None or self.eval_256.nim != nim:
            model, obs = self.theta_to_model(theta, seed=seed, nim=nim)
            self.eval_256 = Evaluator(self.ctx, self.grid, nim, obs.psf, self.hess_grid)
        model, obs = self.theta_to_model(theta, seed=seed, nim=nim)
        out = self.eval_256.loglike(model, obs, self.data_hess, self.data_mom)
        return float(out.item())

    def run_mcmc(self, theta0, n_steps: int, step_scale, rng, screen: bool, nim: int = 256, seed0: int = 10_000_000,
                 temperature: float = 1.0):
        counter = [seed0]

        def sim(th):
            counter[0] += 1
            return self.simulator_loglike(th, counter[0], nim)

        def prior(th):
            th = np.asarray(th)
            return 0.0 if np.all(th >= self.lo) and np.all(th <= self.hi) else -np.inf

        t0 = time.perf_counter()
        chain, lchain, info = delayed_acceptance_mcmc(theta0, n_steps, step_scale, prior, sim, self.surrogate_loglike,
                                                      rng, screen=screen, temperature=temperature)
        info["seconds"] = time.perf_counter() - t0
        return chain, lchain, info
