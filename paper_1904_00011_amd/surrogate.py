"""Surrogate log-Hess network and the delayed-acceptance sampler that uses it as a screen.

The network (BF16 MFMA forward/backward and Adam in libpcmd.so) maps the 12 model parameters to
the log-Hess diagram log((H_j + 1/2) / (N + n_bins / 2)).  Inside Metropolis-Hastings it screens
each proposal: a proposal the surrogate already rejects never reaches the simulator, and one it
accepts is accepted or rejected by the simulator's own log-likelihood with the delayed-acceptance
correction (Christen & Fox 2005), so the chain still targets the simulator's likelihood.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib


class SurrogateNet:
    """Device storage of one network (FP32 master weights, Adam moments, BF16 copies of W, W^T)."""

    def __init__(self, ctx: _lib.Context, dims, master: np.ndarray, device: str = "cuda"):
        self.ctx = ctx
        self.dims = tuple(int(d) for d in dims)
        dev = torch.device(device)
        n = _lib.mlp_param_count(self.dims)
        nw = _lib.mlp_weight_count(self.dims)
        assert master.shape == (n,), (master.shape, n)
        self.master = torch.from_numpy(np.ascontiguousarray(master, np.float32)).to(dev)
        self.m = torch.zeros(n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(n, dtype=torch.float32, device=dev)
        self.w = torch.empty(nw, dtype=torch.bfloat16, device=dev)
        self.wt = torch.empty(nw, dtype=torch.bfloat16, device=dev)
        self.step = 0
        self.struct = _lib.MlpS()
        self.struct.n_layers = len(self.dims) - 1
        for i, d in enumerate(self.dims):
            self.struct.dims[i] = d
        self.struct.master = self.master.data_ptr()
        self.struct.adam_m = self.m.data_ptr()
        self.struct.adam_v = self.v.data_ptr()
        self.struct.w_bf16 = self.w.data_ptr()
        self.struct.wt_bf16 = self.wt.data_ptr()
        ctx.mlp_refresh(self.struct)

    @property
    def n_params(self) -> int:
        return int(self.master.numel())

    def forward(self, x: torch.Tensor, y: torch.Tensor | None = None) -> torch.Tensor:
        if y is None:
            y = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device=x.device)
        self.ctx.mlp_forward(self.struct, x, y)
        return y

    def train_step(self, x, t, lr: float, loss_out=None, grad_out=None, apply_update: bool = True):
        if apply_update:
            self.step += 1
        self.ctx.mlp_train_step(self.struct, x, t, lr, max(self.step, 1), loss_out, grad_out, apply_update)

    def train_step_rows(self, x, t, rows, lr: float, grad, loss_out=None):
        """One Adam step on the batch formed by rows `rows` (int32 device vector) of the set (x, t);
        the gather runs inside the library's kernels.  grad: [n_params] FP32 device buffer."""
        self.step += 1
        self.ctx.mlp_backward(self.struct, x, t, grad, rows=rows, loss_out=loss_out)
        self.ctx.mlp_adam(self.struct, grad, lr, self.step)

    def loss(self, x, t, mse_out, rows=None):
        """Mean squared error over the set (x, t) (or its rows `rows`) into mse_out [1] FP64."""
        self.ctx.mlp_loss(self.struct, x, t, mse_out, rows=rows)

    def state(self) -> dict:
        """Checkpoint: master weights, Adam moments and the step count."""
        return dict(dims=self.dims, master=self.master.cpu().numpy(), m=self.m.cpu().numpy(),
                    v=self.v.cpu().numpy(), step=self.step)

    def load_state(self, st: dict):
        assert tuple(st["dims"]) == self.dims
        self.master.copy_(torch.from_numpy(np.asarray(st["master"], np.float32)))
        self.m.copy_(torch.from_numpy(np.asarray(st["m"], np.float32)))
        self.v.copy_(torch.from_numpy(np.asarray(st["v"], np.float32)))
        self.step = int(st["step"])
        self.ctx.mlp_refresh(self.struct)


def log_hess_target(ctx: _lib.Context, hess: torch.Tensor) -> torch.Tensor:
    """log((H + 1/2) / (N + n_bins / 2)) per row of a [n][n_bins] count tensor (the training
    targets), computed by the library."""
    out = torch.empty(hess.shape, dtype=torch.float32, device=hess.device)
    ctx.log_hess_target(hess, out)
    return out


class Standardizer:
    """Affine map of the 12 parameters onto roughly unit scale (fixed from the prior ranges)."""

    def __init__(self, lo, hi):
        self.lo = np.asarray(lo, np.float64)
        self.hi = np.asarray(hi, np.float64)

    def __call__(self, theta: np.ndarray) -> np.ndarray:
        return ((np.asarray(theta, np.float64) - self.lo) / (self.hi - self.lo) * 2.0 - 1.0).astype(np.float32)


def delayed_acceptance_mcmc(theta0, n_steps: int, step_scale, log_prior, sim_loglike, sur_loglike, rng,
                            screen: bool = True, temperature: float = 1.0):
    """Metropolis-Hastings with a symmetric Gaussian random walk on the target
    prior x exp(L / temperature).  With screen=True a proposal is first accepted with probability
    min(1, exp(dS / temperature + d log prior)) using the surrogate log-likelihood S; survivors are
    then accepted with probability min(1, exp((dL - dS) / temperature)) using the simulator's L
    (delayed acceptance, Christen & Fox 2005), so the chain targets the same distribution as plain
    Metropolis-Hastings (screen=False, every proposal judged by the simulator).  A temperature
    above one tempers the likelihood, e.g. to the scale of its own stochastic scatter.
    Returns (chain [n_steps+1][d], logL chain, counters dict)."""
    inv_t = 1.0 / float(temperature)
    theta = np.asarray(theta0, np.float64)
    L = sim_loglike(theta) * inv_t
    S = sur_loglike(theta) * inv_t if screen else 0.0
    lp = log_prior(theta)
    chain, lchain = [theta.copy()], [L]
    n_sim, n_sur, n_acc, n_stage1 = 1, 1 if screen else 0, 0, 0
    for _ in range(n_steps):
        prop = theta + rng.normal(size=theta.shape) * step_scale
        lpp = log_prior(prop)
        if not np.isfinite(lpp):
            chain.append(theta.copy()); lchain.append(L)
            continue
        if screen:
            Sp = sur_loglike(prop) * inv_t
            n_sur += 1
            a1 = (Sp - S) + (lpp - lp)
            if math.log(rng.uniform()) >= min(0.0, a1):
                chain.append(theta.copy()); lchain.append(L)
                continue
            n_stage1 += 1
            Lp = sim_loglike(prop) * inv_t
            n_sim += 1
            a2 = (Lp - L) - (Sp - S)
            if math.log(rng.uniform()) < min(0.0, a2):
                theta, L, S, lp = prop, Lp, Sp, lpp
                n_acc += 1
        else:
            Lp = sim_loglike(prop) * inv_t
            n_sim += 1
            if math.log(rng.uniform()) < min(0.0, (Lp - L) + (lpp - lp)):
                theta, L, lp = prop, Lp, lpp
                n_acc += 1
        chain.append(theta.copy()); lchain.append(L)
    return np.array(chain), np.array(lchain) / inv_t, dict(simulator_calls=n_sim, surrogate_calls=n_sur, accepted=n_acc,
                                                   passed_screen=n_stage1)
