"""Stochastic-likelihood tooling (Appendix A of the paper).

The simulated diagram is one random realisation of the model, so the log-likelihood of a fixed
parameter point scatters from call to call, with a long positive tail.  The paper's remedy after a
nested-sampling fit: re-simulate the best-fit point 100 times, take the median log-likelihood as a
ceiling L_max, cap every sample's log-likelihood at L_max and recompute the posterior weights and
the remaining-evidence criterion.  This module provides the re-simulations (one batched,
graph-replayed launch through the C ABI), the ceiling, the capped weights and the criterion, and the
study of the scatter against the image size (larger images average over more rare fluctuations).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import _lib
from .pipeline import Evaluator


def resimulate_loglikes(ctx: _lib.Context, ev: Evaluator, model, obs, data_hess: torch.Tensor,
                        data_mom: torch.Tensor, n: int, seed0: int, mode: int = _lib.LL_POISSON,
                        eps: float = 0.01, batch: int = 256, hess_out: torch.Tensor | None = None) -> np.ndarray:
    """log L of one parameter point for n seeds (seed0 .. seed0 + n - 1), as batched launches of up
    to `batch` simulations on the direct convolution path; bit-identical to n single calls.
    hess_out [n][n_bins] (int32, device), if given, receives every simulation's Hess diagram."""
    lam = ev.entries(model).clone()
    psf = ev.psf_d
    out = np.empty(n, dtype=np.float64)
    ll = torch.empty(min(batch, n), dtype=torch.float64, device=ev.dev)
    for b0 in range(0, n, batch):
        b1 = min(n, b0 + batch)
        jobs = [dict(lam=lam, flux=ev.flux_d, obs=dataclasses.replace(obs, seed=seed0 + k), psf=psf,
                     conv_path=_lib.CONV_DIRECT) for k in range(b0, b1)]
        ctx.batch_run(jobs, ev.hess_grid, data_hess, data_mom, ll[: b1 - b0], mode, eps,
                      hess_out=None if hess_out is None else hess_out[b0:b1], use_graph=True, bands=ev.bands)
        out[b0:b1] = ll[: b1 - b0].cpu().numpy()
    return out


def lmax_ceiling(resimulated: np.ndarray) -> float:
    """The ceiling L_max: the median of the best-fit point's re-simulated log-likelihoods."""
    return float(np.median(np.asarray(resimulated, dtype=np.float64)))


def cap_loglikes(logl, lmax: float) -> np.ndarray:
    """Every log-likelihood above L_max is set to L_max (positive fluctuations carry no weight)."""
    return np.minimum(np.asarray(logl, dtype=np.float64), float(lmax))


def nested_weights(logl, log_dx) -> np.ndarray:
    """Normalised posterior weights w_i = L_i dX_i / sum_j L_j dX_j of nested-sampling dead points
    (log-likelihoods logl, log prior-volume widths log_dx)."""
    a = np.asarray(logl, dtype=np.float64) + np.asarray(log_dx, dtype=np.float64)
    a = a - a.max()
    w = np.exp(a)
    return w / w.sum()


def remaining_evidence(logl, log_dx, log_x_final: float, logl_max_live: float) -> float:
    """Delta ln Z: ln(Z + L_max,live X_final) - ln Z, the stopping criterion of nested sampling
    (evidence that could still lie in the remaining prior volume X_final)."""
    a = np.asarray(logl, dtype=np.float64) + np.asarray(log_dx, dtype=np.float64)
    lnz = np.logaddexp.reduce(a)
    return float(np.logaddexp(lnz, logl_max_live + log_x_final) - lnz)


def effective_sample_size(w) -> float:
    """Kish's effective sample size of normalised weights, 1 / sum w^2."""
    w = np.asarray(w, dtype=np.float64)
    return float(1.0 / np.sum(w * w))


def scatter_vs_image_size(ctx: _lib.Context, grid, model, obs, nims, n_seeds: int, hess_bins: int = 100,
                          data_seed: int = 2, mode: int = _lib.LL_POISSON) -> list[dict]:
    """For each image side N: a data image of the model at N (seed data_seed), then n_seeds
    re-simulations scored against it.  Returns per N the mean, standard deviation and median
    (the would-be L_max) of log L, and the standard deviation per pixel."""
    rows = []
    for N in nims:
        o = dataclasses.replace(obs, nim=int(N))
        dev = torch.device("cuda")
        ev = Evaluator(ctx, grid, int(N), o.psf, dict(x0=0.0, dx=0.05, y0=0.0, dy=0.05, nx=hess_bins, ny=hess_bins))
        md = ev.simulate(model, dataclasses.replace(o, seed=data_seed), _lib.CONV_DIRECT).cpu().numpy().astype(np.float64)
        fin = np.isfinite(md).all(axis=0)
        x = float(np.median((md[0] - md[1])[fin]))
        y = float(np.median(md[1][fin]))
        ev.hess_grid = dict(x0=np.floor(x / 0.05) * 0.05 - hess_bins // 2 * 0.05, dx=0.05,
                            y0=np.floor(y / 0.05) * 0.05 - hess_bins // 2 * 0.05, dy=0.05, nx=hess_bins, ny=hess_bins)
        dh = torch.empty(hess_bins * hess_bins, dtype=torch.int32, device=dev)
        dm = torch.empty(3, dtype=torch.float64, device=dev)
        ev.hess_of(ev.mags, dh, dm)
        ll = resimulate_loglikes(ctx, ev, model, o, dh, dm, n_seeds, seed0=1000, mode=mode)
        rows.append(dict(nim=int(N), mean=float(ll.mean()), std=float(ll.std(ddof=1)), median=lmax_ceiling(ll),
                         std_per_pixel=float(ll.std(ddof=1) / (N * N)),
                         skew=float(np.mean((ll - ll.mean()) ** 3) / ll.std() ** 3)))
    return rows
