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

import ctypes as C
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


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def _check(rc: int, what: str) -> None:
    if rc != _lib.OK:
        raise _lib.PcmdError(rc, f"{what} rejected its arguments (NaN, empty, or no finite mass)")


def lmax_ceiling(resimulated) -> float:
    """The ceiling L_max: the median of the best-fit point's re-simulated log-likelihoods."""
    v = _f64(resimulated)
    out = C.c_double(0.0)
    _check(_lib.load().pcmd_lmax_ceiling(v.ctypes.data, v.size, C.byref(out)), "pcmd_lmax_ceiling")
    return out.value


def cap_loglikes(logl, lmax: float) -> np.ndarray:
    """Every log-likelihood above L_max is set to L_max (positive fluctuations carry no weight)."""
    v = _f64(logl)
    out = np.empty_like(v)
    _check(_lib.load().pcmd_cap_loglikes(v.ctypes.data, v.size, float(lmax), out.ctypes.data), "pcmd_cap_loglikes")
    return out


def nested_weights(logl, log_dx) -> np.ndarray:
    """Normalised posterior weights w_i = L_i dX_i / sum_j L_j dX_j of nested-sampling dead points
    (log-likelihoods logl, log prior-volume widths log_dx)."""
    a, d = _f64(logl), _f64(log_dx)
    if a.shape != d.shape:
        raise ValueError("logl and log_dx differ in shape")
    w = np.empty_like(a)
    _check(_lib.load().pcmd_nested_weights(a.ctypes.data, d.ctypes.data, a.size, w.ctypes.data), "pcmd_nested_weights")
    return w


def remaining_evidence(logl, log_dx, log_x_final: float, logl_max_live: float) -> float:
    """Delta ln Z: ln(Z + L_max,live X_final) - ln Z, the stopping criterion of nested sampling
    (evidence that could still lie in the remaining prior volume X_final)."""
    a, d = _f64(logl), _f64(log_dx)
    if a.shape != d.shape:
        raise ValueError("logl and log_dx differ in shape")
    out = C.c_double(0.0)
    _check(_lib.load().pcmd_remaining_evidence(a.ctypes.data, d.ctypes.data, a.size, float(log_x_final),
                                               float(logl_max_live), C.byref(out)), "pcmd_remaining_evidence")
    return out.value


def effective_sample_size(w) -> float:
    """Kish's effective sample size of normalised weights, 1 / sum w^2."""
    v = _f64(w)
    out = C.c_double(0.0)
    _check(_lib.load().pcmd_effective_sample_size(v.ctypes.data, v.size, C.byref(out)), "pcmd_effective_sample_size")
    return out.value


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
