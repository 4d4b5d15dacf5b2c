"""One likelihood evaluation through the C ABI: entries -> simulate -> Hess -> log-likelihood.

Holds the device copy of an isochrone grid and the output buffers so that repeated evaluations
allocate nothing new.  All arithmetic runs in libpcmd.so.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _lib


class Evaluator:
    """Evaluate log L(theta) for a fixed isochrone grid, image size, PSF and Hess grid."""

    def __init__(self, ctx: _lib.Context, grid, nim: int, psf: np.ndarray | None, hess_grid: dict,
                 bands=(0, 1, 1), imf_alpha: float = 2.35, device: str = "cuda", imf: str = "salpeter"):
        self.ctx = ctx
        self.grid = grid
        self.nim = int(nim)
        self.hess_grid = dict(hess_grid)
        self.bands = tuple(bands)
        self.dev = torch.device(device)
        imf_w, flux, self.iso_imf_sum = _lib.grid_prepare(grid.iso_of_entry, grid.mass, grid.absmag, imf_alpha, imf,
                                                          n_iso=grid.n_iso)
        self.iso_d = torch.from_numpy(np.ascontiguousarray(grid.iso_of_entry, np.int32)).to(self.dev)
        self.imf_d = torch.from_numpy(imf_w).to(self.dev)
        self.flux_d = torch.from_numpy(flux).to(self.dev)
        self.E = int(grid.n_entries)
        self.B = int(grid.n_bands)
        self.psf_d = None if psf is None else torch.from_numpy(np.ascontiguousarray(psf, np.float32)).to(self.dev)
        self.lam = torch.empty(self.E, dtype=torch.float64, device=self.dev)
        self.mags = torch.empty((self.B, self.nim * self.nim), dtype=torch.float32, device=self.dev)
        nb = hess_grid["nx"] * hess_grid["ny"]
        self.hess = torch.empty(nb, dtype=torch.int32, device=self.dev)
        self.mom = torch.empty(3, dtype=torch.float64, device=self.dev)
        self.out = torch.empty(1, dtype=torch.float64, device=self.dev)

    def entries(self, model, stream=None):
        w, npix = _lib.iso_weights(model, self.grid)
        self.ctx.entries(self.E, self.iso_d, self.imf_d, self.iso_imf_sum, w, npix, self.lam, stream)
        return self.lam

    def simulate(self, model, obs, conv_path: int = _lib.CONV_AUTO, stream=None):
        self.entries(model, stream)
        self.ctx.simulate(self.lam, self.flux_d, obs, self.mags, psf=self.psf_d, conv_path=conv_path, stream=stream)
        return self.mags

    def hess_of(self, mags, hess_out, mom_out, stream=None):
        self.ctx.hess(mags, self.B, mags.shape[1], self.hess_grid, hess_out, mom_out, self.bands, stream)

    def loglike(self, model, obs, data_hess, data_mom, mode: int = _lib.LL_POISSON, eps: float = 0.01,
                conv_path: int = _lib.CONV_AUTO, stream=None, out=None):
        """Queue one full evaluation; the result lands in `out` (a one-element float64 device
        tensor, e.g. a slot of a results vector) or, by default, in self.out."""
        dst = self.out if out is None else out
        if dst.dtype != torch.float64 or dst.numel() != 1 or not dst.is_cuda:
            raise ValueError("out must be a one-element float64 device tensor")
        self.simulate(model, obs, conv_path, stream)
        self.hess_of(self.mags, self.hess, self.mom, stream)
        self.ctx.loglike(self.hess, data_hess, self.mom, data_mom, dst, mode, eps, stream)
        return dst

    def loglike_multi(self, model, obs, cmds, mode: int = _lib.LL_POISSON, eps: float = 0.01,
                      conv_path: int = _lib.CONV_AUTO, stream=None):
        """Joint log-likelihood of several colour-magnitude diagrams of one simulated image, e.g.
        (b0 - b1, b1) and (b1 - b2, b2) for three bands: one simulation, then per diagram its Hess
        and likelihood, the diagrams' likelihoods added on the device.  cmds: sequence of
        (bands, hess_grid, data_hess, data_mom).  The result lands in self.out (device)."""
        self.simulate(model, obs, conv_path, stream)
        if not hasattr(self, "_multi_h") or len(self._multi_h) < len(cmds):
            self._multi_h = [None] * len(cmds)
        for k, (bands, hgrid, dh, dm) in enumerate(cmds):
            nb = hgrid["nx"] * hgrid["ny"]
            if self._multi_h[k] is None or self._multi_h[k].numel() != nb:
                self._multi_h[k] = torch.empty(nb, dtype=torch.int32, device=self.dev)
            self.ctx.hess(self.mags, self.B, self.mags.shape[1], hgrid, self._multi_h[k], self.mom, bands, stream)
            self.ctx.loglike(self._multi_h[k], dh, self.mom, dm, self.out, mode | (_lib.LL_ACCUMULATE if k else 0), eps,
                             stream)
        return self.out

