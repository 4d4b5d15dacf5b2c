"""Binned log-likelihood of a model Hess against a data Hess (oracle side).

Sec. 2.5.  The paper compares bin counts d_i (data) and m_i (model) with
Gaussian statistics, a floor of 2 on the per-bin uncertainty, and adds a term C
for the difference of mean colour and magnitude with a 0.05 mag error.  It
names a Poisson likelihood only to say that a bin with data but no model pixels
breaks it.

Modes:
* POISSON (0): lam_j = N_d (m_j + eps) / (N_m + eps n_bins), a pseudo-count eps
  per bin so that sum lam = N_d and empty model bins stay finite;
  logL = sum_j [d_j ln lam_j - lam_j - ln d_j!].
* GAUSS_PAPER (1): the counts-domain reading of the printed formula: model
  counts scaled to the data total, mh_j = m_j N_d / N_m,
  sigma_j = max(sqrt(d_j + mh_j), 2), logL = -sum (d_j - mh_j)^2 / (2 sigma_j^2) + C.
* GAUSS_LITERAL (2): the formula as printed, fractions over sigma_j =
  max(sqrt(d_j^2 + m_j^2), 2), plus C.
C = -(C_d - C_m)^2 / (2 * 0.05^2) - (M_d - M_m)^2 / (2 * 0.05^2), with C and M
the mean colour and magnitude over finite pixels.
"""
from __future__ import annotations

import math

import numpy as np

POISSON, GAUSS_PAPER, GAUSS_LITERAL = 0, 1, 2


def mean_term(mom_m, mom_d) -> float:
    Cm, Mm = mom_m[0] / mom_m[2], mom_m[1] / mom_m[2]
    Cd, Md = mom_d[0] / mom_d[2], mom_d[1] / mom_d[2]
    return -(Cd - Cm) ** 2 / (2 * 0.05 ** 2) - (Md - Mm) ** 2 / (2 * 0.05 ** 2)


def loglike(h_model, h_data, mom_model, mom_data, mode: int = POISSON, eps: float = 0.01) -> float:
    m = np.asarray(h_model, dtype=np.float64).ravel()
    d = np.asarray(h_data, dtype=np.float64).ravel()
    Nm, Nd = m.sum(), d.sum()
    nb = m.shape[0]
    if mode == POISSON:
        lam = Nd * (m + eps) / (Nm + eps * nb)
        lgd = np.array([math.lgamma(v + 1.0) for v in d])
        return float(np.sum(d * np.log(lam) - lam - lgd))
    if mode == GAUSS_PAPER:
        mh = m * Nd / Nm
        sig = np.maximum(np.sqrt(d + mh), 2.0)
        return float(-np.sum((d - mh) ** 2 / (2 * sig ** 2)) + mean_term(mom_model, mom_data))
    if mode == GAUSS_LITERAL:
        sig = np.maximum(np.sqrt(d * d + m * m), 2.0)
        return float(-np.sum((d / Nd - m / Nm) ** 2 / (2 * sig ** 2)) + mean_term(mom_model, mom_data))
    raise ValueError(mode)
