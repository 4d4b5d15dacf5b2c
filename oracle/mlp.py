"""Multilayer perceptron surrogate of the log-Hess diagram (oracle side).

The paper evaluates its stochastic likelihood at every sampler point (Sec. 2.5) and notes the
cost of fits (about 100 GPU-hours, Sec. 2.5).  A network that maps the model parameters to the
log-Hess diagram can screen proposals before the simulator judges them.  This module is the plain
reference of that network:

  x_0 = bf16(theta);  z_l = x_l W_l^T + b_l;  x_{l+1} = bf16(GELU(z_l)) for hidden layers;
  y = z_{L-1};  loss = mean((y - t)^2) over samples and outputs.

GELU(z) = z Phi(z) (exact, with the error function).  Weights used by the products are the
BF16-rounded master weights; stored activations and back-propagated gradients are rounded to
BF16 where the network stores them in BF16 (round to nearest even).  Everything else is FP64
here, so that the GPU's FP32 accumulation is the only difference.

Backward (the chain rule written out):
  dy = 2 (y - t) / (n M);  dz_{L-1} = bf16(dy);
  dW_l = dz_l^T x_l;  db_l = sum_n dz_l;  dx_l = dz_l W_l;  dz_{l-1} = bf16(dx_l GELU'(z_{l-1})),
  GELU'(z) = Phi(z) + z phi(z).
Adam (Kingma & Ba 2015) on the FP32 master weights.

Targets: ln((H_j + 1/2) / (N + n_bins / 2)) of a simulated Hess diagram (N its total).

Pins: finite differences of the pure-FP64 network (no rounding) against the backward formulas;
GELU and its derivative against numerical differentiation; the target shares of a diagram sum to
one and equal counts give equal targets (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def bf16_round(x) -> np.ndarray:
    """Round FP32 values to BF16 (nearest, ties to even); returned as FP32."""
    x = np.asarray(x, dtype=np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = (u + np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))) >> np.uint64(16)
    return (r.astype(np.uint32) << np.uint32(16)).view(np.float32)


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + special.erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def param_count(dims) -> int:
    return sum(dims[l + 1] * dims[l] + dims[l + 1] for l in range(len(dims) - 1))


def unpack(master: np.ndarray, dims):
    """Packed master vector -> [(W_l [out][in], b_l [out])]."""
    out, o = [], 0
    for l in range(len(dims) - 1):
        nw = dims[l + 1] * dims[l]
        W = master[o:o + nw].reshape(dims[l + 1], dims[l])
        o += nw
        b = master[o:o + dims[l + 1]]
        o += dims[l + 1]
        out.append((W, b))
    return out


def forward(master, dims, x, rounding: bool = True):
    """Returns (y, cache).  rounding=False gives the pure FP64 network (for finite differences)."""
    rnd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(np.asarray(master, dtype=np.float64), dims)
    xs, zs = [], []
    h = np.asarray(rnd(np.asarray(x, dtype=np.float32) if rounding else x), dtype=np.float64)
    L = len(layers)
    for l, (W, b) in enumerate(layers):
        Wq = np.asarray(rnd(W.astype(np.float32)) if rounding else W, dtype=np.float64)
        bq = np.asarray(b.astype(np.float32) if rounding else b, dtype=np.float64)
        xs.append(h)
        z = h @ Wq.T + bq
        zs.append(z)
        if l < L - 1:
            a = gelu(z)
            h = np.asarray(rnd(a.astype(np.float32)) if rounding else a, dtype=np.float64)
    return zs[-1], dict(xs=xs, zs=zs)


def loss_and_grad(master, dims, x, t, rounding: bool = True):
    """MSE loss and the gradient of every master parameter (packed like `master`)."""
    rnd = bf16_round if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    y, cache = forward(master, dims, x, rounding)
    t = np.asarray(t, dtype=np.float64)
    n, M = y.shape
    loss = float(np.mean((y - t) ** 2))
    layers = unpack(np.asarray(master, dtype=np.float64), dims)
    L = len(layers)
    dy = 2.0 * (y - t) / (n * M)
    dz = np.asarray(rnd(dy.astype(np.float32)) if rounding else dy, dtype=np.float64)
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        W, _ = layers[l]
        Wq = np.asarray(rnd(W.astype(np.float32)) if rounding else W, dtype=np.float64)
        dW = dz.T @ cache["xs"][l]
        db = dz.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            dx = dz @ Wq
            g = dx * gelu_grad(cache["zs"][l - 1])
            dz = np.asarray(rnd(g.astype(np.float32)) if rounding else g, dtype=np.float64)
    packed = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, packed


def adam_update(master, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015); returns (master, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return master - lr * mh / (np.sqrt(vh) + eps), m, v


def log_hess_target(hess):
    """Training target of one or more Hess diagrams (rows of counts): the log of each bin's share
    with half a count added to every bin, ln((H_j + 1/2) / (N + n_bins / 2)), N the row's total.
    The shares of a row sum to one, and an empty bin keeps a finite target."""
    h = np.atleast_2d(np.asarray(hess, dtype=np.float64))
    N = h.sum(axis=1, keepdims=True)
    return np.log((h + 0.5) / (N + 0.5 * h.shape[1]))


def mse(y, t) -> float:
    """Mean squared error over all samples and outputs."""
    return float(np.mean((np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)) ** 2))


def surrogate_loglike(logh_pred, hess_data):
    """Poisson log-likelihood of the data Hess under the predicted bin proportions:
    lam_j = N_d exp(y_j) / sum_k exp(y_k);  logL = sum_j d_j ln lam_j - lam_j - ln d_j!."""
    y = np.asarray(logh_pred, dtype=np.float64)
    d = np.asarray(hess_data, dtype=np.float64).ravel()
    ymax = y.max()
    w = np.exp(y - ymax)
    lam = d.sum() * w / w.sum()
    return float(np.sum(d * np.log(lam) - lam - special.gammaln(d + 1.0)))
