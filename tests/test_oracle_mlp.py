"""Oracle surrogate-network pins: backward formulas against finite differences of the pure FP64
network, GELU against numerical differentiation, BF16 rounding, the surrogate likelihood."""
import math

import numpy as np
import pytest
from scipy import stats

import synth_inputs as si
from oracle import mlp


def test_bf16_rounding():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -7 + 2 ** -8, -2.5, 3.0e-5], dtype=np.float32)
    got = mlp.bf16_round(x)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: even -> 1; 1 + 1.5*2^-8 rounds up to 1 + 2^-7;
    # 1 + 2^-7 + 2^-8 is a tie: even (mantissa ...10) -> 1 + 2^-6
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == np.float32(1 + 2 ** -7)
    assert got[3] == np.float32(1 + 2 ** -6) and got[4] == -2.5
    assert abs(got[5] / 3.0e-5 - 1) < 2 ** -8


def test_gelu_derivative():
    z = np.linspace(-6, 6, 1001)
    h = 1e-6
    num = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.max(np.abs(num - mlp.gelu_grad(z))) < 1e-8
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    assert mlp.gelu(np.array([3.0]))[0] == pytest.approx(3.0 * stats.norm.cdf(3.0), rel=1e-14)


def test_backward_against_finite_differences():
    dims = (5, 7, 6, 4)
    master = si.mlp_init(dims, 1).astype(np.float64)
    r = np.random.default_rng(2)
    x = r.normal(size=(9, 5))
    t = r.normal(size=(9, 4))
    loss, g = mlp.loss_and_grad(master, dims, x, t, rounding=False)
    h = 1e-6
    for i in r.choice(len(master), 40, replace=False):
        mp = master.copy(); mp[i] += h
        mm = master.copy(); mm[i] -= h
        lp, _ = mlp.loss_and_grad(mp, dims, x, t, rounding=False)
        lm, _ = mlp.loss_and_grad(mm, dims, x, t, rounding=False)
        assert abs((lp - lm) / (2 * h) - g[i]) < 1e-7 + 1e-5 * abs(g[i])
    assert mlp.param_count(dims) == len(master)


def test_adam_first_step_moves_by_lr():
    w = np.array([1.0, -2.0, 0.5]); g = np.array([0.3, -0.1, 0.0])
    w2, m, v = mlp.adam_update(w, g, np.zeros(3), np.zeros(3), 1, 0.01)
    # first bias-corrected step is lr * g / (|g| + eps) = lr * sign(g)
    assert np.allclose(w2[:2], w[:2] - 0.01 * np.sign(g[:2]), rtol=0, atol=1e-9) and w2[2] == w[2]


def test_surrogate_loglike_is_poisson():
    r = np.random.default_rng(3)
    d = r.poisson(3.0, 500)
    y = r.normal(0, 0.5, 500)
    lam = d.sum() * np.exp(y) / np.exp(y).sum()
    assert mlp.surrogate_loglike(y, d) == pytest.approx(float(stats.poisson.logpmf(d, lam).sum()), rel=1e-12)
    assert mlp.surrogate_loglike(y + 7.0, d) == pytest.approx(mlp.surrogate_loglike(y, d), rel=1e-12)


def test_log_hess_target_pins():
    # the shares exp(target) of a diagram sum to one; an empty bin gets (1/2) / (N + n/2)
    r = np.random.default_rng(5)
    h = r.poisson(3.0, size=(4, 250))
    h[1] = 0
    h[2, :200] = 0
    t = mlp.log_hess_target(h)
    assert t.shape == (4, 250)
    assert np.allclose(np.exp(t).sum(axis=1), 1.0, rtol=0, atol=1e-13)
    assert t[1] == pytest.approx(np.full(250, np.log(1.0 / 250)), rel=1e-14)
    n2 = h[2].sum()
    assert t[2, 0] == pytest.approx(np.log(0.5 / (n2 + 125.0)), rel=1e-14)
    # a hand case: counts (3, 0, 1), N = 4, denominator 5.5
    assert mlp.log_hess_target([3, 0, 1])[0] == pytest.approx(np.log([3.5 / 5.5, 0.5 / 5.5, 1.5 / 5.5]), rel=1e-15)
    assert mlp.mse([[1.0, 2.0]], [[0.0, 4.0]]) == pytest.approx(2.5)
