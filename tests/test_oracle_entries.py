"""Oracle a0 pins: normalisation, IMF closed form, MDF weights, SFH integrals."""
import math

import numpy as np
import pytest
from scipy import integrate

import synth_inputs as si
from oracle import entries as E


def test_sum_lambda_is_npix_all_models():
    g = si.headline_grid()
    for sfh in ("const", "tau", "dtau"):
        m = si.Model(sfh=sfh, log_npix=3.3, tau_gyr=2.0, mdf="gauss", feh_mu=-0.1)
        lam, _, _ = E.build_entries(m, g)
        assert lam.sum() == pytest.approx(10 ** 3.3, rel=1e-12)
        assert (lam >= 0).all()
    m = si.Model(sfh="nonparam", log_sfh=(1.0, 0.5, 0.0, 1.2, 2.0, 2.5, 1.5), mdf="gauss", feh_mu=0.0)
    lam, _, _ = E.build_entries(m, g)
    assert lam.sum() == pytest.approx(sum(10 ** v for v in m.log_sfh), rel=1e-12)


def test_salpeter_bin_integral_against_quadrature():
    g = si.isochrone_ssp(500)
    w = E.imf_weights(g, 2.35)
    e = E.imf_bin_edges(g.mass)
    for i in (0, 100, 499):
        q, _ = integrate.quad(lambda m: m ** -2.35, e[i], e[i + 1], epsabs=0, epsrel=1e-13)
        assert w[i] == pytest.approx(q, rel=1e-10)
    # bins tile the mass range: their sum is the integral over the whole range
    tot, _ = integrate.quad(lambda m: m ** -2.35, e[0], e[-1], epsabs=0, epsrel=1e-13, limit=200)
    assert w.sum() == pytest.approx(tot, rel=1e-10)
    # edges are geometric midpoints
    assert e[1] == pytest.approx(math.sqrt(g.mass[0] * g.mass[1]), rel=1e-14)


def test_small_case_lambda_range():
    g, m, o = si.small_case()
    lam, _, _ = E.build_entries(m, g)
    assert lam.sum() == pytest.approx(100.0, rel=1e-13)
    assert lam.mean() == pytest.approx(0.2, rel=1e-12)
    assert 5e-4 < lam.min() < 2e-3 and 1.0 < lam.max() < 1.6


def test_mdf_weights_sigma_0p2_on_grid():
    # normal density at 0, +-0.25, +-0.5, +-0.75 for sigma 0.2, normalised: the values worked
    # out by hand are 0.499, 0.228, 0.022 and 4.4e-4 (the last is pruned at 1%)
    grid = np.array([-1.0, -0.75, -0.5, -0.25, 0.0, 0.25, 0.5, 0.75, 1.0])
    m = si.Model(mdf="gauss", feh_mu=0.0, feh_sigma=0.2, mdf_prune=0.0)
    w = E.mdf_weights(m, grid)
    assert w[4] == pytest.approx(0.499, abs=1e-3)
    assert w[3] == pytest.approx(0.228, abs=1e-3) and w[5] == pytest.approx(w[3], rel=1e-14)
    assert w[2] == pytest.approx(0.0219, abs=2e-4)
    assert w[1] == pytest.approx(4.4e-4, abs=2e-5)
    m.mdf_prune = 0.01
    w = E.mdf_weights(m, grid)
    assert (w > 0).sum() == 5 and w.sum() == pytest.approx(1.0, rel=1e-14)


def test_tau_and_delayed_tau_against_quadrature():
    edges = np.linspace(6.0, 10.2, 8)
    T = 10 ** 10.2
    for tau_gyr in (0.1, 3.0, 8.0):
        tau = tau_gyr * 1e9
        w = E.sfh_age_weights(si.Model(sfh="tau", tau_gyr=tau_gyr), edges)
        wd = E.sfh_age_weights(si.Model(sfh="dtau", tau_gyr=tau_gyr), edges)
        for a in range(7):
            t1, t2 = T - 10 ** edges[a + 1], T - 10 ** edges[a]
            q, _ = integrate.quad(lambda t: math.exp(-t / tau), t1, t2, epsabs=0, epsrel=1e-12)
            qd, _ = integrate.quad(lambda t: t * math.exp(-t / tau), t1, t2, epsabs=0, epsrel=1e-12)
            assert w[a] == pytest.approx(q, rel=1e-8, abs=1e-300)
            assert wd[a] == pytest.approx(qd, rel=1e-8, abs=1e-300)
    wc = E.sfh_age_weights(si.Model(sfh="const"), edges)
    assert np.allclose(wc, 10 ** edges[1:] - 10 ** edges[:-1], rtol=1e-14)


def test_flux_is_ten_to_minus_0p4_mag():
    g, m, o = si.small_case()
    _, f64, f32 = E.build_entries(m, g)
    assert np.allclose(-2.5 * np.log10(f64), g.absmag, rtol=0, atol=1e-12)
    assert f32.dtype == np.float32


def test_kroupa_imf_against_quadrature_and_shape():
    """Kroupa (2001) IMF (Sec. 2.2's alternative to Salpeter): bin integrals against numerical
    quadrature of the piecewise density, continuity at 0.08 and 0.5 Msun, and the logarithmic
    slopes -0.3 / -1.3 / -2.3 of its three segments."""
    for lo, hi in ((0.01, 0.05), (0.05, 0.2), (0.07, 0.09), (0.3, 0.7), (0.45, 3.0), (0.02, 20.0), (1.0, 40.0)):
        q, _ = integrate.quad(E.kroupa_pdf, lo, hi, points=[p for p in (0.08, 0.5) if lo < p < hi], epsabs=0,
                              epsrel=1e-12, limit=200)
        assert E.kroupa_bin_weight(lo, hi)[0] == pytest.approx(q, rel=1e-10)
    for b in (0.08, 0.5):
        assert E.kroupa_pdf(b * (1 - 1e-12)) == pytest.approx(E.kroupa_pdf(b), rel=1e-9)
    for m, slope in ((0.02, -0.3), (0.2, -1.3), (5.0, -2.3)):
        d = math.log(E.kroupa_pdf(m * 1.001) / E.kroupa_pdf(m)) / math.log(1.001)
        assert d == pytest.approx(slope, rel=1e-9)
    # sum of lambda is still Npix with the Kroupa weights
    G = si.headline_grid()
    m = si.Model(sfh="tau", log_npix=3.0, tau_gyr=2.0, mdf="gauss", feh_mu=0.0, imf="kroupa")
    lam, _, _ = E.build_entries(m, G)
    assert lam.sum() == pytest.approx(1e3, rel=1e-12)
    # Kroupa holds fewer low-mass stars per high-mass star than Salpeter
    ms = si.Model(sfh="tau", log_npix=3.0, tau_gyr=2.0, mdf="gauss", feh_mu=0.0)
    ls, _, _ = E.build_entries(ms, G)
    low = G.mass < 0.3
    assert lam[low].sum() < ls[low].sum()
