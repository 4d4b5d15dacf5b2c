"""Oracle a3-a6 pins: PSF, noise, Hess and likelihood against closed forms,
hand-worked fixtures and brute-force enumeration."""
import math
import os

import numpy as np
import pytest
from scipy import stats

import synth_inputs as si
from oracle import entries as E
from oracle import hess as H
from oracle import loglike as L
from oracle import noise as N
from oracle import pipeline as P
from oracle import psf as PS
from oracle import sampler as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ---------------- PSF -----------------

def test_delta_psf_is_identity_and_flux_conserved():
    r = np.random.default_rng(0)
    F = r.gamma(0.5, 2.0, size=(2, 32, 32))
    d = np.zeros((2, 1, 1), np.float32); d[:] = 1
    assert np.array_equal(PS.convolve_periodic(F, d), F)
    p = si.psf_stack(5, (1.0, 1.3))
    G = PS.convolve_periodic(F, p)
    for b in range(2):
        assert G[b].sum() == pytest.approx(F[b].sum() * float(p[b].astype(np.float64).sum()), rel=1e-12)


def test_direct_equals_fft_circular_convolution():
    r = np.random.default_rng(1)
    F = r.gamma(0.5, 2.0, size=(1, 24, 24))
    p = si.psf_stack(7, (1.5,))
    G = PS.convolve_periodic(F, p)
    K, Nn = 7, 24
    h = (K - 1) // 2
    ker = np.zeros((Nn, Nn))
    for u in range(K):
        for v in range(K):
            ker[(u - h) % Nn, (v - h) % Nn] = p[0, u, v]
    Gf = np.real(np.fft.ifft2(np.fft.fft2(F[0]) * np.fft.fft2(ker)))
    assert np.allclose(G[0], Gf, rtol=1e-10, atol=1e-12)


def test_iid_variance_scales_by_sum_p2():
    r = np.random.default_rng(2)
    F = r.normal(0, 1, size=(1, 256, 256))
    p = si.psf_stack(9, (1.2,))
    G = PS.convolve_periodic(F, p)
    s2 = float((p[0].astype(np.float64) ** 2).sum())
    assert G.var() == pytest.approx(s2, rel=0.03)


def test_asymmetric_psf_orientation():
    # P[u][v] with a single 1 at (u, v) = (0, 2) shifts the image by (u - h, v - h) = (-1, +1)
    F = np.zeros((1, 8, 8)); F[0, 3, 3] = 1.0
    p = np.zeros((1, 3, 3), np.float32); p[0, 0, 2] = 1.0
    G = PS.convolve_periodic(F, p)
    assert G[0, 2, 4] == 1.0 and G.sum() == 1.0


# ---------------- noise -----------------

def test_gaussian_magnitude_noise_moments():
    G = np.full((2, 100000), 1e-8)
    o = si.Obs(nim=1, seed=4, dmod=0, noise_model=1, noise_sigma_mag=(0.02, 0.05))
    m = N.magnitudes(G, o)
    for b, s in enumerate((0.02, 0.05)):
        d = m[b] - 20.0
        assert abs(d.mean()) < 5 * s / math.sqrt(len(d))
        assert abs(d.std() - s) < 5 * s / math.sqrt(2 * len(d))


def test_shot_noise_variance_equals_counts():
    o = si.Obs(nim=1, seed=5, dmod=0, noise_model=2, exptime=(1000.0,), zp=(25.0,), sky=(0.0,))
    G = np.full((1, 200000), 10 ** (-0.4 * 27.0))          # m = 27 -> c = t 10^(-0.4 (27 - 25))
    m = N.magnitudes(G, o)
    c = 1000.0 * 10 ** (-0.4 * 2.0)
    cp = 1000.0 * 10 ** (-0.4 * (m[0] - 25.0))
    assert abs(cp.mean() - c) < 5 * math.sqrt(c / len(cp))
    assert cp.var() == pytest.approx(c, rel=0.02)
    # with sky: the sky adds to the counts the noise is drawn from and is subtracted after it, so
    # the sky-subtracted counts keep the source mean and take variance source + sky
    sky = 3.0 * c
    os_ = si.Obs(nim=1, seed=6, dmod=0, noise_model=2, exptime=(1000.0,), zp=(25.0,), sky=(sky,))
    ms = N.magnitudes(G, os_)
    fin = np.isfinite(ms[0])
    cs = np.where(fin, 1000.0 * 10 ** (-0.4 * (ms[0] - 25.0)), 0.0)   # +inf magnitude: counts <= 0
    assert (~fin).mean() < 1e-3
    assert abs(cs.mean() - c) < 5 * math.sqrt((c + sky) / len(cs)) + c * (~fin).mean()
    assert cs.var() == pytest.approx(c + sky, rel=0.03)
    # no noise: exact flux -> magnitude
    o0 = si.Obs(nim=1, seed=5, dmod=0, noise_model=0)
    assert N.magnitudes(np.array([[1e-10, 0.0]]), o0)[0, 0] == pytest.approx(25.0, abs=1e-12)
    assert np.isinf(N.magnitudes(np.array([[1e-10, 0.0]]), o0)[0, 1])


# ---------------- Hess -----------------

def load_hess_example():
    rows, Hx = [], []
    for line in open(os.path.join(GOLD, "hess_4x4_example.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        if t[0] == "H":
            Hx.append([int(v) for v in t[1:]])
        else:
            rows.append((float(t[0]), float(t[1]), int(t[2]), int(t[3])))
    return rows, np.array(Hx)


def test_hess_hand_example():
    rows, Hx = load_hess_example()
    mags = np.array([[r[0] for r in rows], [r[1] for r in rows]], dtype=np.float32)
    g = dict(x0=0.0, dx=0.05, nx=4, y0=20.0, dy=0.05, ny=3)
    ix, iy, _, _ = H.pixel_bins(mags, g, 0, 1, 1)
    assert list(ix) == [r[2] for r in rows] and list(iy) == [r[3] for r in rows]
    Hm, mom = H.hess(mags, g, 0, 1, 1)
    assert np.array_equal(Hm, Hx) and Hm.sum() == len(rows)
    fin = np.isfinite(mags).all(axis=0)
    m64 = mags.astype(np.float64)
    assert mom[2] == fin.sum()
    assert mom[0] == pytest.approx((m64[0] - m64[1])[fin].sum(), rel=1e-15)


def test_hess_total_and_distance_shift():
    lam, _, f32 = E.build_entries(*si.small_case()[1::-1])
    o = si.Obs(nim=32, seed=8, dmod=25.0, psf=si.psf_stack(3, (0.8, 0.8)), noise_model=1,
               noise_sigma_mag=(0.02, 0.02))
    out = P.simulate(lam, f32, o)
    x = np.median(out["mags"][0] - out["mags"][1]); y = np.median(out["mags"][1])
    g = si.hess_grid_from_median(x, y, 60, 60)
    H1, _ = H.hess(out["mags64"], g)
    assert H1.sum() == 32 * 32
    o2 = si.Obs(nim=32, seed=8, dmod=25.0 + 0.05 * 3, psf=o.psf, noise_model=1, noise_sigma_mag=(0.02, 0.02))
    out2 = P.simulate(lam, f32, o2)
    assert np.allclose(out2["mags64"] - out["mags64"], 0.15, atol=1e-9)     # colour unchanged, magnitude +0.15
    ix1, iy1, _, _ = H.pixel_bins(out["mags64"], g, 0, 1, 1)
    ix2, iy2, _, _ = H.pixel_bins(out2["mags64"], g, 0, 1, 1)
    ty = (out["mags64"][1] - g["y0"]) / g["dy"]
    safe = (np.abs(ty - np.round(ty)) > 1e-6) & (iy1 < g["ny"] - 4) & (ty >= 0)
    assert np.array_equal(ix1, ix2) and np.array_equal(iy2[safe], iy1[safe] + 3)


def test_end_to_end_brute_force_two_points():
    # two points, delta PSF, no noise, no dust, mu_d = 0: pixel (x, y) is a function of (n1, n2)
    lam = np.array([0.3, 1.7])
    mag = np.array([[1.0, 2.5], [0.4, 2.2]])          # [band][point]: blue, red absolute magnitudes
    f32 = (10 ** (-0.4 * mag)).astype(np.float32)
    o = si.Obs(nim=256, seed=21, dmod=0.0, psf=None, noise_model=0)
    out = P.simulate(lam, f32, o)
    g = dict(x0=-0.2, dx=0.05, nx=30, y0=-4.0, dy=0.05, ny=100)
    Hm, _ = H.hess(out["mags"], g)
    # enumerate (n1, n2) with the exact Poisson pmf
    expect = np.zeros_like(Hm, dtype=np.float64)
    f = f32.astype(np.float64)
    for n1 in range(0, 15):
        for n2 in range(0, 25):
            p = stats.poisson.pmf(n1, 0.3) * stats.poisson.pmf(n2, 1.7)
            Fb = n1 * f[0, 0] + n2 * f[0, 1]
            Fr = n1 * f[1, 0] + n2 * f[1, 1]
            if Fb == 0:
                ix, iy = 0, g["ny"] - 1            # +inf - +inf = NaN colour, +inf magnitude
            else:
                mb = np.float64(np.float32(-2.5 * math.log10(Fb)))
                mr = np.float64(np.float32(-2.5 * math.log10(Fr)))
                ix = min(max(math.floor((mb - mr + 0.2) / 0.05), 0), g["nx"] - 1)
                iy = min(max(math.floor((mr + 4.0) / 0.05), 0), g["ny"] - 1)
            expect[iy, ix] += p
    expect *= Hm.sum()
    keep = expect > 5
    obs_k, exp_k = Hm[keep].astype(np.float64), expect[keep]
    chi2 = ((obs_k - exp_k) ** 2 / exp_k).sum()
    assert stats.chi2.sf(chi2, keep.sum() - 1) > 1e-4
    assert Hm[~keep].sum() < 5 * max(expect[~keep].sum(), 1.0)


# ---------------- likelihood -----------------

def test_poisson_loglike_hand_2x2():
    hm = np.array([[3, 0], [1, 4]]); hd = np.array([[2, 1], [0, 5]])
    eps = 0.01
    lamh = 8 * (np.array([3, 0, 1, 4]) + eps) / (8 + 4 * eps)
    assert lamh.sum() == pytest.approx(8.0, rel=1e-15)
    d = np.array([2, 1, 0, 5])
    # by hand: sum d ln lam - lam - ln d!
    ref = sum(d[j] * math.log(lamh[j]) - lamh[j] - math.log(math.factorial(d[j])) for j in range(4))
    got = L.loglike(hm, hd, [0, 0, 8], [0, 0, 8], L.POISSON, eps)
    assert got == pytest.approx(ref, rel=1e-13)
    assert got == pytest.approx(float(stats.poisson.logpmf(d, lamh).sum()), rel=1e-12)


def test_gaussian_loglike_identical_hess_is_mean_term():
    r = np.random.default_rng(3)
    h = r.poisson(20, size=(10, 10))
    mom_d = np.array([30.0, 2000.0, 100.0]); mom_m = np.array([31.0, 2003.0, 100.0])
    got = L.loglike(h, h, mom_m, mom_d, L.GAUSS_PAPER)
    assert got == pytest.approx(L.mean_term(mom_m, mom_d), rel=1e-14)
    assert L.mean_term(mom_m, mom_d) == pytest.approx(-(0.01 ** 2 + 0.03 ** 2) / (2 * 0.05 ** 2), rel=1e-10)
    assert L.loglike(h, h, mom_d, mom_d, L.GAUSS_PAPER) == 0.0
    assert L.loglike(h, h, mom_d, mom_d, L.GAUSS_LITERAL) == 0.0
    # floor of 2 on sigma: a single-count difference costs 1/8
    h2 = h.copy(); d2 = h.copy(); h2[:] = 0; d2[:] = 0; h2[0, 0] = 1; d2[0, 1] = 1
    assert L.loglike(h2, d2, mom_d, mom_d, L.GAUSS_PAPER) == pytest.approx(-2 * (1.0 / 8.0), rel=1e-14)


def test_gaussian_loglikes_hand_worked_above_the_floor():
    """Both Gaussian forms on a hand-worked 2 x 2 example whose bins all sit above the floor of 2,
    with model and data totals that differ (tests/golden/gauss_loglike_2x2_example.txt)."""
    from fractions import Fraction as Fr
    vals = {}
    for line in open(os.path.join(GOLD, "gauss_loglike_2x2_example.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        vals[t[0]] = t[1:]
    d = np.array([int(v) for v in vals["d"]])
    m = np.array([int(v) for v in vals["m"]])
    mom_d = np.array([float(v) for v in vals["mom_d"]])
    mom_m = np.array([float(v) for v in vals["mom_m"]])
    paper = float(Fr(vals["paper"][0]))
    literal = float(-sum(Fr(v) for v in vals["literal_terms"]) + Fr(vals["mean_term"][0]))
    assert L.mean_term(mom_m, mom_d) == pytest.approx(float(Fr(vals["mean_term"][0])), rel=1e-12)
    assert L.loglike(m, d, mom_m, mom_d, L.GAUSS_PAPER) == pytest.approx(paper, rel=1e-13)
    assert L.loglike(m, d, mom_m, mom_d, L.GAUSS_LITERAL) == pytest.approx(literal, rel=1e-13)
    # the Hess part of the printed form is tiny next to the mean term: its units clash
    assert abs(literal - float(Fr(vals["mean_term"][0]))) < 2e-5


def test_poisson_loglike_scatter_shrinks_with_image_size():
    # Appendix A: larger simulated images give less stochastic likelihoods
    g, m, _ = si.small_case()
    lam, _, f32 = E.build_entries(m, g)
    psf = si.psf_stack(3, (0.8, 0.8))
    od = si.Obs(nim=64, seed=2, dmod=25.0, psf=psf, noise_model=1, noise_sigma_mag=(0.02, 0.02))
    dm = P.simulate(lam, f32, od)["mags"]
    hg = si.hess_grid_from_median(np.median(dm[0] - dm[1]), np.median(dm[1]), 60, 60)
    Hd, md = H.hess(dm, hg)
    spread = {}
    for nim in (16, 48):
        vals = []
        for s in range(6):
            o = si.Obs(nim=nim, seed=100 + s, dmod=25.0, psf=psf, noise_model=1, noise_sigma_mag=(0.02, 0.02))
            Hm, mm = H.hess(P.simulate(lam, f32, o)["mags"], hg)
            vals.append(L.loglike(Hm, Hd, mm, md, L.POISSON))
        spread[nim] = np.std(vals)
    assert spread[48] < spread[16]


def test_multi_cmd_loglike_is_the_sum_over_diagrams():
    """The joint likelihood of several colour-magnitude diagrams: one diagram reproduces the single
    likelihood, the order of the diagrams does not matter, and a diagram whose data and model Hess
    are both the full pixel count in one bin adds exactly the Poisson term of that bin."""
    import math
    from oracle import hess as oh, loglike as ol
    from oracle import pipeline as op
    r = np.random.default_rng(3)
    mags = np.stack([r.normal(25.0, 1.0, 500), r.normal(24.5, 1.0, 500), r.normal(24.0, 1.0, 500)])
    g1 = dict(x0=-3.0, dx=0.1, nx=60, y0=21.0, dy=0.1, ny=70)
    g2 = dict(x0=-3.0, dx=0.2, nx=30, y0=20.0, dy=0.2, ny=40)
    data = np.stack([r.normal(25.1, 1.0, 500), r.normal(24.5, 1.0, 500), r.normal(24.0, 1.0, 500)])
    c1 = ((0, 1, 1), g1, *oh.hess(data, g1, 0, 1, 1))
    c2 = ((1, 2, 2), g2, *oh.hess(data, g2, 1, 2, 2))
    H1, m1 = oh.hess(mags, g1, 0, 1, 1)
    assert op.loglike_multi_cmd(mags, [c1]) == ol.loglike(H1, c1[2], m1, c1[3])
    a = op.loglike_multi_cmd(mags, [c1, c2])
    b = op.loglike_multi_cmd(mags, [c2, c1])
    assert a == pytest.approx(b, rel=1e-14)
    # a one-bin diagram: d = m = 500 in the single bin, lambda = 500, term 500 ln 500 - 500 - ln 500!
    g0 = dict(x0=-100.0, dx=200.0, nx=1, y0=-100.0, dy=200.0, ny=1)
    c0 = ((0, 1, 1), g0, *oh.hess(data, g0, 0, 1, 1))
    one = op.loglike_multi_cmd(mags, [c1, c0]) - op.loglike_multi_cmd(mags, [c1])
    assert one == pytest.approx(500 * math.log(500.0) - 500.0 - math.lgamma(501.0), rel=1e-12)


def test_subpixel_grid_reduces_to_single_psf_and_shifts():
    """The 4 x 4 sub-pixel PSF grid (Sec. 2.2): sixteen copies of one PSF give the single-PSF
    convolution; integer-shifted delta PSFs move each region's pixels by their own shift (exact);
    region boundaries follow floor(4 y / N) also when N is not a multiple of 4."""
    from oracle import psf as P
    r = np.random.default_rng(5)
    for N in (16, 18):
        F = r.uniform(0.0, 1.0, (2, N, N))
        one = si.psf_stack(5, (1.0, 1.5))
        grid = np.repeat(one[:, None], 16, axis=1)
        assert np.array_equal(P.convolve_periodic_subpixel(F, grid), P.convolve_periodic(F, one))
        # delta PSF of region r displaced by (sy, sx) = (r // 4 - 1, r % 4 - 2) pixels
        K, h = 7, 3
        deltas = np.zeros((2, 16, K, K), np.float32)
        for reg in range(16):
            deltas[:, reg, h + reg // 4 - 1, h + reg % 4 - 2] = 1.0
        G = P.convolve_periodic_subpixel(F, deltas)
        reg_of = P.region_of(N, 4)
        for y in range(N):
            for x in range(N):
                rr = reg_of[y, x]
                sy, sx = rr // 4 - 1, rr % 4 - 2
                assert np.array_equal(G[:, y, x], F[:, (y - sy) % N, (x - sx) % N])
        assert reg_of[0, 0] == 0 and reg_of[N - 1, N - 1] == 15
        assert reg_of[(N + 3) // 4, 0] == 4 and reg_of[(N + 3) // 4 - 1, 0] == 0
