"""Oracle a1/a2 pins: Poisson rules against the Poisson law, the dust split by
enumeration, and the flux moments, distance and dust invariants of Sec. 2."""
import math

import numpy as np
import pytest
from scipy import stats

import synth_inputs as si
from oracle import entries as E
from oracle import rng, sampler as S


@pytest.mark.parametrize("lam", [0.0, 1e-6, 3e-3, 0.2, 1.0, 3.7, 9.99])
def test_inversion_thresholds_match_poisson_cdf(lam):
    T = S.inversion_thresholds(lam)
    cdf = stats.poisson.cdf(np.arange(len(T)), lam) if len(T) else np.array([])
    for k, t in enumerate(T):
        # T_k / 2^32 is the cdf to within 2^-32 (floor) plus FP64 summation error
        assert abs(t / 2 ** 32 - cdf[k]) <= 2 ** -32 + 1e-14
        assert t < 2 ** 32 - 1
    # past the table, less than 2^-31 of the Poisson mass is left: outcome K takes it
    assert stats.poisson.sf(len(T), lam) < 2 ** -31


def _table_moments(T):
    """Exact mean and second moment of the count that the inversion table T gives over all 2^32
    words: outcome k (k < K) takes the words [T_{k-1}, T_k), outcome K the words [T_{K-1}, 2^32)."""
    edges = [0] + list(T) + [2 ** 32]
    mass = np.array([edges[k + 1] - edges[k] for k in range(len(T) + 1)], dtype=np.float64)
    k = np.arange(len(T) + 1, dtype=np.float64)
    return float((mass * k).sum() / 2.0 ** 32), float((mass * k * k).sum() / 2.0 ** 32)


def test_inversion_table_moments_by_enumeration():
    """The count an inversion table gives has, over all 2^32 words, mean lambda and variance
    lambda (the Poisson law) to its 2^-32 quantisation, and the table never runs past the support
    of the law: the count of the largest word is one the Poisson law reaches with probability at
    least 2^-33.  A table that ran on to the 63 cap when the FP64 cdf stalls just below 1 (so that
    word 2^32 - 1 drew 63 stars) fails both: it adds 63^2 2^-32 to the second moment, which for the
    faintest-weight, brightest points is many times lambda itself."""
    rs = np.random.default_rng(7)
    lams = np.concatenate([10.0 ** rs.uniform(-10, -6, 2000), 10.0 ** rs.uniform(-6, 0, 2000),
                           rs.uniform(1.0, 2.0, 1000), rs.uniform(2.0, 10.0, 500),
                           [2.0 ** -32 * 1.01, 2.0 ** -32 * 0.99, 1e-10, 3e-10, 1.999999]])
    q = 2.0 ** -32
    for lam in lams:
        lam = float(lam)
        T = S.inversion_thresholds(lam)
        K = len(T)
        # support: the largest count drawn is one the law gives at least 2^-33
        assert K == 0 or stats.poisson.sf(K - 1, lam) >= q / 2, (lam, K)
        m1, m2 = _table_moments(T)
        # each threshold is the cdf floored to 2^-32 (plus FP64 rounding): the moments move by at
        # most (K + 1) 2^-32 and (K + 1)^2 2^-32, plus the law's mass above K (< 2^-31)
        tail = stats.poisson.sf(K, lam)
        tail_m1 = sum(stats.poisson.sf(j, lam) for j in range(K, K + 40))
        tail_m2 = sum((2 * j + 1) * stats.poisson.sf(j, lam) for j in range(K, K + 40))
        assert abs(m1 - lam) <= (K + 1) * q + tail_m1 + 1e-15, (lam, K, m1)
        assert abs((m2 - m1 * m1) - lam) <= (K + 1) ** 2 * q + tail_m2 + 1e-14, (lam, K, m2 - m1 * m1)
        assert tail < 2 ** -31
    # the floor: below lambda ~ 2^-32 the table is empty and no star is ever drawn
    assert S.inversion_thresholds(1e-10) == []
    assert len(S.inversion_thresholds(3e-10)) == 1


@pytest.mark.parametrize("lam", [0.05, 0.9, 6.0])
def test_inversion_counts_on_stratified_words(lam):
    # 65536 equally spaced words: P(n <= k) is hit to within 2^-16
    u = (np.arange(65536, dtype=np.uint64) << np.uint64(16)) + np.uint64(12345)
    n = S.count_from_thresholds(u, S.inversion_thresholds(lam))
    emp = np.array([(n <= k).mean() for k in range(12)])
    assert np.all(np.abs(emp - stats.poisson.cdf(np.arange(12), lam)) <= 2 ** -16 + 1e-12)


@pytest.mark.parametrize("lam", [2.0, 3.3, 10.0, 10.5, 37.3, 100.0, 255.5, 511.9])
def test_alias_masses_match_poisson_pmf(lam):
    """C1b: the cumulative outcome masses are the Poisson cdf times 2^32 to within the floor (and
    the FP64 recurrence), the support is the cdf's, and the masses sum to 2^32."""
    k_lo, m = S.alias_masses(lam)
    m = np.array(m, dtype=np.int64)
    assert m.sum() == 2 ** 32 and (m >= 0).all() and m[0] > 0
    cum = np.cumsum(m)[:-1].astype(np.float64)
    cdf = stats.poisson.cdf(k_lo + np.arange(len(cum)), lam) * 2.0 ** 32
    assert np.max(np.abs(cum - cdf)) <= 1.0 + 2.0 ** 32 * 1e-12
    # below k_lo the cdf is under 2^-32; above the last outcome less than 2^-31 is left
    assert k_lo == 0 or stats.poisson.cdf(k_lo - 1, lam) < 2.0 ** -32
    assert stats.poisson.sf(k_lo + len(m) - 1, lam) < 2.0 ** -31
    assert S.alias_columns(len(m)) <= S.ALIAS_MAX_COLS


@pytest.mark.parametrize("lam", [2.0, 10.0, 63.0, 255.5, 511.9])
def test_alias_table_realises_the_masses_exactly(lam):
    """Summing, over the M columns, the words that select each outcome (h_c to the column,
    2^32/M - h_c to its alias) gives back every outcome mass exactly: the table draws the C1b
    law to the last of the 2^32 words."""
    k_lo, m = S.alias_masses(lam)
    k2, bits, packed = S.alias_table(lam)
    M = 1 << bits
    cap = 2 ** 32 // M
    assert k2 == k_lo and M == S.alias_columns(len(m)) and len(packed) == M
    h = (packed >> bits).astype(np.int64)
    a = (packed & (M - 1)).astype(np.int64)
    # a column whose alias is itself is full (height 2^32/M, stored as 2^32/M - 1)
    ht = np.where(a == np.arange(M), cap, h)
    got = np.zeros(M, dtype=np.int64)
    for c in range(M):
        got[c] += ht[c]
        got[a[c]] += cap - ht[c]
    want = np.zeros(M, dtype=np.int64)
    want[:len(m)] = m
    assert np.array_equal(got, want)
    # the draw, over every word of three columns (the most and least massive and a middle one),
    # selects the column exactly h_c times and its alias the rest
    for c in {int(np.argmax(want)), int(np.argmin(ht)), int(np.argmin(np.abs(ht - cap // 2)))}:
        if cap > 1 << 24:
            r = np.concatenate([np.arange(1 << 20, dtype=np.uint64), np.uint64(cap) - 1 - np.arange(1 << 20, dtype=np.uint64),
                                np.uint64(ht[c]) + np.arange(-4, 4).astype(np.uint64) if 4 <= ht[c] < cap - 4 else
                                np.zeros(0, np.uint64)])
            r = np.unique(r)
        else:
            r = np.arange(cap, dtype=np.uint64)
        u = (np.uint64(c) << np.uint64(32 - bits)) | r
        n = S.count_from_alias(u, k_lo, bits, packed)
        expect = np.where(r < np.uint64(ht[c]), k_lo + c, k_lo + a[c])
        if a[c] == c:
            expect[:] = k_lo + c
        assert np.array_equal(n, expect)


@pytest.mark.parametrize("lam", [12.0, 140.0])
def test_alias_draws_chi_square(lam):
    """Counts from the per-pixel sampler for an entry in the C1b range follow Poisson(lambda)."""
    f = np.ones((1, 1), np.float32)
    n = S.sample_pixels(np.array([lam]), f, 21, np.arange(200000), want_counts=True)["counts"][:, 0]
    lo, hi = int(lam - 4 * math.sqrt(lam)), int(lam + 4 * math.sqrt(lam))
    edges = np.arange(max(lo, 1), hi + 1)
    obs = np.array([(n < edges[0]).sum()] + [(n == k).sum() for k in edges] + [(n > edges[-1]).sum()])
    p = np.concatenate([[stats.poisson.cdf(edges[0] - 1, lam)], stats.poisson.pmf(edges, lam),
                        [stats.poisson.sf(edges[-1], lam)]])
    chi2 = ((obs - p * len(n)) ** 2 / (p * len(n))).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4
    assert abs(n.mean() - lam) < 5 * math.sqrt(lam / len(n))


def test_ln32_accuracy():
    x = np.geomspace(2.0 ** -24, 2.0 ** 24, 200001).astype(np.float32)
    got = S.ln32(x).astype(np.float64)
    ref = np.log(x.astype(np.float64))
    assert np.max(np.abs(got - ref)) < 1.5e-6
    far = np.abs(ref) > 0.01
    ulp = np.spacing(np.abs(ref[far]).astype(np.float32)).astype(np.float64)
    assert np.max(np.abs(got[far] - ref[far]) / ulp) <= 3.0


def test_lnfact32():
    k = np.arange(0, 5000, dtype=np.float32)
    got = S.lnfact32(k).astype(np.float64)
    ref = np.array([math.lgamma(v + 1.0) for v in range(5000)])
    assert np.all(np.abs(got - ref) <= 3e-7 * np.maximum(ref, 1.0))


@pytest.mark.parametrize("lam", [10.0, 30.0, 100.0, 1000.0, 1e4])
def test_ptrs_moments(lam):
    n, used = S.ptrs_draw(S.ptrs_constants(lam), 11, np.arange(300000), 3)
    N = len(n)
    assert abs(n.mean() - lam) < 5 * math.sqrt(lam / N)
    # Var of the sample variance for Poisson: (mu4 - sigma^4)/N with mu4 = lam + 3 lam^2
    sd_var = math.sqrt((lam + 3 * lam * lam - lam * lam) / N)
    assert abs(n.var() - lam) < 5 * sd_var
    assert used.max() < 64


@pytest.mark.parametrize("lam", [10.0, 27.5, 140.0])
def test_ptrs_chi_square(lam):
    n, _ = S.ptrs_draw(S.ptrs_constants(lam), 5, np.arange(400000), 9)
    lo, hi = int(lam - 4 * math.sqrt(lam)), int(lam + 4 * math.sqrt(lam))
    edges = np.arange(max(lo, 1), hi + 1)
    obs = np.array([(n < edges[0]).sum()] + [(n == k).sum() for k in edges] + [(n > edges[-1]).sum()])
    p = np.concatenate([[stats.poisson.cdf(edges[0] - 1, lam)], stats.poisson.pmf(edges, lam),
                        [stats.poisson.sf(edges[-1], lam)]])
    exp = p * len(n)
    chi2 = ((obs - exp) ** 2 / exp).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4


def test_split_half_enumeration():
    # for n <= 8 stars, over all 256 values of the entry's split byte, r ~ Binomial(n, 1/2) exactly
    W = np.arange(256, dtype=np.uint32)
    px = np.zeros(256, dtype=np.int64)
    for n in range(0, 9):
        r = S.split_reddened(np.full(256, n), W, 0.5, 1, px, 0)
        cnt = np.bincount(r, minlength=n + 1)
        expect = np.array([math.comb(n, k) * 2 ** (8 - n) for k in range(n + 1)])
        assert np.array_equal(cnt[:n + 1], expect)
    # the byte of entry i is byte i mod 16 of its 16-entry block
    px = np.arange(1000)
    for i in (0, 5, 16, 31):
        w = rng.philox4x32_10(px, i // 16, rng.TAG_SPLIT, 0, 3)[(i % 16) // 4]
        assert np.array_equal(S.split_first_byte(px, i, 3), (w >> np.uint32(8 * (i % 4))) & np.uint32(255))


def test_split_large_n_and_general_fraction():
    px = np.arange(100000)
    w = S.split_first_byte(px, 7, 3)
    for n in (12, 40, 300):
        r = S.split_reddened(np.full(len(px), n), w, 0.5, 3, px, 7)
        assert abs(r.mean() - n / 2) < 5 * math.sqrt(n / 4 / len(px))
        assert abs(r.var() - n / 4) < 5 * (n / 4) * math.sqrt(2 / len(px))
    for F in (0.3, 0.85):
        for n in (1, 9):
            r = S.split_reddened(np.full(len(px), n), w, F, 3, px, 7)
            assert abs(r.mean() - n * F) < 5 * math.sqrt(n * F * (1 - F) / len(px))
    assert np.array_equal(S.split_reddened(np.full(5, 4), w[:5], 0.0, 3, px[:5], 0), np.zeros(5))
    assert np.array_equal(S.split_reddened(np.full(5, 4), w[:5], 1.0, 3, px[:5], 0), np.full(5, 4))


def _small():
    g, m, o = si.small_case()
    lam, f64, f32 = E.build_entries(m, g)
    return lam, f32, o


def test_flux_mean_and_variance_closed_form():
    # pre-PSF pixel flux: mean sum(lam f), variance sum(lam f^2) (surface-brightness fluctuation)
    lam, f32, o = _small()
    s = S.sample_window(lam, f32, 77, 0, 40000)
    f = f32.astype(np.float64)
    for b in range(2):
        F = s["F_clr"][b]
        mu = (lam * f[b]).sum()
        var = (lam * f[b] ** 2).sum()
        mu4 = (lam * f[b] ** 4).sum() + 3 * var ** 2     # fourth central moment of a compound Poisson sum
        N = len(F)
        assert abs(F.mean() - mu) < 5 * math.sqrt(var / N)
        assert abs(F.var() - var) < 5 * math.sqrt((mu4 - var ** 2) / N)
    cov = (lam * f[0] * f[1]).sum()
    c = np.cov(s["F_clr"][0], s["F_clr"][1])[0, 1]
    assert abs(c - cov) < 0.1 * cov


def test_total_star_count_is_poisson_npix():
    lam, f32, o = _small()
    s = S.sample_window(lam, f32, 5, 0, 8000, want_counts=True)
    tot = s["counts"].sum(axis=1)
    edges = np.arange(70, 131)
    obs = np.array([(tot < 70).sum()] + [(tot == k).sum() for k in edges] + [(tot > 130).sum()])
    p = np.concatenate([[stats.poisson.cdf(69, 100)], stats.poisson.pmf(edges, 100), [stats.poisson.sf(130, 100)]])
    chi2 = ((obs - p * len(tot)) ** 2 / (p * len(tot))).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4


def test_distance_scales_flux_only_and_npix_degeneracy():
    lam, f32, o = _small()
    o1 = si.Obs(nim=32, seed=3, dmod=25.0)
    o2 = si.Obs(nim=32, seed=3, dmod=26.25)
    F1, s1 = S.simulate_flux(lam, f32, o1, want_counts=True)
    F2, s2 = S.simulate_flux(lam, f32, o2, want_counts=True)
    assert np.array_equal(s1["counts"], s2["counts"])
    assert np.allclose(F2, F1 * 10 ** (-0.4 * 1.25), rtol=1e-14, atol=0)
    # equal Npix * 10^(-0.4 mu_d) -> equal expected flux, dispersion differs by the Npix ratio
    f = f32.astype(np.float64)
    mean1 = (lam * f[1]).sum() * 10 ** (-0.4 * 25.0)
    mean2 = (10 * lam * f[1]).sum() * 10 ** (-0.4 * 27.5)
    assert mean1 == pytest.approx(mean2, rel=1e-12)
    var1 = (lam * f[1] ** 2).sum() * 10 ** (-0.8 * 25.0)
    var2 = (10 * lam * f[1] ** 2).sum() * 10 ** (-0.8 * 27.5)
    assert var2 == pytest.approx(var1 / 10, rel=1e-12)


def test_dust_invariants():
    lam, f32, o = _small()
    base = S.sample_window(lam, f32, 9, 0, 512, dust_model=0, want_counts=True)
    for F, expect_r in ((0.0, "zero"), (1.0, "all"), (0.5, None)):
        s = S.sample_window(lam, f32, 9, 0, 512, dust_model=2, dust_frac=F, want_counts=True)
        assert np.array_equal(s["counts"], base["counts"])      # counts never depend on the dust
        if expect_r == "zero":
            assert s["red"].sum() == 0
        elif expect_r == "all":
            assert np.array_equal(s["red"], s["counts"])
        else:
            assert 0 < s["red"].sum() < s["counts"].sum()
    # fixed screen (E1) with F = 1 scales every band by 10^(-0.4 R_b E)
    s = S.sample_window(lam, f32, 9, 0, 512, dust_model=1, dust_frac=1.0)
    px = np.arange(512)
    F_d = S.pixel_flux(s["F_clr"], s["F_red"], px, 9, 25.0, 1, -0.5, 0.0, (3.6, 1.9))
    F_0 = S.pixel_flux(base["F_clr"], base["F_red"], px, 9, 25.0, 0)
    E_ = 10 ** -0.5
    for b, R in enumerate((3.6, 1.9)):
        assert np.allclose(F_d[b], F_0[b] * 10 ** (-0.4 * R * E_), rtol=1e-14)


def test_lognormal_dust_draws():
    px = np.arange(100000)
    e = S.dust_ebv(px, 4, 2, -0.5, 0.2)
    le = np.log10(e)
    assert abs(le.mean() + 0.5) < 5 * 0.2 / math.sqrt(len(px))
    assert abs(le.std() - 0.2) < 0.01


@pytest.mark.parametrize("lam,frac", [(40.0, 0.3), (5.0, 0.7), (2000.0, 0.6), (700.0, 0.8), (64.0, 0.5),
                                      (3000.0, 0.5), (4.0, 0.5), (10.0, 0.5)])
def test_thinning_parts_are_independent_poisson(lam, frac):
    """C3b: for an entry at lambda >= 2 under a split 0 < F < 1 (at F = 1/2: lambda >= 4) the
    unreddened and reddened counts are independent Poisson((1 - F) lambda) and Poisson(F lambda)
    (alias parts below 512, rejection above), so the total is Poisson(lambda) and each star is
    reddened with probability F."""
    f = np.ones((1, 1), np.float32)
    N = 60000
    s = S.sample_pixels(np.array([lam]), f, 31, np.arange(N), dust_model=2, dust_frac=frac, want_counts=True)
    n, r = s["counts"][:, 0], s["red"][:, 0]
    c = n - r
    for x, mu in ((c, lam * (1 - frac)), (r, lam * frac), (n, lam)):
        assert abs(x.mean() - mu) < 5 * math.sqrt(mu / N)
        assert abs(x.var() / mu - 1) < 5 * math.sqrt((2 + 1 / mu) / N)
    assert abs(np.corrcoef(c, r)[0, 1]) < 5 / math.sqrt(N)
    lo, hi = int(lam - 4 * math.sqrt(lam)), int(lam + 4 * math.sqrt(lam))
    edges = np.arange(max(lo, 1), hi + 1)
    obs = np.array([(n < edges[0]).sum()] + [(n == k).sum() for k in edges] + [(n > edges[-1]).sum()])
    p = np.concatenate([[stats.poisson.cdf(edges[0] - 1, lam)], stats.poisson.pmf(edges, lam),
                        [stats.poisson.sf(edges[-1], lam)]])
    chi2 = ((obs - p * N) ** 2 / (p * N)).sum()
    assert stats.chi2.sf(chi2, len(obs) - 1) > 1e-4


def test_thinning_uses_its_own_words():
    """C3b draws the unreddened part from the entry's inversion word through the alias table of
    (1 - F) lambda, and the reddened part from the TAG_RED word through that of F lambda."""
    lam, frac, seed = 30.0, 0.25, 77
    px = np.arange(64)
    s = S.sample_pixels(np.array([0.0, 0.0, lam]), np.ones((1, 3), np.float32), seed, px, dust_model=1,
                        dust_frac=frac, want_counts=True)
    u = rng.philox4x32_10(px, 0, rng.TAG_MAIN, 0, seed)[2]
    v = rng.philox4x32_10(px, 0, rng.TAG_RED, 0, seed)[2]
    want_c = S.count_from_alias(u, *S.alias_table(lam * (1 - frac)))
    want_r = S.count_from_alias(v, *S.alias_table(lam * frac))
    assert np.array_equal(s["red"][:, 2], want_r)
    assert np.array_equal(s["counts"][:, 2] - s["red"][:, 2], want_c)


@pytest.mark.parametrize("lam,thinned", [(4.0, True), (3.999, False), (1500.0, True), (10.0, True), (64.0, True),
                                         (2.5, False)])
def test_half_split_thins_from_lambda_4(lam, thinned):
    """At F = 1/2 an entry at lambda >= 4 draws its two halves from its own words through the
    tables of lambda / 2 (C3b); below 4 its count is drawn whole and split one bit per star
    (C3), so the reddened count is the popcount of its split bits."""
    seed = 78
    px = np.arange(256)
    s = S.sample_pixels(np.array([0.0, 0.0, 0.0, lam]), np.ones((1, 4), np.float32), seed, px, dust_model=2,
                        dust_frac=0.5, want_counts=True)
    n, r = s["counts"][:, 3], s["red"][:, 3]
    u = rng.philox4x32_10(px, 0, rng.TAG_MAIN, 0, seed)[3]
    if thinned:
        v = rng.philox4x32_10(px, 0, rng.TAG_RED, 0, seed)[3]
        want_c = S.draw_part(lam / 2, u.astype(np.uint64), seed, px, 3, rng.TAG_PTRS)
        want_r = S.draw_part(lam / 2, v.astype(np.uint64), seed, px, 3, rng.TAG_PTRS_RED)
        assert np.array_equal(r, want_r)
        assert np.array_equal(n - r, want_c)
    else:
        assert np.array_equal(n, S.draw_part(lam, u.astype(np.uint64), seed, px, 3, rng.TAG_PTRS))
        byte = S.split_first_byte(px, 3, seed)
        want_r = S.split_reddened(n, byte, 0.5, seed, px, 3)
        assert np.array_equal(r, want_r)
