"""The process-parallel oracle driver joins the oracle's own per-slab and per-band results: the
same fluxes, images and count digests as the sequential oracle, and a digest that sees any single
changed count."""
import numpy as np

import synth_inputs as si
from oracle import entries as oe
from oracle import parallel as opar
from oracle import pipeline as op


def test_parallel_oracle_equals_sequential():
    G, = (si.headline_grid().subsample(25),)
    model, obs = si.draw_headline_params(1001, log_npix=4.0)
    lam, _, f32 = oe.build_entries(model, G)
    obs.nim = 24
    obs.psf = si.psf_stack(5, (1.0, 1.2, 1.4))
    seq = op.simulate(lam, f32, obs, want_counts=True)
    par = opar.simulate(lam, f32, obs, with_digest=True, workers=3)
    np.testing.assert_allclose(par["F"], seq["F"], rtol=1e-13, atol=0)
    np.testing.assert_allclose(par["G"], seq["G"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(par["mags64"], seq["mags64"], rtol=0, atol=1e-10)
    mult = opar.digest_multipliers(len(lam))
    assert np.array_equal(par["digest_counts"], opar.count_digest(seq["counts"], mult))
    assert np.array_equal(par["digest_red"], opar.count_digest(seq["red"], mult))
    # windows come back in window order
    F, dc, _ = opar.simulate_flux(lam, f32, obs, [(500, 530), (3, 10)], with_digest=True, workers=2, slab=7)
    np.testing.assert_allclose(F[:, :30], seq["F"][:, 500:530], rtol=1e-13)
    np.testing.assert_allclose(F[:, 30:], seq["F"][:, 3:10], rtol=1e-13)
    assert np.array_equal(dc[30:], opar.count_digest(seq["counts"][3:10], mult))


def test_count_digest_sees_every_single_change():
    r = np.random.default_rng(1)
    E = 5000
    mult = opar.digest_multipliers(E)
    assert np.all(mult & np.uint64(1) == 1)
    c = r.poisson(0.3, (40, E))
    d0 = opar.count_digest(c, mult)
    for k in range(200):
        c2 = c.copy()
        p, i = r.integers(0, 40), r.integers(0, E)
        c2[p, i] += int(r.choice([-1, 1, 2, 63, 2 ** 31 - 1]))
        d1 = opar.count_digest(c2, mult)
        assert d1[p] != d0[p]
        assert np.array_equal(np.delete(d1, p), np.delete(d0, p))
