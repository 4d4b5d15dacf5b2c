"""Stochastic-likelihood tooling (Appendix A): the ceiling, capping, nested-sampling weights and
the remaining-evidence criterion on hand-worked cases (CPU), and the batched re-simulations
against the oracle (GPU)."""
import dataclasses
import math

import numpy as np
import pytest

import synth_inputs as si
from oracle import hess as oh
from oracle import loglike as ol
from oracle import pipeline as op
from tests import parity_utils as pu


@pytest.fixture(scope="module")
def built_lib():
    """The Appendix A helpers are host code in the C library; build it when it is missing."""
    import os
    from paper_1904_00011_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.load()


def test_ceiling_cap_and_weights_hand_worked(built_lib):
    from paper_1904_00011_amd import stochastic as st
    assert st.lmax_ceiling([3.0, 1.0, 2.0, 10.0]) == 2.5
    assert np.array_equal(st.cap_loglikes([1.0, 5.0, 2.5], 2.5), [1.0, 2.5, 2.5])
    # dead points with equal prior widths: weights proportional to L
    logl = np.log([1.0, 2.0, 3.0, 4.0])
    w = st.nested_weights(logl, np.zeros(4))
    assert np.allclose(w, [0.1, 0.2, 0.3, 0.4], rtol=1e-14)
    assert st.effective_sample_size(np.full(8, 1 / 8)) == pytest.approx(8.0)
    # remaining evidence: Z = sum L dX = 10 (dX = 1), remaining L_live X = 10 -> ln 2
    assert st.remaining_evidence(logl, np.zeros(4), 0.0, math.log(10.0)) == pytest.approx(math.log(2.0), rel=1e-14)


def test_helpers_against_library_routines_and_edge_cases(built_lib):
    """The C helpers against numpy's median and scipy's log-sum-exp on random inputs, dead points
    with zero likelihood (-inf), and the rejected inputs (NaN, empty, no finite mass)."""
    from scipy.special import logsumexp
    from paper_1904_00011_amd import _lib
    from paper_1904_00011_amd import stochastic as st
    rng = np.random.default_rng(7)
    for n in (1, 2, 5, 64, 1001):
        v = rng.normal(-5e4, 3e3, n)
        assert st.lmax_ceiling(v) == np.median(v)
        d = np.log(rng.uniform(1e-6, 1.0, n))
        w = st.nested_weights(v, d)
        np.testing.assert_allclose(w, np.exp(v + d - logsumexp(v + d)), rtol=1e-11, atol=1e-300)
        assert w.sum() == pytest.approx(1.0, rel=1e-14)
        lz = logsumexp(v + d)
        r = v.max() - 3.0
        assert st.remaining_evidence(v, d, -1.0, r) == pytest.approx(np.logaddexp(lz, r - 1.0) - lz, rel=1e-12, abs=1e-15)
        assert st.effective_sample_size(w) == pytest.approx(1.0 / np.sum(w * w), rel=1e-13)
    # a dead point of zero likelihood takes zero weight; a live set of zero likelihood adds nothing
    w = st.nested_weights([-np.inf, 0.0, 0.0], np.zeros(3))
    assert np.array_equal(w, [0.0, 0.5, 0.5])
    assert st.remaining_evidence([0.0, 0.0], np.zeros(2), 0.0, -np.inf) == 0.0
    assert np.array_equal(st.cap_loglikes([-np.inf, 3.0], 1.0), [-np.inf, 1.0])
    assert st.cap_loglikes([], 1.0).size == 0
    for bad in (lambda: st.lmax_ceiling([]), lambda: st.lmax_ceiling([1.0, np.nan]),
                lambda: st.nested_weights([-np.inf, -np.inf], np.zeros(2)),
                lambda: st.nested_weights([np.inf, 0.0], np.zeros(2)),
                lambda: st.nested_weights([-np.inf, 0.0], [np.inf, 0.0]),
                lambda: st.remaining_evidence([0.0, 1.0], [0.0, np.inf], 0.0, 0.0),
                lambda: st.remaining_evidence([0.0], [0.0], np.nan, 0.0),
                lambda: st.cap_loglikes([0.0], np.nan), lambda: st.effective_sample_size([0.0, 0.0])):
        with pytest.raises(_lib.PcmdError):
            bad()


def test_cap_spreads_the_weight_of_a_positive_fluctuation(built_lib):
    """The paper's failure mode: the last dead point is a positive fluctuation 20 log-units above
    the rest and takes almost all the weight; capping at the ceiling spreads the weight again and
    shrinks the remaining-evidence criterion."""
    from paper_1904_00011_amd import stochastic as st
    n_live = 50
    i = np.arange(400)
    log_x = -(i + 1) / n_live
    log_dx = log_x + math.log(math.expm1(1.0 / n_live))  # X_{i-1} - X_i
    logl = -0.5 * np.exp(2 * log_x) * 1e3                   # rises to a plateau near 0
    logl[-1] = 20.0                                          # one extreme positive fluctuation
    w = st.nested_weights(logl, log_dx)
    assert w[-1] > 0.99
    capped = st.cap_loglikes(logl, 0.0)
    wc = st.nested_weights(capped, log_dx)
    assert wc[-1] < 0.05 and st.effective_sample_size(wc) > 20 * st.effective_sample_size(w)
    assert st.remaining_evidence(capped, log_dx, log_x[-1], 0.0) < st.remaining_evidence(logl, log_dx, log_x[-1], 20.0)


@pytest.mark.gpu
def test_resimulations_match_the_oracle():
    """Twelve re-simulations of the small case (one batched, graph-replayed launch) against the
    oracle's own simulations with the same seeds: the Hess diagrams agree except for pixels within
    1e-4 mag of a bin edge, and wherever they agree the log-likelihoods agree to 1e-3."""
    import torch
    import paper_1904_00011_amd as P
    from paper_1904_00011_amd import stochastic as st
    ctx = P.Context(0)
    try:
        grid, model, obs = si.small_case()
        dev = torch.device("cuda")
        od = dataclasses.replace(obs, seed=99)
        data = op.simulate(*op.entries.build_entries(model, grid)[::2], od)["mags64"]
        x, y = np.median(data[0] - data[1]), np.median(data[1])
        hgrid = si.hess_grid_from_median(x, y, 100, 100)
        hd, md = oh.hess(data, hgrid)
        ev = P.Evaluator(ctx, grid, obs.nim, obs.psf, hgrid)
        hd_d = torch.from_numpy(hd.ravel().astype(np.int32)).to(dev)
        md_d = torch.from_numpy(md).to(dev)
        n = 12
        hs = torch.empty((n, 100 * 100), dtype=torch.int32, device=dev)
        ll = st.resimulate_loglikes(ctx, ev, model, obs, hd_d, md_d, n, seed0=500, hess_out=hs)
        ctx.sync()
        lam, _, f32 = op.entries.build_entries(model, grid)
        agree = 0
        for k in range(n):
            ok_k = dataclasses.replace(obs, seed=500 + k)
            ok = op.simulate(lam, f32, ok_k)["mags64"]
            ho, mo = oh.hess(ok, hgrid)
            hg = hs[k].cpu().numpy().reshape(100, 100).astype(np.int64)
            # the batched re-simulation's Hess is that of the single-call image, whose pixels are
            # checked against the oracle's one by one
            g = pu.gpu_simulate(ctx, lam, f32, ok_k, want_flux=False)
            assert np.array_equal(hg, oh.hess(g["mags"], hgrid)[0]), k
            _, _, moved = pu.assert_hess_per_pixel(g["mags"], ok, hgrid, what=f"Hess of re-simulation {k}")
            if moved == 0:
                assert np.array_equal(hg, ho), k
                agree += 1
                assert abs(ll[k] - ol.loglike(ho, hd, mo, md)) <= pu.LOGL_ATOL, k
            else:   # a pixel on a bin edge moved: the likelihood is still that of the GPU's own Hess
                hm_g, mm_g = oh.hess(g["mags"], hgrid)
                assert abs(ll[k] - ol.loglike(hm_g, hd, mm_g, md)) <= pu.LOGL_ATOL, k
        print(f"[case] resimulations: {agree}/{n} with identical Hess; L_max = {st.lmax_ceiling(ll):.2f}", flush=True)
        assert agree >= n // 2
    finally:
        ctx.close()
