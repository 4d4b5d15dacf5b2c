"""The device builds each alias table from prefix sums instead of walking Vose's two stacks one
pop at a time (k_prep_alias).  This checks, on the CPU, that the prefix-sum form of the loop gives
the oracle's table word for word.  The form, for smalls s_1, s_2, ... and larges l_1, l_2, ... in
pop order (highest column first), with D(i) the deficits cap - m of the first i smalls and E(j) the
excesses m - cap of the first j larges (all exact integers): s_i takes alias l_j for the first j
with E(j) >= D(i - 1); l_j turns small after the first a with D(a) > E(j), keeping height
cap + E(j) - D(a) and alias l_{j+1}; a large that never turns small is full (height cap, alias
itself).  The GPU tables themselves are compared with the oracle's counts in the parity tests."""
import numpy as np
import pytest

from oracle import sampler as S


def _prefix_form_table(lam: float):
    k_lo, m = S.alias_masses(lam)
    M = S.alias_columns(len(m))
    bits = M.bit_length() - 1
    cap = (1 << 32) // M
    w = list(m) + [0] * (M - len(m))
    smalls = [j for j in range(M) if w[j] < cap][::-1]
    larges = [j for j in range(M) if w[j] >= cap][::-1]
    D = np.cumsum([0] + [cap - w[s] for s in smalls]).astype(np.int64)
    E = np.cumsum([w[l] - cap for l in larges]).astype(np.int64)
    assert D[-1] < 2**32 and (len(E) == 0 or E[-1] < 2**32), "prefix sums fit 32 bits"
    h = [0] * M
    a = [0] * M
    for l in larges:
        h[l], a[l] = cap, l
    for i, s in enumerate(smalls):          # pop index i: needs D(i) = D[i]
        j = int(np.searchsorted(E, D[i], side="left"))
        h[s], a[s] = w[s], larges[j]
    for j, l in enumerate(larges):
        k = int(np.searchsorted(D[1:], E[j], side="right")) + 1   # first k >= 1 with D[k] > E[j]
        if k <= len(smalls) and j + 1 < len(larges):
            h[l], a[l] = cap + int(E[j]) - int(D[k]), larges[j + 1]
    packed = np.array([(min(h[c], cap - 1) << bits) | a[c] for c in range(M)], dtype=np.uint32)
    return k_lo, bits, packed


def _lams():
    rng = np.random.default_rng(1904)
    return np.concatenate([np.linspace(2.0, 512.0, 300, endpoint=False),
                           np.exp(rng.uniform(np.log(2.0), np.log(512.0), 1700)),
                           [2.0, np.nextafter(2.0, 3.0), 31.999, 32.0, 63.999, 64.0, 511.999]])


def test_prefix_form_equals_the_stack_loop():
    for lam in _lams():
        k0, b0, p0 = S.alias_table(lam)
        k1, b1, p1 = _prefix_form_table(lam)
        assert (k0, b0) == (k1, b1), lam
        assert np.array_equal(p0, p1), lam


@pytest.mark.parametrize("lam", [3.0e-9, 0.25])
def test_prefix_form_small_parts(lam):
    # thinned parts can be far below 2 (a part of lambda F); the construction is the same
    k0, b0, p0 = S.alias_table(lam)
    k1, b1, p1 = _prefix_form_table(lam)
    assert (k0, b0) == (k1, b1)
    assert np.array_equal(p0, p1)
