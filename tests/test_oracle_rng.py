"""Oracle RNG pins: published Philox4x32-10 known answers and uniformity."""
import os

import numpy as np
from scipy import stats

from oracle import rng

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def load_kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([int(v, 16) for v in line.split()])
    return rows


def test_philox_known_answers():
    rows = load_kat()
    assert len(rows) == 3
    for r in rows:
        key = r[4] | (r[5] << 32)
        out = rng.philox4x32_10(r[0], r[1], r[2], r[3], key)
        assert [int(v) for v in out] == r[6:10]


def test_philox_vectorised_matches_scalar():
    px = np.arange(1000)
    out = rng.philox4x32_10(px, 7, rng.TAG_MAIN, 0, 12345)
    for p in (0, 1, 517, 999):
        s = rng.philox4x32_10(p, 7, rng.TAG_MAIN, 0, 12345)
        assert [int(o[p]) for o in out] == [int(v) for v in s]


def test_uniformity_and_stream_separation():
    px = np.arange(200000)
    a = rng.philox4x32_10(px, 0, rng.TAG_MAIN, 0, 99)
    b = rng.philox4x32_10(px, 0, rng.TAG_SPLIT, 0, 99)
    for w in a + b:
        top = (w >> np.uint32(24)).astype(np.int64)
        counts = np.bincount(top, minlength=256)
        chi2 = ((counts - len(px) / 256) ** 2 / (len(px) / 256)).sum()
        assert stats.chi2.sf(chi2, 255) > 1e-4
    assert not np.array_equal(a[0], b[0])
    u = rng.u01_open_f64(a[0])
    assert u.min() > 0 and u.max() < 1
    u32 = rng.u01_open_f32(a[1])
    assert u32.min() > 0 and u32.max() < 1 and u32.dtype == np.float32
    z = rng.box_muller_f64(a[2], a[3])
    assert abs(z.mean()) < 5 / np.sqrt(len(z)) and abs(z.var() - 1) < 5 * np.sqrt(2 / len(z))
