"""Pins of the oracle's random-number layer against what is fixed outside it.

* Philox4x32-10: the known-answer vectors published with the generator
  (Salmon et al., SC'11, distributed as Random123's kat_vectors).
* Integer maps: preimage boundaries of the multiply-shift range map, the
  integer crossover threshold against the real inequality u < CR.
* Donors: exhaustive enumeration of every index input for NP in {4, 5, 6};
  the map must be a bijection onto ordered distinct triples excluding i.
* Statistics: chi-square of raw words, KS of the Box-Muller normals.
"""
import itertools

import os

import numpy as np
import pytest
from scipy import stats

import oracle as O

def _load_kat():
    """(counter, key, expected output) rows of tests/golden/philox4x32_10_kat.txt."""
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = []
    with open(path) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(t, 16) for t in line.split()]
            rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


KAT = _load_kat()


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    assert [int(v) for v in O.philox(ctr, key)] == want


def test_philox_words_uniform():
    # chi-square of the top byte over 2^14 counters x 4 words
    words = np.concatenate([O.philox([t, 7, 3 << 24, 0], [11, 250517430]) for t in range(1 << 14)])
    counts = np.bincount(words >> 24, minlength=256)
    chi2 = ((counts - counts.mean()) ** 2 / counts.mean()).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4


def test_u24_u53_exact_and_in_range():
    assert O.u24(0) == 0.0
    assert O.u24(0xFFFFFFFF) == (2**24 - 1) / 2**24
    assert O.u24(0x00000100) == 2.0**-24
    assert O.u53(0, 0) == 0.0
    assert O.u53(0xFFFFFFFF, 0xFFFFFFFF) == (2**53 - 1) / 2**53
    # the 53 bits are (a >> 5) high and (b >> 6) low
    assert O.u53(1 << 5, 0) == 2.0**-27
    assert O.u53(0, 1 << 6) == 2.0**-53
    # u24 values are exact in float32
    for w in (0x12345678, 0xDEADBEEF, 0x80000000):
        u = O.u24(w)
        assert float(np.float32(u)) == u


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 10, 50, 179, 199, 1000, 2**31 + 11])
def test_range_preimage_boundaries(n):
    # value k is produced exactly by words in [ceil(k 2^32/n), ceil((k+1) 2^32/n))
    for k in sorted({k for k in (0, 1, n // 2, n - 1) if 0 <= k < n}):
        lo = -(-(k << 32) // n)
        assert O.rng_range(lo, n) == k
        if lo > 0:
            assert O.rng_range(lo - 1, n) == k - 1
    assert O.rng_range(0, n) == 0
    assert O.rng_range(0xFFFFFFFF, n) == n - 1


@pytest.mark.parametrize("cr", [0.0, 1e-9, 0.1, 0.5, 0.9, 0.9999999, 1.0])
def test_cr_threshold_matches_real_inequality(cr):
    t = O.cr_threshold(cr)
    # u = m 2^-24 < CR  <=>  m < t  for every integer m in [0, 2^24)
    if t > 0:
        assert (t - 1) / 2**24 < cr
    if t < 2**24:
        assert t / 2**24 >= cr
    if cr == 0.9:
        assert t == 15099495           # 0.9 * 2^24 = 15099494.4
    if cr == 1.0:
        assert t == 2**24


def _word_for(k, n):
    """Smallest 32-bit word whose range(., n) equals k."""
    return -(-(k << 32) // n)


@pytest.mark.parametrize("np_", [4, 5, 6])
def test_donors_exhaustive_bijection(np_):
    dim = 3
    for i in range(np_):
        seen = set()
        for a, b, c in itertools.product(range(np_ - 1), range(np_ - 2), range(np_ - 3)):
            w = [_word_for(a, np_ - 1), _word_for(b, np_ - 2), _word_for(c, np_ - 3),
                 _word_for(dim - 1, dim)]
            r1, r2, r3, jr = (int(v) for v in O.donors_from_words(np_, dim, i, w))
            assert len({i, r1, r2, r3}) == 4
            assert all(0 <= r < np_ for r in (r1, r2, r3))
            assert jr == dim - 1
            seen.add((r1, r2, r3))
        # every ordered distinct triple excluding i appears exactly once
        want = {t for t in itertools.permutations([k for k in range(np_) if k != i], 3)}
        assert seen == want


def test_donors_from_stream_are_distinct():
    for np_ in (4, 7, 50, 180):
        for t in range(1, 4):
            for i in range(np_):
                r1, r2, r3, jr = O.de_donors(np_, 10, i, 3, 250517430, t)
                assert len({i, int(r1), int(r2), int(r3)}) == 4
                assert 0 <= jr < 10


def test_box_muller_normals():
    _, _, G = O.instance(O.RASTRIGIN, 100, 0, 250517431, return_gaussian=True)
    g = G.ravel()
    assert stats.kstest(g, "norm").pvalue > 1e-3
    assert abs(g.mean()) < 0.05 and abs(g.var() - 1.0) < 0.05


def test_shift_uniform_on_box():
    o, _ = O.instance(O.ELLIPSOID, 400, 3, 250517431)
    assert o.min() >= -80 and o.max() < 80
    assert stats.kstest((o + 80) / 160, "uniform").pvalue > 1e-3
