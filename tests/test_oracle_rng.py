"""Pins for the reference's counter-based generator and distributions.

The generator is pinned to the published Philox4x32-10 known-answer vectors
(``golden/philox4x32_10_kat.txt``, from the Random123 distribution), to an
independent second implementation (``philox_ref``) agreeing bit for bit on
10^6 calls, and by distributional checks of the uniforms and of every derived
distribution (moments and Kolmogorov-Smirnov against scipy's exact CDFs).
"""
import os

import numpy as np
import pytest
from scipy import stats

import philox_ref as PR

KAT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    """(counter, key, output) word lists of the published known-answer rows."""
    rows = []
    for line in open(KAT):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        w = [int(x, 16) for x in line]
        assert len(w) == 10
        rows.append((w[0:4], w[4:6], w[6:10]))
    assert len(rows) == 3
    return rows


@pytest.mark.parametrize("row", range(3))
def test_philox_known_answers(orc, row):
    ctr, key, want = kat_rows()[row]
    assert orc.philox(ctr, key) == want
    assert PR.philox_int(ctr, key) == want


def kat_as_uniform_call(ctr, key):
    """The known-answer row as the generator's uniform call: counter
    (i, slot | attempt << 8, lo32(id), hi32(id)), key (lo32(seed), hi32(seed));
    returns (seed, id, i, slot, attempt) and the two uniforms
    ((w >> 12) + 1/2) 2^-52 of the output words w = o1:o0 and o3:o2."""
    seed = key[0] | (key[1] << 32)
    sid = ctr[2] | (ctr[3] << 32)
    return (seed, sid, ctr[0], ctr[1] & 0xFF, ctr[1] >> 8)


def kat_uniforms(out):
    w0 = out[0] | (out[1] << 32)
    w1 = out[2] | (out[3] << 32)
    return [((w0 >> 12) + 0.5) * 2.0 ** -52, ((w1 >> 12) + 0.5) * 2.0 ** -52]


@pytest.mark.parametrize("row", range(3))
def test_uniform_call_known_answers(orc, row):
    ctr, key, out = kat_rows()[row]
    seed, sid, i, slot, attempt = kat_as_uniform_call(ctr, key)
    got = orc.uniforms(seed, sid, i, 1, slot, attempt).ravel()
    assert list(got) == kat_uniforms(out)


def test_philox_single_calls_match_independent_implementation(orc):
    rng = np.random.default_rng(123)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**32, 4)]
        key = [int(v) for v in rng.integers(0, 2**32, 2)]
        assert orc.philox(ctr, key) == PR.philox_int(ctr, key)


def test_philox_extreme_words(orc):
    for ctr, key in [([0, 0, 0, 0], [0, 0]),
                     ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
                     ([1, 0, 0, 0], [0, 0]),
                     ([0, 0, 0, 1], [0, 1])]:
        assert orc.philox(ctr, key) == PR.philox_int(ctr, key)


def test_vectorised_reference_agrees_with_integer_reference():
    c = np.arange(50, dtype=np.uint64) * np.uint64(2654435761)
    a = PR.philox_np(c, c + np.uint64(1), c ^ np.uint64(0xABCDEF), np.uint64(7),
                     np.uint64(42), np.uint64(9))
    for j in range(50):
        want = PR.philox_int([int(c[j]), int(c[j]) + 1, int(c[j]) ^ 0xABCDEF, 7], [42, 9])
        got = [int(a[w][j]) & 0xFFFFFFFF for w in range(4)]
        assert got == want


@pytest.mark.parametrize("seed,sid,slot,attempt", [(42, 0, 0, 0), (7, 999, 8, 3),
                                                   (2**40 + 5, 2**33 + 17, 4, 15)])
def test_uniforms_bitwise_million(orc, seed, sid, slot, attempt):
    n = 1_000_000 if (seed, sid) == (42, 0) else 200_000
    got = orc.uniforms(seed, sid, 0, n, slot, attempt)
    want = PR.uniform_pairs(seed, sid, 0, n, slot, attempt)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_uniform_range_and_moments(orc):
    u = orc.uniforms(42, 0, 0, 1_000_000, 1).ravel()
    assert u.min() > 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / u.size)
    assert abs(u.var() - 1 / 12) < 5e-4
    assert stats.kstest(u, "uniform").pvalue > 1e-4
    # the two words of one call and neighbouring counters are uncorrelated
    pairs = orc.uniforms(42, 0, 0, 200_000, 2)
    assert abs(np.corrcoef(pairs[:, 0], pairs[:, 1])[0, 1]) < 0.01
    assert abs(np.corrcoef(pairs[:-1, 0], pairs[1:, 0])[0, 1]) < 0.01


def test_slots_attempts_and_scenarios_are_distinct_streams(orc):
    base = orc.uniforms(42, 0, 0, 1000, 0, 0)
    for other in (orc.uniforms(42, 0, 0, 1000, 1, 0), orc.uniforms(42, 0, 0, 1000, 0, 1),
                  orc.uniforms(42, 1, 0, 1000, 0, 0), orc.uniforms(43, 0, 0, 1000, 0, 0)):
        assert not np.any(base == other)


def _one_param(orc, dist, name="mass", n=200_000):
    from paper_2604_27193_amd import workloads as W
    d = W.single(n)
    d[name] = dist
    return orc.sample(d)[name]


def test_uniform_distribution(orc):
    x = _one_param(orc, ("uniform", 0.4, 0.9), "mu")
    assert x.min() >= 0.4 and x.max() <= 0.9
    assert stats.kstest(x, stats.uniform(loc=0.4, scale=0.5).cdf).pvalue > 1e-4


def test_normal_distribution(orc):
    x = _one_param(orc, ("normal", 1500.0, 75.0), "mass")
    assert abs(x.mean() - 1500.0) < 5 * 75.0 / np.sqrt(x.size)
    assert abs(x.std() / 75.0 - 1.0) < 0.01
    assert stats.kstest(x, stats.norm(1500.0, 75.0).cdf).pvalue > 1e-4


def test_truncated_normal_distribution(orc):
    x = _one_param(orc, ("trunc_normal", 0.2, 0.05, 0.05, 1.5), "mu")
    assert x.min() >= 0.05 and x.max() <= 1.5
    a, b = (0.05 - 0.2) / 0.05, (1.5 - 0.2) / 0.05
    assert stats.kstest(x, stats.truncnorm(a, b, loc=0.2, scale=0.05).cdf).pvalue > 1e-4
    # a normal truncated at +-5 sd is essentially never rejected; one rejection
    # changes the value, so the untruncated and truncated draws agree almost always
    v = _one_param(orc, ("trunc_normal", 25.0, 1.0, 20.0, 30.0), "v0")
    w = _one_param(orc, ("normal", 25.0, 1.0), "v0")
    inside = (w >= 20.0) & (w <= 30.0)
    assert np.array_equal(v[inside], w[inside])


def test_truncated_normal_clamps_after_sixteen_rejections(orc):
    # support 8 sd above the mean: every attempt is rejected, value clamps to lo
    x = _one_param(orc, ("trunc_normal", 0.0, 1.0, 8.0, 9.0), "grade", n=1000)
    assert np.all(x == 8.0)


def test_constant_and_trig_columns(orc):
    from paper_2604_27193_amd import workloads as W
    d = W.single(5000)
    d["tau"] = ("const", 0.15)
    cols = orc.sample(d)
    assert np.all(cols["tau"] == 0.15)
    assert np.allclose(cols["sin_grade"], np.sin(cols["grade"]), rtol=0, atol=1e-16)
    assert np.allclose(cols["cos_grade"], np.cos(cols["grade"]), rtol=0, atol=1e-16)
    # draws are a pure function of (seed, scenario, index): any sub-range agrees
    part = orc.sample(d, first=1234, count=100)
    for k in cols:
        assert np.array_equal(part[k], cols[k][1234:1334])
