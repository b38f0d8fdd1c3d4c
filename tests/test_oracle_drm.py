"""Pins of the oracle's DRM generator (CPU only).

Philox4x32-10 against its published known-answer vectors; the fixed-sequence ln
and cos(2 pi .) against the C library within a few ulps; the Gaussian transform
against the moments and CDF of N(0,1); rounding helpers against IEEE definitions.
"""
import math

import numpy as np
import pytest
from scipy import stats

from conftest import golden_rows
from oracle import drm as R


def test_philox_known_answers():
    rows = list(golden_rows("philox4x32_10_kat.txt"))
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        ctr, key, want = v[0:4], v[4:6], v[6:10]
        got = R.philox4x32_10([np.array([c], dtype=np.uint64) for c in ctr], key)
        assert [int(g[0]) for g in got] == want


def test_philox_vectorised_matches_scalar():
    rng = np.random.default_rng(5)
    c = rng.integers(0, 2**32, size=(4, 64), dtype=np.uint64)
    batch = R.philox4x32_10(list(c), (123, 456))
    for j in range(64):
        one = R.philox4x32_10([np.array([c[i, j]]) for i in range(4)], (123, 456))
        assert [int(o[0]) for o in one] == [int(b[j]) for b in batch]


def _ulps(a, b):
    return abs(a - b) / math.ulp(b) if b != 0 else abs(a - b) / math.ulp(1.0)


def test_ln_fixed_accuracy():
    rng = np.random.default_rng(0)
    u = np.concatenate([
        rng.random(20000) + 2.0**-53,
        np.exp(-rng.random(2000) * 36),                  # wide exponent range
        [1.0, 2.0**-53, 0.5, 0.25, 1.0 - 2.0**-53],
        [R.SQRT2 / 2, np.nextafter(R.SQRT2 / 2, 0), np.nextafter(R.SQRT2 / 2, 1)],
    ])
    got = R.ln_fixed(u)
    for x, g in zip(u, got):
        want = math.log(x)
        if want == 0.0:
            assert g == 0.0
        else:
            assert _ulps(g, want) <= 2.0, (x, g, want)


def test_cos2pi_fixed_accuracy():
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.random(20000), [0.0, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875,
                                            np.nextafter(0.25, 0), np.nextafter(0.5, 1)]])
    got = R.cos2pi_fixed(v)
    want = np.cos(2.0 * np.pi * v)
    # the reference itself carries the rounding of 2 pi v (about 1e-15 absolute)
    assert np.max(np.abs(got - want)) < 2.5e-15
    assert got[v == 0.25][0] == pytest.approx(0.0, abs=1e-16)
    assert got[v == 0.5][0] == -1.0 and got[v == 0.0][0] == 1.0


def test_gaussian_moments_and_ks():
    n = 1_000_000
    rows = np.arange(n // 4, dtype=np.uint64)[:, None]
    cols = np.arange(4, dtype=np.uint64)[None, :]
    z = R.gaussian(7, 3, 1, rows, cols).ravel()
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 6 * math.sqrt(2.0 / n)
    kurt = np.mean(z**4) / z.var() ** 2
    assert abs(kurt - 3.0) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-3
    assert np.all(np.isfinite(z))


def test_streams_uncorrelated():
    n = 200_000
    rows = np.arange(n, dtype=np.uint64)
    streams = [R.gaussian(1, node, kind, rows, 0) for node in range(4) for kind in (0, 1)]
    streams.append(R.gaussian(2, 0, 0, rows, 0))      # other seed
    streams.append(R.gaussian(1, 0, 0, rows, 1))      # other column
    C = np.corrcoef(np.vstack(streams))
    off = C[~np.eye(len(streams), dtype=bool)]
    assert np.max(np.abs(off)) < 5 / math.sqrt(n)


def test_entry_is_pure_function_of_index():
    full = R.drm(11, 2, 0, 37, 5, chunk=16)
    again = R.gaussian(11, 2, 0, np.arange(37, dtype=np.uint64)[:, None], np.arange(5, dtype=np.uint64)[None, :])
    assert np.array_equal(full, again)
    assert np.array_equal(full[13, 3], R.gaussian(11, 2, 0, 13, 3))
    big = R.gaussian(11, 2, 0, np.array([2**33 + 5], dtype=np.uint64), 0)
    assert np.isfinite(big).all()


def test_bf16_rounding_definition():
    f = np.array([1.0, 1.00390625, 1.01171875, -2.5, 3.140625, 1e-30], dtype=np.float32)
    bits = R.bf16_bits(f)
    # 1.00390625 = 0x3F808000 is a tie -> even (0x3F80); 1.01171875 = 0x3F818000 -> 0x3F82
    assert list(bits[:3]) == [0x3F80, 0x3F80, 0x3F82]
    back = R.bf16_to_f64(bits)
    assert back[3] == -2.5 and back[4] == 3.140625
    rng = np.random.default_rng(3)
    x = rng.standard_normal(10000)
    y = R.rounded(x, "bf16")
    assert np.max(np.abs(y - x) / np.abs(x)) <= 2.0**-8
    assert np.array_equal(R.rounded(x, "f32"), x.astype(np.float32).astype(np.float64))


def _box_muller_libm(words):
    x0, x1, x2, x3 = words
    a = ((x1 << 32) | x0) >> 11
    b = ((x3 << 32) | x2) >> 11
    u1 = (a + 1) * 2.0**-53
    u2 = b * 2.0**-53
    return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


def test_gaussian_counter_layout_and_transform_from_kat():
    """G(seed, node, kind, row, col) uses counter (lo32 row, hi32 row, col, 2 node + kind)
    and key (lo32 seed, hi32 seed): each KAT counter/key maps to one G entry, whose
    value follows from the KAT output words through Box-Muller evaluated with libm."""
    for row in golden_rows("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        c0, c1, c2, c3, k0, k1 = v[:6]
        seed = (k1 << 32) | k0
        r = (c1 << 32) | c0
        node, kind = c3 >> 1, c3 & 1
        z = float(R.gaussian(seed, node, kind, np.array([r], dtype=np.uint64), c2)[0])
        want = _box_muller_libm(v[6:10])
        assert abs(z - want) <= 4e-15 * max(1.0, abs(want)), (z, want)


def test_c_evaluation_matches_numpy_definition_bitwise():
    """oracle/cdrm.c (the fast path of oracle.drm.gaussian / drm) against the NumPy
    definition, bit for bit: random indices including rows past 2^32, extreme seeds,
    both map kinds, and a dense block."""
    from oracle import cdrm
    from oracle import drm as D
    assert cdrm.lib() is not None, "oracle/_cdrm.so is built by tests/conftest.py"
    g = np.random.default_rng(123)
    rows = np.concatenate([g.integers(0, 2 ** 48, size=50000, dtype=np.uint64),
                           np.array([0, 1, 2 ** 32 - 1, 2 ** 32, 2 ** 63], dtype=np.uint64)])
    cols = g.integers(0, 2 ** 31, size=rows.size, dtype=np.uint64)
    for seed, node, kind in [(0, 0, 0), (1, 5, 1), (0xFFFFFFFFFFFFFFFF, 63, 1), (0x1234_5678_9abc, 12, 0)]:
        a = D.gaussian(seed, node, kind, rows, cols)
        b = D.gaussian_numpy(seed, node, kind, rows, cols)
        assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (seed, node, kind)
    dense = D.drm(7, 3, 0, 300, 17)
    ref = D.gaussian_numpy(7, 3, 0, np.arange(300, dtype=np.uint64)[:, None], np.arange(17, dtype=np.uint64)[None, :])
    assert np.array_equal(dense.view(np.uint64), ref.view(np.uint64))
