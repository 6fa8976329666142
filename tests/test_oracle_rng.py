"""Pins of the oracle's counter-based generator and sketch matrix (CPU only).

Omega of the Gaussian random projection (arXiv 2103.01380, Section 2) is drawn
from Philox4x32-10 (SC'11) and Box-Muller; pinned by the published
known-answer vectors and by distribution statistics.
"""
import math
import os

import numpy as np
import pytest

import oracle

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    rows = []
    with open(os.path.join(GOLD, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(x, 16) for x in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,want", _kat())
def test_philox_known_answers(ctr, key, want):
    got = oracle.philox4x32_10(ctr, key)
    assert [int(x) for x in got] == want


def test_philox_uniform_chi_square():
    # 256 bins over the top byte of 16384 words from consecutive counters
    seed = 7
    words = []
    for i in range(4096):
        words.extend(oracle.philox4x32_10([i, 0, 0, 0], [seed, 0]))
    w = np.array(words, dtype=np.uint64)
    top = (w >> 24).astype(np.int64)
    counts = np.bincount(top, minlength=256)
    expect = len(top) / 256
    chi2 = ((counts - expect) ** 2 / expect).sum()
    # 255 dof: mean 255, sd ~22.6; 6 sd bound
    assert abs(chi2 - 255) < 6 * math.sqrt(2 * 255)
    # lag-1 correlation of consecutive words
    u = w.astype(np.float64) / 2.0 ** 32 - 0.5
    corr = np.corrcoef(u[:-1], u[1:])[0, 1]
    assert abs(corr) < 5 / math.sqrt(len(u))


def test_normals_moments():
    om = oracle.omega(seed=12345, l=8, m=40000)      # 320k draws
    z = om.ravel()
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    k4 = (z ** 4).mean()
    assert abs(k4 - 3.0) < 5 * math.sqrt(96.0 / n)
    # rows of a Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(om[0], om[1])[0, 1]) < 5 / math.sqrt(om.shape[1])


def test_omega_keying():
    a = oracle.omega(seed=1, l=6, m=50)
    b = oracle.omega(seed=1, l=6, m=50)
    c = oracle.omega(seed=2, l=6, m=50)
    d = oracle.omega(seed=1, l=6, m=50, block_key=3)
    assert np.array_equal(a, b)
    assert not np.allclose(a, c)
    assert not np.allclose(a, d)
    # a block of fewer rows sees the prefix of the shared Omega
    e = oracle.omega(seed=1, l=6, m=20)
    assert np.array_equal(a[:, :20], e)
    # and a shorter sketch sees the row prefix
    f = oracle.omega(seed=1, l=4, m=50)
    assert np.array_equal(a[:4], f)


def test_omega_box_muller_pair_radius():
    # rows 2q and 2q+1 share rho: z0^2 + z1^2 = -2 ln u1 with u1 in (0,1]
    om = oracle.omega(seed=99, l=2, m=2000)
    r2 = om[0] ** 2 + om[1] ** 2
    assert np.all(r2 >= 0)
    # exponential(1/2) distribution of r^2: mean 2
    assert abs(r2.mean() - 2.0) < 5 * 2.0 / math.sqrt(len(r2))


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0), (1.00390625, 1.0),            # tie 1 + 2^-8 -> even (1.0)
    (1.01171875, 1.015625),                   # tie 1 + 3*2^-8 -> even (1 + 2^-6)
    (1.0 + 2 ** -8 + 2 ** -20, 1.0078125),    # above the tie -> up
    (-3.14159265, -3.140625), (0.0, 0.0),
])
def test_round_bf16_cases(x, want):
    assert oracle.round_bf16(x) == want


@pytest.mark.parametrize("x,want", [
    (1.0, 1.0), (1.0625, 1.0), (1.1875, 1.25), (1.07, 1.125), (500.0, 448.0),
    (-2.9, -3.0), (2.0 ** -9, 2.0 ** -9), (3 * 2.0 ** -11, 2.0 ** -9), (2.0 ** -11, 0.0),
])
def test_round_e4m3_cases(x, want):
    assert oracle.round_e4m3(x) == want


def test_round_bf16_matches_float32_truncation_rule():
    # independent route: numpy float32 then bf16 RNE by integer arithmetic on float32 bits,
    # valid whenever the double is exactly a float32
    rng = np.random.default_rng(0)
    xs = rng.standard_normal(2000).astype(np.float32)
    bits = xs.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    want = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    got = np.array([oracle.round_bf16(float(x)) for x in xs])
    assert np.array_equal(got, want)


def test_sketch_probe_and_linearity():
    l, m, n = 7, 30, 5
    seed = 4242
    om = oracle.omega(seed, l, m)
    # probe: A = e_i gives Omega(:, i)
    for i in (0, 13, 29):
        A = np.zeros((m, 1), order="F")
        A[i, 0] = 1.0
        Y = oracle.sketch(A, l, seed)
        assert np.array_equal(Y[:, 0], om[:, i])
    rng = np.random.default_rng(1)
    A1 = np.asfortranarray(rng.standard_normal((m, n)))
    A2 = np.asfortranarray(rng.standard_normal((m, n)))
    Y1 = oracle.sketch(A1, l, seed)
    Y2 = oracle.sketch(A2, l, seed)
    Y12 = oracle.sketch(np.asfortranarray(A1 + A2), l, seed)
    assert np.allclose(Y12, Y1 + Y2, rtol=1e-13, atol=1e-13 * np.abs(Y12).max())
    # float32 storage is widened exactly
    A3 = np.asfortranarray(rng.standard_normal((m, n)).astype(np.float32))
    assert np.array_equal(oracle.sketch(A3, l, seed), oracle.sketch(A3.astype(np.float64), l, seed))


def test_sketch_column_window_is_idempotent():
    rng = np.random.default_rng(3)
    A = np.asfortranarray(rng.standard_normal((40, 9)))
    full = oracle.sketch(A, 6, 5)
    Y = np.zeros((6, 9), order="F")
    for j in range(9):
        oracle.sketch(A, 6, 5, j0=j, w=1, Y=Y)
    assert np.array_equal(Y, full)
    oracle.sketch(A, 6, 5, j0=2, w=3, Y=Y)
    assert np.array_equal(Y, full)


def test_low_precision_omega_is_rounded_normal():
    z = oracle.omega(77, 4, 300)
    zb = oracle.omega(77, 4, 300, prec=oracle.OMEGA_BF16)
    z8 = oracle.omega(77, 4, 300, prec=oracle.OMEGA_FP8E4M3)
    assert np.array_equal(zb, np.vectorize(oracle.round_bf16)(z))
    assert np.array_equal(z8, np.vectorize(oracle.round_e4m3)(z))
    assert np.max(np.abs(zb - z) / np.maximum(np.abs(z), 1e-30)) <= 2.0 ** -8
