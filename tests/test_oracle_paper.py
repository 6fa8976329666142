"""Pins of the oracle against the numbers arXiv 2103.01380 prints (CPU only).

* equation (cf) on the shapes behind the printed compression factors
  (Sections 5.1, 5.2, 5.2.1) and the partition table of Section 3.2;
* the analytic 2D Taylor-Green vortex of Section 5.1: rank one, CF about 80,
  relative Frobenius error at machine precision on structured and random grids
  and over spatial partitions;
* the 3D analytic TGV workloads: closed-form coefficients and noise floors.
"""
import math
import os

import numpy as np
import pytest

import oracle
import spid_inputs as si

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                yield [c.strip() for c in line.split("|")]


@pytest.mark.parametrize("row", list(_rows("paper_compression_factors.txt")))
def test_printed_compression_factors(row):
    label, m, ms, n, k, cf, rel = row
    got = oracle.compression_factor([int(m)], [int(n)], [int(k)], m_stored=[int(ms)])
    assert abs(got - float(cf)) <= float(rel) * float(cf), (label, got)


def test_partition_table_gain_almost_70_percent():
    rows = {int(p): [int(x) for x in r.split()] for p, r in _rows("paper_partition_ranks.txt")}
    cfs = {}
    for p, ranks in rows.items():
        m = [100 // p] * p
        cfs[p] = oracle.compression_factor(m, [100] * p, ranks)
    gain = cfs[5] / cfs[1] - 1.0
    assert 0.60 <= gain < 0.70          # "almost 70 %"
    assert cfs[1] == pytest.approx(100 * 100 / (48 * 200))


@pytest.mark.parametrize("unstructured", [False, True])
@pytest.mark.parametrize("blocks", [(1, 1), (2, 1), (1, 5), (10, 10)])
def test_tgv2d_rank_one_machine_precision(unstructured, blocks):
    parts = si.tgv2d_u1(20, 100, T=10.0, nu=0.01, unstructured=unstructured, seed=8,
                        blocks=blocks)
    parts = [p for p in parts if p.shape[0] > 0]
    res = oracle.run_batch(parts, l=min(8, min(p.shape[0] for p in parts)), k_max=1, seed=5)
    assert np.all(res.k == 1)
    assert res.rel_error < 1e-14
    if blocks == (1, 1):
        cf = oracle.compression_factor([400], [100], [1])
        assert cf == pytest.approx(80.0)
    # with a tolerance the rank is found to be one
    res_t = oracle.run_batch(parts, l=min(8, min(p.shape[0] for p in parts)), k_max=5, seed=5,
                             tol=1e-10)
    assert np.all(res_t.k == 1)


def test_tgv3d_single_block_fixed_rank_and_rank_floor():
    w = si.WORKLOADS["tgv32_single_f64"]
    A = si.tgv_blocks(w).numpy()
    blk = np.asfortranarray(A[0].T)                       # m x n column-major
    res = oracle.run_batch([blk], l=w.l, k_max=w.k_max, seed=w.omega_seed)
    # the field is exactly rank one; eight pivots keep the error at rounding level
    assert res.rel_error < 1e-13
    assert res.S[0][0] == 0                                # largest column: t = 0
    assert res.gaps[0][0] > 1e-3
    # rank floor: one pivot and the closed-form coefficients exp(-3 nu (t_j - t_0))
    resf = oracle.run_batch([blk], l=w.l, k_max=w.k_max, seed=w.omega_seed, rank_floor=1e-13)
    assert resf.k[0] == 1 and resf.S[0][0] == 0
    t = si.tgv_times(w.n, w.T)
    want = np.exp(-3.0 * w.nu * (t - t[0]))
    assert np.allclose(resf.P[0][0], want, rtol=1e-14, atol=1e-15)
    assert resf.rel_error < 1e-14
    cf8 = oracle.compression_factor([w.m_b], [w.n], [8])
    cf1 = oracle.compression_factor([w.m_b], [w.n], [1])
    assert cf8 == pytest.approx(7.995, abs=1e-3) and cf1 == pytest.approx(63.96, abs=1e-2)


def test_tgv_clean_rms_closed_form():
    w = si.scaled(si.WORKLOADS["tgv128_b512_f64"], N=32, B=2, n=20)
    A = si.tgv_blocks(si.scaled(w, noise=0.0)).numpy()
    assert math.sqrt((A ** 2).mean()) == pytest.approx(si.tgv_clean_rms(w), rel=1e-12)


def test_tgv_noise_floor_and_companion_tolerance():
    # scaled-down tgv128 workload: 8 blocks of 8^3, n = 64
    w = si.scaled(si.WORKLOADS["tgv128_b512_f64"], N=16, B=2, n=64)
    A = si.tgv_blocks(w).numpy()
    blocks = [np.asfortranarray(A[b].T) for b in range(A.shape[0])]
    res = oracle.run_batch(blocks, l=w.l, k_max=w.k_max, seed=w.omega_seed, tol=w.tol)
    # tolerance 1e-8 is below the 1e-6 noise: every block runs to k_max
    assert np.all(res.k == w.k_max)
    assert np.all(res.status == oracle.ST_TOL_NOT_MET)
    # the error sits at the noise level: 1e-6 * sqrt((n-k)/n) within a factor 2
    noise_rel = w.noise * math.sqrt((w.n - w.k_max) / w.n)
    assert 0.5 * noise_rel < res.rel_error < 2.0 * noise_rel
    # companion tolerance above the noise: the rank-one signal is found in every block
    res5 = oracle.run_batch(blocks, l=w.l, k_max=w.k_max, seed=w.omega_seed, tol=1e-5)
    assert np.all(res5.k == 1) and np.all(res5.S[:, 0] == 0)
    assert res5.rel_error < 3e-6
