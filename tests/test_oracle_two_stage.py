"""Pins of the oracle's modified (two-stage) ID, Section 3.4.2 (CPU only).

* the final coefficients equal C^1 C^{0'} assembled independently with a
  dense block-diagonal C^{0'} (scipy) from per-window and stage-2 IDs;
* the selected columns are I_U(I_1) and P(:, S) is the identity;
* one window with k1 = n is the plain tolerance ID;
* exact low-rank data is recovered through both stages;
* the sketch-space error obeys the triangle bound of the two stages;
* windows of unequal width (nwin not dividing n) and a non-finite window.
"""
import numpy as np
import pytest
from scipy.linalg import block_diag

import oracle


def _lowrank(l, n, r, seed, noise=0.0, decay=0.3):
    rng = np.random.default_rng(seed)
    Y = (rng.standard_normal((l, r)) * 10.0 ** (-decay * np.arange(r))) @ rng.standard_normal((r, n))
    return np.asfortranarray(Y + noise * rng.standard_normal((l, n)))


def _windows(n, nwin):
    return [(w * n // nwin, (w + 1) * n // nwin) for w in range(nwin)]


def _two_stage_dense(Y, nwin, k1, k_max, tol2):
    """Reference assembly from single-stage oracle calls and numpy/scipy."""
    blocks, IU = [], []
    for c0, c1 in _windows(Y.shape[1], nwin):
        sel = oracle.select(Y[:, c0:c1], k1)
        C = oracle.coeffs(sel, c1 - c0)[:sel.k]
        blocks.append(C)
        IU += [c0 + int(j) for j in sel.S[:sel.k]]
    C0 = block_diag(*blocks)                     # sum k_w x n
    Y0 = Y[:, IU]
    sel2 = oracle.select(Y0, k_max, tol2)
    C1 = oracle.coeffs(sel2, len(IU))[:sel2.k]
    return np.array(IU)[sel2.S[:sel2.k]], C1 @ C0, sel2


@pytest.mark.parametrize("n,nwin,k1,seed", [(60, 4, 6, 1), (64, 3, 5, 2), (37, 5, 4, 3), (40, 1, 8, 4)])
def test_matches_dense_assembly(n, nwin, k1, seed):
    Y = _lowrank(20, n, 12, seed, noise=1e-9)
    ts = oracle.two_stage(Y, nwin, k1, 16, 1e-4)
    S_ref, P_ref, sel2 = _two_stage_dense(Y, nwin, k1, 16, 1e-4)
    assert ts.k == sel2.k and ts.status == sel2.status
    assert np.array_equal(ts.S[:ts.k], S_ref)
    assert np.all(ts.S[ts.k:] == -1)
    assert np.allclose(ts.P[:ts.k], P_ref, rtol=0, atol=1e-12 * max(1.0, np.abs(P_ref).max()))
    assert np.all(ts.P[ts.k:] == 0.0)
    assert np.array_equal(ts.P[:ts.k][:, ts.S[:ts.k]], np.eye(ts.k))


def test_one_full_window_is_the_plain_tolerance_id():
    Y = _lowrank(24, 50, 10, 7, noise=1e-8)
    ts = oracle.two_stage(Y, 1, 50, 20, 1e-5)
    sel = oracle.select(Y, 20, 1e-5)
    P = oracle.coeffs(sel, 50)
    # stage 1 at full rank selects min(l, n) = 24 columns; stage 2 works on those
    S1 = oracle.select(Y, 50).S[:24]
    sel2 = oracle.select(Y[:, S1], 20, 1e-5)
    assert np.array_equal(ts.S[:ts.k], S1[sel2.S[:sel2.k]])
    res_ts = np.linalg.norm(Y - Y[:, ts.S[:ts.k]] @ ts.P[:ts.k])
    res_id = np.linalg.norm(Y - Y[:, sel.S[:sel.k]] @ P[:sel.k])
    assert res_ts <= 1e-5 * np.linalg.norm(Y) * 1.01 and res_id <= 1e-5 * np.linalg.norm(Y)


@pytest.mark.parametrize("nwin", [2, 4, 8])
def test_exact_low_rank_through_both_stages(nwin):
    Y = _lowrank(30, 96, 5, 9, decay=0.1)
    ts = oracle.two_stage(Y, nwin, 6, 12, 1e-12)
    assert ts.k == 5
    err = np.linalg.norm(Y - Y[:, ts.S[:5]] @ ts.P[:5]) / np.linalg.norm(Y)
    assert err < 1e-12


@pytest.mark.parametrize("seed", range(4))
def test_triangle_bound_of_the_two_stages(seed):
    Y = _lowrank(18, 72, 14, 20 + seed, noise=1e-6, decay=0.15)
    nwin, k1, tol2 = 4, 6, 1e-3
    ts = oracle.two_stage(Y, nwin, k1, 16, tol2)
    blocks, IU = [], []
    for c0, c1 in _windows(72, nwin):
        sel = oracle.select(Y[:, c0:c1], k1)
        blocks.append(oracle.coeffs(sel, c1 - c0)[:sel.k])
        IU += [c0 + int(j) for j in sel.S[:sel.k]]
    C0 = block_diag(*blocks)
    Y0 = Y[:, IU]
    e1 = np.linalg.norm(Y - Y0 @ C0)
    sel2 = oracle.select(Y0, 16, tol2)
    C1 = oracle.coeffs(sel2, len(IU))[:sel2.k]
    e2 = np.linalg.norm(Y0 - Y0[:, sel2.S[:sel2.k]] @ C1)
    total = np.linalg.norm(Y - Y[:, ts.S[:ts.k]] @ ts.P[:ts.k])
    assert total <= (e1 + e2 * np.linalg.norm(C0, 2)) * (1 + 1e-10)
    assert e2 <= tol2 * np.linalg.norm(Y0) * (1 + 1e-12)       # the stage-2 tolerance stop


def test_non_finite_window_reports_status():
    Y = _lowrank(10, 40, 4, 11)
    Y[3, 25] = np.nan
    ts = oracle.two_stage(Y, 4, 3, 8, 1e-6)
    assert ts.status == oracle.ST_NONFINITE and ts.k == 0
    assert np.all(ts.P == 0.0)


def test_invalid_arguments():
    Y = _lowrank(10, 20, 4, 12)
    with pytest.raises(ValueError):
        oracle.two_stage(Y, 0, 3, 8, 1e-6)
    with pytest.raises(ValueError):
        oracle.two_stage(Y, 21, 3, 8, 1e-6)
