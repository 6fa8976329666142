"""Pins of the oracle's column selection, coefficients and error pass (CPU only).

Each test checks the oracle against something other than itself: LAPACK's
pivoted QR (dgeqp3), least squares (Section 2 defines the coefficients as
least-squares solutions), brute force over all column subsets, the SVD tail
(Eckart-Young), closed forms of structured matrices, and the properties of
Lemma A.1 of arXiv 2103.01380.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg

import oracle


def _rand(m, n, seed, rank=None, decay=None):
    rng = np.random.default_rng(seed)
    if rank is None:
        A = rng.standard_normal((m, n))
    else:
        U = np.linalg.qr(rng.standard_normal((m, rank)))[0]
        V = np.linalg.qr(rng.standard_normal((n, rank)))[0]
        s = np.ones(rank) if decay is None else 10.0 ** (-decay * np.arange(rank))
        A = (U * s) @ V.T
    return np.asfortranarray(A)


def _id_of(A, k, tol=0.0, rank_floor=0.0):
    """Apply the ID stages directly to A (sketch = identity)."""
    sel = oracle.select(A, k, tol, rank_floor)
    P = oracle.coeffs(sel, A.shape[1])
    return sel, P


# ------------------------------------------------------------------ library routine: dgeqp3
@pytest.mark.parametrize("m,n,k,seed", [(30, 12, 6, 0), (8, 20, 8, 1), (50, 50, 20, 2),
                                        (17, 9, 9, 3)])
def test_pivots_match_lapack_pivoted_qr(m, n, k, seed):
    A = _rand(m, n, seed)
    sel, P = _id_of(A, k)
    Q, R, piv = scipy.linalg.qr(A, pivoting=True, mode="economic")
    # gap rule: compare the pivot prefix while the top-two gap is decidable
    for s in range(sel.k):
        if sel.gaps[s] <= 1e-10:
            break
        assert sel.S[s] == piv[s], f"step {s}"
    # |R_ss| agree with LAPACK's diagonal (same pivots, same subspaces)
    kk = sel.k
    Rss = np.array([sel.R[s, sel.S[s]] for s in range(kk)])
    assert np.allclose(np.abs(Rss), np.abs(np.diag(R))[:kk], rtol=1e-10)
    # coefficients are R11^-1 R12 of LAPACK's factor (sign invariant)
    R11 = R[:kk, :kk]
    R12 = R[:kk, kk:]
    T = scipy.linalg.solve_triangular(R11, R12)
    P_perm = P[:kk][:, piv]
    assert np.allclose(P_perm[:, :kk], np.eye(kk), atol=0)
    if T.size:
        assert np.allclose(P_perm[:, kk:], T, rtol=1e-9, atol=1e-9 * max(1, np.abs(T).max()))


# ------------------------------------------------------------------ least squares definition
@pytest.mark.parametrize("l,n,k,seed", [(12, 40, 5, 4), (30, 30, 10, 5), (9, 100, 9, 6)])
def test_coefficients_are_least_squares(l, n, k, seed):
    Y = _rand(l, n, seed)
    sel, P = _id_of(Y, k)
    S = sel.S[:sel.k]
    X, *_ = np.linalg.lstsq(Y[:, S], Y, rcond=None)
    assert np.allclose(P[:sel.k], X, rtol=1e-9, atol=1e-9 * np.abs(X).max())


# ------------------------------------------------------------------ Lemma A.1 properties
def test_identity_block_is_exact():
    Y = _rand(20, 35, 7)
    sel, P = _id_of(Y, 12)
    S = sel.S[:sel.k]
    assert np.array_equal(P[:sel.k][:, S], np.eye(sel.k))        # Lemma A.1 (1), bitwise


@pytest.mark.parametrize("seed", range(5))
def test_cpqr_coefficient_bound_and_report(seed):
    # For pivoted QR |R(s,j)| <= |R_ss| on unselected columns, which bounds |P| by 2^(k-1);
    # Lemma A.1 (2)-(3) are existence statements, CPQR gives them only approximately.
    k = 8
    Y = _rand(16, 60, 10 + seed)
    sel, P = _id_of(Y, k)
    assert np.abs(P).max() <= 2.0 ** (k - 1)


@pytest.mark.parametrize("m,n", [(10, 6), (7, 7), (40, 12)])
def test_full_rank_k_equals_n_is_exact(m, n):
    # Lemma A.1 (5): A = A(:,I) C when k = n
    A = _rand(m, n, 11)
    sel, P = _id_of(A, n)
    assert sel.k == n
    Pk = P[:n]
    assert np.array_equal(np.sort(sel.S), np.arange(n))
    assert np.array_equal(np.abs(Pk).sum(0), np.ones(n))         # a permutation matrix
    e2, a2 = oracle.reconstruct(A, sel.S, sel.k, P)
    assert e2 == 0.0


def test_lemma_error_bound_holds_with_margin():
    # Lemma A.1 (6) (existence) compared with the CPQR result on a decaying spectrum:
    # report-only check that the pivoted-QR ID stays within sqrt(k(n-k)+1) * sigma_{k+1} * 10
    A = _rand(60, 40, 12, rank=40, decay=0.2)
    k = 10
    sel, P = _id_of(A, k)
    approx = A[:, sel.S[:k]] @ P[:k]
    err = np.linalg.norm(A - approx, 2)
    s = np.linalg.svd(A, compute_uv=False)
    assert err <= 10 * math.sqrt(k * (40 - k) + 1) * s[k]


# ------------------------------------------------------------------ CPQR invariants
@pytest.mark.parametrize("seed", range(4))
def test_cpqr_invariants(seed):
    Y = _rand(24, 50, 20 + seed, rank=24, decay=0.1)
    k = 15
    sel, P = _id_of(Y, k)
    S = sel.S[:sel.k]
    Rss = np.abs([sel.R[s, S[s]] for s in range(sel.k)])
    assert np.all(np.diff(Rss) <= 1e-12 * Rss[0])                  # non-increasing pivots
    sel_set = set()
    for s in range(sel.k):
        for j in range(Y.shape[1]):
            if j in sel_set or j == S[s]:
                continue
            assert abs(sel.R[s, j]) <= Rss[s] * (1 + 1e-12)
        sel_set.add(S[s])
    # sketch-space identity: ||Y - Y(:,S) P||_F^2 = sum of residual norms
    resid = Y - Y[:, S] @ P[:sel.k]
    assert np.isclose((resid ** 2).sum(), sel.res2, rtol=1e-9, atol=1e-14 * (Y ** 2).sum())


# ------------------------------------------------------------------ closed forms
def test_orthogonal_columns_select_by_norm():
    rng = np.random.default_rng(30)
    m, n, k = 40, 12, 5
    Q = np.linalg.qr(rng.standard_normal((m, n)))[0]
    norms = rng.permutation(np.linspace(1.0, 12.0, n))
    A = np.asfortranarray(Q * norms)
    sel, P = _id_of(A, k)
    want = np.argsort(-norms)[:k]
    assert np.array_equal(sel.S[:k], want)
    # least-squares coefficients on orthogonal columns vanish off the identity block
    mask = np.ones(n, bool)
    mask[want] = False
    assert np.abs(P[:k][:, mask]).max() < 1e-12
    e2, a2 = oracle.reconstruct(A, sel.S, k, P)
    assert np.isclose(e2, (norms[mask] ** 2).sum(), rtol=1e-12)
    assert np.isclose(a2, (norms ** 2).sum(), rtol=1e-12)


def test_ties_go_to_lowest_index():
    A = np.asfortranarray(np.eye(6) * np.array([1.0, 3.0, 3.0, 2.0, 3.0, 1.0]))
    sel, _ = _id_of(A, 4)
    assert list(sel.S[:4]) == [1, 2, 4, 3]


def test_column_permutation_equivariance():
    A = _rand(30, 14, 31)
    perm = np.random.default_rng(5).permutation(14)
    sel, P = _id_of(A, 6)
    sel2, P2 = _id_of(np.asfortranarray(A[:, perm]), 6)
    inv = np.argsort(perm)
    assert np.array_equal(perm[sel2.S[:6]], sel.S[:6])
    assert np.allclose(P2[:, inv], P, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("e", [-7, 3, 40])
def test_power_of_two_scaling_is_bitwise_invariant(e):
    A = _rand(25, 18, 32)
    sel, P = _id_of(A, 7)
    sel2, P2 = _id_of(np.asfortranarray(A * 2.0 ** e), 7)
    assert np.array_equal(sel.S, sel2.S)
    assert np.array_equal(P, P2)


def test_rank_deficient_stops():
    A = _rand(30, 20, 33, rank=3)
    A[:, 5] = 0.0
    sel, P = _id_of(A, 10, rank_floor=1e-12)
    assert sel.k == 3
    assert sel.status == oracle.ST_RANK_DEFICIENT
    e2, a2 = oracle.reconstruct(A, sel.S, sel.k, P)
    assert e2 <= 1e-26 * a2
    Z = np.zeros((5, 4), order="F")
    selz = oracle.select(Z, 3)
    assert selz.k == 0 and selz.status == oracle.ST_RANK_DEFICIENT


def test_tolerance_stop():
    A = _rand(40, 30, 34, rank=30, decay=0.25)
    # singular values 10^(-i/4): residual after k pivots ~ sqrt(sum_{i>=k} s_i^2)
    sel, P = _id_of(A, 30, tol=1e-3)
    res = math.sqrt(sel.res2) / np.linalg.norm(A)
    assert res <= 1e-3
    # one fewer pivot would not have met it
    sel2, _ = _id_of(A, sel.k - 1)
    assert math.sqrt(sel2.res2) / np.linalg.norm(A) > 1e-3
    sel3, _ = _id_of(A, 5, tol=1e-12)
    assert sel3.k == 5 and sel3.status == oracle.ST_TOL_NOT_MET


def test_nonfinite_sketch_reports_status():
    Y = _rand(6, 8, 35)
    Y[2, 3] = np.nan
    sel = oracle.select(Y, 3)
    assert sel.status == oracle.ST_NONFINITE and sel.k == 0


# ------------------------------------------------------------------ brute force (tiny)
@pytest.mark.parametrize("seed", range(6))
def test_brute_force_subsets(seed):
    rng = np.random.default_rng(100 + seed)
    m, n, k = int(rng.integers(6, 13)), int(rng.integers(5, 11)), int(rng.integers(1, 4))
    A = _rand(m, n, 200 + seed, rank=min(m, n), decay=0.3)
    sel, P = _id_of(A, k)
    e2, a2 = oracle.reconstruct(A, sel.S, sel.k, P)
    best = np.inf
    for sub in itertools.combinations(range(n), k):
        X, *_ = np.linalg.lstsq(A[:, sub], A, rcond=None)
        best = min(best, ((A - A[:, sub] @ X) ** 2).sum())
    s = np.linalg.svd(A, compute_uv=False)
    tail = (s[k:] ** 2).sum()
    assert best <= e2 * (1 + 1e-10)                 # greedy is never better than the best subset
    assert best >= tail * (1 - 1e-10)                # no subset beats the SVD tail
    # the oracle's error equals the least-squares residual of its own subset
    X, *_ = np.linalg.lstsq(A[:, sel.S[:k]], A, rcond=None)
    lsq = ((A - A[:, sel.S[:k]] @ X) ** 2).sum()
    assert np.isclose(e2, lsq, rtol=1e-9, atol=1e-14 * a2)


def test_brute_force_orthogonal_family_exact_subset():
    rng = np.random.default_rng(41)
    Q = np.linalg.qr(rng.standard_normal((10, 7)))[0]
    A = np.asfortranarray(Q * np.array([0.5, 3.0, 1.0, 2.5, 0.1, 4.0, 2.0]))
    k = 3
    sel, P = _id_of(A, k)
    best, arg = np.inf, None
    for sub in itertools.combinations(range(7), k):
        X, *_ = np.linalg.lstsq(A[:, sub], A, rcond=None)
        e = ((A - A[:, sub] @ X) ** 2).sum()
        if e < best:
            best, arg = e, sub
    assert set(sel.S[:k]) == set(arg)


# ------------------------------------------------------------------ sketched ID on exact low rank
@pytest.mark.parametrize("rank,l", [(1, 6), (4, 10), (7, 12)])
def test_sketched_id_recovers_exact_low_rank(rank, l):
    A = _rand(300, 40, 50 + rank, rank=rank)
    res = oracle.run_batch([A], l=l, k_max=rank, seed=9)
    assert res.rel_error < 1e-12
    assert res.k[0] == rank


def test_batch_matches_single_block_calls():
    blocks = [_rand(60 + 7 * b, 20 + b, 60 + b) for b in range(5)]
    res = oracle.run_batch(blocks, l=10, k_max=6, seed=3, nthreads=3)
    for b, A in enumerate(blocks):
        Y = oracle.sketch(A, 10, 3)
        sel = oracle.select(Y, 6)
        P = oracle.coeffs(sel, A.shape[1])
        e2, a2 = oracle.reconstruct(A, sel.S, sel.k, P)
        assert np.array_equal(res.Y[b], Y)
        assert np.array_equal(res.S[b], sel.S)
        assert np.array_equal(res.P[b], P)
        assert res.err2[b] == e2 and res.nrm2[b] == a2


def test_subsampling_sketch_thm_a1_bound():
    # Theorem A.1 (SubID) with the reading eps(tau) = lambda_max(A^T A - tau B^T B):
    # ||A - A(:,I_B) C_B||_2 <= min over tau of rho_k(tau).  Here B = A(J,:) (every 3rd row).
    rng = np.random.default_rng(70)
    m, n, k = 240, 30, 4
    x = np.linspace(0, 2 * np.pi, m, endpoint=False)
    t = np.linspace(0, 1, n)
    A = np.asfortranarray(sum(np.outer(np.sin((q + 1) * x), np.exp(-(q + 1) * t)) * 0.5 ** q
                              for q in range(8)) + 1e-6 * rng.standard_normal((m, n)))
    J = np.arange(0, m, 3)
    B = np.asfortranarray(A[J])
    sel, C = _id_of(B, k)
    S = sel.S[:k]
    lhs = np.linalg.norm(A - A[:, S] @ C[:k], 2)
    sB = np.linalg.svd(B, compute_uv=False)
    Bhat = B[:, S] @ C[:k]
    eB = np.linalg.norm(B - Bhat, 2)
    Cn = np.linalg.norm(C[:k], 2)
    best = np.inf
    for tau in np.geomspace(1e-2, 1e3, 200):
        eps = max(np.linalg.eigvalsh(A.T @ A - tau * B.T @ B).max(), 0.0)
        rho = (1 + Cn) * math.sqrt(tau * sB[k] ** 2 + eps) + eB * math.sqrt(tau + eps / sB[k - 1] ** 2)
        best = min(best, rho)
    assert lhs <= best
