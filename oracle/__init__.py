"""Double-precision CPU oracle of the sketched column ID (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2103_01380_amd``) and never imports it.

The arithmetic lives in ``spid_oracle.c`` (plain C, ``-O2 -ffp-contract=off``,
no BLAS); this module only marshals numpy arrays into it.  What each function
follows in arXiv 2103.01380:

* ``omega`` / ``sketch``      -- Section 2, Gaussian random projection B = Omega A.
* ``select``                  -- Section 2 / Algorithm 1, rank-k pivoted
                                 modified Gram-Schmidt ("mgsqr"), Remark 2.1
                                 tolerance stop.
* ``coeffs``                  -- Section 2 / Algorithm 1, C = [I | R11^+ R12] Z^T.
* ``reconstruct``             -- Section 5.1, relative Frobenius error.
* ``compression_factor``      -- equation (cf), summed over blocks (Section 3.2).
* ``coarse_rows`` / ``subsample`` -- Section 2 / Algorithm 2, the deterministic
                                 coarse-grid sketch B = A(J,:) (every s-th point
                                 per direction, Section 5.2).
* ``interp_row`` / ``interp_matrix`` / ``interp_error`` -- Section 2,
                                 equation (single_ID) / Algorithm 3, the
                                 single-pass approximation M B(:,S) C with a
                                 trilinear M (Section 5.2).
* ``two_stage``               -- Section 3.4.2, the modified (two-stage) ID:
                                 rank-k IDs of temporal windows, then a
                                 tolerance ID of the concatenated skeletons,
                                 C^{1'} = C^1 C^{0'}.
* ``run_batch``               -- Section 3.2, independent blocks, threaded.

Parity pins: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` (closed forms, LAPACK special case, brute force,
invariants, the paper's printed compression factors).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spid_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

A_F64, A_F32 = 0, 1
OMEGA_F64, OMEGA_BF16, OMEGA_FP8E4M3 = 0, 1, 2
ST_OK, ST_RANK_DEFICIENT, ST_NONFINITE, ST_TOL_NOT_MET = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (plain C, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
             "-pthread", "-Wall", _SRC, "-o", tmp, "-lm"],
            check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        c = ctypes
        P = c.c_void_p
        lib.spid_ref_philox4x32_10.argtypes = [P, P, P]
        lib.spid_ref_philox4x32_10.restype = None
        lib.spid_ref_omega.argtypes = [c.c_uint64, c.c_uint32, c.c_int64, c.c_int64, c.c_int32]
        lib.spid_ref_omega.restype = c.c_double
        lib.spid_ref_omega_matrix.argtypes = [c.c_uint64, c.c_uint32, c.c_int32, c.c_int64,
                                              c.c_int32, P]
        lib.spid_ref_omega_matrix.restype = None
        lib.spid_ref_round_bf16.argtypes = [c.c_double]
        lib.spid_ref_round_bf16.restype = c.c_double
        lib.spid_ref_round_e4m3.argtypes = [c.c_double]
        lib.spid_ref_round_e4m3.restype = c.c_double
        lib.spid_ref_sketch.argtypes = [c.c_int64, c.c_int32, P, c.c_int64, c.c_int32, c.c_int32,
                                        c.c_uint64, c.c_uint32, c.c_int32, c.c_int32, c.c_int32, P]
        lib.spid_ref_sketch.restype = c.c_int
        lib.spid_ref_select.argtypes = [c.c_int32, c.c_int32, P, c.c_int32, c.c_double, c.c_double,
                                        P, P, P, P, P, P, P]
        lib.spid_ref_select.restype = c.c_int
        lib.spid_ref_coeffs.argtypes = [c.c_int32, c.c_int32, c.c_int32, P, P, P]
        lib.spid_ref_coeffs.restype = c.c_int
        lib.spid_ref_reconstruct.argtypes = [c.c_int64, c.c_int32, P, c.c_int64, c.c_int32,
                                             c.c_int32, c.c_int32, P, P, P, P]
        lib.spid_ref_reconstruct.restype = c.c_int
        lib.spid_ref_compression_factor.argtypes = [c.c_int32, P, P, P, P]
        lib.spid_ref_compression_factor.restype = c.c_double
        lib.spid_ref_run_batch.argtypes = [
            c.c_int32, P, P, P, P, c.c_int32, c.c_int32, c.c_int32, c.c_double, c.c_double,
            c.c_uint64, c.c_int32, c.c_int32, P, P, c.c_int32,
            P, P, P, P, P, P, P, P, P, P]
        lib.spid_ref_coarse_count.argtypes = [P]
        lib.spid_ref_coarse_count.restype = c.c_int32
        lib.spid_ref_coarse_rows.argtypes = [P, P]
        lib.spid_ref_coarse_rows.restype = c.c_int32
        lib.spid_ref_interp_row.argtypes = [P, c.c_int64, P, P]
        lib.spid_ref_interp_row.restype = c.c_int
        lib.spid_ref_subsample.argtypes = [c.c_int64, c.c_int32, P, c.c_int64, c.c_int32, P,
                                           c.c_int32, c.c_int32, c.c_int32, c.c_int32, P]
        lib.spid_ref_subsample.restype = c.c_int
        lib.spid_ref_interp_error.argtypes = [P, c.c_int64, c.c_int32, P, c.c_int64, c.c_int32,
                                              P, c.c_int32, c.c_int32, c.c_int32, P, P, P, P]
        lib.spid_ref_interp_error.restype = c.c_int
        lib.spid_ref_two_stage.argtypes = [c.c_int32, c.c_int32, P, c.c_int32, c.c_int32,
                                           c.c_double, c.c_int32, c.c_double, P, P, P, P, P]
        lib.spid_ref_two_stage.restype = c.c_int
        lib.spid_ref_run_batch.restype = c.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _a_args(A: np.ndarray):
    """Column-major view of a block: returns (array, lda, dtype code)."""
    if A.dtype == np.float64:
        code = A_F64
    elif A.dtype == np.float32:
        code = A_F32
    else:
        raise TypeError("A must be float32 or float64")
    if not A.flags.f_contiguous:
        A = np.asfortranarray(A)
    return A, A.shape[0], code


# --------------------------------------------------------------------------- RNG
def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 block function (SC'11) on one counter/key."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    _load().spid_ref_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def omega_entry(seed: int, r: int, i: int, block_key: int = 0, prec: int = OMEGA_F64) -> float:
    return _load().spid_ref_omega(seed, block_key, r, i, prec)


def omega(seed: int, l: int, m: int, block_key: int = 0, prec: int = OMEGA_F64) -> np.ndarray:
    """The l x m sketch matrix Omega (Section 2, Gaussian random projection)."""
    out = np.zeros((l, m), dtype=np.float64, order="F")
    _load().spid_ref_omega_matrix(seed, block_key, l, m, prec, _ptr(out))
    return out


def round_bf16(x: float) -> float:
    return _load().spid_ref_round_bf16(float(x))


def round_e4m3(x: float) -> float:
    return _load().spid_ref_round_e4m3(float(x))


# ------------------------------------------------------------------------ stages
def sketch(A: np.ndarray, l: int, seed: int, block_key: int = 0, prec: int = OMEGA_F64,
           j0: int = 0, w: int | None = None, Y: np.ndarray | None = None) -> np.ndarray:
    """Y(:, j0:j0+w) = Omega A(:, j0:j0+w), l x n column-major float64."""
    A, lda, code = _a_args(A)
    m, n = A.shape
    if w is None:
        w = n - j0
    if Y is None:
        Y = np.zeros((l, n), dtype=np.float64, order="F")
    rc = _load().spid_ref_sketch(m, n, _ptr(A), lda, code, l, seed, block_key, prec, j0, w, _ptr(Y))
    if rc != 0:
        raise ValueError("spid_ref_sketch: invalid arguments")
    return Y


# ------------------------------------------------------------- coarse-grid sketch
def _grid(grid) -> np.ndarray:
    g = np.ascontiguousarray(grid, dtype=np.int32)
    if g.shape != (7,):
        raise ValueError("grid = (nx, ny, nz, nfields, sx, sy, sz)")
    return g


def coarse_rows(grid) -> np.ndarray:
    """Rows J of the coarse grid (every s-th point per direction, all fields)."""
    g = _grid(grid)
    mc = _load().spid_ref_coarse_count(_ptr(g))
    if mc < 0:
        raise ValueError("invalid grid")
    J = np.zeros(mc, dtype=np.int32)
    _load().spid_ref_coarse_rows(_ptr(g), _ptr(J))
    return J


def subsample(A: np.ndarray, grid) -> np.ndarray:
    """B = A(J,:) for the grid's coarse rows J, m_c x n column-major float64."""
    A, lda, code = _a_args(A)
    m, n = A.shape
    J = coarse_rows(grid)
    Y = np.zeros((len(J), n), dtype=np.float64, order="F")
    rc = _load().spid_ref_subsample(m, n, _ptr(A), lda, code, _ptr(J), len(J), len(J), 0, n,
                                    _ptr(Y))
    if rc != 0:
        raise ValueError("spid_ref_subsample: invalid arguments")
    return Y


def interp_row(grid, i: int):
    """(coarse rows[8], weights[8]) of row i of the trilinear operator M."""
    g = _grid(grid)
    idx = np.zeros(8, dtype=np.int32)
    w = np.zeros(8, dtype=np.float64)
    if _load().spid_ref_interp_row(_ptr(g), int(i), _ptr(idx), _ptr(w)) != 0:
        raise ValueError("invalid grid or row")
    return idx, w


def interp_matrix(grid) -> np.ndarray:
    """Dense M (m x m_c), for small grids."""
    g = _grid(grid)
    m = int(g[0]) * int(g[1]) * int(g[2]) * int(g[3])
    M = np.zeros((m, len(coarse_rows(g))))
    for i in range(m):
        idx, w = interp_row(g, i)
        for c in range(8):
            M[i, idx[c]] += w[c]
    return M


def interp_error(grid, A: np.ndarray, B: np.ndarray, S: np.ndarray, k: int, P: np.ndarray):
    """(err2, nrm2) = (||A - M B(:,S) P||_F^2, ||A||_F^2), Algorithm 3's approximation."""
    g = _grid(grid)
    A, lda, code = _a_args(A)
    m, n = A.shape
    B = np.asfortranarray(B, dtype=np.float64)
    P = np.asfortranarray(P, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.int32)
    e = np.zeros(1)
    a = np.zeros(1)
    rc = _load().spid_ref_interp_error(_ptr(g), m, n, _ptr(A), lda, code, _ptr(B), B.shape[0], k,
                                       P.shape[0], _ptr(S), _ptr(P), _ptr(e), _ptr(a))
    if rc != 0:
        raise ValueError("spid_ref_interp_error: invalid arguments")
    return float(e[0]), float(a[0])


@dataclass
class Selection:
    S: np.ndarray        # int32 [k_max], pivot order, -1 past k_eff
    k: int               # number of pivots taken
    R: np.ndarray        # k_max x n, R(s, j) in original column numbering
    nu: np.ndarray       # final squared residual column norms
    gaps: np.ndarray     # relative top-two gap at every step
    status: int
    res2: float          # sum of nu = ||Y - Y(:,S) P||_F^2


def select(Y: np.ndarray, k_max: int, tol: float = 0.0, rank_floor: float = 0.0) -> Selection:
    """Rank-k (or tolerance) pivoted modified Gram-Schmidt on the sketch."""
    Y = np.asfortranarray(Y, dtype=np.float64)
    l, n = Y.shape
    S = np.full(k_max, -1, dtype=np.int32)
    k = np.zeros(1, dtype=np.int32)
    R = np.zeros((k_max, n), dtype=np.float64)  # row-major
    nu = np.zeros(n, dtype=np.float64)
    gaps = np.zeros(k_max, dtype=np.float64)
    st = np.zeros(1, dtype=np.int32)
    res2 = np.zeros(1, dtype=np.float64)
    rc = _load().spid_ref_select(l, n, _ptr(Y), k_max, tol, rank_floor, _ptr(S), _ptr(k), _ptr(R),
                                 _ptr(nu), _ptr(gaps), _ptr(st), _ptr(res2))
    if rc != 0:
        raise ValueError("spid_ref_select: invalid arguments")
    return Selection(S, int(k[0]), R, nu, gaps, int(st[0]), float(res2[0]))


def coeffs(sel: Selection, n: int) -> np.ndarray:
    """P = [I | R11^+ R12] Z^T, k_max x n column-major float64."""
    k_max = sel.S.shape[0]
    P = np.zeros((k_max, n), dtype=np.float64, order="F")
    R = np.ascontiguousarray(sel.R)
    rc = _load().spid_ref_coeffs(sel.k, k_max, n, _ptr(R), _ptr(sel.S), _ptr(P))
    if rc != 0:
        raise ValueError("spid_ref_coeffs: invalid arguments")
    return P


def reconstruct(A: np.ndarray, S: np.ndarray, k: int, P: np.ndarray):
    """(err2, nrm2) = (||A - A(:,S) P||_F^2, ||A||_F^2) against the stored A."""
    A, lda, code = _a_args(A)
    m, n = A.shape
    P = np.asfortranarray(P, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.int32)
    e = np.zeros(1)
    a = np.zeros(1)
    rc = _load().spid_ref_reconstruct(m, n, _ptr(A), lda, code, k, P.shape[0], _ptr(S), _ptr(P),
                                      _ptr(e), _ptr(a))
    if rc != 0:
        raise ValueError("spid_ref_reconstruct: invalid arguments")
    return float(e[0]), float(a[0])


def compression_factor(m, n, k, m_stored=None) -> float:
    """Equation (cf) summed over blocks; ``m_stored`` = rows of the stored skeleton
    (the coarse grid size for the single-pass ID), defaults to m."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    k = np.ascontiguousarray(k, dtype=np.int32)
    if m_stored is None:
        return _load().spid_ref_compression_factor(len(m), _ptr(m), _ptr(n), _ptr(k), None)
    ms = np.ascontiguousarray(m_stored, dtype=np.int64)
    return _load().spid_ref_compression_factor(len(m), _ptr(m), _ptr(n), _ptr(k), _ptr(ms))


@dataclass
class TwoStage:
    S: np.ndarray        # int32 [k_max], columns of A in stage-2 pivot order, -1 past k
    k: int
    status: int
    P: np.ndarray        # k_max x n, C^1 C^{0'}
    gaps: np.ndarray     # stage-2 relative top-two gaps


def two_stage(Y: np.ndarray, nwin: int, k1: int, k_max: int, tol2: float,
              rank_floor: float = 0.0) -> TwoStage:
    """Modified (two-stage) ID on a block's sketch Y (Section 3.4.2)."""
    Y = np.asfortranarray(Y, dtype=np.float64)
    l, n = Y.shape
    S = np.full(k_max, -1, dtype=np.int32)
    k = np.zeros(1, dtype=np.int32)
    st = np.zeros(1, dtype=np.int32)
    P = np.zeros((k_max, n), dtype=np.float64, order="F")
    gaps = np.zeros(k_max, dtype=np.float64)
    rc = _load().spid_ref_two_stage(l, n, _ptr(Y), nwin, k1, rank_floor, k_max, tol2, _ptr(S),
                                    _ptr(k), _ptr(st), _ptr(P), _ptr(gaps))
    if rc != 0:
        raise ValueError("spid_ref_two_stage: invalid arguments")
    return TwoStage(S, int(k[0]), int(st[0]), P, gaps)


@dataclass
class BatchResult:
    Y: list
    S: np.ndarray        # [nblocks, k_max]
    k: np.ndarray        # [nblocks]
    status: np.ndarray   # [nblocks]
    P: list              # per block k_max x n_b
    gaps: np.ndarray     # [nblocks, k_max]
    err2: np.ndarray
    nrm2: np.ndarray
    ierr2: np.ndarray | None = None   # single-pass (interpolated) error, grids only

    @property
    def rel_error(self) -> float:
        return float(np.sqrt(self.err2.sum() / self.nrm2.sum()))

    @property
    def rel_interp_error(self) -> float:
        return float(np.sqrt(self.ierr2.sum() / self.nrm2.sum()))


def run_batch(blocks, l: int, k_max: int, seed: int, tol: float = 0.0, rank_floor: float = 0.0,
              omega_per_block: bool = False, prec: int = OMEGA_F64,
              block_ids=None, nthreads: int | None = None, grids=None) -> BatchResult:
    """The whole pipeline on a list of column-major blocks, one thread pool.

    ``block_ids`` gives each block's index in the full batch (it keys Omega
    when ``omega_per_block``); defaults to 0..len-1.  ``grids`` (one
    ``(nx, ny, nz, nfields, sx, sy, sz)`` per block) switches the sketch to the
    coarse-grid subsample B = A(J,:) (SubID) and adds the single-pass error
    (``ierr2``); l must then be at least every block's m_c.
    """
    blocks = [np.asfortranarray(b) for b in blocks]
    dt = blocks[0].dtype
    if any(b.dtype != dt for b in blocks):
        raise TypeError("all blocks must share a dtype")
    code = A_F64 if dt == np.float64 else A_F32
    nb = len(blocks)
    m = np.array([b.shape[0] for b in blocks], dtype=np.int64)
    n = np.array([b.shape[1] for b in blocks], dtype=np.int32)
    lda = m.copy()
    ptrs = (ctypes.c_void_p * nb)(*[b.ctypes.data for b in blocks])
    offY = np.zeros(nb, dtype=np.int64)
    offP = np.zeros(nb, dtype=np.int64)
    offY[1:] = np.cumsum(l * n[:-1].astype(np.int64))
    offP[1:] = np.cumsum(k_max * n[:-1].astype(np.int64))
    Y = np.zeros(int(l * n.astype(np.int64).sum()), dtype=np.float64)
    P = np.zeros(int(k_max * n.astype(np.int64).sum()), dtype=np.float64)
    S = np.full((nb, k_max), -1, dtype=np.int32)
    k = np.zeros(nb, dtype=np.int32)
    st = np.zeros(nb, dtype=np.int32)
    gaps = np.zeros((nb, k_max), dtype=np.float64)
    err2 = np.zeros(nb)
    nrm2 = np.zeros(nb)
    if nthreads is None:
        nthreads = len(os.sched_getaffinity(0))
    g_arr = None
    ierr2 = None
    if grids is not None:
        g_arr = np.ascontiguousarray(np.asarray(grids, dtype=np.int32).reshape(nb, 7))
        ierr2 = np.zeros(nb)
    if block_ids is not None and omega_per_block and grids is None:
        # per-block keys follow the caller's numbering: run blocks one by one
        for idx, (blk, bid) in enumerate(zip(blocks, block_ids)):
            bkey = int(bid) + 1
            Yb = sketch(blk, l, seed, block_key=bkey, prec=prec)
            sel = select(Yb, k_max, tol, rank_floor)
            Pb = coeffs(sel, blk.shape[1])
            e2, a2 = reconstruct(blk, sel.S, sel.k, Pb)
            Y[offY[idx]:offY[idx] + Yb.size] = Yb.ravel(order="F")
            P[offP[idx]:offP[idx] + Pb.size] = Pb.ravel(order="F")
            S[idx] = sel.S
            k[idx] = sel.k
            st[idx] = sel.status
            gaps[idx] = sel.gaps
            err2[idx], nrm2[idx] = e2, a2
    else:
        rc = _load().spid_ref_run_batch(nb, _ptr(m), _ptr(n), ptrs, _ptr(lda), code, l, k_max, tol,
                                        rank_floor, seed, int(bool(omega_per_block)), prec,
                                        _ptr(offY), _ptr(offP), int(nthreads), _ptr(Y), _ptr(S),
                                        _ptr(k), _ptr(st), _ptr(P), _ptr(gaps), _ptr(err2),
                                        _ptr(nrm2), None if g_arr is None else _ptr(g_arr),
                                        None if ierr2 is None else _ptr(ierr2))
        if rc != 0:
            raise ValueError("spid_ref_run_batch: invalid arguments")
    Ys = [Y[offY[b]:offY[b] + l * n[b]].reshape((l, n[b]), order="F") for b in range(nb)]
    Ps = [P[offP[b]:offP[b] + k_max * n[b]].reshape((k_max, n[b]), order="F") for b in range(nb)]
    return BatchResult(Ys, S, k, st, Ps, gaps, err2, nrm2, ierr2)
