"""Python binding of the gfx950 sketched column-ID library (``libspid.so``).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI of ``include/spid.h``.  PyTorch supplies device memory and
streams.  Importing this package on a machine without the built library raises
immediately; there is no CPU fallback.

The functions carry the C names (``spid_workspace_bytes``, ``spid_create``,
``spid_bind_A``, ``spid_sketch_update``, ``spid_select``, ``spid_coeffs``,
``spid_reconstruct``, ``spid_copy_sketch``, ``spid_destroy``,
``spid_last_error``, the launch-shape variants ``spid_workspace_bytes_tuned``,
``spid_create_tuned``, ``spid_get_tuning``, ``spid_reconstruct_interp`` of the
coarse-grid sketch and ``spid_select_two_stage`` of the modified two-stage ID);
:class:`SPID` bundles them for a batch of blocks.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspid.so")

SPID_OK, SPID_EINVAL, SPID_EWORKSPACE, SPID_EHIP, SPID_ESTATE = 0, -1, -2, -3, -4
BLOCK_OK, BLOCK_RANK_DEFICIENT, BLOCK_NONFINITE, BLOCK_TOL_NOT_MET = 0, 1, 2, 3
A_F64, A_F32 = 0, 1
SK_F64, SK_BF16, SK_FP8E4M3, SK_SUBSAMPLE = 0, 1, 2, 3

EXPORTS = ("spid_workspace_bytes", "spid_workspace_bytes_tuned", "spid_create",
           "spid_create_tuned", "spid_get_tuning", "spid_bind_A", "spid_sketch_update",
           "spid_select", "spid_coeffs", "spid_reconstruct", "spid_copy_sketch",
           "spid_destroy", "spid_last_error", "spid_reconstruct_interp",
           "spid_select_two_stage", "spid_create_static")


class SpidError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"spid status {status}: {msg}")
        self.status = status


class spid_grid(ctypes.Structure):
    _fields_ = [(f, ctypes.c_int32) for f in ("nx", "ny", "nz", "nfields", "sx", "sy", "sz")]


class spid_desc(ctypes.Structure):
    _fields_ = [
        ("nblocks", ctypes.c_int32),
        ("h_m", ctypes.POINTER(ctypes.c_int64)),
        ("h_n", ctypes.POINTER(ctypes.c_int32)),
        ("l", ctypes.c_int32),
        ("k_max", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("rank_floor", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("omega_per_block", ctypes.c_int32),
        ("a_dtype", ctypes.c_int32),
        ("prec", ctypes.c_int32),
        ("lp_terms", ctypes.c_int32),
        ("h_grid", ctypes.c_void_p),
        ("ts_windows", ctypes.c_int32),
        ("ts_k1", ctypes.c_int32),
    ]


class spid_tuning(ctypes.Structure):
    _fields_ = [
        ("sk_tn", ctypes.c_int32),
        ("sk_nw", ctypes.c_int32),
        ("sk_items", ctypes.c_int32),
        ("rc_rpi", ctypes.c_int32),
        ("st_groups", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


def make_tuning(t=None):
    """A spid_tuning from a dict (missing keys = 0 = library default), or None."""
    if t is None:
        return None
    tu = spid_tuning()
    for f, _ in spid_tuning._fields_:
        setattr(tu, f, int(t.get(f, 0)))
    return tu


_lib = None


def load_library(path: str = LIB_PATH):
    """Load ``libspid.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build it with paper_2103_01380_amd._build.build() "
            "(hipcc --offload-arch=gfx950); there is no fallback path")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    D = ctypes.POINTER(spid_desc)
    lib.spid_workspace_bytes.argtypes = [D]
    lib.spid_workspace_bytes.restype = ctypes.c_size_t
    T = ctypes.POINTER(spid_tuning)
    lib.spid_workspace_bytes_tuned.argtypes = [D, T]
    lib.spid_workspace_bytes_tuned.restype = ctypes.c_size_t
    lib.spid_create.argtypes = [D, P, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.spid_create.restype = ctypes.c_int
    lib.spid_create_tuned.argtypes = [D, T, P, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.spid_create_tuned.restype = ctypes.c_int
    lib.spid_create_static.argtypes = [D, T, ctypes.POINTER(P)]
    lib.spid_create_static.restype = ctypes.c_int
    lib.spid_get_tuning.argtypes = [P, T]
    lib.spid_get_tuning.restype = ctypes.c_int
    lib.spid_bind_A.argtypes = [P, P, P]
    lib.spid_bind_A.restype = ctypes.c_int
    lib.spid_sketch_update.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P]
    lib.spid_sketch_update.restype = ctypes.c_int
    lib.spid_select.argtypes = [P, P, P, P, P]
    lib.spid_select.restype = ctypes.c_int
    lib.spid_coeffs.argtypes = [P, P, P]
    lib.spid_coeffs.restype = ctypes.c_int
    lib.spid_reconstruct.argtypes = [P, P, P, P, P, P]
    lib.spid_reconstruct.restype = ctypes.c_int
    lib.spid_reconstruct_interp.argtypes = [P, P, P, P, P, P]
    lib.spid_reconstruct_interp.restype = ctypes.c_int
    lib.spid_select_two_stage.argtypes = [P, P, P, P, P, P]
    lib.spid_select_two_stage.restype = ctypes.c_int
    lib.spid_copy_sketch.argtypes = [P, P, P]
    lib.spid_copy_sketch.restype = ctypes.c_int
    lib.spid_destroy.argtypes = [P]
    lib.spid_destroy.restype = ctypes.c_int
    lib.spid_last_error.argtypes = []
    lib.spid_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def spid_last_error() -> str:
    return load_library().spid_last_error().decode()


def _check(st: int):
    if st != SPID_OK:
        raise SpidError(st, spid_last_error())


def _ptr(t):
    """Device (or host) address of a torch tensor, or None."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def make_desc(m, n, l, k_max, tol=0.0, rank_floor=0.0, seed=0, omega_per_block=False,
              a_dtype=A_F64, prec=SK_F64, lp_terms=1, grids=None, ts_windows=0, ts_k1=0):
    """``grids``: ``[nblocks, 7]`` (nx, ny, nz, nfields, sx, sy, sz) for the coarse-grid
    sketch, else None."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    d = spid_desc()
    d.nblocks = len(m)
    d.h_m = m.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    d.h_n = n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.l, d.k_max, d.tol, d.rank_floor = int(l), int(k_max), float(tol), float(rank_floor)
    d.seed = int(seed)
    d.omega_per_block = int(bool(omega_per_block))
    d.a_dtype, d.prec, d.lp_terms = int(a_dtype), int(prec), int(lp_terms)
    d.ts_windows, d.ts_k1 = int(ts_windows), int(ts_k1)
    g = None
    if grids is not None:
        g = np.ascontiguousarray(np.asarray(grids, dtype=np.int32).reshape(len(m), 7))
        d.h_grid = g.ctypes.data
    d._keep = (m, n, g)    # keep the host arrays alive with the struct
    return d


# ----------------------------------------------------------------------- C names
def spid_workspace_bytes(desc: spid_desc) -> int:
    return int(load_library().spid_workspace_bytes(ctypes.byref(desc)))


def spid_workspace_bytes_tuned(desc: spid_desc, tuning) -> int:
    t = None if tuning is None else ctypes.byref(tuning)
    return int(load_library().spid_workspace_bytes_tuned(ctypes.byref(desc), t))


def spid_create(desc: spid_desc, workspace) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(load_library().spid_create(ctypes.byref(desc), _ptr(workspace),
                                      workspace.numel() * workspace.element_size(),
                                      ctypes.byref(ctx)))
    return ctx


def spid_create_tuned(desc: spid_desc, tuning, workspace) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    t = None if tuning is None else ctypes.byref(tuning)
    _check(load_library().spid_create_tuned(ctypes.byref(desc), t, _ptr(workspace),
                                            workspace.numel() * workspace.element_size(),
                                            ctypes.byref(ctx)))
    return ctx


def spid_create_static(desc: spid_desc, tuning=None) -> ctypes.c_void_p:
    """Context whose workspace is the library's static per-device array (no allocation)."""
    ctx = ctypes.c_void_p()
    t = None if tuning is None else ctypes.byref(tuning)
    _check(load_library().spid_create_static(ctypes.byref(desc), t, ctypes.byref(ctx)))
    return ctx


def spid_get_tuning(ctx) -> dict:
    t = spid_tuning()
    _check(load_library().spid_get_tuning(ctx, ctypes.byref(t)))
    return t.as_dict()


def spid_bind_A(ctx, block_ptrs, lda):
    ptrs = np.ascontiguousarray(block_ptrs, dtype=np.uint64)
    ld = np.ascontiguousarray(lda, dtype=np.int64)
    _check(load_library().spid_bind_A(ctx, ptrs.ctypes.data_as(ctypes.c_void_p),
                                      ld.ctypes.data_as(ctypes.c_void_p)))


def spid_sketch_update(ctx, j0: int, w: int, stream=None):
    _check(load_library().spid_sketch_update(ctx, int(j0), int(w), _stream(stream)))


def spid_select(ctx, k=None, S=None, status=None, stream=None):
    _check(load_library().spid_select(ctx, _ptr(k), _ptr(S), _ptr(status), _stream(stream)))


def spid_coeffs(ctx, P, stream=None):
    _check(load_library().spid_coeffs(ctx, _ptr(P), _stream(stream)))


def spid_reconstruct(ctx, P, err2, nrm2, skeleton=None, stream=None):
    _check(load_library().spid_reconstruct(ctx, _ptr(P), _ptr(err2), _ptr(nrm2),
                                           _ptr(skeleton), _stream(stream)))


def spid_reconstruct_interp(ctx, P, err2, nrm2, coarse_skeleton=None, stream=None):
    _check(load_library().spid_reconstruct_interp(ctx, _ptr(P), _ptr(err2), _ptr(nrm2),
                                                  _ptr(coarse_skeleton), _stream(stream)))


def spid_select_two_stage(ctx, P, k=None, S=None, status=None, stream=None):
    _check(load_library().spid_select_two_stage(ctx, _ptr(k), _ptr(S), _ptr(status), _ptr(P),
                                                _stream(stream)))


def spid_copy_sketch(ctx, Y, stream=None):
    _check(load_library().spid_copy_sketch(ctx, _ptr(Y), _stream(stream)))


def spid_destroy(ctx):
    _check(load_library().spid_destroy(ctx))


# ------------------------------------------------------------------- convenience
_PREC = {"f64": SK_F64, "bf16": SK_BF16, "fp8": SK_FP8E4M3, "subsample": SK_SUBSAMPLE}


def coarse_rows_count(grid) -> int:
    """m_c of one block grid (nx, ny, nz, nfields, sx, sy, sz)."""
    nx, ny, nz, nf, sx, sy, sz = (int(v) for v in grid)
    return nf * (-(-nx // sx)) * (-(-ny // sy)) * (-(-nz // sz))


class SPID:
    """A batch of blocks on the current GPU: workspace, outputs and the four stages.

    ``blocks`` is a list of device tensors (column-major blocks given as
    ``[n_b, m_b]`` contiguous tensors, i.e. transposed views of A_b) or a single
    ``[nblocks, n, m]`` tensor of equal blocks.  Outputs are torch tensors on the
    same device: ``k``, ``S`` ([nblocks, k_max]), ``status``, ``P`` (flat,
    per-block k_max x n_b column-major), ``err2``, ``nrm2``.

    ``ts_windows`` / ``ts_k1`` reserve the modified two-stage ID
    (:meth:`select_two_stage` in place of :meth:`select` + :meth:`coeffs`).

    ``static_scratch=True`` creates the context with ``spid_create_static`` (the
    library's per-device scratch array as the workspace: nothing is allocated for
    it; one such context per device at a time).

    ``prec="subsample"`` with ``grids`` (one ``(nx, ny, nz, nfields, sx, sy, sz)`` per
    block, or one for all) selects the coarse-grid sketch B = A(J,:); ``l`` then
    defaults to the largest coarse row count, and :meth:`reconstruct_interp` gives
    the single-pass error into ``err2_interp``.
    """

    def __init__(self, m, n, l, k_max, tol=0.0, rank_floor=0.0, seed=0, omega_per_block=False,
                 a_dtype="f64", prec="f64", lp_terms=1, device="cuda", tuning=None, grids=None,
                 ts_windows=0, ts_k1=0, static_scratch=False):
        import torch
        self.m = np.ascontiguousarray(m, dtype=np.int64)
        self.n = np.ascontiguousarray(n, dtype=np.int32)
        self.nblocks = len(self.m)
        self.grids = None
        if grids is not None:
            g = np.asarray(grids, dtype=np.int32)
            self.grids = np.ascontiguousarray(np.broadcast_to(g.reshape(-1, 7),
                                                              (self.nblocks, 7)))
            self.mc = np.array([coarse_rows_count(x) for x in self.grids], dtype=np.int64)
            if l is None:
                l = int(self.mc.max())
        self.l, self.k_max = int(l), int(k_max)
        self.desc = make_desc(self.m, self.n, l, k_max, tol, rank_floor, seed, omega_per_block,
                              A_F64 if a_dtype == "f64" else A_F32, _PREC[prec], lp_terms,
                              self.grids, ts_windows, ts_k1)
        self._tuning = make_tuning(tuning)
        nbytes = spid_workspace_bytes_tuned(self.desc, self._tuning)
        if nbytes == 0:
            raise SpidError(SPID_EINVAL, spid_last_error())
        self.device = torch.device(device)
        if static_scratch:
            # the library's static scratch array instead of a workspace (spid_create_static)
            self._ws_raw = self.workspace = None
            with torch.cuda.device(self.device):
                self.ctx = spid_create_static(self.desc, self._tuning)
        else:
            # 256-byte aligned workspace carved from a torch allocation
            self._ws_raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self._ws_raw.data_ptr()) % 256
            self.workspace = self._ws_raw[off:off + nbytes]
            self.ctx = spid_create_tuned(self.desc, self._tuning, self.workspace)
        self.tuning = spid_get_tuning(self.ctx)
        sum_n = int(self.n.astype(np.int64).sum())
        self.k = torch.zeros(self.nblocks, dtype=torch.int32, device=self.device)
        self.S = torch.full((self.nblocks, self.k_max), -1, dtype=torch.int32, device=self.device)
        self.status = torch.zeros(self.nblocks, dtype=torch.int32, device=self.device)
        self.P = torch.zeros(self.k_max * sum_n, dtype=torch.float64, device=self.device)
        self.err2 = torch.zeros(self.nblocks, dtype=torch.float64, device=self.device)
        self.nrm2 = torch.zeros(self.nblocks, dtype=torch.float64, device=self.device)
        self.err2_interp = torch.zeros(self.nblocks, dtype=torch.float64, device=self.device)
        self.p_off = np.zeros(self.nblocks, dtype=np.int64)
        self.p_off[1:] = np.cumsum(self.k_max * self.n[:-1].astype(np.int64))
        self.y_off = np.zeros(self.nblocks, dtype=np.int64)
        self.y_off[1:] = np.cumsum(self.l * self.n[:-1].astype(np.int64))
        self._A = None

    def bind(self, A, offsets=None, lda=None):
        """A: [nblocks, n, m] tensor of equal blocks, or a flat tensor with element
        ``offsets`` per block (each block column-major with leading dimension lda)."""
        es = A.element_size()
        base = A.data_ptr()
        if offsets is None:
            assert A.dim() == 3 and A.shape[0] == self.nblocks
            offsets = np.arange(self.nblocks, dtype=np.int64) * (A.shape[1] * A.shape[2])
            if lda is None:
                lda = np.full(self.nblocks, A.shape[2], dtype=np.int64)
        if lda is None:
            lda = self.m
        ptrs = np.asarray([base + int(o) * es for o in offsets], dtype=np.uint64)
        spid_bind_A(self.ctx, ptrs, lda)
        self._A = A

    def sketch_update(self, j0=0, w=None, stream=None):
        spid_sketch_update(self.ctx, j0, int(self.n.max()) - j0 if w is None else w, stream)

    def select(self, stream=None):
        spid_select(self.ctx, self.k, self.S, self.status, stream)

    def coeffs(self, stream=None):
        spid_coeffs(self.ctx, self.P, stream)

    def reconstruct(self, skeleton=None, stream=None):
        spid_reconstruct(self.ctx, self.P, self.err2, self.nrm2, skeleton, stream)

    def select_two_stage(self, stream=None):
        """Modified two-stage ID (needs ``ts_windows``): S, k, status and P in one call."""
        spid_select_two_stage(self.ctx, self.P, self.k, self.S, self.status, stream)

    def reconstruct_interp(self, coarse_skeleton=None, stream=None):
        """Single-pass error ||A - M B(:,S) P||^2 per block into ``err2_interp``."""
        spid_reconstruct_interp(self.ctx, self.P, self.err2_interp, self.nrm2, coarse_skeleton,
                                stream)

    def run(self, stream=None):
        """One pass of the whole method: sketch, select, coeffs, reconstruct."""
        self.sketch_update(stream=stream)
        self.select(stream)
        self.coeffs(stream)
        self.reconstruct(stream=stream)

    def sketch(self):
        import torch
        Y = torch.empty(self.l * int(self.n.astype(np.int64).sum()), dtype=torch.float64,
                        device=self.device)
        spid_copy_sketch(self.ctx, Y)
        return Y

    def block_P(self, b: int):
        """Host copy of P_b as a k_max x n_b array."""
        o, nb = int(self.p_off[b]), int(self.n[b])
        return self.P[o:o + self.k_max * nb].cpu().numpy().reshape(nb, self.k_max).T


    def close(self):
        if self.ctx is not None:
            spid_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


load_library()
