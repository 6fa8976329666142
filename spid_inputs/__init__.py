"""Seeded synthetic inputs shared by the tests, the oracle runs and the benchmark.

This module generates snapshot matrices and holds the workload descriptions.
It contains none of the compression method's arithmetic (no sketch, no
pivoted QR, no coefficients, no error pass), so the GPU library and the CPU
oracle can both be fed from it without sharing any of the method's code.

Layout of a batch of equal blocks: a tensor ``[nblocks, n, m_b]`` whose
block ``b`` is the column-major ``m_b x n`` snapshot matrix A_b (leading
dimension m_b): column j is the flattened snapshot at time t_j (Section 2 of
arXiv 2103.01380: rows are spatial values, columns are time steps).  Uneven
batches are one flat buffer with per-block element offsets.

Row order inside a block: field-major (u, v, w[, rho, p] or the fields of the
workload), then z, y, x with x fastest, local to the block.  Block id =
bx + B*(by + B*bz) on a B x B x B decomposition of the periodic grid
x_i = 2*pi*i/N (Section 3.2: the spatial domain is split into independent
sub-blocks).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch


# ----------------------------------------------------------------------------- workloads
@dataclass
class Workload:
    """One named workload: shapes, method parameters and seeds."""
    name: str
    description: str
    kind: str                     # "tgv" | "turbulence" | "lowrank"
    N: int = 0                    # grid points per direction
    B: int = 1                    # blocks per direction
    n: int = 0                    # snapshots (equal-block workloads)
    fields: int = 3
    nu: float = 0.0               # viscosity (TGV)
    T: float = 10.0               # final time (TGV)
    dt: float = 0.02              # snapshot spacing (turbulence)
    noise: float = 0.0            # relative noise amplitude
    nmodes: int = 4096
    kmax: int = 16
    a_dtype: str = "f64"          # stored A
    l: int = 0
    k_max: int = 0
    tol: float = 0.0
    prec: str = "f64"             # sketch precision: f64 | bf16 | fp8
    lp_terms: int = 1
    stream: bool = False          # one snapshot per sketch update
    data_seed: int = 0
    omega_seed: int = 0
    nblocks_uneven: int = 0       # lowrank
    subsample: int = 0            # > 0: coarse-grid sketch, every s-th point per direction
    ts_windows: int = 0           # > 0: modified two-stage ID with this many temporal windows
    ts_k1: int = 0                # two-stage: stage-1 rank per window
    extra: dict = field(default_factory=dict)

    @property
    def nblocks(self) -> int:
        if self.kind == "lowrank":
            return self.nblocks_uneven
        return self.B ** 3

    @property
    def edge(self) -> int:
        return self.N // self.B

    @property
    def m_b(self) -> int:
        return self.fields * self.edge ** 3

    @property
    def elem_bytes(self) -> int:
        return 8 if self.a_dtype == "f64" else 4

    def grids(self) -> np.ndarray:
        """Per-block grids (nx, ny, nz, fields, sx, sy, sz) of the coarse-grid sketch:
        every block is an E^3 cube (E = N / B) of ``fields`` stacked fields."""
        E, s = self.N // self.B, self.subsample
        return np.tile(np.array([E, E, E, self.fields, s, s, s], dtype=np.int32),
                       (self.nblocks, 1))

    @property
    def coarse_rows(self) -> int:
        E, s = self.N // self.B, self.subsample
        return self.fields * (-(-E // s)) ** 3


WORKLOADS = {
    # analytic TGV, one block, fixed rank 8, l = k + 10, double precision
    "tgv32_single_f64": Workload(
        name="tgv32_single_f64",
        description="analytic TGV 32^3 (u,v,w), 64 snapshots in [0,10], nu=0.01, one block, "
                    "k=8, l=18, FP64 sketch",
        kind="tgv", N=32, B=1, n=64, fields=3, nu=0.01, T=10.0, a_dtype="f64",
        l=18, k_max=8, prec="f64", data_seed=2001, omega_seed=1001),
    # analytic TGV + 1e-6 noise, 512 blocks of 16^3, tolerance 1e-8 capped at k=32, l=42
    "tgv128_b512_f64": Workload(
        name="tgv128_b512_f64",
        description="analytic TGV 128^3 (u,v,w) + 1e-6 relative Gaussian noise, 512 blocks of "
                    "16^3 (m_b=12288), 256 snapshots in [0,10], nu=0.005, tolerance 1e-8 with "
                    "k<=32, l=42, FP64 sketch",
        kind="tgv", N=128, B=8, n=256, fields=3, nu=0.005, T=10.0, noise=1e-6, a_dtype="f64",
        l=42, k_max=32, tol=1e-8, prec="f64", data_seed=2002, omega_seed=1002),
    # turbulence-like field, 4096 blocks of 16^3, k=32, l=48, BF16 sketch
    "turb256_b4096_bf16": Workload(
        name="turb256_b4096_bf16",
        description="turbulence-like 256^3 (rho,u,v,w,p) FP32, 4096 Fourier modes |k|<=16 with "
                    "-5/3 spectrum, 512 snapshots dt=0.02, 4096 blocks of 16^3 (m_b=20480), "
                    "k=32, l=48, BF16 sketch",
        kind="turbulence", N=256, B=16, n=512, fields=5, dt=0.02, a_dtype="f32",
        l=48, k_max=32, prec="bf16", lp_terms=2, data_seed=2003, omega_seed=1003),
    # uneven low-rank batch
    "lowrank_uneven2000_bf16": Workload(
        name="lowrank_uneven2000_bf16",
        description="2000 blocks, edge log-uniform in [4,32] (m_b=5*edge^3), n_b log-uniform in "
                    "[128,1024], rank U{2..40}, sigma_i=10^(-i/4), FP32; tolerance 1e-4 with "
                    "k<=40, l=50, BF16 sketch",
        kind="lowrank", fields=5, a_dtype="f32", l=50, k_max=40, tol=1e-4, prec="bf16",
        lp_terms=2, nblocks_uneven=2000, data_seed=2004, omega_seed=1004),
    # large resident set, streamed one snapshot at a time, FP8 sketch
    "turb256_b32768_fp8_stream": Workload(
        name="turb256_b32768_fp8_stream",
        description="turbulence-like 256^3 (rho,u,v,w,p) FP32, 384 snapshots, 32768 blocks of "
                    "8^3 (m_b=2560), k=64, l=96, FP8-e4m3 sketch, one snapshot per update",
        kind="turbulence", N=256, B=32, n=384, fields=5, dt=0.02, a_dtype="f32",
        l=96, k_max=64, prec="fp8", lp_terms=3, stream=True, data_seed=2005, omega_seed=1005),
    # counter runs of the BF16 sketch at the BF16 turbulence workload's block shape
    # (20480 x 512, l = 48, k = 32) on 512 synthetic low-rank blocks (21.5 GB)
    "lowrank_b512_bf16": Workload(
        name="lowrank_b512_bf16",
        description="512 blocks of 20480 x 512 (5 fields x 16^3, the BF16 turbulence block "
                    "shape), rank 40 with Gaussian factors, sigma_i=10^(-i/4), FP32; k=32, "
                    "l=48, BF16 sketch",
        kind="lowrank", fields=5, a_dtype="f32", l=48, k_max=32, prec="bf16", lp_terms=2,
        nblocks_uneven=512, data_seed=2007, omega_seed=1007,
        extra={"shape": {"edge_range": (16, 16), "n_range": (512, 512), "rank_range": (40, 40)},
               "orthonormal": False}),
    # the paper's own sketch (Section 2, Algorithms 2-3; Section 5.2.3's 64^3 single
    # partition at interval 3): coarse-grid subsample, trilinear single-pass error
    "tgv64_single_sub3": Workload(
        name="tgv64_single_sub3",
        description="analytic TGV 64^3 (u,v,w), 100 snapshots in [0,10], nu=0.01, one block, "
                    "coarse-grid sketch every 3rd point per direction (3*22^3=31944 rows), "
                    "tolerance 1e-10 with k<=4, single-pass (trilinear) error",
        kind="tgv", N=64, B=1, n=100, fields=3, nu=0.01, T=10.0, a_dtype="f64",
        l=31944, k_max=4, tol=1e-10, prec="subsample", subsample=3, data_seed=2006),
    # the 512-block TGV data of the double-precision Gaussian workload, coarse-grid sketch
    "tgv128_b512_sub3": Workload(
        name="tgv128_b512_sub3",
        description="analytic TGV 128^3 (u,v,w) + 1e-6 relative Gaussian noise, 512 blocks of "
                    "16^3 (m_b=12288), 256 snapshots in [0,10], nu=0.005, coarse-grid sketch "
                    "every 3rd point (648 rows), tolerance 1e-8 with k<=32, single-pass error",
        kind="tgv", N=128, B=8, n=256, fields=3, nu=0.005, T=10.0, noise=1e-6, a_dtype="f64",
        l=648, k_max=32, tol=1e-8, prec="subsample", subsample=3, data_seed=2002),
    # the 512-block TGV data compressed by the modified two-stage ID (Section 3.4.2):
    # 8 windows of 32 snapshots at rank 16, then a tolerance ID of the 128 window skeletons
    "tgv128_b512_f64_2stage": Workload(
        name="tgv128_b512_f64_2stage",
        description="as tgv128_b512_f64, modified two-stage ID: 8 temporal windows of 32 "
                    "snapshots at rank 16, stage 2 with tolerance 1e-8 and k<=32, l=42",
        kind="tgv", N=128, B=8, n=256, fields=3, nu=0.005, T=10.0, noise=1e-6, a_dtype="f64",
        l=42, k_max=32, tol=1e-8, prec="f64", data_seed=2002, omega_seed=1002,
        ts_windows=8, ts_k1=16),
    "tgv128_b512_sub7": Workload(
        name="tgv128_b512_sub7",
        description="as tgv128_b512_sub3 with every 7th point (3*3^3=81 coarse rows)",
        kind="tgv", N=128, B=8, n=256, fields=3, nu=0.005, T=10.0, noise=1e-6, a_dtype="f64",
        l=81, k_max=32, tol=1e-8, prec="subsample", subsample=7, data_seed=2002),
}


def scaled(w: Workload, **changes) -> Workload:
    """A copy of a workload with some fields changed (smaller test cases)."""
    d = dict(w.__dict__)
    d.update(changes)
    return Workload(**d)


# ----------------------------------------------------------------------------- TGV
def tgv_times(n: int, T: float) -> np.ndarray:
    """Snapshot times t_j = T j / (n - 1), endpoints included."""
    if n == 1:
        return np.zeros(1)
    return T * np.arange(n, dtype=np.float64) / (n - 1)


def _block_coords(N: int, B: int, device, dtype):
    """Per block, the local grid coordinates (z, y, x fastest) as [nb, E^3] tensors."""
    E = N // B
    h = 2.0 * math.pi / N
    loc = torch.arange(E, device=device, dtype=torch.int64)
    bidx = torch.arange(B, device=device, dtype=torch.int64)
    # global index of local point l in block coordinate b: b*E + l
    g = (bidx[:, None] * E + loc[None, :]).to(dtype) * h       # [B, E]
    nb = B ** 3
    b = torch.arange(nb, device=device)
    bx, by, bz = b % B, (b // B) % B, b // (B * B)
    X = g[bx][:, None, None, :].expand(nb, E, E, E)            # x fastest
    Y = g[by][:, None, :, None].expand(nb, E, E, E)
    Z = g[bz][:, :, None, None].expand(nb, E, E, E)
    return X.reshape(nb, -1), Y.reshape(nb, -1), Z.reshape(nb, -1)


def tgv_blocks(w: Workload, device="cpu", dtype=torch.float64, block_range=None) -> torch.Tensor:
    """Analytic 3D Taylor-Green vortex snapshots, [nblocks, n, m_b].

    u = sin x cos y cos z e^{-3 nu t}, v = -cos x sin y cos z e^{-3 nu t}, w = 0.
    With ``w.noise > 0``, adds noise * RMS(A_clean over the whole grid) * N(0,1),
    drawn from a torch generator seeded with ``w.data_seed`` (on ``device``).
    ``block_range=(b0, b1)`` returns only those blocks (the noise is then
    drawn for the sub-range only, so use it for noise-free fields).
    """
    assert w.fields == 3
    N, B, n = w.N, w.B, w.n
    X, Y, Z = _block_coords(N, B, device, torch.float64)
    if block_range is not None:
        b0, b1 = block_range
        X, Y, Z = X[b0:b1], Y[b0:b1], Z[b0:b1]
    fu = torch.sin(X) * torch.cos(Y) * torch.cos(Z)
    fv = -torch.cos(X) * torch.sin(Y) * torch.cos(Z)
    fw = torch.zeros_like(fu)
    F = torch.cat([fu, fv, fw], dim=1)                         # [nb, m_b]
    t = torch.as_tensor(tgv_times(n, w.T), device=device)
    g = torch.exp(-3.0 * w.nu * t)                             # [n]
    nb = F.shape[0]
    out = torch.empty((nb, n, F.shape[1]), device=device, dtype=dtype)
    for j in range(n):
        out[:, j, :] = (F * g[j]).to(dtype)
    if w.noise > 0:
        rms = math.sqrt(float((F.double() ** 2).mean()) * float((g.double() ** 2).mean()))
        gen = torch.Generator(device=device)
        gen.manual_seed(w.data_seed)
        amp = w.noise * rms
        for b in range(nb):
            out[b] += amp * torch.randn(out[b].shape, generator=gen, device=device, dtype=dtype)
    return out


def tgv_clean_rms(w: Workload) -> float:
    """RMS of the noise-free TGV data matrix over the whole grid (closed form).

    Over a periodic grid with N >= 3, mean(sin^2 x cos^2 y cos^2 z) = 1/8, the
    same for v, and w = 0: mean over the three fields = 1/12 of the time factor.
    """
    t = tgv_times(w.n, w.T)
    return math.sqrt((1.0 / 12.0) * float(np.mean(np.exp(-6.0 * w.nu * t))))


# ----------------------------------------------------------------------------- turbulence
@dataclass
class Modes:
    kappa: np.ndarray     # [M, 3] integer wavevectors (half space, distinct)
    amp: np.ndarray       # [M] |kappa|^(-11/6) normalised
    omega: np.ndarray     # [M] |kappa|^(2/3)
    pol: np.ndarray       # [M, 3] unit vectors orthogonal to kappa
    phase: np.ndarray     # [3, M] phases for velocity, rho, p
    samp: np.ndarray      # [2, M] scalar amplitudes (rho, p)


def turbulence_modes(nmodes: int, kmax: int, seed: int) -> Modes:
    """Draw the random Fourier modes of the turbulence-like field.

    Integer wavevectors with 1 <= |kappa| <= kmax, one of each +-kappa pair,
    drawn uniformly without replacement; amplitude |kappa|^(-11/6) so that the
    shell energy ~ |kappa|^2 * amp^2 ~ |kappa|^(-5/3); frequency |kappa|^(2/3);
    velocity polarisation a random unit vector orthogonal to kappa
    (divergence free); independent uniform phases.
    """
    rng = np.random.default_rng(seed)
    r = np.arange(-kmax, kmax + 1)
    K = np.stack(np.meshgrid(r, r, r, indexing="ij"), axis=-1).reshape(-1, 3)
    k2 = (K ** 2).sum(1)
    keep = (k2 >= 1) & (k2 <= kmax * kmax)
    # half space: first nonzero component positive
    first = np.where(K[:, 2] != 0, K[:, 2], np.where(K[:, 1] != 0, K[:, 1], K[:, 0]))
    keep &= first > 0
    K = K[keep]
    if nmodes > len(K):
        raise ValueError(f"only {len(K)} half-space modes with |k| <= {kmax}")
    idx = rng.choice(len(K), size=nmodes, replace=False)
    idx.sort()
    kap = K[idx].astype(np.int64)
    kn = np.sqrt((kap ** 2).sum(1).astype(np.float64))
    amp = kn ** (-11.0 / 6.0)
    omega = kn ** (2.0 / 3.0)
    v = rng.standard_normal((nmodes, 3))
    khat = kap / kn[:, None]
    v -= (v * khat).sum(1, keepdims=True) * khat
    pol = v / np.linalg.norm(v, axis=1, keepdims=True)
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(3, nmodes))
    samp = rng.uniform(0.5, 1.5, size=(2, nmodes))
    # normalise the velocity so that its mean square over the grid is ~1
    # (mean of cos^2 is 1/2 for every nonzero integer mode)
    ms = 0.5 * (amp ** 2).sum()
    amp = amp / math.sqrt(3.0 * ms)
    return Modes(kap, amp, omega, pol, phase, samp)


def _field_coeffs(modes: Modes):
    """Per field (rho, u, v, w, p): amplitude [M] and phase [M] of each mode;
    rho = 1 + 0.05 s_rho, p = 1 + 0.1 s_p with s normalised scalar sums."""
    a = modes.amp
    scal = []
    for q in range(2):
        s = a * modes.samp[q]
        s = s / math.sqrt(0.5 * (s ** 2).sum())
        scal.append(s)
    amps = [0.05 * scal[0], a * modes.pol[:, 0], a * modes.pol[:, 1], a * modes.pol[:, 2],
            0.1 * scal[1]]
    phases = [modes.phase[1], modes.phase[0], modes.phase[0], modes.phase[0], modes.phase[2]]
    offsets = [1.0, 0.0, 0.0, 0.0, 1.0]
    return amps, phases, offsets


def turbulence_direct(w: Workload, points: np.ndarray, t: np.ndarray, modes: Modes | None = None):
    """Direct mode sum at grid points (integer indices [P, 3] as (x, y, z)) and times t.

    Returns [5, P, len(t)] float64.  Used to validate the FFT generator.
    """
    modes = modes or turbulence_modes(w.nmodes, w.kmax, w.data_seed)
    h = 2.0 * math.pi / w.N
    x = points.astype(np.float64) * h
    amps, phases, offsets = _field_coeffs(modes)
    arg_x = x @ modes.kappa.T.astype(np.float64)               # [P, M]
    out = np.zeros((5, len(points), len(t)))
    for f in range(5):
        for jt, tt in enumerate(t):
            out[f, :, jt] = offsets[f] + (amps[f][None, :] * np.cos(
                arg_x + phases[f][None, :] - modes.omega[None, :] * tt)).sum(1)
    return out


def turbulence_blocks(w: Workload, device="cpu", out_dtype=torch.float32,
                      modes: Modes | None = None, progress=None) -> torch.Tensor:
    """Turbulence-like snapshots, [nblocks, n, m_b] in ``out_dtype``.

    Each snapshot of each field is one inverse real FFT of the sparse mode
    spectrum on the N^3 grid (double precision), then scattered into the
    block layout.  Snapshot times t_j = dt * j.
    """
    assert w.fields == 5
    modes = modes or turbulence_modes(w.nmodes, w.kmax, w.data_seed)
    N, B, n, E = w.N, w.B, w.n, w.edge
    if 2 * w.kmax + 1 > N:
        raise ValueError("grid too coarse for kmax")
    amps, phases, offsets = _field_coeffs(modes)
    kap = modes.kappa
    # rfft half spectrum indices: last axis is z? torch.fft.irfftn over dims (0,1,2) treats the
    # LAST dim as the halved one.  Our array axes are (z, y, x); exp(i k.x) with x fastest, so
    # axis 2 is x.  Store modes at [kz, ky, kx] with kx >= 0 (use -kappa if kx < 0).
    kx, ky, kz = kap[:, 0], kap[:, 1], kap[:, 2]
    flip = kx < 0
    on_plane = kx == 0
    sx = np.where(flip, -kx, kx)
    sy = np.where(flip, -ky, ky) % N
    sz = np.where(flip, -kz, kz) % N
    sgn = np.where(flip, -1.0, 1.0)
    # conjugate partner for modes on the kx = 0 plane
    py_ = (-np.where(flip, -ky, ky)) % N
    pz_ = (-np.where(flip, -kz, kz)) % N
    dev = torch.device(device)
    sx_t = torch.as_tensor(sx, device=dev)
    sy_t = torch.as_tensor(sy, device=dev)
    sz_t = torch.as_tensor(sz, device=dev)
    pl = torch.as_tensor(np.nonzero(on_plane)[0], device=dev)
    py_t = torch.as_tensor(py_, device=dev)[pl]
    pz_t = torch.as_tensor(pz_, device=dev)[pl]
    om = torch.as_tensor(modes.omega, device=dev)
    sgn_t = torch.as_tensor(sgn, device=dev)
    nb = B ** 3
    out = torch.empty((nb, n, w.m_b), device=dev, dtype=out_dtype)
    scale = float(N) ** 3 / 2.0
    H = torch.zeros((N, N, N // 2 + 1), device=dev, dtype=torch.complex128)
    for f in range(5):
        a_t = torch.as_tensor(amps[f], device=dev)
        ph_t = torch.as_tensor(phases[f], device=dev)
        for j in range(n):
            tt = w.dt * j
            ang = sgn_t * (ph_t - om * tt)
            c = torch.polar(a_t * scale, ang)
            H.zero_()
            H[sz_t, sy_t, sx_t] = c
            if len(pl):
                H[pz_t, py_t, sx_t[pl]] = torch.conj(c[pl])
            g = torch.fft.irfftn(H, s=(N, N, N), dim=(0, 1, 2)) + offsets[f]   # [z, y, x]
            blk = g.reshape(B, E, B, E, B, E).permute(0, 2, 4, 1, 3, 5).reshape(nb, E ** 3)
            out[:, j, f * E ** 3:(f + 1) * E ** 3] = blk.to(out_dtype)
            if progress is not None:
                progress(f, j)
    return out


# ----------------------------------------------------------------------------- low rank uneven
@dataclass
class UnevenBatch:
    m: np.ndarray          # int64 [nb]
    n: np.ndarray          # int32 [nb]
    rank: np.ndarray       # int32 [nb]
    offsets: np.ndarray    # int64 [nb] element offsets into the flat buffer
    total: int             # elements


def lowrank_shapes(w: Workload, nblocks: int | None = None, edge_range=(4, 32),
                   n_range=(128, 1024), rank_range=(2, 40)) -> UnevenBatch:
    """Block shapes of the uneven batch: edge and n_b log-uniform, rank uniform."""
    nb = nblocks or w.nblocks_uneven
    rng = np.random.default_rng(w.data_seed)
    e = np.rint(np.exp(rng.uniform(math.log(edge_range[0]), math.log(edge_range[1]), nb)))
    e = e.astype(np.int64)
    nn = np.rint(np.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1]), nb)))
    nn = nn.astype(np.int32)
    r = rng.integers(rank_range[0], rank_range[1] + 1, nb).astype(np.int32)
    m = (w.fields * e ** 3).astype(np.int64)
    r = np.minimum(r, np.minimum(m, nn)).astype(np.int32)
    sizes = m * nn.astype(np.int64)
    off = np.zeros(nb, dtype=np.int64)
    off[1:] = np.cumsum(sizes[:-1])
    return UnevenBatch(m, nn, r, off, int(sizes.sum()))


def lowrank_blocks(w: Workload, shapes: UnevenBatch, device="cpu", out_dtype=torch.float32,
                   decay=0.25, orthonormal=True) -> torch.Tensor:
    """Flat buffer of the uneven low-rank batch.

    A_b = U_b diag(sigma) V_b^T with U_b (m_b x r_b) and V_b (n_b x r_b)
    orthonormal (QR of Gaussian matrices, double precision) and
    sigma_i = 10^(-decay * i), i = 0..r_b-1.  Block b is column-major
    m_b x n_b at ``shapes.offsets[b]``.  ``orthonormal=False`` uses the
    Gaussian factors scaled by 1/sqrt(rows) instead (nearly orthonormal, no QR).
    """
    dev = torch.device(device)
    out = torch.empty(shapes.total, device=dev, dtype=out_dtype)
    gen = torch.Generator(device=dev)
    gen.manual_seed(w.data_seed)
    for b in range(len(shapes.m)):
        m, n, r = int(shapes.m[b]), int(shapes.n[b]), int(shapes.rank[b])
        U = torch.randn((m, r), generator=gen, device=dev, dtype=torch.float64)
        V = torch.randn((n, r), generator=gen, device=dev, dtype=torch.float64)
        if orthonormal:
            U, V = torch.linalg.qr(U)[0], torch.linalg.qr(V)[0]
        else:
            U, V = U / math.sqrt(m), V / math.sqrt(n)
        sig = 10.0 ** (-decay * torch.arange(r, device=dev, dtype=torch.float64))
        Ab = (U * sig[None, :]) @ V.T                            # m x n
        o = int(shapes.offsets[b])
        out[o:o + m * n] = Ab.T.contiguous().reshape(-1).to(out_dtype)   # column-major
    return out


# ----------------------------------------------------------------------------- helpers
def generate(w: Workload, device="cpu", progress=None):
    """Generate a workload's A.  Returns (tensor, m[], n[], offsets[]) with
    offsets in elements into the flattened tensor."""
    if w.kind == "tgv":
        A = tgv_blocks(w, device=device, dtype=torch.float64 if w.a_dtype == "f64" else torch.float32)
    elif w.kind == "turbulence":
        A = turbulence_blocks(w, device=device, progress=progress,
                              out_dtype=torch.float32 if w.a_dtype == "f32" else torch.float64)
    elif w.kind == "lowrank":
        sh = lowrank_shapes(w, **w.extra.get("shape", {}))
        A = lowrank_blocks(w, sh, device=device,
                           out_dtype=torch.float32 if w.a_dtype == "f32" else torch.float64,
                           orthonormal=w.extra.get("orthonormal", True))
        return A, sh.m, sh.n, sh.offsets
    else:
        raise ValueError(w.kind)
    nb = A.shape[0]
    m = np.full(nb, A.shape[2], dtype=np.int64)
    n = np.full(nb, A.shape[1], dtype=np.int32)
    off = np.arange(nb, dtype=np.int64) * (A.shape[1] * A.shape[2])
    return A, m, n, off


def gaussian_like(w: Workload, device="cpu", seed: int | None = None):
    """A batch with the workload's block shapes and data type but i.i.d. N(0, 1)
    entries, drawn with a handful of generator calls (profiling runs, where the
    streaming kernels' traffic and instruction counts do not depend on the
    values; the selection then takes k_max pivots in every block).  Returns
    (tensor, m[], n[], offsets[]) as ``generate``."""
    dt = torch.float32 if w.a_dtype == "f32" else torch.float64
    gen = torch.Generator(device=device)
    gen.manual_seed(w.data_seed if seed is None else seed)
    if w.kind == "lowrank":
        sh = lowrank_shapes(w, **w.extra.get("shape", {}))
        m, n, off, total = sh.m, sh.n, sh.offsets, sh.total
        A = torch.empty(total, device=device, dtype=dt)
    else:
        nb = w.nblocks
        m = np.full(nb, w.m_b, dtype=np.int64)
        n = np.full(nb, w.n, dtype=np.int32)
        off = np.arange(nb, dtype=np.int64) * (w.n * w.m_b)
        A = torch.empty((nb, w.n, w.m_b), device=device, dtype=dt)
    flat = A.view(-1)
    chunk = 1 << 30
    for o in range(0, flat.numel(), chunk):
        flat[o:o + chunk].normal_(generator=gen)
    return A, m, n, off


def block_view(A: torch.Tensor, m, n, off, b: int) -> np.ndarray:
    """Host numpy column-major view (copy) of block b."""
    flat = A.reshape(-1)
    mb, nb_ = int(m[b]), int(n[b])
    o = int(off[b])
    v = flat[o:o + mb * nb_].detach().cpu().numpy()
    return np.asfortranarray(v.reshape(nb_, mb).T)


# ----------------------------------------------------------------------------- 2D TGV
def tgv2d_u1(npts: int, n: int, T: float = 10.0, nu: float = 0.01, unstructured: bool = False,
             seed: int = 0, blocks=(1, 1)):
    """u1 of the 2D incompressible Taylor-Green vortex (Section 5.1 of arXiv 2103.01380),
    u1 = sin x1 cos x2 exp(-2 nu t) on [0, 2 pi)^2, npts^2 points (a structured grid, or
    uniform random points when ``unstructured``), n snapshots uniform in [0, T].

    Returns a list of column-major float64 blocks, partitioned into blocks[0] x blocks[1]
    equal slabs along x1 and x2 (points assigned by coordinate for the random grid).
    """
    if unstructured:
        rng = np.random.default_rng(seed)
        x1 = rng.uniform(0.0, 2 * math.pi, npts * npts)
        x2 = rng.uniform(0.0, 2 * math.pi, npts * npts)
    else:
        g = 2 * math.pi * np.arange(npts) / npts
        x1, x2 = (a.ravel() for a in np.meshgrid(g, g, indexing="xy"))
    t = tgv_times(n, T)
    bx = np.minimum((x1 / (2 * math.pi) * blocks[0]).astype(int), blocks[0] - 1)
    by = np.minimum((x2 / (2 * math.pi) * blocks[1]).astype(int), blocks[1] - 1)
    out = []
    for j in range(blocks[1]):
        for i in range(blocks[0]):
            sel = (bx == i) & (by == j)
            f = np.sin(x1[sel]) * np.cos(x2[sel])
            out.append(np.asfortranarray(np.outer(f, np.exp(-2.0 * nu * t))))
    return out


def turbulence_block_direct(w: Workload, b: int, modes: Modes | None = None,
                            out_dtype=np.float32) -> np.ndarray:
    """Block b of the turbulence-like workload evaluated directly from the mode sum
    (no FFT), column-major m_b x n.  Modes sharing a frequency are summed first:
    cos(k.x + phi - w t) = cos(k.x + phi) cos(w t) + sin(k.x + phi) sin(w t)."""
    modes = modes or turbulence_modes(w.nmodes, w.kmax, w.data_seed)
    N, B, E = w.N, w.B, w.edge
    bx, by, bz = b % B, (b // B) % B, b // (B * B)
    loc = np.arange(E)
    zz, yy, xx = np.meshgrid(bz * E + loc, by * E + loc, bx * E + loc, indexing="ij")
    pts = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1).astype(np.float64)
    h = 2.0 * math.pi / N
    arg = (pts * h) @ modes.kappa.T.astype(np.float64)              # [P, M]
    amps, phases, offsets = _field_coeffs(modes)
    om_u, inv = np.unique(np.round(modes.omega, 12), return_inverse=True)
    t = w.dt * np.arange(w.n)
    Ct = np.cos(np.outer(om_u, t))                                   # [U, n]
    St = np.sin(np.outer(om_u, t))
    out = np.empty((w.fields * E ** 3, w.n), dtype=np.float64)
    for f in range(5):
        th = arg + phases[f][None, :]
        ind = np.zeros((len(inv), len(om_u)))
        ind[np.arange(len(inv)), inv] = amps[f]
        Gc = np.cos(th) @ ind                                        # [P, U]
        Gs = np.sin(th) @ ind
        out[f * E ** 3:(f + 1) * E ** 3] = offsets[f] + Gc @ Ct + Gs @ St
    return np.asfortranarray(out.astype(out_dtype))


# ----------------------------------------------------------------------------- in-situ stand-in
class StandInSolver:
    """Stand-in for the paper's flow solver in the in-situ measurements: the three
    Taylor-Green velocity components on the periodic N^3 grid advanced by linear
    advection-diffusion (second-order central differences, explicit Euler) with
    torch element-wise operations on the GPU.  ``store`` writes the current field
    as snapshot column j of the block-major data matrix [B^3, n, 3 E^3] (the store
    task that precedes a sketch update).  This is the application, not the
    compression method."""

    def __init__(self, N: int, B: int, nu: float, device, vel=(1.0, 0.5, 0.25), cfl=0.2):
        self.N, self.B, self.E = N, B, N // B
        self.h = 2.0 * math.pi / N
        self.nu, self.vel = nu, vel
        self.dt = cfl * self.h
        g = torch.arange(N, device=device, dtype=torch.float64) * self.h
        Z, Yc, X = torch.meshgrid(g, g, g, indexing="ij")        # [z, y, x], x fastest
        self.F0 = torch.stack([torch.sin(X) * torch.cos(Yc) * torch.cos(Z),
                               -torch.cos(X) * torch.sin(Yc) * torch.cos(Z),
                               torch.zeros_like(X)])

    def step(self, F):
        h = self.h
        lap = -6.0 * F
        adv = torch.zeros_like(F)
        for d, c in zip((3, 2, 1), self.vel):                     # x, y, z axes of [f, z, y, x]
            fp = torch.roll(F, -1, d)
            fm = torch.roll(F, 1, d)
            lap += fp + fm
            adv += (c / (2.0 * h)) * (fp - fm)
        F += self.dt * (self.nu / (h * h) * lap - adv)

    def store(self, F, A, j):
        B, E = self.B, self.E
        V = F.reshape(3, B, E, B, E, B, E).permute(1, 3, 5, 0, 2, 4, 6)   # bz, by, bx, f, z, y, x
        A[:, j, :] = V.reshape(B ** 3, 3 * E ** 3)
