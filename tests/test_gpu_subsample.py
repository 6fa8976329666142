"""GPU parity of the coarse-grid sketch (Section 2; Algorithm 2, SubID) and the
single-pass error M B(:,S) C (Algorithm 3) against the oracle, through the C ABI.

The sketch is a copy, so it must equal the oracle's bit for bit.  Selection
follows the gap rule (FP64, gap > 1e-10), coefficients and both errors match
to FP64 rounding.  Short coarse grids (m_c <= 128) take the register
selection kernels, taller ones the global-memory selection kernel.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from _harness import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _field_blocks(grids, n, seed, dtype=np.float64, noise=1e-7, rank=6):
    """Smooth low-rank space-time fields on each block's grid plus noise."""
    rng = np.random.default_rng(seed)
    out = []
    for g in grids:
        nx, ny, nz, nf = g[:4]
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        t = np.linspace(0.0, 1.0, n)
        A = np.zeros((nf * nx * ny * nz, n))
        for q in range(rank):
            a, b, c = rng.uniform(0.05, 0.4, 3)
            sp = np.concatenate([(np.sin(a * (q + 1) * x + f) * np.cos(b * y - f) * np.cos(c * z)).ravel()
                                 for f in range(nf)])
            A += np.outer(sp, np.exp(-(q + 1) * t) * 0.5 ** q)
        A += noise * rng.standard_normal(A.shape)
        out.append(np.asfortranarray(A.astype(dtype)))
    return out


def _check(g, o, blocks, grids, gamma=1e-10):
    for b in range(len(blocks)):
        assert np.array_equal(g.Y[b], o.Y[b]), b              # a copy: bitwise
    compare(g, o, gamma=gamma, y_rtol=0.0)
    for b, (A, gr) in enumerate(zip(blocks, grids)):
        eg = math.sqrt(g.ierr2[b] / g.nrm2[b])
        eo = math.sqrt(o.ierr2[b] / o.nrm2[b])
        assert abs(eg - eo) <= 1e-12 + 1e-11 * eo, (b, eg, eo)
        k = int(g.k[b])
        J = oracle.coarse_rows(gr)
        want = A[J][:, g.S[b][:k]]
        assert np.array_equal(g.cskel[b][:, :k], want), b   # B(:,S), exact


def test_short_coarse_grids_register_selection():
    """16^3 x 3-field blocks at interval 7 (81 coarse rows), 8 blocks, tolerance."""
    grids = [(16, 16, 16, 3, 7, 7, 7)] * 8
    blocks = _field_blocks(grids, 96, 1)
    print("case: subsample 16^3 s=7", flush=True)
    g = gpu_run(blocks, None, 12, 0, tol=1e-6, grids=grids)
    o = oracle_run(blocks, 81, 12, 0, tol=1e-6, grids=grids)
    _check(g, o, blocks, grids)


def test_tall_coarse_grids_global_selection_uneven_f32():
    """Interval 3 on 16^3 blocks (648 coarse rows: the global-memory selection),
    uneven grids with clamped edges, FP32 data, padded sketch rows."""
    grids = [(16, 16, 16, 3, 3, 3, 3), (20, 12, 9, 2, 3, 2, 4), (7, 30, 11, 1, 2, 5, 3),
             (16, 16, 16, 3, 3, 3, 3)]
    blocks = _field_blocks(grids, 80, 2, dtype=np.float32, noise=1e-5)
    l = 700
    print("case: subsample tall f32", flush=True)
    g = gpu_run(blocks, l, 10, 0, grids=grids)
    o = oracle_run(blocks, l, 10, 0, grids=grids)
    _check(g, o, blocks, grids)


def test_tall_coarse_grid_tolerance_and_rank_floor():
    grids = [(24, 20, 16, 2, 2, 2, 2)] * 3          # 2 * 12*10*8 = 1920 coarse rows
    blocks = _field_blocks(grids, 64, 3, noise=1e-9)
    print("case: subsample tall tol", flush=True)
    for kw in ({"tol": 1e-5}, {"rank_floor": 1e-7}):
        g = gpu_run(blocks, None, 16, 0, grids=grids, **kw)
        o = oracle_run(blocks, 1920, 16, 0, grids=grids, **kw)
        _check(g, o, blocks, grids)


def test_tgv64_interval3_single_partition():
    """u1 of the analytic Taylor-Green vortex on 64^3 points, 100 snapshots,
    interval 3 (Section 5.2.3's setting): rank one, SubID error at machine
    precision, single-pass error about 2 %, CF about 2400."""
    N, n = 64, 100
    h = 2 * np.pi / N
    grid = (N, N, N, 1, 3, 3, 3)
    z, y, x = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
    f = (np.sin(h * x) * np.cos(h * y) * np.cos(h * z)).ravel()
    A = np.asfortranarray(np.outer(f, np.exp(-0.03 * np.linspace(0.0, 1.0, n))))
    print("case: tgv64 s=3", flush=True)
    g = gpu_run([A], None, 4, 0, tol=1e-10, grids=[grid])
    o = oracle_run([A], 10648, 4, 0, tol=1e-10, grids=[grid])
    _check(g, o, [A], [grid])
    assert g.k[0] == 1 and g.rel_error < 1e-13
    assert abs(g.rel_interp_error - o.rel_interp_error) < 1e-12
    assert 0.01 < g.rel_interp_error < 0.03
    cf = oracle.compression_factor([N ** 3], [n], [int(g.k[0])], m_stored=[10648])
    assert abs(cf - 2400) <= 0.02 * 2400


def test_interval_one_equals_the_plain_id_and_state_errors():
    import paper_2103_01380_amd as sp
    grids = [(10, 8, 6, 1, 1, 1, 1)] * 2              # 480 rows: B = A, tall selection
    blocks = _field_blocks(grids, 40, 4)
    g = gpu_run(blocks, None, 6, 0, grids=grids)
    o = oracle_run(blocks, 480, 6, 0, grids=grids)
    _check(g, o, blocks, grids)
    for b in range(2):
        assert abs(g.ierr2[b] - g.err2[b]) <= 1e-12 * g.nrm2[b]   # M = I
    # the single-pass error needs the coarse-grid sketch, and coefficients
    ctx = sp.SPID([100], [10], 4, 2)
    with pytest.raises(sp.SpidError) as e:
        ctx.reconstruct_interp()
    assert e.value.status == sp.SPID_EINVAL
    ctx.close()
    ctx = sp.SPID([480], [10], None, 2, prec="subsample", grids=[(10, 8, 6, 1, 1, 1, 1)])
    with pytest.raises(sp.SpidError) as e:
        ctx.reconstruct_interp()
    assert e.value.status == sp.SPID_ESTATE
    ctx.close()


@pytest.mark.parametrize("grid", [(16, 16, 16, 1, 3, 3, 3), (24, 20, 12, 2, 2, 2, 2)])
def test_tall_selection_row_caching_variants(grid):
    """Coarse sketches of 129..256 and 1025+ rows (the register-cached and the
    streaming forms of the global-memory selection)."""
    grids = [grid] * 5
    l = len(oracle.coarse_rows(grid))
    assert 128 < l <= 256 or l > 1024
    blocks = _field_blocks(grids, 120, 5, noise=1e-8)
    print("case: tall variant", l, flush=True)
    g = gpu_run(blocks, None, 24, 0, tol=1e-7, grids=grids)
    o = oracle_run(blocks, l, 24, 0, tol=1e-7, grids=grids)
    _check(g, o, blocks, grids)


def test_tall_selection_one_workgroup_per_block_streaming_rows():
    """128 blocks of 1440 coarse rows: the one-workgroup-per-block selection in its
    streaming form (fewer blocks take the row-split selection)."""
    grids = [(24, 20, 12, 2, 2, 2, 2)] * 128
    blocks = _field_blocks(grids[:1], 32, 6, noise=1e-8) * 128
    print("case: tall 128 blocks", flush=True)
    g = gpu_run(blocks, None, 10, 0, tol=1e-6, grids=grids)
    o = oracle_run(blocks[:2], 1440, 10, 0, tol=1e-6, grids=grids[:2])
    for b in range(128):                    # identical blocks: identical results
        assert np.array_equal(g.S[b], g.S[0]) and g.err2[b] == g.err2[0]
    sub = type(g)(g.Y[:2], g.S[:2], g.k[:2], g.status[:2], g.P[:2], g.err2[:2], g.nrm2[:2],
                  None, g.ierr2[:2], g.cskel[:2])
    _check(sub, o, blocks[:2], grids[:2])
