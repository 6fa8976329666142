"""The synthetic input generators (CPU): the FFT-based turbulence generator equals
the direct mode sum, the TGV closed form, the uneven-batch shapes."""
import math

import numpy as np
import pytest
import torch

import spid_inputs as si


def test_turbulence_fft_matches_direct_mode_sum():
    w = si.scaled(si.WORKLOADS["turb256_b4096_bf16"], N=48, B=3, n=5)
    A = si.turbulence_blocks(w, device="cpu", out_dtype=torch.float64)
    for b in (0, 13, 26):
        d = si.turbulence_block_direct(w, b, out_dtype=np.float64)
        assert np.abs(d - A[b].numpy().T).max() < 1e-12


def test_turbulence_modes_properties():
    m = si.turbulence_modes(4096, 16, 5)
    k2 = (m.kappa ** 2).sum(1)
    assert np.all((k2 >= 1) & (k2 <= 256))
    keys = {tuple(k) for k in m.kappa}
    assert len(keys) == 4096
    assert not any(tuple(-k) in keys for k in m.kappa)          # one of each +-k pair
    assert np.allclose((m.pol * m.kappa).sum(1), 0.0, atol=1e-12)  # divergence free
    assert np.allclose(np.linalg.norm(m.pol, axis=1), 1.0)
    kn = np.sqrt(k2)
    assert np.allclose(m.omega, kn ** (2.0 / 3.0))
    # shell energy ~ |k|^2 amp^2 ~ |k|^(-5/3)
    assert np.allclose(m.amp / m.amp[0], (kn / kn[0]) ** (-11.0 / 6.0))


def test_tgv_blocks_layout_and_closed_form():
    w = si.scaled(si.WORKLOADS["tgv128_b512_f64"], N=8, B=2, n=3, noise=0.0)
    A = si.tgv_blocks(w).numpy()                 # [8, 3, 3*64]
    E, h = 4, 2 * math.pi / 8
    b = 5                                        # bx=1, by=0, bz=1
    t = si.tgv_times(3, w.T)
    for (z, y, x) in [(0, 0, 0), (3, 2, 1)]:
        gx, gy, gz = (1 * E + x) * h, (0 * E + y) * h, (1 * E + z) * h
        i = z * 16 + y * 4 + x
        for j in range(3):
            g = math.exp(-3 * w.nu * t[j])
            assert A[b, j, i] == pytest.approx(math.sin(gx) * math.cos(gy) * math.cos(gz) * g)
            assert A[b, j, 64 + i] == pytest.approx(-math.cos(gx) * math.sin(gy) * math.cos(gz) * g)
            assert A[b, j, 128 + i] == 0.0


def test_uneven_shapes():
    w = si.WORKLOADS["lowrank_uneven2000_bf16"]
    sh = si.lowrank_shapes(w)
    e = np.rint((sh.m / 5) ** (1 / 3))
    assert np.all((e >= 4) & (e <= 32))
    assert np.all((sh.n >= 128) & (sh.n <= 1024))
    assert np.all((sh.rank >= 2) & (sh.rank <= 40))
    assert 80e9 < sh.total * 4 < 100e9


def test_lowrank_block_singular_values():
    w = si.WORKLOADS["lowrank_uneven2000_bf16"]
    sh = si.lowrank_shapes(w, nblocks=3, edge_range=(4, 6), n_range=(128, 160))
    A = si.lowrank_blocks(w, sh, out_dtype=torch.float64)
    for b in range(3):
        m, n, r = int(sh.m[b]), int(sh.n[b]), int(sh.rank[b])
        blk = A[sh.offsets[b]:sh.offsets[b] + m * n].numpy().reshape(n, m).T
        s = np.linalg.svd(blk, compute_uv=False)
        assert np.allclose(s[:r], 10.0 ** (-0.25 * np.arange(r)), rtol=1e-10)
        assert np.all(s[r:] < 1e-12)


@pytest.mark.parametrize("name", ["tgv64_single_sub3", "tgv128_b512_sub3", "tgv128_b512_sub7"])
def test_coarse_grid_workloads_match_the_oracle_grid(name):
    import oracle
    w = si.WORKLOADS[name]
    g = w.grids()
    assert g.shape == (w.nblocks, 7)
    assert int(np.prod(g[0][:4])) == (w.N // w.B) ** 3 * w.fields
    assert len(oracle.coarse_rows(g[0])) == w.coarse_rows == w.l
