"""GPU parity of the HIP path (through the C ABI) against the CPU oracle.

Double-precision path: selected indices bit-exact on every step whose oracle
top-two pivot gap exceeds 1e-10 of the largest sketch column norm, relative
reconstruction errors within 1e-12, sketch within 1e-13 relative, P within
1e-9 when every pivot matches, identity block exact.
"""
import math

import numpy as np
import pytest
import torch

import spid_inputs as si
from _harness import compare, gpu_run, oracle_run

pytestmark = pytest.mark.gpu


def _rand_blocks(shapes, seed, dtype=np.float64, rank=None, decay=0.2):
    rng = np.random.default_rng(seed)
    out = []
    for (m, n) in shapes:
        if rank is None:
            A = rng.standard_normal((m, n))
        else:
            r = min(rank, m, n)
            U = np.linalg.qr(rng.standard_normal((m, r)))[0]
            V = np.linalg.qr(rng.standard_normal((n, r)))[0]
            A = (U * 10.0 ** (-decay * np.arange(r))) @ V.T
        out.append(np.asfortranarray(A.astype(dtype)))
    return out


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    print(f"\n[gpu] {torch.cuda.get_device_name(0)}", flush=True)


def test_tgv32_single_block_full_size():
    """Analytic TGV 32^3, one block 98304 x 64, k = 8, l = 18 (full workload size)."""
    w = si.WORKLOADS["tgv32_single_f64"]
    A = si.tgv_blocks(w).numpy()
    blk = [np.asfortranarray(A[0].T)]
    g = gpu_run(blk, w.l, w.k_max, w.omega_seed)
    o = oracle_run(blk, w.l, w.k_max, w.omega_seed)
    st = compare(g, o)
    assert g.S[0][0] == 0 and st["prefix"][0] >= 1
    assert g.rel_error < 1e-13 and o.rel_error < 1e-13
    # rank-floor reading: one pivot and closed-form coefficients
    gf = gpu_run(blk, w.l, w.k_max, w.omega_seed, rank_floor=1e-13)
    assert gf.k[0] == 1 and gf.S[0][0] == 0
    t = si.tgv_times(w.n, w.T)
    assert np.allclose(gf.P[0][0], np.exp(-3.0 * w.nu * (t - t[0])), rtol=1e-13, atol=1e-14)


def test_tgv_noise_tolerance_blocks_at_workload_block_size():
    """TGV + 1e-6 noise, blocks of 16^3 x 256 (the 512-block workload's block shape),
    8 blocks, tolerance 1e-8 capped at 32, l = 42."""
    w = si.scaled(si.WORKLOADS["tgv128_b512_f64"], N=32, B=2)
    A = si.tgv_blocks(w).numpy()
    blocks = [np.asfortranarray(A[b].T) for b in range(A.shape[0])]
    g = gpu_run(blocks, w.l, w.k_max, w.omega_seed, tol=w.tol)
    o = oracle_run(blocks, w.l, w.k_max, w.omega_seed, tol=w.tol)
    st = compare(g, o)
    assert np.all(g.k == w.k_max)
    assert np.all(g.status == 3)
    print("prefix", st["prefix"], "full", st["full_match"], "e", g.rel_error, o.rel_error)
    # companion tolerance above the noise floor: k = 1 everywhere
    g5 = gpu_run(blocks, w.l, w.k_max, w.omega_seed, tol=1e-5)
    o5 = oracle_run(blocks, w.l, w.k_max, w.omega_seed, tol=1e-5)
    compare(g5, o5)
    assert np.all(g5.k == 1)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_ragged_uneven_blocks_fixed_rank(dtype):
    # rows not multiples of 32, columns not multiples of 16/64, odd l
    shapes = [(1000, 37), (33, 70), (4097, 129), (260, 5), (2049, 300)]
    blocks = _rand_blocks(shapes, 5, dtype=dtype, rank=40, decay=0.1)
    l, k = 5, 5
    g = gpu_run(blocks, l, k, 77, skeleton=True)
    o = oracle_run(blocks, l, k, 77)
    compare(g, o)
    for b, blk in enumerate(blocks):
        kk = int(g.k[b])
        assert np.array_equal(g.skel[b][:, :kk], blk[:, g.S[b][:kk]])


@pytest.mark.parametrize("l,k", [(13, 9), (33, 20), (48, 32)])
def test_random_blocks_various_l(l, k):
    shapes = [(3000, 64), (5000, 256), (777, 100), (12288, 256)]
    blocks = _rand_blocks(shapes, l * 100 + k, rank=60, decay=0.05)
    g = gpu_run(blocks, l, k, 1234 + l)
    o = oracle_run(blocks, l, k, 1234 + l)
    st = compare(g, o)
    assert st["full_match"] >= 1


def test_tolerance_mode_uneven():
    shapes = [(2000, 80), (640, 200), (5000, 150)]
    blocks = _rand_blocks(shapes, 9, rank=30, decay=0.25)
    g = gpu_run(blocks, 40, 30, 5, tol=1e-4)
    o = oracle_run(blocks, 40, 30, 5, tol=1e-4)
    compare(g, o)
    assert np.array_equal(g.k, o.k)


def test_omega_per_block_keys():
    shapes = [(1500, 40)] * 3
    blocks = _rand_blocks(shapes, 10, rank=10, decay=0.3)
    g = gpu_run(blocks, 12, 6, 99, omega_per_block=True)
    o = oracle_run(blocks, 12, 6, 99, omega_per_block=True)
    compare(g, o)


def test_padded_leading_dimension():
    shapes = [(1000, 30), (513, 64)]
    blocks = _rand_blocks(shapes, 12, rank=8, decay=0.3)
    g = gpu_run(blocks, 12, 8, 21, lda_pad=7)
    o = oracle_run(blocks, 12, 8, 21)
    compare(g, o)


def test_k_equals_n_is_exact_and_degenerate_blocks():
    rng = np.random.default_rng(13)
    full = np.asfortranarray(rng.standard_normal((300, 6)))
    zero = np.zeros((200, 6), order="F")
    rank1 = np.asfortranarray(np.outer(rng.standard_normal(250), rng.standard_normal(6)))
    nanb = np.asfortranarray(rng.standard_normal((100, 6)))
    nanb[10, 2] = np.nan
    blocks = [full, zero, rank1, nanb]
    g = gpu_run(blocks, 6, 6, 8, tol=1e-14)
    o = oracle_run(blocks, 6, 6, 8, tol=1e-14)
    assert g.k[0] == 6 and g.err2[0] <= 1e-24 * g.nrm2[0]
    assert g.k[1] == 0 and g.status[1] == 1 and g.err2[1] == 0.0
    assert g.k[2] == 1
    assert g.status[3] == 2 and g.k[3] == 0
    assert np.array_equal(g.status, o.status) and np.array_equal(g.k, o.k)


def test_call_order_is_enforced():
    import paper_2103_01380_amd as sp
    m, n = np.array([100]), np.array([10])
    ctx = sp.SPID(m, n, 4, 2)
    with pytest.raises(sp.SpidError) as e:
        ctx.sketch_update()
    assert e.value.status == sp.SPID_ESTATE
    A = torch.randn(1, 10, 100, dtype=torch.float64, device="cuda")
    ctx.bind(A)
    with pytest.raises(sp.SpidError) as e:
        ctx.select()
    assert e.value.status == sp.SPID_ESTATE
    ctx.sketch_update(0, 5)
    with pytest.raises(sp.SpidError):
        ctx.select()
    ctx.sketch_update(5, 5)
    ctx.select()
    ctx.coeffs()
    ctx.reconstruct()
    torch.cuda.synchronize()
    ctx.close()


def test_repeat_runs_are_bitwise_identical():
    shapes = [(4096, 256)] * 4
    blocks = _rand_blocks(shapes, 14, rank=50, decay=0.05)
    a = gpu_run(blocks, 42, 32, 6)
    b = gpu_run(blocks, 42, 32, 6)
    assert np.array_equal(a.S, b.S)
    assert np.array_equal(a.err2, b.err2)
    for x, y in zip(a.P, b.P):
        assert np.array_equal(x, y)
