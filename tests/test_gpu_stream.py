"""GPU parity of one-snapshot sketch updates (blocks as the MFMA column
dimension) and exactness of the low-precision sketch matrix.

One-snapshot updates (w <= 4) take a different kernel shape than batch
updates: blocks of equal m are grouped, each group shares one Omega chunk per
row range, and large groups are split along their rows with a fixed-order
reduction.  The sketch must still equal the oracle's to FP64 rounding, and the
selection must follow the gap rule.  The low-precision sketch matrix is the
double-precision normal rounded to bfloat16 / e4m3; a sketch of identity
columns returns it exactly, entry by entry.
"""
import numpy as np
import pytest
import torch

import oracle
import spid_inputs as si
from _harness import compare, gpu_run, matched_prefix, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rand_blocks(shapes, seed, rank, decay):
    rng = np.random.default_rng(seed)
    out = []
    for m, n in shapes:
        U = rng.standard_normal((m, rank))
        V = rng.standard_normal((n, rank))
        A = (U * (10.0 ** (-decay * np.arange(rank)))) @ V.T + 1e-9 * rng.standard_normal((m, n))
        out.append(np.asfortranarray(A))
    return out


def test_stream_groups_split_and_ragged_fp64():
    """Several m values (partial groups, one group split along its rows), blocks with
    fewer snapshots than others (j >= n_b), streamed one snapshot per call."""
    shapes = [(6000, 40)] * 3 + [(1000, 48)] * 130 + [(257, 33)] * 2 + [(4100, 48)]
    blocks = _rand_blocks(shapes, 31, rank=10, decay=0.3)
    print("case: stream fp64 groups", len(blocks), flush=True)
    g = gpu_run(blocks, 14, 8, 17, stream_columns=True)
    o = oracle_run(blocks, 14, 8, 17)
    stats = compare(g, o)
    assert stats["full_match"] > 0


def test_stream_equals_batch_within_rounding():
    shapes = [(3000, 48), (1200, 64)]
    blocks = _rand_blocks(shapes, 11, rank=12, decay=0.2)
    a = gpu_run(blocks, 16, 8, 3)
    b = gpu_run(blocks, 16, 8, 3, stream_columns=True)
    for x, y in zip(a.Y, b.Y):
        scale = np.linalg.norm(x, axis=0).max()
        assert np.abs(x - y).max() <= 1e-13 * scale
    assert np.array_equal(a.S, b.S)


def test_stream_with_block_keys_falls_back_to_batch_shape():
    shapes = [(900, 20), (700, 24)]
    blocks = _rand_blocks(shapes, 12, rank=6, decay=0.4)
    g = gpu_run(blocks, 10, 6, 5, omega_per_block=True, stream_columns=True)
    o = oracle_run(blocks, 10, 6, 5, omega_per_block=True)
    compare(g, o)


def test_stream_fp8_turbulence_8cubed_blocks():
    """Blocks of the streamed 256^3 turbulence-like workload (8^3 x 5 fields, n = 384),
    FP8 sketch with per-32-row scales, k = 64, l = 96, one snapshot per call."""
    w = si.WORKLOADS["turb256_b32768_fp8_stream"]
    modes = si.turbulence_modes(w.nmodes, w.kmax, w.data_seed)
    ids = list(range(0, 32768, 32768 // 160))[:160]
    blocks = [si.turbulence_block_direct(w, b, modes) for b in ids]
    print("case: stream fp8 blocks", len(blocks), flush=True)
    g = gpu_run(blocks, w.l, w.k_max, w.omega_seed, prec="fp8", lp_terms=w.lp_terms,
                stream_columns=True)
    o = oracle_run(blocks, w.l, w.k_max, w.omega_seed, prec="fp8")
    e_gpu, r2, pre = _fp8_gates(blocks, g, o)
    print(f"stream fp8 e_gpu={e_gpu:.3e} e_oracle={o.rel_error:.3e} R2={r2:.3e} "
          f"min prefix={min(pre)}")
    assert e_gpu <= 1e-3 and r2 <= 1e-3


def _fp8_gates(blocks, g, o, gamma=1e-2, y_rtol=2e-4):
    """FP8 sketch against the oracle (same e4m3 sketch matrix): sketch within the
    split-term rounding, the pivots of every step whose oracle gap exceeds gamma,
    the status where the whole selection is decided, and the error gates
    (e_gpu = ||A - A(:,S~)P~|| / ||A||, R2 = ||A(:,S~)P~ - A(:,S)P|| / ||A||)."""
    num = den = rd = 0.0
    prefixes = []
    for b, A in enumerate(blocks):
        Ad = A.astype(np.float64)
        scale = np.linalg.norm(o.Y[b], axis=0).max()
        assert np.abs(g.Y[b] - o.Y[b]).max() <= y_rtol * scale, (b, np.abs(g.Y[b] - o.Y[b]).max() / scale)
        s_star, ok = matched_prefix(g.S[b], o.S[b], o.gaps[b], g.k[b], o.k[b], gamma)
        assert ok, (b, s_star, g.S[b][:s_star], o.S[b][:s_star])
        prefixes.append(s_star)
        kg, ko = int(g.k[b]), int(o.k[b])
        if s_star == ko and kg == ko:
            assert g.status[b] == o.status[b], (b, g.status[b], o.status[b])
        assert np.array_equal(g.P[b][:kg][:, g.S[b][:kg]], np.eye(kg)), b
        ag = Ad[:, g.S[b][:kg]] @ g.P[b][:kg]
        ao = Ad[:, o.S[b][:ko]] @ o.P[b][:ko]
        num += ((Ad - ag) ** 2).sum()
        rd += ((ag - ao) ** 2).sum()
        den += (Ad ** 2).sum()
    return float(np.sqrt(num / den)), float(np.sqrt(rd / den)), prefixes


@pytest.mark.parametrize("groups", [2, 4, 0])
def test_stream_fp8_multi_group(groups):
    """One-snapshot FP8 updates with several groups of 128 equal-m blocks per work
    item (st_groups; 0 = the library's choice, one): three groups of 2560-row blocks
    and a 128 + 2 block run of 1000-row blocks (a partial group, a ragged last
    chunk: 1000 = 7 x 128 + 104)."""
    shapes = [(2560, 80)] * 384 + [(1000, 80)] * 130
    rng = np.random.default_rng(41)
    blocks = []
    for m, n in shapes:
        U = rng.standard_normal((m, 12))
        V = rng.standard_normal((n, 12)) * 10.0 ** (-0.3 * np.arange(12))
        # columns decaying in time keep the first pivots decidable at the FP8 gap
        A = (U @ V.T + 1e-5 * rng.standard_normal((m, n))) * (0.85 ** np.arange(n))
        blocks.append(np.asfortranarray(A.astype(np.float32)))
    print(f"case: fp8 one-snapshot st_groups={groups}", flush=True)
    g = gpu_run(blocks, 64, 40, 19, prec="fp8", lp_terms=3, stream_columns=True,
                tuning={"st_groups": groups} if groups else None)
    if groups:
        assert g.tuning["st_groups"] == groups
    o = oracle_run(blocks, 64, 40, 19, prec="fp8")
    e_gpu, r2, pre = _fp8_gates(blocks, g, o)
    print(f"fp8 one-snapshot groups={g.tuning['st_groups']} e_gpu={e_gpu:.3e} "
          f"e_oracle={o.rel_error:.3e} R2={r2:.3e} min prefix={min(pre)}")
    # the oracle decides 3.6 pivots per block on average at the FP8 gap (0 to 7)
    assert np.mean(pre) >= 3 and max(pre) >= 6
    assert e_gpu <= 1e-3 and r2 <= 1e-3


@pytest.mark.parametrize("prec,code", [("bf16", oracle.OMEGA_BF16), ("fp8", oracle.OMEGA_FP8E4M3)])
def test_low_precision_omega_is_exact(prec, code):
    """Sketch of identity columns: Y(:, j) = Omega(:, row of column j) exactly, for
    rows spread over eight blocks (262144 entries at l = 64)."""
    l, n, m = 64, 512, 8192
    blocks = []
    for b in range(8):
        A = np.zeros((m, n), dtype=np.float32, order="F")
        rows = (np.arange(n) * 7 + 512 * b) % m
        A[rows, np.arange(n)] = 1.0
        blocks.append(A)
    g = gpu_run(blocks, l, 8, 77, prec=prec, lp_terms=1)
    om = oracle.omega(77, l, m, prec=code)
    bad = 0
    for b in range(8):
        rows = (np.arange(n) * 7 + 512 * b) % m
        bad += int(np.count_nonzero(g.Y[b] != om[:, rows]))
    assert bad == 0
