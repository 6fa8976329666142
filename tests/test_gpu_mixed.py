"""GPU parity of the mixed-precision (bfloat16 sketch, FP32 accumulation) path.

The oracle runs in FP64 with the same sketch matrix (Omega rounded to bfloat16);
the GPU additionally splits A into bfloat16 terms.  Checks: the sketch within the
split-term rounding, selected indices on every step whose oracle gap exceeds 1e-3,
and the reconstruction gates: R1 e_gpu <= 1e-3 where the oracle's own error is
<= 5e-4, R2 ||A(:,S~)P~ - A(:,S)P||_F / ||A||_F <= 1e-3.
"""
import math

import numpy as np
import pytest
import torch

import spid_inputs as si
from _harness import gpu_run, matched_prefix, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _gates(blocks, g, o, gamma=1e-3, y_rtol=2e-6):
    """y_rtol: the split-term sketch against the oracle's FP64 sketch with the same
    sketch matrix, relative to the largest sketch column norm (two bfloat16 terms
    leave about 2e-7, three e4m3 terms about 6e-5; FP32 accumulation over the rows
    adds about 1e-6 at most).  The error pass is held to the rounding of its
    split-bfloat16 product: with delta the error of the product A(:,S) P,
    |err2 - e_direct| <= 2 |<r, delta>| + |delta|^2; the cross term is bounded by
    2 sqrt(e_direct) |delta| (|delta| about 1e-7 ||A||) and in practice far smaller,
    since the residual and the rounding are uncorrelated (measured at most 4.2e-9
    sqrt(e_direct) ||A|| on these blocks), so the test holds it to 5e-8; the squares
    are summed in FP32 over 16 terms before the FP64 sum (at most 16 * 2^-24 < 1e-6
    of e_direct)."""
    num = den = rdiff = 0.0
    worst = 0.0
    for b, A in enumerate(blocks):
        Ad = A.astype(np.float64)
        scale = np.linalg.norm(o.Y[b], axis=0).max()
        assert np.abs(g.Y[b] - o.Y[b]).max() <= y_rtol * scale, (b, np.abs(g.Y[b] - o.Y[b]).max() / scale)
        s_star, ok = matched_prefix(g.S[b], o.S[b], o.gaps[b], g.k[b], o.k[b], gamma)
        assert ok, (b, s_star, g.S[b][:s_star], o.S[b][:s_star])
        kg, ko = int(g.k[b]), int(o.k[b])
        ag = Ad[:, g.S[b][:kg]] @ g.P[b][:kg]
        ao = Ad[:, o.S[b][:ko]] @ o.P[b][:ko]
        rdiff += ((ag - ao) ** 2).sum()
        num += g.err2[b]
        den += g.nrm2[b]
        # the GPU's error pass agrees with a direct FP64 evaluation of its own factors
        e_direct = ((Ad - ag) ** 2).sum()
        a_norm = math.sqrt((Ad ** 2).sum())
        gap = abs(g.err2[b] - e_direct)
        worst = max(worst, gap / (math.sqrt(e_direct) * a_norm + 1e-300))
        assert gap <= 5e-8 * math.sqrt(e_direct) * a_norm + 1e-6 * e_direct + 1e-13 * a_norm ** 2, \
            (b, g.err2[b], e_direct, gap / (math.sqrt(e_direct) * a_norm + 1e-300))
    e_gpu = math.sqrt(num / den)
    r2 = math.sqrt(rdiff / den)
    print(f"error pass: max |err2 - e_direct| / (sqrt(e_direct) ||A||) = {worst:.3e}")
    return e_gpu, o.rel_error, r2


@pytest.mark.parametrize("terms", [2, 3])
def test_turbulence_blocks_bf16(terms):
    """Blocks of the 256^3 turbulence-like workload (16^3 x 5 fields, n = 512), k = 32, l = 48."""
    w = si.WORKLOADS["turb256_b4096_bf16"]
    modes = si.turbulence_modes(w.nmodes, w.kmax, w.data_seed)
    blocks = [si.turbulence_block_direct(w, b, modes) for b in (0, 2049)]
    g = gpu_run(blocks, w.l, w.k_max, w.omega_seed, prec="bf16", lp_terms=terms)
    o = oracle_run(blocks, w.l, w.k_max, w.omega_seed, prec="bf16")
    e_gpu, e_ora, r2 = _gates(blocks, g, o)
    print(f"terms={terms} e_gpu={e_gpu:.3e} e_oracle={e_ora:.3e} R2={r2:.3e}")
    assert e_ora <= 5e-4 and e_gpu <= 1e-3 and r2 <= 1e-3


def test_ragged_lowrank_bf16():
    rng = np.random.default_rng(21)
    blocks = []
    for (m, n, r) in [(1000, 150, 10), (4097, 300, 25), (640, 129, 40), (20480, 512, 20)]:
        U = np.linalg.qr(rng.standard_normal((m, r)))[0]
        V = np.linalg.qr(rng.standard_normal((n, r)))[0]
        blocks.append(np.asfortranarray(((U * 10.0 ** (-0.25 * np.arange(r))) @ V.T).astype(np.float32)))
    g = gpu_run(blocks, 50, 40, 11, tol=1e-4, prec="bf16", lp_terms=2)
    o = oracle_run(blocks, 50, 40, 11, tol=1e-4, prec="bf16")
    e_gpu, e_ora, r2 = _gates(blocks, g, o)
    print(f"e_gpu={e_gpu:.3e} e_oracle={e_ora:.3e} R2={r2:.3e} k_gpu={g.k} k_ora={o.k}")
    assert e_gpu <= 1e-3 and r2 <= 1e-3
    assert np.all(np.abs(g.k - o.k) <= 1)


def test_bf16_split_term_sketch_accuracy_orders():
    """More split terms bring the sketch closer to the FP64 sketch with the same Omega."""
    rng = np.random.default_rng(22)
    blocks = [np.asfortranarray(rng.standard_normal((5000, 64)).astype(np.float32))]
    o = oracle_run(blocks, 16, 8, 4, prec="bf16")
    errs = []
    for terms in (1, 2, 3):
        g = gpu_run(blocks, 16, 8, 4, prec="bf16", lp_terms=terms)
        scale = np.abs(o.Y[0]).max()
        errs.append(np.abs(g.Y[0] - o.Y[0]).max() / scale)
    print("sketch rel err by terms", errs)
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 2e-2 and errs[1] < 1e-4 and errs[2] < 1e-5


def test_turbulence_8cubed_blocks_fp8():
    """Blocks of the 32768-block workload (8^3 x 5 fields, n = 384), k = 64, l = 96, e4m3 sketch
    with three split terms and per-32-row power-of-two scales."""
    w = si.WORKLOADS["turb256_b32768_fp8_stream"]
    modes = si.turbulence_modes(w.nmodes, w.kmax, w.data_seed)
    blocks = [si.turbulence_block_direct(w, b, modes) for b in (0, 20000)]
    g = gpu_run(blocks, w.l, w.k_max, w.omega_seed, prec="fp8", lp_terms=3)
    o = oracle_run(blocks, w.l, w.k_max, w.omega_seed, prec="fp8")
    e_gpu, e_ora, r2 = _gates(blocks, g, o, gamma=1e-2, y_rtol=2e-4)
    print(f"fp8 e_gpu={e_gpu:.3e} e_oracle={e_ora:.3e} R2={r2:.3e}")
    assert e_ora <= 5e-4 and e_gpu <= 1e-3 and r2 <= 1e-3


def test_fp8_split_term_sketch_accuracy_orders():
    rng = np.random.default_rng(23)
    blocks = [np.asfortranarray((rng.standard_normal((3000, 40)) *
                                 np.exp(rng.uniform(-5, 5, (3000, 1)))).astype(np.float32))]
    o = oracle_run(blocks, 20, 8, 5, prec="fp8")
    errs = []
    for terms in (1, 2, 3):
        g = gpu_run(blocks, 20, 8, 5, prec="fp8", lp_terms=terms)
        scale = np.abs(o.Y[0]).max()
        errs.append(np.abs(g.Y[0] - o.Y[0]).max() / scale)
    print("fp8 sketch rel err by terms", errs)
    assert errs[0] > errs[1] > errs[2]
    assert errs[0] < 1e-1 and errs[1] < 3e-3 and errs[2] < 1e-4


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_wide_blocks_hybrid_selection(prec):
    """n up to 1000 and l = 50 (the uneven workload's limits): selection keeps part of the
    sketch in LDS."""
    rng = np.random.default_rng(24)
    dt = np.float64 if prec == "f64" else np.float32
    blocks = []
    for (m, n, r) in [(1600, 1000, 30), (640, 700, 12), (3000, 130, 40)]:
        U = np.linalg.qr(rng.standard_normal((m, r)))[0]
        V = np.linalg.qr(rng.standard_normal((n, r)))[0]
        blocks.append(np.asfortranarray(((U * 10.0 ** (-0.25 * np.arange(r))) @ V.T).astype(dt)))
    g = gpu_run(blocks, 50, 40, 12, tol=1e-4, prec=prec, lp_terms=2)
    o = oracle_run(blocks, 50, 40, 12, tol=1e-4, prec=prec)
    if prec == "f64":
        from _harness import compare
        compare(g, o)
    else:
        e_gpu, e_ora, r2 = _gates(blocks, g, o)
        assert e_gpu <= 1e-3 and r2 <= 1e-3


def test_tall_sketch_pair_selection_f64():
    """l = 96, n = 384 in double precision: the two-lanes-per-column selection kernel
    against the oracle by the FP64 gap rule."""
    rng = np.random.default_rng(25)
    blocks = []
    for (m, n, r) in [(2560, 384, 80), (3000, 200, 50)]:
        U = np.linalg.qr(rng.standard_normal((m, r)))[0]
        V = np.linalg.qr(rng.standard_normal((n, r)))[0]
        blocks.append(np.asfortranarray((U * 10.0 ** (-0.05 * np.arange(r))) @ V.T))
    from _harness import compare
    g = gpu_run(blocks, 96, 64, 13)
    o = oracle_run(blocks, 96, 64, 13)
    st = compare(g, o)
    assert min(st["prefix"]) >= 10


@pytest.mark.parametrize("l,k,shapes,tol", [
    (60, 40, [(2560, 600, 50), (1800, 520, 30)], 0.0),     # n > 512: register + LDS rows
    (120, 70, [(3000, 300, 90), (2000, 256, 40)], 1e-6),   # l > 96: 64 rows per lane, tolerance
])
def test_tall_sketch_selection_variants_f64(l, k, shapes, tol):
    rng = np.random.default_rng(26 + l)
    blocks = []
    for (m, n, r) in shapes:
        U = np.linalg.qr(rng.standard_normal((m, r)))[0]
        V = np.linalg.qr(rng.standard_normal((n, r)))[0]
        blocks.append(np.asfortranarray((U * 10.0 ** (-0.05 * np.arange(r))) @ V.T))
    from _harness import compare
    print(f"case: tall selection l={l} k={k} shapes={shapes}", flush=True)
    g = gpu_run(blocks, l, k, 14, tol=tol)
    o = oracle_run(blocks, l, k, 14, tol=tol)
    st = compare(g, o)
    assert min(st["prefix"]) >= 10


@pytest.mark.parametrize("l,k,shapes,decay", [
    (16, 8, [(1000, 100, 12), (777, 50, 20)], 0.5),                # one 16-row coefficient block
    (96, 80, [(3000, 200, 90), (1500, 130, 100), (641, 97, 95)], 0.07),   # six blocks, three k-steps
])
def test_bf16_coefficient_term_orders(l, k, shapes, decay):
    """The split coefficient terms are written in 16-byte pieces of the coefficients
    kernel's own rows and the error pass gathers its selected columns in that order:
    ranks that fill one and six 16-row coefficient blocks (one and three 32-column
    k-steps of the error pass), against the oracle and a direct evaluation.  Every
    block has more than k singular values above the sketch's rounding, so the
    selections stay well conditioned."""
    rng = np.random.default_rng(27 + k)
    blocks = []
    for (m, n, r) in shapes:
        U = np.linalg.qr(rng.standard_normal((m, r)))[0]
        V = np.linalg.qr(rng.standard_normal((n, r)))[0]
        blocks.append(np.asfortranarray(((U * 10.0 ** (-decay * np.arange(r))) @ V.T)
                                        .astype(np.float32)))
    print(f"case: bf16 coefficient terms l={l} k={k} shapes={shapes}", flush=True)
    g = gpu_run(blocks, l, k, 15, prec="bf16", lp_terms=2)
    o = oracle_run(blocks, l, k, 15, prec="bf16")
    e_gpu, e_ora, r2 = _gates(blocks, g, o)
    print(f"e_gpu={e_gpu:.3e} e_oracle={e_ora:.3e} R2={r2:.3e} k_gpu={g.k}")
    assert e_gpu <= 1e-3 and r2 <= 1e-3
