"""The four stages captured into one HIP graph (torch.cuda.CUDAGraph on the
capture stream) and replayed: every replay equals the eager run bitwise.  The
library enqueues only kernels (no memset, no host synchronisation)."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec,dtype", [("f64", torch.float64), ("bf16", torch.float32)])
def test_graph_replays_equal_eager(prec, dtype):
    import paper_2103_01380_amd as sp
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    nb, n, m = 24, 96, 3000
    A = torch.randn((nb, n, m), generator=g, device="cuda", dtype=dtype)
    # low rank + noise so that the selection is well defined
    U = torch.randn((nb, 6, m), generator=g, device="cuda", dtype=dtype)
    C = torch.randn((nb, n, 6), generator=g, device="cuda", dtype=dtype)
    A = torch.bmm(C, U) + 1e-3 * A
    mm = np.full(nb, m)
    nn = np.full(nb, n)
    ctx = sp.SPID(mm, nn, 16, 8, tol=1e-6, seed=3, a_dtype="f64" if prec == "f64" else "f32",
                  prec=prec, lp_terms=2)
    ctx.bind(A)
    ctx.run()
    torch.cuda.synchronize()
    ref = [t.clone() for t in (ctx.S, ctx.k, ctx.P, ctx.err2, ctx.nrm2)]
    for t in (ctx.S, ctx.k, ctx.P, ctx.err2, ctx.nrm2):
        t.zero_()
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            ctx.run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in (ctx.S, ctx.k, ctx.P, ctx.err2, ctx.nrm2):
            t.fill_(7)                      # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip((ctx.S, ctx.k, ctx.P, ctx.err2, ctx.nrm2), ref):
            assert torch.equal(a, b), rep
    ctx.close()


def _capture_and_check(ctx, step, outs):
    step()
    torch.cuda.synchronize()
    ref = [t.clone() for t in outs]
    graph = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(graph, stream=s):
            step(s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        for t in outs:
            t.fill_(7)                      # eager work between replays
        graph.replay()
        torch.cuda.synchronize()
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), rep


@pytest.mark.parametrize("nblocks,interval", [(24, 2), (2, 1)])
def test_graph_coarse_grid_single_pass(nblocks, interval):
    """Coarse-grid sketch, selection (one workgroup per block, or the row-split
    form for two tall blocks), coefficients and the single-pass error in one graph."""
    import paper_2103_01380_amd as sp
    g = torch.Generator(device="cuda")
    g.manual_seed(6)
    grid = (20, 16, 12, 2, interval, interval, interval)
    m, n = 20 * 16 * 12 * 2, 64
    U = torch.randn((nblocks, 5, m), generator=g, device="cuda", dtype=torch.float64)
    C = torch.randn((nblocks, n, 5), generator=g, device="cuda", dtype=torch.float64)
    A = torch.bmm(C, U) + 1e-6 * torch.randn((nblocks, n, m), generator=g, device="cuda",
                                             dtype=torch.float64)
    ctx = sp.SPID(np.full(nblocks, m), np.full(nblocks, n), None, 8, tol=1e-4, prec="subsample",
                  grids=[grid] * nblocks)
    ctx.bind(A)

    def step(stream=None):
        ctx.sketch_update(stream=stream)
        ctx.select(stream)
        ctx.coeffs(stream)
        ctx.reconstruct_interp(stream=stream)

    _capture_and_check(ctx, step, (ctx.S, ctx.k, ctx.P, ctx.err2_interp, ctx.nrm2))
    ctx.close()


def test_graph_two_stage():
    import paper_2103_01380_amd as sp
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    nb, n, m = 16, 120, 2000
    U = torch.randn((nb, 7, m), generator=g, device="cuda", dtype=torch.float64)
    C = torch.randn((nb, n, 7), generator=g, device="cuda", dtype=torch.float64)
    A = torch.bmm(C, U) + 1e-7 * torch.randn((nb, n, m), generator=g, device="cuda",
                                             dtype=torch.float64)
    ctx = sp.SPID(np.full(nb, m), np.full(nb, n), 20, 12, tol=1e-5, seed=4, ts_windows=6,
                  ts_k1=5)
    ctx.bind(A)

    def step(stream=None):
        ctx.sketch_update(stream=stream)
        ctx.select_two_stage(stream)
        ctx.reconstruct(stream=stream)

    _capture_and_check(ctx, step, (ctx.S, ctx.k, ctx.P, ctx.err2, ctx.nrm2))
    ctx.close()


def test_graph_uneven_batch_matches_oracle():
    """A ragged batch shaped like the uneven workload (edges log-uniform in [4, 16]:
    m_b = 5 e^3 from 320 to 20480 rows, mostly not multiples of 4; n_b log-uniform in
    [40, 300]; low rank with decaying singular values, FP32), BF16 sketch with a
    tolerance: the four stages captured into one graph replay the eager results bit
    for bit, and the eager results pass the mixed-precision gates against the oracle
    (pivot prefix by the 1e-3 gap rule, sketch to the split-term rounding, R2 and the
    error of the factors)."""
    import math
    from _harness import gpu_run, matched_prefix, oracle_run
    rng = np.random.default_rng(33)
    blocks = []
    for b in range(40):
        e = int(round(math.exp(rng.uniform(math.log(4), math.log(16)))))
        m = 5 * e ** 3
        n = int(round(math.exp(rng.uniform(math.log(40), math.log(300)))))
        r = int(rng.integers(2, 16))
        U = rng.standard_normal((m, r))
        V = rng.standard_normal((n, r)) * 10.0 ** (-0.25 * np.arange(r))
        blocks.append(np.asfortranarray((U @ V.T + 1e-7 * rng.standard_normal((m, n))).astype(np.float32)))
    print("case: graph uneven", [b.shape for b in blocks[:4]], flush=True)
    g = gpu_run(blocks, 30, 20, 17, tol=1e-4, prec="bf16", lp_terms=2, graph_replays=3)
    o = oracle_run(blocks, 30, 20, 17, tol=1e-4, prec="bf16")
    num = den = rd = 0.0
    for b, A in enumerate(blocks):
        Ad = A.astype(np.float64)
        scale = np.linalg.norm(o.Y[b], axis=0).max()
        assert np.abs(g.Y[b] - o.Y[b]).max() <= 2e-6 * scale, b
        s_star, ok = matched_prefix(g.S[b], o.S[b], o.gaps[b], g.k[b], o.k[b], 1e-3)
        assert ok, (b, s_star)
        kg, ko = int(g.k[b]), int(o.k[b])
        ag = Ad[:, g.S[b][:kg]] @ g.P[b][:kg]
        ao = Ad[:, o.S[b][:ko]] @ o.P[b][:ko]
        e_direct = ((Ad - ag) ** 2).sum()
        a_norm = math.sqrt((Ad ** 2).sum())
        assert abs(g.err2[b] - e_direct) <= 5e-8 * math.sqrt(e_direct) * a_norm + \
            1e-6 * e_direct + 1e-13 * a_norm ** 2, b
        num += e_direct
        rd += ((ag - ao) ** 2).sum()
        den += (Ad ** 2).sum()
    assert math.sqrt(num / den) <= 1e-3 and math.sqrt(rd / den) <= 1e-3
