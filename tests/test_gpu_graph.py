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
