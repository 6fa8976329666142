"""The allocation-free context (spid_create_static, for callers that cannot
allocate device memory) against the workspace context (spid_create_tuned) through
the C ABI: the same kernels on the same data, so every output must be equal bit
for bit, on two contexts in a row, the second on a smaller batch (the static
array keeps the first call's contents).  Also: a descriptor beyond the array is
rejected with EWORKSPACE, and a static context replaced by a later one is
rejected with ESTATE instead of reading the newer tables."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _batch(shapes, seed, dtype):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    parts = []
    for m, n in shapes:
        U = torch.randn((n, 6), generator=g, device="cuda", dtype=torch.float64)
        V = torch.randn((6, m), generator=g, device="cuda", dtype=torch.float64)
        E = torch.randn((n, m), generator=g, device="cuda", dtype=torch.float64)
        parts.append((U @ V + 1e-4 * E).to(dtype).reshape(-1))     # [n, m]: column-major A
    m = np.array([s[0] for s in shapes], dtype=np.int64)
    n = np.array([s[1] for s in shapes], dtype=np.int32)
    off = np.zeros(len(shapes), dtype=np.int64)
    off[1:] = np.cumsum((m * n)[:-1])
    return torch.cat(parts), m, n, off


def _run(static, A, m, n, off, **kw):
    import paper_2103_01380_amd as sp
    ctx = sp.SPID(m, n, static_scratch=static, **kw)
    ctx.bind(A, offsets=off)
    ctx.run()
    torch.cuda.synchronize()
    out = [t.clone() for t in (ctx.S, ctx.k, ctx.status, ctx.P, ctx.err2, ctx.nrm2)]
    out.append(ctx.sketch())
    torch.cuda.synchronize()
    ctx.close()
    return out


@pytest.mark.parametrize("prec", ["f64", "bf16"])
def test_static_context_equals_workspace_context(prec):
    dtype = torch.float64 if prec == "f64" else torch.float32
    kw = dict(l=24, k_max=12, tol=1e-6, seed=13, a_dtype="f64" if prec == "f64" else "f32",
              prec=prec, lp_terms=2)
    # second call smaller than the first
    for case, shapes in enumerate([[(7000, 200)] * 6 + [(300, 130), (20000, 96)],
                                   [(900, 40), (1500, 33)]]):
        A, m, n, off = _batch(shapes, 3 + case, dtype)
        print(f"case: static scratch {prec} call {case} blocks {len(shapes)}", flush=True)
        ref = _run(False, A, m, n, off, **kw)
        got = _run(True, A, m, n, off, **kw)
        for i, (a, b) in enumerate(zip(got, ref)):
            assert torch.equal(a, b), (case, i)


def test_static_context_limits():
    import paper_2103_01380_amd as sp
    # 400 blocks of 1000 x 512 at l = 48: about 313 MiB of workspace
    d = sp.make_desc(np.full(400, 1000), np.full(400, 512), 48, 8, tol=1e-3)
    assert sp.spid_workspace_bytes(d) > (64 << 20)
    with pytest.raises(sp.SpidError) as e:
        sp.spid_create_static(d)
    assert e.value.status == sp.SPID_EWORKSPACE and "static scratch" in str(e.value)
    # a replaced static context is refused
    A, m, n, off = _batch([(500, 30)] * 2, 9, torch.float64)
    first = sp.SPID(m, n, 10, 4, static_scratch=True)
    second = sp.SPID(m, n, 10, 4, static_scratch=True)
    with pytest.raises(sp.SpidError) as e:
        first.bind(A, offsets=off)
    assert e.value.status == sp.SPID_ESTATE
    second.bind(A, offsets=off)
    second.run()
    torch.cuda.synchronize()
    first.close()
    second.close()
