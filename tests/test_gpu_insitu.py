"""In-situ compression on the GPU (Sections 3.3-3.4, Algorithms 4-5): a stand-in
solver advances the flow field on the default stream and stores every snapshot
into the resident data matrix; the one-snapshot sketch update of that snapshot
runs on a second stream behind an event, overlapping the next solver step.
After the last snapshot the selection, coefficients and error pass run on the
second stream.  The result must equal the oracle's on the stored snapshots
(FP64 gap rule, coefficients, errors), and the overlapped sketch must equal a
batch sketch of the same data to FP64 rounding."""
import numpy as np
import pytest
import torch

import spid_inputs as si
from _harness import compare, oracle_run

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_overlapped_sketch_updates_match_the_oracle():
    import paper_2103_01380_amd as sp
    N, B, n, l, k_max, tol, seed = 32, 2, 48, 20, 12, 1e-9, 41
    dev = torch.device("cuda")
    solver = si.StandInSolver(N, B, 0.01, dev)
    nb, m = B ** 3, 3 * (N // B) ** 3
    A = torch.empty((nb, n, m), dtype=torch.float64, device=dev)
    ctx = sp.SPID(np.full(nb, m), np.full(nb, n), l, k_max, tol=tol, seed=seed)
    ctx.bind(A)
    prod = torch.cuda.current_stream()
    sk = torch.cuda.Stream()
    F = solver.F0.clone()
    print("case: in-situ overlap", flush=True)
    for j in range(n):
        for _ in range(3):
            solver.step(F)
        solver.store(F, A, j)
        ev = torch.cuda.Event()
        ev.record(prod)
        sk.wait_event(ev)
        ctx.sketch_update(j, 1, stream=sk)
    ctx.select(sk)
    ctx.coeffs(sk)
    ctx.reconstruct(stream=sk)
    torch.cuda.synchronize()
    Y_situ = ctx.sketch().cpu().numpy()
    S, k, st = ctx.S.cpu().numpy(), ctx.k.cpu().numpy(), ctx.status.cpu().numpy()
    P = [ctx.block_P(b) for b in range(nb)]
    err2, nrm2 = ctx.err2.cpu().numpy(), ctx.nrm2.cpu().numpy()
    # the same data sketched in one batch update
    ctx.sketch_update()
    torch.cuda.synchronize()
    Y_batch = ctx.sketch().cpu().numpy()
    ctx.close()
    scale = np.abs(Y_batch).max()
    assert np.abs(Y_situ - Y_batch).max() <= 1e-13 * scale
    blocks = [np.asfortranarray(A[b].cpu().numpy().T) for b in range(nb)]
    o = oracle_run(blocks, l, k_max, seed, tol=tol)
    from _harness import GpuResult
    Ys = [Y_situ[b * l * n:(b + 1) * l * n].reshape(n, l).T for b in range(nb)]
    g = GpuResult(Ys, S, k, st, P, err2, nrm2)
    stats = compare(g, o)
    e_gpu = float(np.sqrt(err2.sum() / nrm2.sum()))
    print(f"in-situ: e_gpu={e_gpu:.3e} e_oracle={o.rel_error:.3e} k={k} "
          f"prefix={stats['prefix']}")
    assert min(stats["prefix"]) >= 1
