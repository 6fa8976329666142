"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the CPU oracle on the same bytes, and compare them by the gap rule."""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import torch

import oracle

PREC_OMEGA = {"f64": oracle.OMEGA_F64, "bf16": oracle.OMEGA_BF16, "fp8": oracle.OMEGA_FP8E4M3}


@dataclass
class GpuResult:
    Y: list
    S: np.ndarray
    k: np.ndarray
    status: np.ndarray
    P: list
    err2: np.ndarray
    nrm2: np.ndarray
    skel: list | None = None
    ierr2: np.ndarray | None = None      # single-pass (interpolated) error, coarse grids
    cskel: list | None = None            # coarse skeleton B(:,S), coarse grids
    tuning: dict | None = None           # launch shapes in effect

    @property
    def rel_interp_error(self):
        return float(math.sqrt(self.ierr2.sum() / self.nrm2.sum()))

    @property
    def rel_error(self):
        return float(math.sqrt(self.err2.sum() / self.nrm2.sum()))


def gpu_run(blocks, l, k_max, seed, tol=0.0, rank_floor=0.0, omega_per_block=False,
            prec="f64", lp_terms=1, skeleton=False, stream_columns=False, lda_pad=0,
            grids=None, tuning=None, graph_replays=0):
    """Run the four stages on the GPU for host column-major blocks.  ``grids``: the
    coarse-grid sketch (SubID) plus the single-pass error and coarse skeleton.
    ``graph_replays``: after the eager run, capture the four stages into one HIP
    graph and replay it that many times (eager work between the replays),
    asserting every replay equal to the eager results bit for bit."""
    import paper_2103_01380_amd as sp
    dt = blocks[0].dtype
    a_dtype = "f64" if dt == np.float64 else "f32"
    m = np.array([b.shape[0] for b in blocks], dtype=np.int64)
    n = np.array([b.shape[1] for b in blocks], dtype=np.int32)
    lda = m + lda_pad
    sizes = lda * n
    off = np.zeros(len(blocks), dtype=np.int64)
    off[1:] = np.cumsum(sizes[:-1])
    flat = np.zeros(int(sizes.sum()), dtype=dt)
    for b, blk in enumerate(blocks):
        v = np.zeros((n[b], lda[b]), dtype=dt)
        v[:, :m[b]] = blk.T
        flat[off[b]:off[b] + sizes[b]] = v.ravel()
    A = torch.from_numpy(flat).cuda()
    if grids is not None:
        prec = "subsample"
    ctx = sp.SPID(m, n, l, k_max, tol=tol, rank_floor=rank_floor, seed=seed,
                  omega_per_block=omega_per_block, a_dtype=a_dtype, prec=prec,
                  lp_terms=lp_terms, grids=grids, tuning=tuning)
    l = ctx.l
    ctx.bind(A, offsets=off, lda=lda)
    if stream_columns:
        for j in range(int(n.max())):
            ctx.sketch_update(j, 1)
    else:
        ctx.sketch_update()
    ctx.select()
    ctx.coeffs()
    skel_t = None
    if skeleton:
        skel_t = torch.full((int((m * k_max).sum()),), float("nan"), dtype=A.dtype, device=A.device)
    ctx.reconstruct(skeleton=skel_t)
    if graph_replays:
        torch.cuda.synchronize()
        outs = (ctx.S, ctx.k, ctx.status, ctx.P, ctx.err2, ctx.nrm2)
        ref = [t.clone() for t in outs]
        ref_y = ctx.sketch()
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cap):
            with torch.cuda.graph(graph, stream=cap):
                ctx.run(cap)
        torch.cuda.current_stream().wait_stream(cap)
        torch.cuda.synchronize()
        for rep in range(graph_replays):
            for t in outs:
                t.fill_(7)                      # eager work between replays
            graph.replay()
            torch.cuda.synchronize()
            for a, b in zip(outs, ref):
                assert torch.equal(a, b), rep
            assert torch.equal(ctx.sketch(), ref_y), rep
    cs_t = None
    if grids is not None:
        mc = ctx.mc
        cs_t = torch.full((int((mc * k_max).sum()),), float("nan"), dtype=A.dtype, device=A.device)
        ctx.reconstruct_interp(coarse_skeleton=cs_t)
    torch.cuda.synchronize()
    Yf = ctx.sketch().cpu().numpy()
    Ys = [Yf[ctx.y_off[b]:ctx.y_off[b] + l * n[b]].reshape(n[b], l).T for b in range(len(blocks))]
    Ps = [ctx.block_P(b) for b in range(len(blocks))]
    skel = None
    if skeleton:
        sk = skel_t.cpu().numpy()
        so = np.zeros(len(blocks), dtype=np.int64)
        so[1:] = np.cumsum((m * k_max)[:-1])
        skel = [sk[so[b]:so[b] + m[b] * k_max].reshape(k_max, m[b]).T for b in range(len(blocks))]
    ierr2 = cskel = None
    if grids is not None:
        ierr2 = ctx.err2_interp.cpu().numpy()
        cs = cs_t.cpu().numpy()
        co = np.zeros(len(blocks), dtype=np.int64)
        co[1:] = np.cumsum((ctx.mc * k_max)[:-1])
        cskel = [cs[co[b]:co[b] + ctx.mc[b] * k_max].reshape(k_max, ctx.mc[b]).T
                 for b in range(len(blocks))]
    res = GpuResult(Ys, ctx.S.cpu().numpy(), ctx.k.cpu().numpy(), ctx.status.cpu().numpy(), Ps,
                    ctx.err2.cpu().numpy(), ctx.nrm2.cpu().numpy(), skel, ierr2, cskel,
                    dict(ctx.tuning))
    ctx.close()
    return res


def oracle_run(blocks, l, k_max, seed, tol=0.0, rank_floor=0.0, omega_per_block=False,
               prec="f64", block_ids=None, grids=None):
    return oracle.run_batch(blocks, l=l, k_max=k_max, seed=seed, tol=tol, rank_floor=rank_floor,
                            omega_per_block=omega_per_block, prec=PREC_OMEGA[prec],
                            block_ids=block_ids, grids=grids)


def matched_prefix(S_gpu, S_ora, gaps, k_gpu, k_ora, gamma):
    """Length of the decidable prefix (oracle gap > gamma) and whether it matches."""
    s_star = 0
    kk = min(int(k_gpu), int(k_ora))
    while s_star < kk and gaps[s_star] > gamma:
        s_star += 1
    ok = np.array_equal(S_gpu[:s_star], S_ora[:s_star])
    return s_star, ok


def compare(gpu: GpuResult, ora, gamma=1e-10, y_rtol=1e-13, err_atol=1e-12, p_rtol=1e-9,
            check_k=True):
    """Assert the FP64-path parity rules block by block; returns summary stats."""
    nb = len(gpu.Y)
    stats = {"prefix": [], "full_match": 0}
    for b in range(nb):
        Yg, Yo = gpu.Y[b], ora.Y[b]
        if y_rtol is not None:
            scale = np.linalg.norm(Yo, axis=0).max() + 1e-300
            assert np.abs(Yg - Yo).max() <= y_rtol * scale, (b, np.abs(Yg - Yo).max() / scale)
        s_star, ok = matched_prefix(gpu.S[b], ora.S[b], ora.gaps[b], gpu.k[b], ora.k[b], gamma)
        assert ok, (b, gpu.S[b][:s_star], ora.S[b][:s_star])
        stats["prefix"].append(s_star)
        full = s_star == ora.k[b] and gpu.k[b] == ora.k[b]
        if check_k and full:
            assert gpu.status[b] == ora.status[b], (b, gpu.status[b], ora.status[b])
        if full:
            stats["full_match"] += 1
            kk = int(ora.k[b])
            Pg, Po = gpu.P[b][:kk], ora.P[b][:kk]
            # P = R11^-1 R12 amplifies the rounding-level difference of the two sketches
            # by the condition number of the selected sketch columns
            cond = np.linalg.cond(ora.Y[b][:, ora.S[b][:kk]]) if kk else 1.0
            tol_p = max(p_rtol, 1e-15 * cond) * max(1.0, np.abs(Po).max())
            assert np.abs(Pg - Po).max() <= tol_p, (b, np.abs(Pg - Po).max(), cond)
            assert np.all(gpu.P[b][kk:] == 0.0)
        # identity block is exact
        kg = int(gpu.k[b])
        Sg = gpu.S[b][:kg]
        if kg:
            assert np.array_equal(gpu.P[b][:kg][:, Sg], np.eye(kg)), b
        eg = math.sqrt(gpu.err2[b] / gpu.nrm2[b]) if gpu.nrm2[b] > 0 else 0.0
        eo = math.sqrt(ora.err2[b] / ora.nrm2[b]) if ora.nrm2[b] > 0 else 0.0
        if err_atol is not None:
            assert abs(eg - eo) <= err_atol, (b, eg, eo)
        assert abs(gpu.nrm2[b] - ora.nrm2[b]) <= 1e-13 * ora.nrm2[b] + 1e-300, b
    return stats
