"""Launch-shape autotuner for the batched sketched column ID.

The two streaming stages (sketch update, error pass) have launch shapes that
do not change the method's results, only how the independent blocks of
Section 3.2 are mapped onto the GPU: 16-column MFMA tiles per wave and waves
per workgroup of the sketch, the number of sketch work items (how far blocks
are split along their rows), and the row sub-tiles per error-pass work item.
``autotune`` times every candidate shape on the caller's resident batch with
HIP events (the stage's own stream), keeps the fastest per stage and caches the
choice in a JSON table keyed by the batch signature, so the same workload
reuses it.  Selection and coefficients have no tunable shape.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import SPID

_HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(_HERE, "tuned_shapes.json")


def _mfma_tiles(l: int) -> int:
    t = (l + 15) // 16
    return t if t <= 4 else (6 if t <= 6 else 8)


def signature(m, n, l, k_max, tol, a_dtype, prec, lp_terms, stream_columns=False) -> str:
    """Key of a batch: method parameters plus a digest of the block shapes."""
    m = np.ascontiguousarray(m, dtype=np.int64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    h = hashlib.sha1(m.tobytes() + n.tobytes()).hexdigest()[:16]
    return (f"{prec}|{a_dtype}|l{l}|k{k_max}|tol{tol:g}|t{lp_terms}|nb{len(m)}|"
            f"{'stream' if stream_columns else 'batch'}|{h}")


def sketch_candidates(prec: str, l: int, max_n: int):
    """Sketch shapes the library instantiates for this precision and l."""
    mt = _mfma_tiles(l)
    if prec == "f64":
        tns = [1, 2] if mt <= 4 else [1]
    elif prec == "bf16":
        tns = [1, 2, 4] if mt < 6 else [1, 2]
    else:
        tns = [1]
    shapes = [(tn, 8) for tn in tns if 16 * 8 * tn <= max(128, 2 * max_n)] + [(1, 4)]
    if prec == "bf16":
        shapes = [(0, 8)] + shapes   # tiles sized per block (the library's default)
    out = []
    for tn, nw in shapes:
        for items in (1024, 2048, 4096, 8192):
            out.append({"sk_tn": tn, "sk_nw": nw, "sk_items": items})
    return out


def recon_candidates(a_dtype: str, prec: str):
    if a_dtype == "f32" and prec != "f64":
        return [{}]                      # split-bfloat16 error pass: no shape knob
    return [{"rc_rpi": r} for r in (1, 2, 4, 8, 12, 16)]


def _time(fn, stream, reps):
    import torch
    fn()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps)]
    for r in range(reps):
        ev[2 * r].record(stream)
        fn()
        ev[2 * r + 1].record(stream)
    torch.cuda.synchronize()
    return min(ev[2 * r].elapsed_time(ev[2 * r + 1]) for r in range(reps))


def load_table(path: str = CACHE) -> dict:
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def _store(path: str, key: str, entry: dict):
    table = load_table(path)
    table[key] = entry
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(A, m, n, l, k_max, offsets=None, lda=None, tol=0.0, rank_floor=0.0, seed=0,
             omega_per_block=False, a_dtype="f64", prec="f64", lp_terms=1,
             stream_columns=False, reps=3, cache=CACHE, use_cache=True, log=None) -> dict:
    """Fastest launch shapes for this batch (a ``spid_tuning`` dict).

    ``A``, ``offsets`` and ``lda`` as for :meth:`SPID.bind`.  With
    ``stream_columns`` the sketch is timed as one update per column (w = 1),
    the way a stream of snapshots drives it."""
    import torch
    m = np.ascontiguousarray(m, dtype=np.int64)
    n = np.ascontiguousarray(n, dtype=np.int32)
    key = signature(m, n, l, k_max, tol, a_dtype, prec, lp_terms, stream_columns)
    if use_cache:
        hit = load_table(cache).get(key)
        if hit is not None:
            return dict(hit["tuning"])
    stream = torch.cuda.current_stream()
    kw = dict(tol=tol, rank_floor=rank_floor, seed=seed, omega_per_block=omega_per_block,
              a_dtype=a_dtype, prec=prec, lp_terms=lp_terms, device=A.device)
    nmax = int(n.max())
    t0 = time.time()

    def sketch_all(ctx):
        if stream_columns:
            for j in range(nmax):
                ctx.sketch_update(j, 1, stream=stream)
        else:
            ctx.sketch_update(stream=stream)

    records = []
    best_sk, best_sk_ms = None, float("inf")
    for cand in sketch_candidates(prec, l, nmax):
        ctx = SPID(m, n, l, k_max, tuning=cand, **kw)
        try:
            ctx.bind(A, offsets=offsets, lda=lda)
            ms = _time(lambda: sketch_all(ctx), stream, reps)
        finally:
            ctx.close()
        records.append({"stage": "sketch", **cand, "ms": round(ms, 4)})
        if log:
            log(f"autotune sketch {cand}: {ms:.3f} ms")
        if ms < best_sk_ms:
            best_sk, best_sk_ms = cand, ms
    best_rc, best_rc_ms = {}, float("inf")
    for cand in recon_candidates(a_dtype, prec):
        ctx = SPID(m, n, l, k_max, tuning={**best_sk, **cand}, **kw)
        try:
            ctx.bind(A, offsets=offsets, lda=lda)
            ctx.sketch_update(stream=stream)
            ctx.select(stream)
            ctx.coeffs(stream)
            ms = _time(lambda: ctx.reconstruct(stream=stream), stream, reps)
        finally:
            ctx.close()
        records.append({"stage": "reconstruct", **cand, "ms": round(ms, 4)})
        if log:
            log(f"autotune reconstruct {cand}: {ms:.3f} ms")
        if ms < best_rc_ms:
            best_rc, best_rc_ms = cand, ms
    tuning = {**best_sk, **best_rc}
    if cache:
        _store(cache, key, {"tuning": tuning, "sketch_ms": round(best_sk_ms, 4),
                            "reconstruct_ms": round(best_rc_ms, 4),
                            "seconds": round(time.time() - t0, 2),
                            "device": torch.cuda.get_device_name(A.device),
                            "candidates": records})
    return tuning
