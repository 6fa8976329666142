"""Benchmark: snapshot GB/s compressed by the sketched column ID on one MI355X.

A step is one pass of the whole method over the resident batch: sketch
update over every column, column selection, coefficients and the
reconstruction-error pass.  The timed region starts with the snapshot matrices
already in HBM.  Prints one JSON line (rank 0).

Default workload: the turbulence-like 256^3 field (rho, u, v, w, p; FP32),
4096 blocks of 16^3 (m_b = 20480), 512 snapshots, k = 32, l = 48, bfloat16
sketch with FP32 accumulation and FP64 selection / coefficients, timed beside
the plain FP64 method on the same resident data.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"f64": 78.6, "f64_vector": 78.6, "f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="turb256_b4096_bf16")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-max-blocks", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--graph", action="store_true",
                    help="capture one step into a HIP graph and time graph replays")
    ap.add_argument("--no-autotune", action="store_true",
                    help="library default launch shapes instead of the autotuned ones")
    ap.add_argument("--tune-cache", default=None,
                    help="JSON table of tuned shapes (default: the package's table)")
    ap.add_argument("--no-fp64-compare", action="store_true",
                    help="skip timing the plain FP64 path on a mixed-precision workload")
    ap.add_argument("--insitu", action="store_true",
                    help="measure the in-situ overhead instead: a stand-in solver produces the "
                         "snapshots on one stream, the sketch updates run on another")
    ap.add_argument("--solver-substeps", type=int, default=1,
                    help="--insitu: solver steps per stored snapshot")
    ap.add_argument("--data", choices=("workload", "gaussian"), default="workload",
                    help="gaussian: the workload's block shapes with i.i.d. N(0,1) entries drawn "
                         "by a few generator calls (profiling runs with few non-library kernels)")
    ap.add_argument("--profile-region", action="store_true",
                    help="mark only the timed steps for rocprofv3 --selected-regions "
                         "(roctxProfilerResume / roctxProfilerPause): data generation, tuning, "
                         "the oracle and the FP64 comparison are left out of the profile")
    return ap.parse_args()


class ProfileRegion:
    """roctxProfilerResume(0) / roctxProfilerPause(0) around the timed steps when
    --profile-region is given (no-op otherwise)."""

    def __init__(self, on: bool):
        self.lib = None
        if on:
            import ctypes
            self.lib = ctypes.CDLL(os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib",
                                                "librocprofiler-sdk-roctx.so"))
            self.lib.roctxProfilerResume.argtypes = [ctypes.c_uint64]
            self.lib.roctxProfilerPause.argtypes = [ctypes.c_uint64]

    def resume(self):
        if self.lib is not None:
            self.lib.roctxProfilerResume(0)

    def pause(self):
        if self.lib is not None:
            self.lib.roctxProfilerPause(0)


def log(args, *a):
    if not args.quiet:
        print("[bench]", *a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this build measures one GPU only: the blocks are "
                          "independent and a multi-GPU run would shard them with no exchange; "
                          "run with --gpus 1"}))
        sys.exit(2)
    import torch
    import spid_inputs as si
    import paper_2103_01380_amd as sp

    w = si.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    if args.insitu:
        insitu(args, w, dev)
        return
    t0 = time.time()
    def progress(f, j):
        if j == 0 or j == w.n - 1:
            log(args, f"  generating field {f} snapshot {j}")
    if args.data == "gaussian":
        A, m, n, off = si.gaussian_like(w, device=dev)
    else:
        A, m, n, off = si.generate(w, device=dev, progress=progress)
    torch.cuda.synchronize()
    log(args, f"generated {w.name}: {A.numel() * A.element_size() / 1e9:.2f} GB in "
              f"{time.time() - t0:.1f}s")
    nbytes = int((m * n.astype(np.int64)).sum()) * w.elem_bytes
    stream = torch.cuda.current_stream()
    tuning = None
    coarse = w.subsample > 0
    if not args.no_autotune and not coarse and not w.ts_windows:
        from paper_2103_01380_amd import autotune as at
        t0 = time.time()
        tuning = at.autotune(A, m, n, w.l, w.k_max, offsets=off, tol=w.tol, seed=w.omega_seed,
                             a_dtype=w.a_dtype, prec=w.prec, lp_terms=w.lp_terms,
                             stream_columns=w.stream, cache=args.tune_cache or at.CACHE,
                             log=(lambda s: log(args, s)))
        log(args, f"launch shapes {tuning} ({time.time() - t0:.1f}s)")
    ctx = sp.SPID(m, n, w.l, w.k_max, tol=w.tol, seed=w.omega_seed,
                  a_dtype=w.a_dtype, prec=w.prec, lp_terms=w.lp_terms, device=dev, tuning=tuning,
                  grids=w.grids() if coarse else None, ts_windows=w.ts_windows, ts_k1=w.ts_k1)
    ctx.bind(A, offsets=off)
    region = ProfileRegion(args.profile_region)
    region.resume()
    ms_step, stage, wall = time_steps(args, ctx, w, stream)
    torch.cuda.synchronize()
    region.pause()
    graph_ms = None
    if args.graph:
        # one step captured into a HIP graph, replayed for the same number of steps
        graph = torch.cuda.CUDAGraph()
        cap = torch.cuda.Stream()
        cap.wait_stream(stream)
        with torch.cuda.stream(cap):
            with torch.cuda.graph(graph, stream=cap):
                ctx.run(stream=cap)
        stream.wait_stream(cap)
        graph.replay()
        torch.cuda.synchronize()
        t0g = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0g) * 1e3 / args.steps
        log(args, f"graph replay: {graph_ms:.3f} ms per step")
    value = nbytes / (ms_step * 1e-3) / 1e9
    kk = ctx.k.cpu().numpy()
    if coarse:
        # single-pass ID: the error of M B(:,S) C, the stored skeleton has m_c rows
        rel_err = float((ctx.err2_interp.sum() / ctx.nrm2.sum()).sqrt())
        ms_rows = ctx.mc
    else:
        rel_err = rel_error(ctx)
        ms_rows = m
    cf = float((m * n.astype(np.int64)).sum() / max(1, (kk * (ms_rows + n)).sum()))
    # bytes-CF: the stored skeleton in the data's type, the coefficients in FP64
    cf_bytes = float(nbytes / max(1, (kk * (ms_rows * w.elem_bytes + n.astype(np.int64) * 8)).sum()))
    blocks_err = per_block_errors(ctx, coarse)
    log(args, f"stage ms: sketch {stage[0]:.3f} select {stage[1]:.3f} coeffs {stage[2]:.3f} "
              f"recon {stage[3]:.3f}; step {ms_step:.3f} ms; rel err {rel_err:.3e}")

    work = stage_work(w, m, n, kk, nbytes, ctx)
    roof = dominant_roofline(w, stage, work)
    step_roof = step_roofline(w, stage, work, ms_step)

    cpu = None
    agree = None
    if not args.no_cpu_baseline:
        cpu, agree = cpu_baseline(args, w, A, m, n, off, ctx)

    fp64 = None
    if w.prec not in ("f64", "subsample") and not args.no_fp64_compare:
        # the plain FP64 method on the same resident data: FP64 sketch and FP64 error pass
        ctx64 = sp.SPID(m, n, w.l, w.k_max, tol=w.tol, seed=w.omega_seed, a_dtype=w.a_dtype,
                        prec="f64", device=dev)
        ctx64.bind(A, offsets=off)
        ms64, stage64, _ = time_steps(args, ctx64, w, stream)
        fp64 = {"ms_per_step": round(ms64, 4), "value": round(nbytes / (ms64 * 1e-3) / 1e9, 2),
                "rel_error": rel_error(ctx64),
                "stage_ms": {k: round(v, 4) for k, v in zip(STAGES, stage64)}}
        log(args, f"plain FP64 path: {ms64:.3f} ms per step, rel err {fp64['rel_error']:.3e}")
        ctx64.close()

    out = {
        "metric": "snapshot GB/s compressed at rel. err <= 1e-3 (sketched column ID: sketch + "
                  "CPQR select + coefficients + reconstruction error)",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if w.prec in ("f64", "subsample") else f"{w.prec}-sketch/f64",
        "data": "synthetic" if args.data == "workload" else "synthetic, i.i.d. gaussian entries",
        "config": {"workload": w.name, "description": w.description,
                   "nblocks": int(len(m)), "bytes": nbytes, "l": w.l, "k_max": w.k_max,
                   "tol": w.tol, "sketch_update": "one snapshot per call" if w.stream
                   else "all snapshots in one call",
                   "sketch": (f"coarse grid, every {w.subsample}th point; error of M B(:,S) C"
                              if coarse else "Gaussian, " + w.prec),
                   "two_stage": ({"windows": w.ts_windows, "k1": w.ts_k1}
                                 if w.ts_windows else None)},
        "rel_error": rel_err,
        "error_gate_1e-3": bool(rel_err <= 1e-3),
        "compression_factor": round(cf, 3),
        "compression_factor_bytes": round(cf_bytes, 3),
        "k_mean": float(kk.mean()),
        "k_histogram": k_histogram(kk),
        "block_rel_error": blocks_err,
        "graph_ms_per_step": None if graph_ms is None else round(graph_ms, 4),
        "stage_ms": {k: round(v, 4) for k, v in zip(STAGES, stage)},
        "launch_shapes": ctx.tuning,
        "roofline": roof,
        "roofline_step": step_roof,
        "cpu_baseline": cpu,
        "oracle_agreement": agree,
        "fp64_path": fp64,
        "speedup_vs_fp64": None if fp64 is None else round(fp64["ms_per_step"] / ms_step, 3),
    }
    print(json.dumps(out), flush=True)
    ctx.close()


STAGES = ("sketch", "select", "coeffs", "reconstruct")


def per_block_errors(ctx, coarse):
    """Distribution of the per-block relative errors sqrt(err2_b / nrm2_b) (the gate
    uses the global error; Section 5.1 reports field-level errors)."""
    e2 = (ctx.err2_interp if coarse else ctx.err2).cpu().numpy()
    n2 = ctx.nrm2.cpu().numpy()
    e = np.sqrt(e2 / np.where(n2 > 0, n2, 1.0))
    q = np.quantile(e, [0.5, 0.9, 0.99])
    return {"max": float(e.max()), "argmax_block": int(e.argmax()), "p50": float(q[0]),
            "p90": float(q[1]), "p99": float(q[2]), "mean": float(e.mean()),
            "blocks_over_1e-3": int((e > 1e-3).sum())}


def k_histogram(kk):
    """Selected ranks: {k: number of blocks}."""
    vals, cnt = np.unique(kk, return_counts=True)
    return {str(int(v)): int(c) for v, c in zip(vals, cnt)}


def insitu(args, w, dev):
    """In-situ compression (Sections 3.3-3.4, Algorithms 4-5): a stand-in solver
    advances the velocity field one step at a time and stores each snapshot into
    the resident data matrix (the store task); the sketch update of that snapshot
    runs on a second stream behind an event, so it overlaps the next solver step.
    The overhead is the extra wall time over the solver alone; the selection,
    coefficients and error pass run once after the last step.

    Stand-in solver: ``spid_inputs.StandInSolver`` (linear advection-diffusion of
    the three Taylor-Green velocity components, the application, not the
    compression path)."""
    import torch
    import paper_2103_01380_amd as sp
    assert w.kind == "tgv" and not w.subsample and not w.ts_windows
    import spid_inputs as si
    N, B = w.N, w.B
    E = N // B
    nb = B ** 3
    solver = si.StandInSolver(N, B, w.nu, dev)
    F0 = solver.F0
    solver_step = solver.step
    A = torch.empty((nb, w.n, 3 * E ** 3), dtype=torch.float64, device=dev)

    def store(F, j):
        solver.store(F, A, j)

    m = np.full(nb, 3 * E ** 3, dtype=np.int64)
    n = np.full(nb, w.n, dtype=np.int32)
    ctx = sp.SPID(m, n, w.l, w.k_max, tol=w.tol, seed=w.omega_seed, device=dev)
    ctx.bind(A)
    prod = torch.cuda.current_stream()
    sk = torch.cuda.Stream()

    def run(mode):
        F = F0.clone()
        evs = [torch.cuda.Event() for _ in range(w.n)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for j in range(w.n):
            for _ in range(args.solver_substeps):
                solver_step(F)
            store(F, j)
            if mode == "overlap":
                evs[j].record(prod)
                sk.wait_event(evs[j])
                ctx.sketch_update(j, 1, stream=sk)
            elif mode == "serial":
                ctx.sketch_update(j, 1, stream=prod)
        torch.cuda.synchronize()
        t_loop = time.perf_counter() - t0
        t1 = time.perf_counter()
        if mode != "solver":
            s = sk if mode == "overlap" else prod
            ctx.select(s)
            ctx.coeffs(s)
            ctx.reconstruct(stream=s)
            torch.cuda.synchronize()
        return t_loop, time.perf_counter() - t1

    run("overlap")                                               # warm-up (compiles, caches)
    reps = max(1, args.steps // 5)
    t = {}
    for mode in ("solver", "overlap", "serial"):
        best = None
        for _ in range(reps):
            r = run(mode)
            best = r if best is None or r[0] < best[0] else best
        t[mode] = best
        log(args, f"in-situ {mode}: loop {best[0] * 1e3:.2f} ms, after-loop {best[1] * 1e3:.2f} ms")
    over = (t["overlap"][0] / t["solver"][0] - 1.0) * 100.0
    rel = rel_error(ctx)
    kk = ctx.k.cpu().numpy()
    out = {
        "metric": "in-situ overhead of the per-snapshot sketch updates over the stand-in solver",
        "value": round(over, 2), "unit": "%", "n_gpus": 1, "steps": reps, "warmup": 1,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name + "_insitu", "snapshots": w.n, "nblocks": nb,
                   "solver": f"advection-diffusion, {N}^3 x 3 fields, central differences, "
                             f"explicit Euler, {args.solver_substeps} step(s) per snapshot",
                   "l": w.l, "k_max": w.k_max, "tol": w.tol},
        "solver_ms": round(t["solver"][0] * 1e3, 3),
        "solver_plus_sketch_overlapped_ms": round(t["overlap"][0] * 1e3, 3),
        "solver_plus_sketch_serial_ms": round(t["serial"][0] * 1e3, 3),
        "serial_overhead_pct": round((t["serial"][0] / t["solver"][0] - 1.0) * 100.0, 2),
        "after_last_step_ms": round(t["overlap"][1] * 1e3, 3),
        "rel_error": rel, "k_mean": float(kk.mean()),
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def time_steps(args, ctx, w, stream):
    """Warm-up, then ``args.steps`` timed steps; returns (ms per step, stage ms, wall s).
    A step is the whole method: the sketch of every snapshot (one update per
    snapshot for a streamed workload), selection, coefficients, error pass."""
    import torch
    nmax = int(ctx.n.max())

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        if w.stream:
            for j in range(nmax):
                ctx.sketch_update(j, 1, stream=stream)
        else:
            ctx.sketch_update(stream=stream)
        if ev is not None:
            ev[1].record(stream)
        if w.ts_windows:
            # both stages, pivots and coefficients in one call (reported as "select")
            ctx.select_two_stage(stream)
        else:
            ctx.select(stream)
        if ev is not None:
            ev[2].record(stream)
        if not w.ts_windows:
            ctx.coeffs(stream)
        if ev is not None:
            ev[3].record(stream)
        if w.subsample:
            ctx.reconstruct_interp(stream=stream)
        else:
            ctx.reconstruct(stream=stream)
        if ev is not None:
            ev[4].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        step(evs[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    stage = np.zeros(4)
    for e in evs:
        for i in range(4):
            stage[i] += e[i].elapsed_time(e[i + 1])
    stage /= args.steps
    return wall * 1e3 / args.steps, stage, wall


def rel_error(ctx) -> float:
    """The gate's global relative Frobenius error: sqrt(sum err2 / sum nrm2)."""
    return float((ctx.err2.sum() / ctx.nrm2.sum()).sqrt())


def stage_work(w, m, n, kk, nbytes, ctx=None):
    """Algorithmic (bytes, flops, flop peak) per stage: what the method must do."""
    n64 = n.astype(np.int64)
    k64 = kk.astype(np.int64)
    if w.subsample:
        # coarse grid: the sketch gathers m_c rows and writes the l-row sketch; the
        # error pass reads A once, 2k flops per entry plus the 8-point stencil of each
        # skeleton entry (FP64 vector arithmetic)
        mc = ctx.mc.astype(np.int64)
        sk_bytes = int((mc * n64).sum()) * w.elem_bytes + 8 * w.l * int(n64.sum())
        sel_flops = float((4.0 * w.l * k64 * (n64 - (k64 - 1) / 2.0)).sum())
        co_flops = float((k64 * k64 * (n64 - k64)).sum())
        ip_flops = 2.0 * float((m * n64 * k64).sum()) + 16.0 * float((m * k64).sum())
        sel_bytes = 0
        if w.l > 128:
            # tall sketch selected in global memory: what the method must move is one
            # read of the sketch (the kernel's own per-step streaming of its working copy
            # is design traffic, not algorithmic)
            sel_bytes = int(8 * w.l * int(n64.sum()))
        return {
            "sketch": (sk_bytes, 0.0, PEAK_TFLOPS["f64_vector"]),
            "select": (sel_bytes, sel_flops, PEAK_TFLOPS["f64_vector"]),
            "coeffs": (0, co_flops, PEAK_TFLOPS["f64_vector"]),
            "reconstruct": (nbytes, ip_flops, PEAK_TFLOPS["f64_vector"]),
        }
    sk_flops = 2.0 * w.l * float((m * n64).sum())
    sel_flops = float((4.0 * w.l * k64 * (n64 - (k64 - 1) / 2.0)).sum())
    co_flops = float((k64 * k64 * (n64 - k64)).sum())
    if w.ts_windows:
        # stage 1 on every window at rank k1, stage 2 on nwin * k1 columns, and C^1 C^{0'}
        nw, k1 = w.ts_windows, w.ts_k1
        n2 = nw * k1
        sel_flops = float((nw * 4.0 * w.l * k1 * (n64 / nw - (k1 - 1) / 2.0)
                           + 4.0 * w.l * k64 * (n2 - (k64 - 1) / 2.0)).sum())
        co_flops = float((nw * k1 * k1 * (n64 / nw - k1) + k64 * k64 * (n2 - k64)
                          + 2.0 * k64 * k1 * n64).sum())
    rc_flops = 2.0 * float((m * (n64 - k64) * k64).sum())
    sk_peak = PEAK_TFLOPS["f64" if w.prec == "f64" else w.prec]
    rc_peak = PEAK_TFLOPS["f64" if (w.a_dtype == "f64" or w.prec == "f64") else "bf16"]
    return {
        "sketch": (nbytes, sk_flops, sk_peak),
        "select": (0, sel_flops, PEAK_TFLOPS["f64"]),
        "coeffs": (0, co_flops, PEAK_TFLOPS["f64"]),
        "reconstruct": (nbytes, rc_flops, rc_peak),
    }


def dominant_roofline(w, stage, work):
    """Roofline of the slowest streaming kernel: algorithmic bytes or flops over its
    average launch time (HIP events on its launch stream), against the closer roof."""
    t = dict(zip(STAGES, stage))
    # streaming kernels: the sketch, the error pass, and a selection that streams
    # its working copy through HBM (tall coarse sketches)
    cand = [x for x in STAGES if x in ("sketch", "reconstruct") or work[x][0] > 0]
    dom = max(cand, key=lambda x: t[x])
    b_alg, f_alg, peak_t = work[dom]
    t_s = t[dom] * 1e-3
    gbs = b_alg / t_s / 1e9
    tfl = f_alg / t_s / 1e12
    if tfl / peak_t > gbs / PEAK_HBM_GBS:
        roof = {"bound": "alu" if w.subsample else "mfma", "achieved": round(tfl, 3),
                "peak": peak_t, "unit": "TFLOP/s", "frac": round(tfl / peak_t, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(gbs / PEAK_HBM_GBS, 4)}
    roof["kernel"] = dom
    roof["traffic"] = measured_traffic(w.name, dom)
    return roof


def kernel_source_digest() -> str:
    """Digest of the kernel sources; counter records are valid only for this digest."""
    import hashlib
    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2103_01380_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith(".h"):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the recorded rocprofv3 counters
    (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, each scaled by what the counter
    reads for a plain copy of known size); None when no record exists or the kernels
    changed since it was taken."""
    path = os.path.join(ROOT, "paper_2103_01380_amd", "measured_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(workload)
    if not rec or rec.get("kernel_source_sha1") != kernel_source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k:
        return None
    kib = rec["fetch_factor"] * k["fetch_kib"] + rec["write_factor"] * (k.get("write_kib") or 0.0)
    return round(kib * 1024.0)


def step_roofline(w, stage, work, ms_step):
    """T_roof = sum over stages of max(bytes / HBM peak, flops / matrix-core peak);
    frac = T_roof / measured step time."""
    per = {}
    t_roof = 0.0
    for name, ms in zip(STAGES, stage):
        b, f, peak_t = work[name]
        t = max(b / (PEAK_HBM_GBS * 1e9), f / (peak_t * 1e12)) * 1e3
        per[name] = {"t_roof_ms": round(t, 4), "frac": round(t / ms, 4) if ms > 0 else None}
        t_roof += t
    return {"t_roof_ms": round(t_roof, 4), "frac": round(t_roof / ms_step, 4), "stages": per}


def oracle_agreement(w, A, m, n, off, ctx, idx, res):
    """The GPU's factors against the oracle's on the oracle's sample of blocks:
    relative errors of both, the A-space difference of the two reconstructions
    (R2) and how many blocks select the oracle's columns over the decidable prefix."""
    import torch
    gamma = {"f64": 1e-10, "subsample": 1e-10, "bf16": 1e-3, "fp8": 1e-2}[w.prec]
    S = ctx.S.cpu().numpy()
    k = ctx.k.cpu().numpy()
    e2g = ctx.err2.cpu().numpy()
    n2g = ctx.nrm2.cpu().numpy()
    num = den = 0.0
    match = full = 0
    flat = A.reshape(-1)
    for r, b in enumerate(idx):
        b = int(b)
        mb, nb_ = int(m[b]), int(n[b])
        Ad = flat[int(off[b]):int(off[b]) + mb * nb_].view(nb_, mb).t().double()
        kg, ko = int(k[b]), int(res.k[r])
        Pg = torch.from_numpy(np.ascontiguousarray(ctx.block_P(b)[:kg])).to(Ad.device)
        Po = torch.from_numpy(np.ascontiguousarray(res.P[r][:ko])).to(Ad.device)
        ag = Ad[:, torch.from_numpy(S[b][:kg].astype(np.int64)).to(Ad.device)] @ Pg
        ao = Ad[:, torch.from_numpy(res.S[r][:ko].astype(np.int64)).to(Ad.device)] @ Po
        num += float(((ag - ao) ** 2).sum())
        den += float(n2g[b])
        s_star = 0
        while s_star < min(kg, ko) and res.gaps[r][s_star] > gamma:
            s_star += 1
        if np.array_equal(S[b][:s_star], res.S[r][:s_star]):
            match += 1
        if s_star == ko and kg == ko and np.array_equal(S[b][:kg], res.S[r][:ko]):
            full += 1
    extra = {}
    if w.subsample:
        i2g = ctx.err2_interp.cpu().numpy()
        extra = {"gpu_rel_interp_error": float(np.sqrt(i2g[idx].sum() / n2g[idx].sum())),
                 "oracle_rel_interp_error": res.rel_interp_error}
    return {"blocks": int(len(idx)), **extra,
            # the coarse-grid step measures the single-pass error only (no SubID pass)
            "gpu_rel_error": (None if w.subsample else
                              float(np.sqrt(e2g[idx].sum() / n2g[idx].sum()))),
            "oracle_rel_error": res.rel_error,
            "R2": float(np.sqrt(num / den)) if den > 0 else 0.0,
            "gap_gamma": gamma,
            "prefix_match_blocks": int(match),
            "identical_selection_blocks": int(full)}


def cpu_baseline(args, w, A, m, n, off, ctx):
    """The oracle, as it stands, timed on a bounded sample of the same blocks.

    A first batch (one block per thread) measures the per-block cost; the
    sample then grows to about ``--cpu-seconds`` of wall time."""
    import spid_inputs as si
    import oracle
    nb = len(m)
    threads = len(os.sched_getaffinity(0))
    rng = np.random.default_rng(0)
    order = rng.permutation(nb)
    prec = {"f64": oracle.OMEGA_F64, "bf16": oracle.OMEGA_BF16, "fp8": oracle.OMEGA_FP8E4M3,
            "subsample": oracle.OMEGA_F64}
    grids = w.grids() if w.subsample else None

    def two_stage_batch(blocks):
        # sketch, both stages and the error per block, one block per thread
        from concurrent.futures import ThreadPoolExecutor

        def one(Ab):
            Y = oracle.sketch(Ab, w.l, w.omega_seed, prec=prec[w.prec])
            ts = oracle.two_stage(Y, w.ts_windows, w.ts_k1, w.k_max, w.tol)
            e2, a2 = oracle.reconstruct(Ab, ts.S, ts.k, ts.P)
            return Y, ts, e2, a2
        with ThreadPoolExecutor(threads) as ex:
            out = list(ex.map(one, blocks))
        return oracle.BatchResult([o[0] for o in out], np.stack([o[1].S for o in out]),
                                  np.array([o[1].k for o in out]),
                                  np.array([o[1].status for o in out]),
                                  [o[1].P for o in out], np.stack([o[1].gaps for o in out]),
                                  np.array([o[2] for o in out]), np.array([o[3] for o in out]))

    def run(idx):
        blocks = [si.block_view(A, m, n, off, int(b)) for b in idx]
        t0 = time.perf_counter()
        if w.ts_windows:
            res = two_stage_batch(blocks)
        else:
            res = oracle.run_batch(blocks, l=w.l, k_max=w.k_max, seed=w.omega_seed, tol=w.tol,
                                   prec=prec[w.prec], nthreads=threads,
                                   grids=None if grids is None else grids[idx])
        dt = time.perf_counter() - t0
        return dt, int(sum(b.shape[0] * b.shape[1] for b in blocks)) * w.elem_bytes, res

    first = order[:min(threads, nb)]
    dt1, b1, _ = run(first)
    per_block = dt1 / len(first)
    want = int(max(len(first), min(nb, args.cpu_seconds / max(per_block, 1e-9))))
    want = min(want, args.cpu_max_blocks)
    idx = np.sort(order[:want])
    dt, sbytes, res = run(idx)
    log(args, f"cpu oracle: {len(idx)} blocks, {threads} threads, {dt:.1f}s, "
              f"rel err {res.rel_error:.3e}")
    agree = oracle_agreement(w, A, m, n, off, ctx, idx, res)
    log(args, f"oracle agreement: {agree}")
    total_bytes = int((m * n.astype(np.int64)).sum()) * w.elem_bytes
    # one core: the first blocks of the sample, about a tenth of the multi-thread time
    one = None
    if not w.ts_windows:
        n1 = int(max(1, min(len(idx), round(0.1 * args.cpu_seconds / max(per_block * threads,
                                                                           1e-9)))))
        sel1 = idx[:n1]
        blocks1 = [si.block_view(A, m, n, off, int(b)) for b in sel1]
        t0 = time.perf_counter()
        oracle.run_batch(blocks1, l=w.l, k_max=w.k_max, seed=w.omega_seed, tol=w.tol,
                         prec=prec[w.prec], nthreads=1,
                         grids=None if grids is None else grids[sel1])
        dt1c = time.perf_counter() - t0
        b1c = int(sum(b.shape[0] * b.shape[1] for b in blocks1)) * w.elem_bytes
        one = {"value": round(b1c / dt1c / 1e9, 5), "unit": "GB/s", "cores": 1,
               "blocks": int(n1), "seconds": round(dt1c, 2),
               "full_config_s_extrapolated": round(total_bytes / (b1c / dt1c), 1)}
        log(args, f"cpu oracle, one core: {n1} blocks in {dt1c:.1f}s")
    return {"value": round(sbytes / dt / 1e9, 5), "unit": "GB/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{len(idx)} of {nb} blocks (seeded choice), whole method per block "
                      f"(sketch, select, coefficients, error), {dt:.1f} s wall on {threads} "
                      f"threads" + ("; the oracle also forms the SubID error (a second pass "
                                    "over A)" if w.subsample else ""),
            "full_config_s_extrapolated": round(total_bytes / (sbytes / dt), 1),
            "one_core": one}, agree


if __name__ == "__main__":
    main()
