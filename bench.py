#!/usr/bin/env python3
"""Throughput of the converged steady solve: 512 x 512 leakage + variation thermal maps per second.

Workload (one step): a batch of 256 distinct Monte Carlo samples of one 64-block floorplan on a
512 x 512 grid of a 10 mm x 10 mm, 0.5 mm die; threshold-voltage variation (lognormal leakage
scale) and +-5 % conductivity variation, k(T) = k0 (300/T)^1.3, exponential leakage with
beta = 0.017 / K, FP32 maps, Picard iteration to max increment <= tol (default 1e-3 K, fifty
times inside the metric's 0.05 K accuracy bar), then one FP64 application of the fixed-point
map per sample for its residual.  Inputs are resident in HBM before the timed region; the
Green's-function table is built once during warm-up.  The oracle leg solves samples 0, 85, 170
and 255 with the same stopping rule and reports the largest distance of the GPU maps from them;
a side leg repeats the timed steps at tol 0.01 K.

Prints one JSON line (see the keys below).  Only one GPU is used; --gpus > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "converged 512² thermal maps/s at ≤0.05 K max err; surrogate vs plain, same GPU"
HBM_PEAK_GBS = 8000.0


def _sample(i: int, n: int, fft_workers: int = 1, floorplan: int = 0):
    import numpy as np

    import workloads.gen as W

    W.FFT_WORKERS = fft_workers
    inp = W.config2(sample=i, n=n, floorplan=floorplan)
    f = lambda a: a.astype(np.float32)
    return f(inp.q_dyn), f(inp.q_leak0), f(inp.leak_var), f(inp.cond_map)


def _sample_small(seed: int):
    import numpy as np

    import workloads.gen as W

    inp = W.config1(seed=seed, n=64)
    return inp.q_dyn.astype(np.float64), inp.q_leak0.astype(np.float64)


def _sample_mixed(size_class: int, i: int):
    import numpy as np

    import workloads.gen as W

    W.FFT_WORKERS = 1
    inp = W.config3(size_class, i)
    f = lambda a: a.astype(np.float32)
    return size_class, f(inp.q_dyn), f(inp.q_leak0), f(inp.leak_var), f(inp.cond_map)


def generate_extra(args):
    """Inputs of the small-grid and mixed-size legs, made before the GPU is touched."""
    import multiprocessing as mp

    small = mixed = unseen = None
    jobs = []
    if not args.no_small:
        jobs.append("small")
    if not args.no_mixed:
        jobs.append("mixed")
    if not args.no_surrogate and args.unseen_batch > 0:
        jobs.append("unseen")
    if not jobs:
        return None, None, None
    pool = mp.get_context("fork").Pool(max(1, args.workers))
    try:
        if "small" in jobs:
            small = pool.map(_sample_small, range(args.small_batch))
        if "mixed" in jobs:
            # size classes interleaved in the problem array
            mixed = pool.starmap(_sample_mixed, [(c, i) for i in range(args.mixed_batch) for c in range(4)])
        if "unseen" in jobs:
            unseen = pool.starmap(_sample, [(i, args.n, 1, UNSEEN_FLOORPLAN) for i in range(args.unseen_batch)])
    finally:
        pool.close()
        pool.join()
    return small, mixed, unseen


def generate(batch: int, n: int, workers: int):
    if workers <= 1:
        import workloads.gen as W

        saved, W.FFT_WORKERS = W.FFT_WORKERS, -1
        try:
            return [_sample(i, n, fft_workers=-1) for i in range(batch)]
        finally:
            W.FFT_WORKERS = saved
    import multiprocessing as mp

    pool = mp.get_context("fork").Pool(workers)
    try:
        out = pool.starmap(_sample, [(i, n) for i in range(batch)])
    finally:
        pool.close()  # workers exit on their own (no signal)
        pool.join()
    return out


def stream_ceiling(n: int, batch: int, buffers: int = 6, reps: int = 24) -> dict:
    """What plain streaming reaches on this GPU at the batch's footprint, as context for the
    roofline fraction (the fraction itself is taken against the published 8 TB/s): an in-place
    scale (read + write, the access pattern of the solver's passes) and a copy, over `buffers`
    rotating arrays of one batch-sized plane each, so that the 256 MB last-level cache holds
    none of the next launch's data."""
    import torch

    dev = torch.device("cuda", 0)
    planes = [torch.ones((batch, n, n), dtype=torch.float32, device=dev) for _ in range(buffers)]
    nbytes = 2 * planes[0].numel() * 4

    def timed(fn):
        for k in range(buffers):
            fn(k)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for k in range(reps):
            fn(k)
        e1.record()
        e1.synchronize()
        return nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9

    inplace = timed(lambda k: planes[k % buffers].mul_(1.0001))
    copy = timed(lambda k: planes[(k + 1) % buffers].copy_(planes[k % buffers]))
    del planes
    torch.cuda.empty_cache()
    return {"inplace_GBps": round(inplace, 1), "copy_GBps": round(copy, 1),
            "method": f"torch in-place mul_ / copy_ over {buffers} rotating {batch}x{n}x{n} FP32 planes"}


def algorithmic_bytes(n: int) -> dict:
    """Bytes each kernel class must move per map it processes (FP32 maps, FP64 residual pass), with
    the conductivity factor on the source side (the default): the FP32 passes read q_dyn / m and
    QL / m, which the prep pass writes once per solve."""
    c = n * n
    return {
        "prep": 32 * c,         # read q_leak0, v, m, q_dyn; write QL, 1/m, q_dyn / m, QL / m
        "row_head": 12 * c,     # read q_dyn / m, QL / m; write spectrum
        "col": 8 * c,           # read + write spectrum
        "row_merged": 24 * c,   # read spectrum, dT, q_dyn / m, QL / m; write dT, spectrum
        "row_last": 12 * c,     # read spectrum, dT; write dT
        "resid_head": 24 * c,   # read dT, q_dyn, QL, 1/m; write FP64 spectrum
        "resid_col": 16 * c,    # read + write FP64 spectrum
        "resid_tail": 12 * c,   # read FP64 spectrum, dT
    }


def measured_traffic(kernel: str, n: int, batch: int):
    """HBM bytes per map-pass of `kernel` from the committed rocprofv3 counter record, if the
    record's kernel sources are still the current ones (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"steady_{n}x{n}_batch{batch}_{kernel}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    h = hashlib.sha256()
    for f in rec["source_files"]:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    if h.hexdigest() != rec["source_sha256"]:
        return None
    return rec["traffic_bytes_per_map_pass"]


TRAFFIC_SOURCES = {
    "row_merged": ["paper_2307_12119_amd/csrc/common.hpp", "paper_2307_12119_amd/csrc/fft.hpp",
                   "paper_2307_12119_amd/csrc/passes.hpp", "paper_2307_12119_amd/csrc/rowops.hpp",
                   "paper_2307_12119_amd/csrc/rowpass.hpp", "paper_2307_12119_amd/csrc/steady.hip"],
    "col": ["paper_2307_12119_amd/csrc/common.hpp", "paper_2307_12119_amd/csrc/fft.hpp",
            "paper_2307_12119_amd/csrc/passes.hpp", "paper_2307_12119_amd/csrc/colpass.hip"],
}


def traffic_record(fetch_dir: str, write_dir: str, kernel: str, symbol: str, maps: float, probe_mb: int,
                   fetch_cmd: str, write_cmd: str, workload: str) -> dict:
    """profiles/*_traffic.json from two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) of the
    same bench command with a copy probe: the kernel's KiB per dispatch, scaled by what the same
    counter reads for the plain copy of probe_mb MiB (which reads and writes exactly that many
    bytes), per map-pass (every map active in every dispatch).  The record carries the hash of
    the kernel's sources, so that the bench drops it once they change."""
    import csv
    import glob
    import hashlib
    import re

    def per_dispatch(d, counter):
        out = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r["Counter_Name"] == counter:
                    v = out.setdefault(r["Dispatch_Id"], [r["Kernel_Name"], 0.0])
                    v[1] += float(r["Counter_Value"])  # summed in case a counter is split per XCD
        return out

    probe = probe_mb << 20
    got = {}
    for d, ctr in ((fetch_dir, "FETCH_SIZE"), (write_dir, "WRITE_SIZE")):
        disp = per_dispatch(d, ctr)
        copies = [v for v in disp.values() if "copyBuffer" in v[0] or ("elementwise_kernel" in v[0] and "copy" in v[0])]
        if not copies:
            raise SystemExit(f"no copy-probe dispatch in {d}")
        hits = [v[1] for v in disp.values() if re.search(symbol, v[0])]
        if not hits:
            raise SystemExit(f"no dispatch of {symbol} in {d}")
        got[ctr] = (sum(hits) / len(hits), max(copies, key=lambda v: v[1])[1], len(hits))
    fetch_kib, fetch_probe, n_disp = got["FETCH_SIZE"]
    write_kib, write_probe, _ = got["WRITE_SIZE"]
    fscale, wscale = (probe / 1024) / fetch_probe, (probe / 1024) / write_probe
    sources = TRAFFIC_SOURCES[kernel]
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    per_disp = (fetch_kib * fscale + write_kib * wscale) * 1024
    return {"kernel": kernel, "kernel_symbol_regex": symbol, "workload": workload, "fetch_cmd": fetch_cmd,
            "write_cmd": write_cmd, "dispatches": n_disp, "fetch_kib_per_dispatch": fetch_kib,
            "write_kib_per_dispatch": write_kib, "copy_probe_bytes": probe, "copy_probe_fetch_kib": fetch_probe,
            "copy_probe_write_kib": write_probe, "fetch_scale": fscale, "write_scale": wscale,
            "map_passes_per_dispatch": maps, "source_sha256": h.hexdigest(), "source_files": sources,
            "traffic_bytes_per_dispatch": per_disp, "traffic_bytes_per_map_pass": per_disp / maps}


def main() -> int:
    if len(sys.argv) > 1 and sys.argv[1] == "--traffic-record":
        # bench.py --traffic-record FETCH_DIR WRITE_DIR KERNEL SYMBOL_REGEX MAPS PROBE_MB OUT_JSON WORKLOAD
        #                           FETCH_CMD WRITE_CMD  (no GPU use)
        fd, wd, kernel, sym, maps, probe_mb, out, workload, fcmd, wcmd = sys.argv[2:12]
        rec = traffic_record(fd, wd, kernel, sym, float(maps), int(probe_mb), fcmd, wcmd, workload)
        json.dump(rec, open(out, "w"), indent=1)
        print(json.dumps(rec))
        return 0
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="diagnostic: time the steps without per-kernel events (no roofline figures)")
    ap.add_argument("--inputs-cache", default="",
                    help="npy file to reuse the generated inputs from (written when missing)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="run one plain device-to-device copy of this size first (counter calibration)")
    ap.add_argument("--no-transient", action="store_true", help="skip the 1024^2 x 1000-step transient run")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate-warm-started solve")
    ap.add_argument("--unseen-batch", type=int, default=64,
                    help="maps of a floorplan outside the training set for the surrogate's generalisation check")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the compensated-twiddle leg (FP32 error at fixed iterations, time cost)")
    ap.add_argument("--no-anderson", action="store_true", help="skip the Anderson(1)-accelerated leg")
    ap.add_argument("--no-oneshot", action="store_true",
                    help="skip the one-shot modified-Green's-function leg (solver, warm start, ablation)")
    ap.add_argument("--no-autotune", action="store_true", help="default launch shapes (no timing of candidates)")
    ap.add_argument("--no-small", action="store_true", help="skip the 64^2 FP64 small-grid leg")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-size Monte Carlo leg")
    ap.add_argument("--small-batch", type=int, default=4096)
    ap.add_argument("--mixed-batch", type=int, default=256, help="samples per size class")
    ap.add_argument("--transient-runs", type=int, default=3)
    ap.add_argument("--no-transient-models", action="store_true",
                    help="transient leg: the single-pole full-history run and its FP64 shadow only (no "
                         "multi-pole or truncated-history runs)")
    ap.add_argument("--tol", type=float, default=1e-3, help="fixed-point tolerance (max increment, K)")
    ap.add_argument("--side-tol", type=float, default=1e-2,
                    help="tolerance of the side leg timed without kernel events (0: skip it)")
    ap.add_argument("--no-oracle-timings", action="store_true",
                    help="skip the oracle timings of the other workloads (64^2, mixed sizes, transient)")
    ap.add_argument("--graph-iterations", type=int, default=2,
                    help="iterations per captured HIP graph in the launch-mode comparison (0: skip it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU only: sharding the samples over several GPUs is not built",
                          "n_gpus": args.gpus}))
        return 2

    t_gen = time.perf_counter()
    cached = None
    if args.inputs_cache and os.path.exists(args.inputs_cache):
        import numpy as np

        cached = np.load(args.inputs_cache)
        if cached.shape[0] != args.batch or cached.shape[-2:] != (args.n, args.n):
            cached = None  # written for another workload: generate and overwrite
    if cached is not None:
        samples = [tuple(cached[i]) for i in range(cached.shape[0])]
    else:
        samples = generate(args.batch, args.n, args.workers)
        if args.inputs_cache:
            import numpy as np

            np.save(args.inputs_cache, np.stack([np.stack(s) for s in samples]))
    small_in, mixed_in, unseen_in = generate_extra(args)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] generated {args.batch} samples of {args.n}^2 (+ extra legs) in {t_gen:.1f} s", file=sys.stderr,
          flush=True)

    import numpy as np
    import torch

    import workloads.gen as W
    from paper_2307_12119_amd import varsim as V

    dev = torch.device("cuda", 0)
    stack = lambda k: torch.from_numpy(np.stack([s[k] for s in samples])).to(dev)
    qd, ql, lv, cm = stack(0), stack(1), stack(2), stack(3)
    out = torch.zeros_like(qd)
    d = W.Die(eta=1.3)
    die = V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)
    items = [{"die": die, "q_dyn": qd[i], "q_leak0": ql[i], "leak_var": lv[i], "cond_map": cm[i], "dT_out": out[i]}
             for i in range(args.batch)]
    if args.copy_probe_mb:
        src = torch.ones(args.copy_probe_mb << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = V.Context(0)
    ctx.set_autotune(0 if args.no_autotune else 1)  # column-pass strip width timed during warm-up
    opts = V.make_options(V.F32, V.LEAK_EXP, 0.017, 50, args.tol, f64_residual=True)
    batch = ctx.prepare(items)
    ws = torch.empty(ctx.workspace_bytes(batch, opts), dtype=torch.uint8, device=dev)

    for _ in range(args.warmup):
        ctx.solve_batch(batch, opts, ws)
    torch.cuda.synchronize()
    print(f"[bench] warm-up done ({args.warmup} steps)", file=sys.stderr, flush=True)

    per_map = algorithmic_bytes(args.n)

    def passes_of(it):
        """map-passes per kernel class over steps with iteration counts `it` (steps x maps)"""
        steps = it.shape[0]
        return {"prep": args.batch * steps, "row_head": args.batch * steps,
                "col": int(it.sum()), "row_merged": int(it.sum()), "row_last": 0,
                "resid_head": args.batch * steps, "resid_col": args.batch * steps,
                "resid_tail": args.batch * steps}

    def kernel_table(ktimes, passes):
        out = {}
        for name, v in ktimes.items():
            if name not in per_map:
                continue
            b = per_map[name] * passes[name]
            out[name] = {"launches": v["count"], "avg_ms": v["total_ms"] / max(v["count"], 1),
                         "total_ms": v["total_ms"],
                         "GB/s": b / (v["total_ms"] * 1e-3) / 1e9 if v["total_ms"] else None}
        return out

    # one untimed-region step with every kernel class bracketed by events: the per-class table
    # and the dominant class, which alone carries events during the timed steps
    kernels, dom = {}, None
    if not args.no_kernel_timing:
        ctx.reset_timing()
        ctx.set_timing_only(None)
        ctx.set_timing(True)
        st_all = ctx.solve_batch(batch, opts, ws)
        torch.cuda.synchronize()
        ctx.set_timing(False)
        kernels = kernel_table(ctx.kernel_times(), passes_of(np.array([st_all["iterations"]])))
        dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
        ctx.reset_timing()
        ctx.set_timing_only(dom)
        ctx.set_timing(True)
    # per-step statistics stay on the device (each call returns once its kernels are enqueued, so
    # the next call's host setup overlaps this call's last passes); read after the timed region
    import ctypes
    dstats = torch.empty((args.steps, args.batch * ctypes.sizeof(V.Stats)), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.solve_batch(batch, opts, ws, stats_out=dstats[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.set_timing(False)
    ktimes = ctx.kernel_times()
    ctx.set_timing_only(None)
    print(f"[bench] timed {args.steps} steps in {elapsed:.3f} s", file=sys.stderr, flush=True)

    # the same steps with no events at all: direct launches, then the fixed-point loop as
    # captured graphs of --graph-iterations iterations (same results, bitwise)
    launch_modes = None
    if args.graph_iterations > 0:
        launch_modes = {"graph_iterations": args.graph_iterations}
        lstats = torch.empty_like(dstats)
        for name, k_graph in (("direct_ms_per_step", 0), ("graph_ms_per_step", args.graph_iterations)):
            ctx.set_graph_iterations(k_graph)
            ctx.solve_batch(batch, opts, ws, stats_out=lstats[0])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for k in range(args.steps):
                ctx.solve_batch(batch, opts, ws, stats_out=lstats[k])
            torch.cuda.synchronize()
            launch_modes[name] = round((time.perf_counter() - t1) / args.steps * 1e3, 4)
        ctx.set_graph_iterations(0)
        # consecutive batches alternating between two streams, each with its own workspace and
        # outputs: a call with device-side statistics returns once its iterations have been
        # read, so its FP64 residual passes overlap the next batch's iterations on the other
        # stream
        out2 = torch.zeros_like(out)
        batch2 = ctx.prepare([dict(it, dT_out=out2[i]) for i, it in enumerate(items)])
        ws2 = torch.empty_like(ws)
        streams = (torch.cuda.current_stream(), torch.cuda.Stream())
        jobs = ((batch, ws), (batch2, ws2))
        for s_, (b_, w_) in zip(streams, jobs):
            with torch.cuda.stream(s_):
                ctx.solve_batch(b_, opts, w_, stats_out=lstats[0])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.steps):
            with torch.cuda.stream(streams[k & 1]):
                ctx.solve_batch(jobs[k & 1][0], opts, jobs[k & 1][1], stats_out=lstats[k])
        torch.cuda.synchronize()
        t2 = time.perf_counter() - t1
        launch_modes["two_streams_ms_per_step"] = round(t2 / args.steps * 1e3, 4)
        launch_modes["two_streams_maps_per_s"] = round(args.batch * args.steps / t2, 2)
        launch_modes["two_streams_bitwise_equal"] = bool(torch.equal(out, out2))
        del out2, batch2, ws2
        print(f"[bench] launch modes {launch_modes}", file=sys.stderr, flush=True)

    # the same steps at the side tolerance (no kernel events)
    side = None
    if args.side_tol > 0:
        opts_side = V.make_options(V.F32, V.LEAK_EXP, 0.017, 50, args.side_tol, f64_residual=True)
        out_side = torch.zeros_like(out)
        batch_side = ctx.prepare([dict(it, dT_out=out_side[i]) for i, it in enumerate(items)])
        sstats = torch.empty_like(dstats)
        for _ in range(args.warmup):
            ctx.solve_batch(batch_side, opts_side, ws, stats_out=sstats[0])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(args.steps):
            ctx.solve_batch(batch_side, opts_side, ws, stats_out=sstats[k])
        torch.cuda.synchronize()
        t_side = time.perf_counter() - t1
        ss = [V.stats_from_bytes(sstats[k], args.batch) for k in range(args.steps)]
        it_side = np.array([s_["iterations"] for s_ in ss])
        side = {"tol_K": args.side_tol, "maps_per_s": round(args.batch * args.steps / t_side, 2),
                "ms_per_step": round(t_side / args.steps * 1e3, 4), "iterations_mean": float(it_side.mean()),
                "residual_f64_max_K": float(max(np.max(s_["residual_f64_K"]) for s_ in ss)),
                "statuses": sorted({int(x) for s_ in ss for x in s_["status"]}),
                "max_diff_vs_headline_K": float((out_side - out).abs().max())}
        del out_side, batch_side, sstats
        print(f"[bench] side tolerance {side}", file=sys.stderr, flush=True)

    per_step = [V.stats_from_bytes(dstats[k], args.batch) for k in range(args.steps)]
    stats = per_step[-1]
    statuses = sorted({int(x) for s_ in per_step for x in s_["status"]})
    it = np.array([s_["iterations"] for s_ in per_step])
    maps_per_s = args.batch * args.steps / elapsed
    passes = passes_of(it)
    if args.no_kernel_timing:
        print(json.dumps({"metric": METRIC, "value": round(maps_per_s, 2), "unit": "maps/s",
                          "ms_per_step": round(elapsed / args.steps * 1e3, 4), "kernel_timing": False,
                          "iterations_mean": float(it.mean())}))
        return 0
    # the dominant class over the timed steps (its events only)
    kernels[dom] = kernel_table({dom: ktimes[dom]}, passes)[dom]
    dom_bytes_per_launch = per_map[dom] * passes[dom] / kernels[dom]["launches"]
    per_pass = measured_traffic(dom, args.n, args.batch)
    traffic = None if per_pass is None else int(per_pass * passes[dom] / kernels[dom]["launches"])
    achieved = kernels[dom]["GB/s"]
    total_alg = sum(per_map[k] * passes[k] for k in kernels)
    resid = stats["residual_f64_K"]

    result = {
        "metric": METRIC,
        "value": round(maps_per_s, 2),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"steady {args.n}x{args.n} FP32 leakage+variation solve, batch of {args.batch} "
                               f"Monte Carlo samples, tol {args.tol:g} K, FP64 residual per map",
                   "n": args.n, "batch": args.batch, "tol_K": args.tol, "precision": "f32"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "bytes_per_launch": int(dom_bytes_per_launch), "avg_launch_ms": kernels[dom]["avg_ms"],
                     "stream_ceiling": stream_ceiling(args.n, args.batch)},
        "solve": {"iterations_mean": float(it.mean()), "iterations_max": int(it.max()), "statuses": statuses,
                  "residual_f64_max_K": float(np.max(resid)),
                  "effective_GBps_all_kernels": round(total_alg / elapsed / 1e9, 1),
                  "kernels_note": f"{dom}: timed steps; other classes: one step timed with every class "
                                  "before the timed region",
                  "kernels": kernels,
                  "launch_modes": launch_modes,
                  "side_tolerance": side,
                  "autotune": ctx.autotune_report().strip().split("\n")},
        "surrogate": None,
    }

    out_w = None
    if not args.no_surrogate:
        result["surrogate"], out_w = surrogate_bench(ctx, items, qd, lv, cm, out, opts, ws, args, maps_per_s,
                                                     float(it.mean()))
        if unseen_in is not None and out_w is not None:
            result["surrogate"]["unseen_floorplan"] = surrogate_unseen(ctx, unseen_in, die, opts, args)
    if not args.no_anderson:
        result["anderson"] = anderson_bench(ctx, items, out, ws, args, maps_per_s, float(it.mean()))
    if not args.no_precision:
        result["precision"] = precision_bench(ctx, items, out, opts, ws, args, maps_per_s)
    if not args.no_oneshot:
        ql_all = np.stack([s_[1] * s_[2] / s_[3] for s_ in samples]).astype(np.float64)
        mu = float(ql_all.mean())  # the batch's (one floorplan's) mean leakage per unit m
        del ql_all
        result["oneshot"] = oneshot_bench(ctx, items, out, opts, ws, args, mu, maps_per_s, float(it.mean()))
    if not args.no_transient:
        del ws
        result["transient"] = transient_bench(ctx, args.transient_runs, not args.no_transient_models)
    if small_in is not None:
        result["small"] = small_bench(ctx, small_in, args)
    if mixed_in is not None:
        result["mixed"] = mixed_bench(ctx, mixed_in, args)
    if not args.no_cpu_baseline:
        check = [i for i in (0, 85, 170, 255) if i < args.batch]
        gpu_maps = {i: out[i].cpu().numpy() for i in check}
        warm = None if out_w is None else {i: out_w[i].cpu().numpy() for i in check}
        result["cpu_baseline"], errs, errs_w, per_iter_s = cpu_baseline(args.n, gpu_maps, args.tol, warm)
        result["max_err_K"] = max(errs.values())
        result["max_err_K_per_map"] = {str(k): v for k, v in errs.items()}
        if errs_w is not None:
            result["surrogate"]["max_err_vs_oracle_K"] = max(errs_w.values())
        if not args.no_oracle_timings:
            result["oracle_timings"] = oracle_timings(ctx, per_iter_s, args)
    check_rec = result["transient"].pop("_check_record", None) if result.get("transient") else None
    if check_rec is not None and not args.no_cpu_baseline:
        result["transient"]["oracle_check"] = transient_oracle_check(check_rec)
    if result.get("mixed") and not args.no_cpu_baseline:
        result["mixed"]["oracle_check"] = mixed_oracle_check(result["mixed"].pop("_first_maps"), args.tol)
    elif result.get("mixed"):
        result["mixed"].pop("_first_maps", None)
    print(json.dumps(result))
    return 0


def small_bench(ctx, samples, args) -> dict:
    """64 x 64 FP64 steady solves (16 blocks, no variation, k constant, exp leakage), tol 1e-6 K,
    at most 20 iterations: one map at a time (latency) and a batch of all seeds (throughput),
    with the LDS-resident path and with the two-pass path."""
    import numpy as np
    import torch

    import workloads.gen as W
    from paper_2307_12119_amd import varsim as V

    dev = torch.device("cuda", 0)
    d = W.Die(eta=0.0)
    die = V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)
    q = torch.from_numpy(np.stack([s[0] for s in samples])).to(dev)
    ql = torch.from_numpy(np.stack([s[1] for s in samples])).to(dev)
    out = torch.zeros_like(q)
    B = q.shape[0]
    opts = V.make_options(V.F64, V.LEAK_EXP, 0.017, 20, 1e-6)
    one = ctx.prepare([{"die": die, "q_dyn": q[0], "q_leak0": ql[0], "dT_out": out[0]}])
    many = ctx.prepare([{"die": die, "q_dyn": q[i], "q_leak0": ql[i], "dT_out": out[i]} for i in range(B)])
    res = {"workload": f"steady 64x64 FP64, 16 blocks, no variation, tol 1e-6 K, max 20 iterations; "
                       f"single map and a batch of {B} seeds"}
    try:
        for name, limit in (("lds_resident", -1), ("two_pass", 0)):
            ctx.set_small_path(limit)
            ws1 = torch.empty(ctx.workspace_bytes(one, opts), dtype=torch.uint8, device=dev)
            wsb = torch.empty(ctx.workspace_bytes(many, opts), dtype=torch.uint8, device=dev)
            for _ in range(3):
                ctx.solve_batch(one, opts, ws1)
            torch.cuda.synchronize()
            reps = 50
            t0 = time.perf_counter()
            for _ in range(reps):
                st1 = ctx.solve_batch(one, opts, ws1)
            torch.cuda.synchronize()
            lat = (time.perf_counter() - t0) / reps
            ctx.solve_batch(many, opts, wsb)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                stb = ctx.solve_batch(many, opts, wsb)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) / args.steps
            res[name] = {"us_per_single_solve": round(lat * 1e6, 1), "batch_maps_per_s": round(B / el, 1),
                         "batch_ms": round(el * 1e3, 3), "iterations_mean": float(np.mean(stb["iterations"])),
                         "statuses": sorted({int(x) for x in stb["status"]})}
    finally:
        ctx.set_small_path(-1)
    return res


def mixed_bench(ctx, samples, args) -> dict:
    """Mixed-size Monte Carlo batch: per size class 128, 256, 512, 1024 the same number of
    variation samples of that class's floorplan, classes interleaved in one varsim_solve_batch
    (FP32, tolerance --tol, FP64 residual per map); per-sample mean / max rises come with the stats."""
    import numpy as np
    import torch

    import workloads.gen as W
    from paper_2307_12119_amd import varsim as V

    dev = torch.device("cuda", 0)
    d = W.Die(eta=1.3)
    die = V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)
    items, cls = [], []
    for c, qd, ql, lv, cm in samples:
        t = lambda a: torch.from_numpy(a).to(dev)
        items.append({"die": die, "q_dyn": t(qd), "q_leak0": t(ql), "leak_var": t(lv), "cond_map": t(cm),
                      "dT_out": torch.zeros_like(t(qd))})
        cls.append(c)
    cls = np.array(cls)
    opts = V.make_options(V.F32, V.LEAK_EXP, 0.017, 50, args.tol, f64_residual=True)
    batch = ctx.prepare(items)
    ws = torch.empty(ctx.workspace_bytes(batch, opts), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        ctx.solve_batch(batch, opts, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = ctx.solve_batch(batch, opts, ws)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    graph = None
    if args.graph_iterations > 0:
        # the same steps with the fixed-point loop as captured graphs; the first maps of every
        # class must come out bitwise equal
        ref = [items[i]["dT_out"].clone() for i in range(min(8, len(items)))]
        ctx.set_graph_iterations(args.graph_iterations)
        ctx.solve_batch(batch, opts, ws)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            st_g = ctx.solve_batch(batch, opts, ws)
        torch.cuda.synchronize()
        el_g = (time.perf_counter() - t1) / args.steps
        ctx.set_graph_iterations(0)
        graph = {"graph_iterations": args.graph_iterations, "maps_per_s": round(len(items) / el_g, 1),
                 "ms_per_step": round(el_g * 1e3, 3),
                 "bitwise_equal": bool(all(torch.equal(r, items[i]["dT_out"]) for i, r in enumerate(ref))
                                       and np.array_equal(st_g["iterations"], st["iterations"]))}
    first = {}
    for c in range(4):
        i0 = int(np.flatnonzero(cls == c)[0])
        first[c] = items[i0]["dT_out"].cpu().numpy()
    per = {}
    for c in range(4):
        sel = st[cls == c]
        n = 128 << c
        per[f"{n}x{n}"] = {"maps": int(sel.size), "iterations_mean": float(sel["iterations"].mean()),
                           "dT_max_K_mean": float(sel["dT_max_K"].mean()),
                           "residual_f64_max_K": float(sel["residual_f64_K"].max())}
    return {"workload": f"{len(items)} steady FP32 problems, {args.mixed_batch} variation samples per size class "
                        f"128/256/512/1024 (one floorplan per class), classes interleaved, tol {args.tol:g} K, "
                        "FP64 residual",
            "maps_per_s": round(len(items) / el, 1), "ms_per_step": round(el * 1e3, 3),
            "statuses": sorted({int(x) for x in st["status"]}), "classes": per, "graph_launched": graph,
            "_first_maps": first}


def anderson_bench(ctx, items, out_plain, ws, args, plain_maps_per_s, plain_iters) -> dict:
    """The same batch with Anderson(1) mixing (a classical acceleration, same stop rule and
    accuracy): maps/s, iterations and the speedup over the plain Picard solve."""
    import numpy as np
    import torch

    from paper_2307_12119_amd import varsim as V

    opts = V.make_options(V.F32, V.LEAK_EXP, 0.017, 50, args.tol, f64_residual=True, anderson=True)
    out_a = torch.zeros_like(out_plain)
    items_a = ctx.prepare([dict(it, dT_out=out_a[i]) for i, it in enumerate(items)])
    ws_a = torch.empty(ctx.workspace_bytes(items_a, opts), dtype=torch.uint8, device=out_plain.device)
    for _ in range(args.warmup):
        ctx.solve_batch(items_a, opts, ws_a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = ctx.solve_batch(items_a, opts, ws_a)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    return {"maps_per_s": round(args.batch / el, 2), "ms_per_step": round(el * 1e3, 4),
            "speedup_vs_plain": round(args.batch / el / plain_maps_per_s, 4),
            "iterations_mean": float(np.mean(st["iterations"])), "plain_iterations_mean": plain_iters,
            "residual_f64_max_K": float(np.max(st["residual_f64_K"])),
            "max_diff_vs_plain_K": float((out_a - out_plain).abs().max()),
            "statuses": sorted({int(x) for x in st["status"]}),
            "note": "two row passes per iteration (evaluation with the residual dot products, then mixing)"}


def precision_bench(ctx, items, out_plain, opts, ws, args, plain_maps_per_s) -> dict:
    """FP32 with compensated twiddles (hi + lo pairs for every twiddle and butterfly constant):
    the headline batch timed with it (no kernel events), and the FP32 arithmetic error with and
    without it -- iterate 5 of the FP32 solve against iterate 5 of the FP64 solve of the same map
    (the GPU's FP64 path, within 1e-9 of the oracle) -- at 512^2 (maps 0-3 of the batch) and
    1024^2 (two samples of the mixed batch's 1024^2 floorplan)."""
    import numpy as np
    import torch

    import workloads.gen as W
    from paper_2307_12119_amd import varsim as V

    dev = out_plain.device
    ct = V.make_options(V.F32, V.LEAK_EXP, opts.beta_per_K, opts.max_iter, opts.tol_K, f64_residual=True,
                        compensated_twiddles=True)
    out_c = torch.zeros_like(out_plain)
    items_c = ctx.prepare([dict(it, dT_out=out_c[i]) for i, it in enumerate(items)])
    for _ in range(args.warmup):
        ctx.solve_batch(items_c, ct, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st = ctx.solve_batch(items_c, ct, ws)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    res = {"compensated": {"maps_per_s": round(args.batch / el, 2), "ms_per_step": round(el * 1e3, 4),
                           "time_vs_plain": round(plain_maps_per_s / (args.batch / el), 4),
                           "iterations_mean": float(np.mean(st["iterations"])),
                           "residual_f64_max_K": float(np.max(st["residual_f64_K"])),
                           "max_diff_vs_plain_K": float((out_c - out_plain).abs().max())},
           "note": "errors: FP32 iterate 5 against FP64 iterate 5 of the same map (fixed iteration count)"}

    def errs(maps):
        out = {}
        for name, prec, dtype, comp in (("rounded", V.F32, torch.float32, False),
                                        ("compensated", V.F32, torch.float32, True),
                                        ("fp64", V.F64, torch.float64, False)):
            its = [dict(m, q_dyn=m["q_dyn"].to(dtype), q_leak0=m["q_leak0"].to(dtype), leak_var=m["leak_var"].to(dtype),
                        cond_map=m["cond_map"].to(dtype), dT_out=torch.zeros_like(m["q_dyn"], dtype=dtype))
                   for m in maps]
            o = V.make_options(prec, V.LEAK_EXP, opts.beta_per_K, 5, 1e-30, compensated_twiddles=comp)
            ctx.solve_batch(its, o, raise_on=())
            out[name] = [it["dT_out"].double() for it in its]
        return {k: float(max((a - b).abs().max().item() for a, b in zip(out[k], out["fp64"])))
                for k in ("rounded", "compensated")}

    res["error_512_K"] = errs([items[i] for i in range(min(4, len(items)))])
    d = W.Die(eta=1.3)
    die = V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)
    big = []
    for smp in range(2):
        inp = W.config3(3, smp)
        t = lambda a: torch.from_numpy(a.astype(np.float32)).to(dev)  # FP32 inputs for every precision
        big.append({"die": die, "q_dyn": t(inp.q_dyn), "q_leak0": t(inp.q_leak0), "leak_var": t(inp.leak_var),
                    "cond_map": t(inp.cond_map)})
    res["error_1024_K"] = errs(big)
    return res


def oneshot_bench(ctx, items, out_plain, opts, ws, args, mu, plain_maps_per_s, plain_iters) -> dict:
    """The paper's one-shot modified Green's functions (Sec. IV-C) on the same batch: as a
    zero-iteration solver (deterministic part only -- the paper's "ignoring f_rand" -- and with
    the random part), their distance from the converged plain result and their FP64 residual;
    then as a non-learned warm start of the fixed point (one-shot time included, same stop rule);
    and the high-variance ablation (leakage variation with twice the log-spread)."""
    import numpy as np
    import torch

    from paper_2307_12119_amd import varsim as V

    dev = out_plain.device
    res = {"mu_W_m2": mu, "note": "mu: mean leakage density per unit conductivity multiplier over the batch"}
    out_os = torch.zeros_like(out_plain)
    items_os = ctx.prepare([dict(it, dT_out=out_os[i]) for i, it in enumerate(items)])
    for name, rnd in (("deterministic_only", False), ("with_random_part", True)):
        for _ in range(args.warmup):
            ctx.solve_oneshot(items_os, opts, mu, rnd, ws)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            st = ctx.solve_oneshot(items_os, opts, mu, rnd, ws)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / args.steps
        err = (out_os - out_plain).abs()
        res[name] = {"maps_per_s": round(args.batch / el, 2), "ms_per_step": round(el * 1e3, 4),
                     "max_err_vs_converged_K": float(err.max()),
                     "mean_err_vs_converged_K": float(err.mean()),
                     "max_err_pct_of_max_rise": float((err.amax(dim=(1, 2)) / out_plain.amax(dim=(1, 2))).max() * 100),
                     "residual_f64_max_K": float(np.max(st["residual_f64_K"])),
                     "statuses": sorted({int(x) for x in st["status"]})}
    # warm start: one-shot (with the random part, no residual) then the fixed point from it
    opts_os = V.make_options(V.F32, V.LEAK_EXP, opts.beta_per_K, opts.max_iter, opts.tol_K)
    init = torch.zeros_like(out_plain)
    out_w = torch.zeros_like(out_plain)
    items_i = ctx.prepare([dict(it, dT_out=init[i]) for i, it in enumerate(items)])
    items_w = ctx.prepare([dict(it, dT_init=init[i], dT_out=out_w[i]) for i, it in enumerate(items)])
    for _ in range(args.warmup):
        ctx.solve_oneshot(items_i, opts_os, mu, True, ws)
        ctx.solve_batch(items_w, opts, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(args.steps):
        ctx.solve_oneshot(items_i, opts_os, mu, True, ws)
        st = ctx.solve_batch(items_w, opts, ws)
        iters.append(st["iterations"])
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / args.steps
    res["warm_start"] = {"maps_per_s": round(args.batch / el, 2), "ms_per_step": round(el * 1e3, 4),
                         "speedup_vs_plain": round(args.batch / el / plain_maps_per_s, 4),
                         "iterations_mean": float(np.mean(iters)), "plain_iterations_mean": plain_iters,
                         "max_diff_vs_plain_K": float((out_w - out_plain).abs().max()),
                         "statuses": sorted({int(x) for x in st["status"]})}
    # ablation on high-variance maps: the first 64 samples with v squared (twice the log-spread)
    B = min(64, len(items))
    v2 = torch.stack([items[i]["leak_var"] for i in range(B)]) ** 2
    conv, one = torch.zeros_like(out_plain[:B]), torch.zeros_like(out_plain[:B])
    hv = [dict(items[i], leak_var=v2[i], dT_out=conv[i]) for i in range(B)]
    hv_os = [dict(items[i], leak_var=v2[i], dT_out=one[i]) for i in range(B)]
    st_c = ctx.solve_batch(hv, opts, raise_on=())
    ok = np.array([s_["status"] == V.OK for s_ in st_c])
    mu2 = float(sum((items[i]["q_leak0"].double() * v2[i].double() / items[i]["cond_map"].double()).mean().item()
                    for i in range(B)) / B)
    abl = {"maps": B, "converged_maps": int(ok.sum()), "mu_W_m2": mu2}
    for name, rnd in (("deterministic_only", False), ("with_random_part", True)):
        st_o = ctx.solve_oneshot(hv_os, opts, mu2, rnd)
        good = ok & np.array([s_["status"] == V.OK for s_ in st_o])
        idx = torch.from_numpy(np.flatnonzero(good)).to(dev)
        e = (one[idx] - conv[idx]).abs()
        abl[name] = {"max_err_K": float(e.max()), "mean_err_K": float(e.mean()),
                     "max_err_pct_of_max_rise": float((e.amax(dim=(1, 2)) / conv[idx].amax(dim=(1, 2))).max() * 100)}
    res["high_variance_ablation"] = abl
    return res


SURROGATE_WEIGHTS = os.path.join(ROOT, "paper_2307_12119_amd", "weights", "surrogate_512.npy")
MFMA_BF16_PEAK_TFLOPS = 2500.0


def conv_flops_per_map(spec) -> float:
    """Dense multiply-adds (x2) of the network's convolutions for one map (stem: 48 inputs)."""
    w, m = spec.width, spec.n // 4
    f = 2.0 * 48 * w[0] * m * m + 2.0 * w[0] * 16 * m * m
    for l in range(5):
        px = (m >> l) ** 2
        cin = w[0] if l == 0 else w[l - 1]
        f += 2.0 * 9 * px * (cin * w[l] + w[l] * w[l])
        if l < 4:
            f += 2.0 * 9 * px * (w[l + 1] + w[l]) * w[l]
    return f


def surrogate_bench(ctx, items, qd, lv, cm, out_plain, opts, ws, args, plain_maps_per_s, plain_iters):
    """The same batch solved from the network's prediction (inference time included), against the
    plain cold start: throughput, iterations, agreement with the plain result."""
    import numpy as np
    import torch

    from paper_2307_12119_amd import varsim as V

    if not os.path.exists(SURROGATE_WEIGHTS):
        return {"status": "no trained weights"}, None
    dev = qd.device
    spec = V.NetSpec(n=args.n)
    net = V.Net(ctx, spec)
    net.set_params(torch.from_numpy(np.load(SURROGATE_WEIGHTS)).to(dev))
    init = torch.empty_like(qd)
    out_w = torch.empty_like(qd)
    items_w = ctx.prepare([dict(it, dT_init=init[i], dT_out=out_w[i]) for i, it in enumerate(items)])
    wsf = torch.empty(net.workspace_bytes(args.batch, False), dtype=torch.uint8, device=dev)
    for _ in range(args.warmup):
        net.forward(qd, lv, cm, init, workspace=wsf)
        ctx.solve_batch(items_w, opts, ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(args.steps):
        net.forward(qd, lv, cm, init, workspace=wsf)
        stats = ctx.solve_batch(items_w, opts, ws)
        iters.append(stats["iterations"])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # network alone, with per-kernel events
    ctx.reset_timing()
    ctx.set_timing(True)
    t1 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(qd, lv, cm, init, workspace=wsf)
    torch.cuda.synchronize()
    t_net = (time.perf_counter() - t1) / args.steps
    ctx.set_timing(False)
    kt = ctx.kernel_times()
    layer_ms = {k: round(v["total_ms"] / args.steps, 4) for k, v in kt.items() if k.startswith("fwd:")}
    conv_ms = sum(v for k, v in layer_ms.items() if k.startswith("fwd:conv:"))
    flops = conv_flops_per_map(spec) * args.batch
    achieved = flops / (conv_ms * 1e-3) / 1e12 if conv_ms else None
    maps_per_s = args.batch * args.steps / elapsed
    pred_err = (init - out_plain).abs()
    training = surrogate_training(ctx, spec, qd, lv, cm, out_plain, args)
    return ({"value": round(maps_per_s, 2), "unit": "maps/s", "speedup_vs_plain": round(maps_per_s / plain_maps_per_s, 4),
             "ms_per_step": round(elapsed / args.steps * 1e3, 4), "iterations_mean": float(np.mean(iters)),
             "plain_iterations_mean": plain_iters, "statuses": sorted({int(x) for x in stats["status"]}),
             "max_diff_vs_plain_K": float((out_w - out_plain).abs().max()),
             "prediction_mae_K": float(pred_err.mean()), "prediction_max_err_K": float(pred_err.max()),
             "network_ms_per_batch": round(t_net * 1e3, 4), "layer_ms_per_batch": layer_ms,
             "roofline": {"bound": "mfma", "kernel": "conv_kernel (all forward convolutions)", "achieved": None if achieved is None else
                          round(achieved, 1), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": None if achieved is None else round(achieved / MFMA_BF16_PEAK_TFLOPS, 4),
                          "flops_per_launch_batch": flops, "conv_ms_per_batch": conv_ms},
             "weights": os.path.relpath(SURROGATE_WEIGHTS, ROOT), "training": training}, out_w)


UNSEEN_FLOORPLAN = 8  # the network was trained on floorplans 0..7


def surrogate_unseen(ctx, samples, die, opts, args) -> dict:
    """Maps of a floorplan the network never saw in training: its prediction error against the
    plain solve's converged maps, and the iterations the warm start needs against the cold one."""
    import numpy as np
    import torch

    from paper_2307_12119_amd import varsim as V

    dev = torch.device("cuda", 0)
    stack = lambda k: torch.from_numpy(np.stack([s_[k] for s_ in samples])).to(dev)
    qd, ql, lv, cm = stack(0), stack(1), stack(2), stack(3)
    b = len(samples)
    out_p, out_w, init = torch.zeros_like(qd), torch.zeros_like(qd), torch.empty_like(qd)
    items = [{"die": die, "q_dyn": qd[i], "q_leak0": ql[i], "leak_var": lv[i], "cond_map": cm[i], "dT_out": out_p[i]}
             for i in range(b)]
    plain = ctx.prepare(items)
    warm = ctx.prepare([dict(it, dT_init=init[i], dT_out=out_w[i]) for i, it in enumerate(items)])
    ws = torch.empty(ctx.workspace_bytes(plain, opts), dtype=torch.uint8, device=dev)
    st_p = ctx.solve_batch(plain, opts, ws)
    net = V.Net(ctx, V.NetSpec(n=args.n))
    net.set_params(torch.from_numpy(np.load(SURROGATE_WEIGHTS)).to(dev))
    net.forward(qd, lv, cm, init, workspace=torch.empty(net.workspace_bytes(b, False), dtype=torch.uint8, device=dev))
    st_w = ctx.solve_batch(warm, opts, ws)
    torch.cuda.synchronize()
    err = (init - out_p).abs()
    return {"floorplan": UNSEEN_FLOORPLAN, "maps": b, "trained_floorplans": "0..7",
            "prediction_mae_K": float(err.mean()), "prediction_max_err_K": float(err.max()),
            "iterations_mean": float(np.mean(st_w["iterations"])), "plain_iterations_mean": float(np.mean(st_p["iterations"])),
            "statuses": sorted({int(x) for x in st_w["status"]} | {int(x) for x in st_p["status"]}),
            "max_diff_vs_plain_K": float((out_w - out_p).abs().max())}


def surrogate_training(ctx, spec, qd, lv, cm, target, args, batch: int = 64, steps: int = 10) -> dict:
    """Training steps of the network (forward, MSE gradient through every layer, Adam) on batches
    of 64 of this batch's maps against the plain solve's converged rises, from a fresh He
    initialisation (the trained weights are not touched).  MFMA figure: dense convolution flops
    of forward + input gradient + weight gradient over the summed time of those kernels."""
    import numpy as np
    import torch

    from paper_2307_12119_amd import varsim as V

    dev = qd.device
    net = V.Net(ctx, spec)
    net.set_params(torch.from_numpy(spec.he_init(0)).to(dev))
    grad = torch.empty(net.param_count, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    wst = torch.empty(net.workspace_bytes(batch, True), dtype=torch.uint8, device=dev)
    n_maps = qd.shape[0]
    idx = [torch.arange(k * batch, (k + 1) * batch, dtype=torch.int32, device=dev) % n_maps for k in range(steps)]

    def step(k):
        net.gradient(qd, lv, cm, target, grad, loss, batch, sample_idx=idx[k % steps], workspace=wst)
        net.adam(grad, 1e-3)

    for k in range(2):
        step(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    ctx.reset_timing()
    ctx.set_timing(True)
    for k in range(steps):
        step(k)
    torch.cuda.synchronize()
    ctx.set_timing(False)
    kt = ctx.kernel_times()
    conv_ms = sum(v["total_ms"] for k, v in kt.items()
                  if k.startswith("fwd:conv:") or k in ("nn_conv_dgrad", "nn_wgrad")) / steps
    # forward, input gradient (every layer but the stem, whose inputs are features) and weight
    # gradient
    m = spec.n // 4
    flops = (3.0 * conv_flops_per_map(spec) - 2.0 * 48 * spec.width[0] * m * m) * batch
    achieved = flops / (conv_ms * 1e-3) / 1e12 if conv_ms else None
    classes = {}
    for k, v in kt.items():
        c = "fwd:conv" if k.startswith("fwd:conv:") else ("fwd:elem" if k.startswith("fwd:") else k)
        classes[c] = round(classes.get(c, 0.0) + v["total_ms"] / steps, 4)
    return {"batch": batch, "ms_per_step": round(wall * 1e3, 4), "samples_per_s": round(batch / wall, 1),
            "last_loss_K2": float(loss.item()), "conv_ms_per_step": round(conv_ms, 4), "class_ms_per_step": classes,
            "roofline": {"bound": "mfma", "kernel": "conv_kernel / wgrad_kernel (forward, input and weight gradients)",
                         "achieved": None if achieved is None else round(achieved, 1),
                         "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": None if achieved is None else round(achieved / MFMA_BF16_PEAK_TFLOPS, 4)}}


TRANSIENT_BYTES_PER_CELL = {"tr_row": 20, "tr_col": 24}  # FP32: see transient_bench


def transient_bench(ctx, runs: int, models: bool = True) -> dict:
    """One 1000-step transient of a 64-block, 1024 x 1024 die (10 us steps, block powers redrawn
    every 1 ms, leakage + variation, k(T) with eta = 1.3), FP32, snapshots every 100 steps; the
    same run in FP64 (untimed) gives the FP32 error at every snapshot."""
    import numpy as np
    import torch

    import workloads.gen as W
    from paper_2307_12119_amd import varsim as V

    n, steps, every = 1024, 1000, 100
    inp = W.transient_problem(n=n, n_steps=steps, dt_s=10e-6, n_blocks=64, hold_s=1e-3, seed=0)
    dev = torch.device("cuda", 0)
    d = inp.die
    die = V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)

    def setup(dtype):
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=dev, dtype=dtype)
        item = {"die": die, "q_leak0": t(inp.q_leak0), "leak_var": t(inp.leak_var), "cond_map": t(inp.cond_map),
                "dT_out": torch.zeros((n, n), dtype=dtype, device=dev)}
        snaps = torch.zeros((steps // every, n, n), dtype=dtype, device=dev)
        return item, t(inp.block_rects).to(torch.int32), t(inp.trace), snaps

    item, rects, trace, snaps = setup(torch.float32)
    opts = V.make_options(V.F32, V.LEAK_EXP, inp.beta, 1, 1e-3)
    ws = torch.empty(ctx.transient_workspace_bytes(item, rects, trace, inp.dt_s, opts, every), dtype=torch.uint8,
                     device=dev)
    st = ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snaps, every, workspace=ws)  # warm-up, table
    torch.cuda.synchronize()
    ctx.reset_timing()
    ctx.set_timing(True)
    t0 = time.perf_counter()
    for _ in range(runs):
        st = ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snaps, every, workspace=ws)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / runs
    ctx.set_timing(False)
    kt = ctx.kernel_times()
    ctx.set_timing(False)
    # untimed: no per-kernel events
    t0 = time.perf_counter()
    ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snaps, every, workspace=ws)
    torch.cuda.synchronize()
    wall_untimed = time.perf_counter() - t0
    got = snaps.cpu().numpy().astype(np.float64)
    # the first TRANSIENT_CHECK_STEPS steps again, every step recorded, for the oracle check at
    # sampled cells (cpu_baseline leg)
    rec = torch.zeros((TRANSIENT_CHECK_STEPS, n, n), dtype=torch.float32, device=dev)
    ctx.solve_transient(item, rects, trace[:TRANSIENT_CHECK_STEPS], inp.dt_s, opts, rec, 1)
    torch.cuda.synchronize()
    check_rec = rec.cpu().numpy().astype(np.float64)
    del rec
    modal = truncated = None
    if models:
        modal, truncated = transient_models(ctx, item, rects, trace, inp, opts, every, snaps, dev)
    item64, rects64, trace64, snaps64 = setup(torch.float64)
    opts64 = V.make_options(V.F64, V.LEAK_EXP, inp.beta, 1, 1e-3)
    ctx.solve_transient(item64, rects64, trace64, inp.dt_s, opts64, snaps64, every)
    torch.cuda.synchronize()
    ref = snaps64.cpu().numpy()
    kernels = {}
    for name in ("tr_row", "tr_col"):
        v = kt.get(name)
        if not v:
            continue
        avg = v["total_ms"] / v["count"]
        kernels[name] = {"launches": v["count"], "avg_ms": avg,
                         "GB/s": TRANSIENT_BYTES_PER_CELL[name] * n * n / (avg * 1e-3) / 1e9}
    return {"workload": "transient 1024x1024 FP32, 1000 steps of 10 us, 64 blocks redrawn every 1 ms, "
                        "leakage + variation, eta 1.3, snapshots every 100 steps",
            "ms_per_run": round(wall_untimed * 1e3, 3), "ms_per_run_with_kernel_events": round(wall * 1e3, 3),
            "steps_per_s": round(steps / wall_untimed, 1), "status": st["status"],
            "dT_max_K": st["dT_max_K"], "fp64_shadow_max_diff_K": float(np.max(np.abs(got - ref))),
            "kernels": kernels, "modal": modal, "truncated_history": truncated,
            "autotune": [l for l in ctx.autotune_report().strip().split("\n") if l.startswith("transient")],
            "_check_record": check_rec}


TRANSIENT_CHECK_STEPS = 20


def transient_oracle_check(rec) -> dict:
    """The oracle's superposition (Eq. tranapprox over the whole history, FP64 direct sums) of the
    transient leg's first steps at sampled cells -- the hottest cell, the corners, the die centre
    and random cells -- with the power history rebuilt from the recorded rises, against the
    GPU's FP32 rise of the last of those steps."""
    import numpy as np

    import workloads.gen as W
    from oracle import steady as S
    from oracle import transient as T

    t0 = time.perf_counter()
    steps, n = rec.shape[0], rec.shape[1]
    inp = W.transient_problem(n=n, n_steps=1000, dt_s=10e-6, n_blocks=64, hold_s=1e-3, seed=0)
    g = S.geometry_from_die(inp.die, n)
    model = T.TransientModel(g, inp.die.rho_c)
    ql = inp.q_leak0 * inp.leak_var
    hist = [np.zeros((n, n))]
    prev = np.zeros((n, n))
    for k in range(steps):
        q = W.raster_trace_step(inp.block_rects, inp.trace[k], n) + ql * np.exp(inp.beta * prev)
        hist.append(g.hx * g.hy * q / inp.cond_map)  # conductivity factor on the source side
        prev = rec[k]
    last = rec[-1]
    hot = np.unravel_index(int(np.argmax(last)), last.shape)
    rng = np.random.default_rng(17)
    rows = np.concatenate([[hot[0], 0, 0, n - 1, n - 1, n // 2], rng.integers(0, n, 10)])
    cols = np.concatenate([[hot[1], 0, n - 1, 0, n - 1, n // 2], rng.integers(0, n, 10)])
    theta = np.zeros(len(rows))
    for j in range(1, steps + 1):
        op = S.DirectSum(g, table=model.step_kernel(j * inp.dt_s))
        theta += op.apply_at(hist[steps - j + 1] - hist[steps - j], rows, cols)
    expect, ok = S.kirchhoff_inverse(theta, g.t_amb, g.eta)
    err = np.abs(last[rows, cols] - expect)
    return {"steps": steps, "cells": len(rows), "max_err_K": float(np.max(err)) if np.all(ok) else None,
            "rise_at_hottest_K": float(expect[0]), "seconds": round(time.perf_counter() - t0, 1),
            "note": "FP32 rise of the leg's first steps (same problem, same tuned passes) against the "
                    "oracle's superposition at sampled cells"}


def transient_models(ctx, item, rects, trace, inp, opts, every, snaps, dev):
    """The transient of transient_bench with the multi-pole model (the slab's 3 slowest depth modes
    + 1 lumped pole per cosine mode) and with the paper's truncated history (step responses
    saturated after 5 ms), each timed once after a warm-up, against the single-pole full-history
    snapshots."""
    import torch

    from paper_2307_12119_amd import varsim as V

    ws4 = torch.empty(ctx.transient_workspace_bytes(item, rects, trace, inp.dt_s, opts, every, V.TAU_MODAL, 4),
                      dtype=torch.uint8, device=dev)
    snaps4 = torch.zeros_like(snaps)
    ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snaps4, every, tau_model=V.TAU_MODAL, workspace=ws4,
                        n_poles=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snaps4, every, tau_model=V.TAU_MODAL, workspace=ws4,
                        n_poles=4)
    torch.cuda.synchronize()
    wall4 = time.perf_counter() - t0
    modal = {"poles": 4, "ms_per_run": round(wall4 * 1e3, 3),
             "max_diff_vs_single_pole_K": float((snaps4 - snaps).abs().max())}
    del ws4, snaps4
    # the paper's truncated history: step responses saturated after 5 ms (500 steps of 10 us)
    h = int(round(5e-3 / inp.dt_s))
    wsh = torch.empty(ctx.transient_workspace_bytes(item, rects, trace, inp.dt_s, opts, every, history_steps=h),
                      dtype=torch.uint8, device=dev)
    snapsh = torch.zeros_like(snaps)
    ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snapsh, every, workspace=wsh, history_steps=h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.solve_transient(item, rects, trace, inp.dt_s, opts, snapsh, every, workspace=wsh, history_steps=h)
    torch.cuda.synchronize()
    wallh = time.perf_counter() - t0
    truncated = {"history_steps": h, "horizon_ms": h * inp.dt_s * 1e3, "ms_per_run": round(wallh * 1e3, 3),
                 "workspace_MiB": round(wsh.numel() / 2 ** 20, 1),
                 "max_diff_vs_full_history_K": float((snapsh - snaps).abs().max())}
    del wsh, snapsh
    return modal, truncated


def host_info() -> dict:
    """CPU model and counts of the host the oracle runs on."""
    model = None
    try:
        import subprocess

        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except Exception:  # lscpu missing: /proc/cpuinfo
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        affinity = os.cpu_count() or 1
    return {"cpu_model": model, "os_cpu_count": os.cpu_count(), "affinity_cpus": affinity}


def oracle_threads() -> int:
    """BLAS threads for the oracle: the process's CPU share (OMP_NUM_THREADS when set, else the
    CPUs it may run on)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return host_info()["affinity_cpus"]


def cpu_baseline(n: int, gpu_maps: dict, tol: float, warm_maps=None, min_s: float = 10.0, max_maps: int = 24):
    """The oracle (FP64 direct sum + Picard, the GPU's stopping rule: max increment <= tol) on
    the samples of gpu_maps (their errors are reported), then samples 1, 2, ... until at least
    min_s seconds of solving (at most max_maps maps), with BLAS on the process's CPU share; the
    Green's table is built before the clock starts.  Returns the baseline record, the plain
    solve's max error per checked sample, the warm-started one's (or None) and the oracle's
    seconds per fixed-point iteration."""
    import contextlib

    import numpy as np

    import workloads.gen as W
    from oracle import steady as S

    threads = oracle_threads()
    try:
        from threadpoolctl import threadpool_limits

        limiter = threadpool_limits(limits=threads, user_api="blas")
    except Exception:  # pragma: no cover
        limiter = contextlib.nullcontext()
    with limiter:
        inp0 = W.config2(sample=0, n=n)
        op = S.DirectSum(S.geometry_from_die(inp0.die, n))  # the table, shared by every sample
        order = list(gpu_maps) + [i for i in range(1, 4 * max_maps) if i not in gpu_maps]
        solved, iters, dt, refs = 0, [], 0.0, {}
        for smp in order:
            if solved >= max_maps or (solved >= len(gpu_maps) and dt >= min_s):
                break
            prob, opts = S.problem_from_inputs(W.config2(sample=smp, n=n), op)
            opts.tol, opts.max_iter = tol, 50
            t0 = time.perf_counter()
            ref, st = S.solve_steady(prob, opts, residual=False)
            dt += time.perf_counter() - t0
            if smp in gpu_maps:
                refs[smp] = ref
            iters.append(st.iterations)
            solved += 1
    errs = {i: float(np.max(np.abs(gpu_maps[i].astype(np.float64) - refs[i]))) for i in gpu_maps}
    errs_w = None
    if warm_maps is not None:
        errs_w = {i: float(np.max(np.abs(warm_maps[i].astype(np.float64) - refs[i]))) for i in warm_maps}
    rec = {"value": round(solved / dt, 6), "unit": "maps/s", "cores": threads, "kind": "oracle",
           "sample": f"{solved} converged {n}x{n} maps (samples {sorted(gpu_maps)} then 1, 2, ...; {sum(iters)} "
                     f"iterations, {dt:.1f} s of solving, tol {tol:g} K as on the GPU), FP64 direct image sum "
                     f"with numpy/BLAS on {threads} threads, Green's table built before timing",
           "host": host_info()}
    return rec, errs, errs_w, dt / max(sum(iters), 1)


def _time_solve(inp, tol, max_iter):
    from oracle import steady as S

    prob, opts = S.problem_from_inputs(inp)
    opts.tol, opts.max_iter = tol, max_iter
    t0 = time.perf_counter()
    _, st = S.solve_steady(prob, opts, residual=False)
    return time.perf_counter() - t0, st


def oracle_timings(ctx, per_iter_512: float, args) -> dict:
    """Oracle wall-clock on the other workloads (same host threads as the baseline), and the
    GPU's Green's-table build time per geometry.  Entries marked extrapolated scale a measured
    direct sum by its O(N^4) cost; nothing else is extrapolated."""
    import numpy as np
    import torch

    import workloads.gen as W
    from oracle import steady as S
    from oracle import transient as T
    from paper_2307_12119_amd import varsim as V

    out = {"threads": oracle_threads()}
    try:
        from threadpoolctl import threadpool_limits

        threadpool_limits(limits=out["threads"], user_api="blas")
    except Exception:  # pragma: no cover
        pass
    # 64^2 FP64, tol 1e-6 K, <= 20 iterations: 16 seeds, median
    t64 = [_time_solve(W.config1(seed=s, n=64), 1e-6, 20)[0] for s in range(16)]
    out["steady_64x64_fp64"] = {"median_s_per_map": float(np.median(t64)), "maps_per_s": 1.0 / float(np.median(t64)),
                                "seeds": 16}
    # mixed sizes: one sample per class; 1024^2 extrapolated from the 512^2 iteration cost
    cls = {}
    for c in range(3):
        inp = W.config3(c, 0)
        dt, st = _time_solve(inp, args.tol, 50)
        cls[f"{inp.n}x{inp.n}"] = {"s_per_map": dt, "iterations": st.iterations}
    it1024 = cls["512x512"]["iterations"]
    cls["1024x1024"] = {"s_per_map": 16.0 * per_iter_512 * it1024, "iterations": it1024,
                        "extrapolated": "16 x the 512^2 direct-sum iteration time (O(N^4)) x the 512^2 class's "
                                        "iteration count"}
    out["mixed_one_sample_per_class"] = cls
    # transient: full-history superposition at 32^2 x 200 steps, measured; 1024^2 x 1000 extrapolated
    inp = W.transient_problem(n=32, n_steps=200, dt_s=10e-6, n_blocks=64, hold_s=1e-3, seed=0)
    geom = S.geometry_from_die(inp.die, 32)
    model = T.TransientModel(geom, inp.die.rho_c)
    q = np.stack([W.raster_trace_step(inp.block_rects, inp.trace[k], 32) for k in range(200)])
    t0 = time.perf_counter()
    T.solve_transient(model, q, inp.dt_s, inp.q_leak0 * inp.leak_var, inp.cond_map, "exp", inp.beta, 100)
    t_fir = time.perf_counter() - t0
    sums_1024 = 1000 * 1001 // 2
    out["transient"] = {"fir_32x32_200_steps_s": t_fir, "direct_sums": 200 * 201 // 2,
                        "fir_1024x1024_1000_steps_s": sums_1024 * 16.0 * per_iter_512,
                        "extrapolated_1024": f"{sums_1024} direct sums at 1024^2, each 16 x a 512^2 direct-sum "
                                             "iteration (O(N^4))"}
    # GPU Green's-table build (FP64 tabulation, cosine eigenvalues, column coefficients)
    d = W.Die(eta=1.3)
    die = V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)
    fresh = V.Context(0)
    tb = {}
    try:
        for n in (64, 128, 256, 512, 1024):
            fresh.reset_timing()
            fresh.set_timing(True)
            fresh.green_table(die, n)
            torch.cuda.synchronize()
            kt = fresh.kernel_times()
            fresh.set_timing(False)
            tb[f"{n}x{n}"] = round(kt["green_table"]["total_ms"], 4)
    finally:
        fresh.close()
    out["gpu_green_table_build_ms"] = tb
    out["cpu_fft_context"] = cpu_fft_context(args.n, args.tol, out["threads"])
    return out


def cpu_fft_context(n: int, tol: float, threads: int) -> dict:
    """Context only, not the oracle: the same Picard loop with scipy's FFT-based cosine transforms
    (FP64, workers = threads) on sample 0, and its distance from the oracle's direct sum."""
    import numpy as np
    import scipy.fft as sfft

    import workloads.gen as W
    from oracle import steady as S

    inp = W.config2(sample=0, n=n)
    prob, opts = S.problem_from_inputs(inp)
    g = prob.geom
    lam = sfft.dct(sfft.dct(prob.op.table, type=1, axis=0), type=1, axis=1)[:n, :n]
    minv = 1.0 / prob.m
    dT = np.zeros((n, n))
    t0 = time.perf_counter()
    for it in range(1, 51):
        p = g.hx * g.hy * (prob.q_dyn + prob.q_leak * np.exp(inp.beta * dT)) * minv
        theta = sfft.idctn(lam * sfft.dctn(p, type=2, workers=threads), type=2, workers=threads)
        new, _ = S.kirchhoff_inverse(theta, g.t_amb, g.eta)
        inc = float(np.max(np.abs(new - dT)))
        dT = new
        if inc <= tol:
            break
    dt = time.perf_counter() - t0
    opts.tol, opts.max_iter = tol, 50
    ref, _ = S.solve_steady(prob, opts, residual=False)
    return {"s_per_map": dt, "maps_per_s": 1.0 / dt, "iterations": it, "workers": threads,
            "max_diff_vs_oracle_K": float(np.max(np.abs(dT - ref))),
            "note": "context only: FFT-based transforms on the host, not the oracle's direct sum"}


def mixed_oracle_check(first_maps: dict, tol: float) -> dict:
    """The first sample of every size class of the mixed batch against the oracle: the full
    converged oracle map at 128^2 - 512^2 (max |dT_gpu - dT_oracle|); at 1024^2 the oracle's
    fixed-point map applied to the GPU result at 32 sampled cells (max |G(dT_gpu) - dT_gpu| there,
    computed cell by cell)."""
    import numpy as np

    import workloads.gen as W
    from oracle import steady as S

    out = {}
    for c, got in first_maps.items():
        inp = W.config3(c, 0)
        key = f"{inp.n}x{inp.n}"
        got = got.astype(np.float64)
        if inp.n <= 512:
            prob, opts = S.problem_from_inputs(inp)
            opts.tol, opts.max_iter = tol, 50
            ref, _ = S.solve_steady(prob, opts, residual=False)
            out[key] = {"max_err_K": float(np.max(np.abs(got - ref)))}
            continue
        prob, opts = S.problem_from_inputs(inp)
        rng = np.random.default_rng(1024)
        rows = rng.integers(0, inp.n, 32)
        cols = rng.integers(0, inp.n, 32)
        hot = np.unravel_index(int(np.argmax(got)), got.shape)
        rows[0], cols[0] = hot
        p = prob.power(got, opts) / prob.m
        theta = prob.op.apply_at(p, rows, cols)
        g_at, _ = S.kirchhoff_inverse(theta, prob.geom.t_amb, prob.geom.eta)
        out[key] = {"max_residual_at_32_cells_K": float(np.max(np.abs(g_at - got[rows, cols]))),
                    "cells": "32 seeded cells including the hot spot"}
    return out


if __name__ == "__main__":
    sys.exit(main())
