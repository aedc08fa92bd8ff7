#!/usr/bin/env python3
"""Train the learned warm start on maps the solver itself generates (GPU, the library's kernels).

Data: `--samples` problems of the 512 x 512 leakage + variation family (64-block floorplans
f = i mod `--floorplans`, variation sample 100000 + i, so that none coincides with an evaluation
map, whose sample ids are below 100000); target = the converged FP32 rise from
varsim_solve_batch at tol 1e-4 K.  Training: mean-squared error, Adam, batch `--batch`, learning
rate with linear warm-up and cosine decay.  Held-out: samples 0 .. `--holdout` - 1 of floorplan 0.
Writes <out>.npy (FP32 parameters in the order of varsim.h) and <out>.json (recipe and metrics).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

CHUNK = 256


def _sample(floorplan: int, sample: int, n: int):
    import numpy as np

    import workloads.gen as W

    W.FFT_WORKERS = 1
    inp = W.config2(sample=sample, n=n, floorplan=floorplan)
    f = lambda a: a.astype(np.float32)
    return f(inp.q_dyn), f(inp.q_leak0), f(inp.leak_var), f(inp.cond_map)


def log(msg: str):
    print(f"[train] {msg}", flush=True)


def solve_targets(ctx, V, die, Q, QL, Vv, M, T, lo, hi, opts, ws):
    """Converged rises of maps lo..hi-1; a map without a converged target (thermal runaway of an
    extreme variation sample) is reported so that training leaves it out."""
    items = [{"die": die, "q_dyn": Q[i], "q_leak0": QL[i - lo], "leak_var": Vv[i], "cond_map": M[i], "dT_out": T[i]}
             for i in range(lo, hi)]
    stats = ctx.solve_batch(items, opts, ws, raise_on=(V.ERR_INVALID, V.ERR_UNSUPPORTED, V.ERR_DEVICE,
                                                       V.ERR_NO_MEMORY))
    return stats


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--samples", type=int, default=20000)
    ap.add_argument("--floorplans", type=int, default=8)
    ap.add_argument("--holdout", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--out", default="surrogate_512", help="output path stem (.npy weights, .json record)")
    args = ap.parse_args()

    import multiprocessing as mp

    pool = mp.get_context("fork").Pool(args.workers)  # forked before the GPU is touched
    import numpy as np
    import torch

    import workloads.gen as W
    from paper_2307_12119_amd import varsim as V

    n, N, H = args.n, args.samples, args.holdout
    dev = torch.device("cuda", 0)
    d = W.Die(eta=1.3)
    die = V.Die(d.lx_m, d.ly_m, d.t_m, d.k0, d.eta, d.t_amb, d.rho_c)
    ctx = V.Context(0)
    spec = V.NetSpec(n=n, k0=d.k0)
    net = V.Net(ctx, spec)
    net.set_params(torch.from_numpy(spec.he_init(args.seed)).to(dev))
    log(f"network: {net.param_count} parameters, widths {spec.width}")

    total = N + H
    Q = torch.empty((total, n, n), dtype=torch.float32, device=dev)
    Vv, M, T = torch.empty_like(Q), torch.empty_like(Q), torch.empty_like(Q)
    opts = V.make_options(V.F32, V.LEAK_EXP, 0.017, 100, 1e-4)
    ws = None
    t0 = time.perf_counter()
    iters = []
    valid = []
    statuses = {}
    for lo in range(0, total, CHUNK):
        hi = min(total, lo + CHUNK)
        jobs = [((i % args.floorplans, 100000 + i) if i < N else (0, i - N)) for i in range(lo, hi)]
        res = pool.starmap(_sample, [(f, s, n) for f, s in jobs])
        up = lambda k: torch.from_numpy(np.stack([r[k] for r in res])).to(dev)
        Q[lo:hi], QL, Vv[lo:hi], M[lo:hi] = up(0), up(1), up(2), up(3)
        if ws is None:
            items = [{"die": die, "q_dyn": Q[0], "q_leak0": QL[0], "leak_var": Vv[0], "cond_map": M[0],
                      "dT_out": T[0]}] * CHUNK
            ws = torch.empty(ctx.workspace_bytes(items, opts), dtype=torch.uint8, device=dev)
        st = solve_targets(ctx, V, die, Q, QL, Vv, M, T, lo, hi, opts, ws)
        for i, s_ in enumerate(st):
            statuses[s_["status"]] = statuses.get(s_["status"], 0) + 1
            if s_["status"] == V.OK:
                iters.append(s_["iterations"])
                if lo + i < N:
                    valid.append(lo + i)
            elif lo + i >= N:
                raise RuntimeError(f"held-out map {lo + i - N} did not converge (status {s_['status']})")
        if (lo // CHUNK) % 8 == 0 or hi == total:
            log(f"data {hi}/{total} maps ({time.perf_counter() - t0:.0f} s), target iterations mean "
                f"{np.mean(iters):.2f}")
    pool.close()
    pool.join()
    t_data = time.perf_counter() - t0

    log(f"target statuses {statuses}; {len(valid)} of {N} training maps converged")
    valid_idx = torch.tensor(valid, dtype=torch.int32, device=dev)
    NV = len(valid)
    B = args.batch
    steps_per_epoch = NV // B
    total_steps = steps_per_epoch * args.epochs
    warm = max(1, total_steps // 50)
    grad = torch.empty(net.param_count, dtype=torch.float32, device=dev)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    losses = torch.zeros(total_steps, dtype=torch.float32, device=dev)
    wst = torch.empty(net.workspace_bytes(B, True), dtype=torch.uint8, device=dev)
    wsf = torch.empty(net.workspace_bytes(CHUNK, False), dtype=torch.uint8, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    pred = torch.empty((CHUNK, n, n), dtype=torch.float32, device=dev)

    def holdout_error():
        err_abs, err_max = 0.0, 0.0
        for lo in range(N, total, CHUNK):
            hi = min(total, lo + CHUNK)
            net.forward(Q[lo:hi], Vv[lo:hi], M[lo:hi], pred[:hi - lo], workspace=wsf)
            e = (pred[:hi - lo] - T[lo:hi]).abs()
            err_abs += float(e.sum())
            err_max = max(err_max, float(e.max()))
        return err_abs / (H * n * n), err_max

    log(f"data ready in {t_data:.0f} s; training {args.epochs} epochs x {steps_per_epoch} steps, batch {B}")
    history = []
    t1 = time.perf_counter()
    step = 0
    for ep in range(args.epochs):
        perm = valid_idx[torch.randperm(NV, generator=gen, device=dev)]
        for k in range(steps_per_epoch):
            lr = args.lr * min(1.0, (step + 1) / warm) * 0.5 * (1.0 + math.cos(math.pi * step / total_steps))
            net.gradient(Q, Vv, M, T, grad, loss, B, sample_idx=perm[k * B:(k + 1) * B], workspace=wst)
            losses[step:step + 1].copy_(loss)
            net.adam(grad, lr)
            step += 1
        torch.cuda.synchronize()
        ep_loss = float(losses[step - steps_per_epoch:step].mean())
        mae, mx = holdout_error()
        history.append({"epoch": ep + 1, "train_mse": ep_loss, "holdout_mae_K": mae, "holdout_max_K": mx})
        log(f"epoch {ep + 1}: train MSE {ep_loss:.4g} K^2, held-out MAE {mae:.4f} K, max {mx:.3f} K "
            f"({time.perf_counter() - t1:.0f} s)")
    t_train = time.perf_counter() - t1

    params = net.get_params().cpu().numpy()
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    np.save(args.out + ".npy", params)
    rec = {"spec": {"n": spec.n, "width": list(spec.width), "shift": list(spec.shift), "scale": list(spec.scale),
                    "out_scale": spec.out_scale, "k0": spec.k0},
           "data": {"family": "512x512 steady, 64 blocks, Vth + conductivity variation, eta 1.3, exp leakage "
                              "beta 0.017/K", "samples": N, "converged_samples": NV,
                    "target_statuses": {str(k): v for k, v in statuses.items()}, "floorplans": args.floorplans,
                    "sample_ids": "100000 + i (floorplan i mod floorplans)",
                    "targets": "varsim_solve_batch FP32, tol 1e-4 K", "target_iterations_mean": float(np.mean(iters)),
                    "holdout": f"floorplan 0, samples 0..{H - 1}"},
           "training": {"epochs": args.epochs, "batch": B, "optimizer": "Adam(0.9, 0.999, 1e-8)", "lr": args.lr,
                        "schedule": "linear warm-up over 2 % of steps, cosine decay", "seed": args.seed,
                        "data_seconds": round(t_data, 1), "train_seconds": round(t_train, 1),
                        "steps": total_steps},
           "history": history}
    json.dump(rec, open(args.out + ".json", "w"), indent=1)
    log(f"wrote {args.out}.npy and .json")
    return 0


if __name__ == "__main__":
    sys.exit(main())
