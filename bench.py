#!/usr/bin/env python3
"""Near-field force benchmark (one GPU).

A step is one pass of the whole hot path over one synthetic box already
resident in HBM:
    bin (cell offsets + stable sort)  ->  accel (plain FP32)
    ->  accel (compensated FP32)      ->  VJP (compensated FP32)
``value`` counts the pair interactions those three force passes evaluate
(3 x I per step, I = sum over sinks of the sources in their 5x5x5 block,
self pairs included) per second of step time, in G pair-interactions/s.

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic work per pair interaction.
FLOP_ACCEL = 23    # the paper's count: 22 add/mul + rsqrt as one (Sec. 2.3)
FLOP_VJP = 36      # the adjoint's operation list
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered2m")
    ap.add_argument("--cpu-sinks", type=int, default=1 << 18,
                    help="sinks in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU; multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1810_02916_amd import nearfield as nfp
    from paper_1810_02916_amd.synth import WORKLOADS, gaussian_cotangent, make_box, occupancy_stats

    sp = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pos_np = make_box(sp)
    occ = occupancy_stats(pos_np, sp.K, sp.L)
    I = occ["interactions"]
    pos = torch.from_numpy(pos_np).to(dev)
    cot = torch.from_numpy(gaussian_cotangent(sp.n, sp.seed * 10 + 2).astype(np.float32)).to(dev)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        b = nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s)
        if ev is not None:
            ev[1].record(stream)
        a0 = nfp.accel(b, 1.0)
        if ev is not None:
            ev[2].record(stream)
        a1 = nfp.accel(b, 1.0, compensated=True)
        if ev is not None:
            ev[3].record(stream)
        g = nfp.accel_vjp(b, cot, 1.0, compensated=True)
        if ev is not None:
            ev[4].record(stream)
        return b, a0, a1, g

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()

    ms_step = (t1 - t0) * 1e3 / args.steps
    parts = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(4)]
                      for k in range(args.steps)])
    t_bin, t_plain, t_comp, t_vjp = parts.mean(axis=0)   # ms

    value = 3.0 * I / (ms_step * 1e-3) / 1e9

    kern = {
        "accel_plain": (t_plain, FLOP_ACCEL),
        "accel_compensated": (t_comp, FLOP_ACCEL),
        "vjp_compensated": (t_vjp, FLOP_VJP),
    }
    dom = max(kern, key=lambda k: kern[k][0])
    tdom, fdom = kern[dom]
    achieved = fdom * I / (tdom * 1e-3)

    b, a_plain, a_comp, g = out
    result = {
        "metric": "G pair-interactions/s and particles/s (FP32 vs compensated, err vs FP64)",
        "value": round(value, 3),
        "unit": "G pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": sp.name, "n": sp.n, "K": sp.K, "L": sp.L, "eps_s": sp.eps_s,
            "sigma_ln": sp.sigma_ln, "interactions": I, "max_cell": occ["max_cell"],
            "step": "bin + accel plain + accel compensated + vjp compensated",
        },
        "breakdown_ms": {"bin": round(t_bin, 4), "accel_plain": round(t_plain, 4),
                         "accel_compensated": round(t_comp, 4), "vjp_compensated": round(t_vjp, 4)},
        "gdips": {"accel_plain": round(I / t_plain / 1e6, 2),
                  "accel_compensated": round(I / t_comp / 1e6, 2),
                  "vjp_compensated": round(I / t_vjp / 1e6, 2)},
        "mparticles_per_s": {"accel_plain": round(sp.n / t_plain / 1e3, 2),
                             "bin_plus_accel_plain": round(sp.n / (t_bin + t_plain) / 1e3, 2),
                             "bin_plus_accel_compensated": round(sp.n / (t_bin + t_comp) / 1e3, 2)},
        "bin_hbm_gbs": round(40.0 * sp.n / (t_bin * 1e-3) / 1e9, 1),
        "roofline": {"kernel": dom, "bound": "alu", "achieved": round(achieved / 1e12, 3),
                     "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32, 4), "traffic": None,
                     "flop_per_pair": fdom, "pairs_per_launch": I},
    }

    if not args.no_cpu:
        import oracle
        from tests.errstats import err_stats
        rng = np.random.default_rng(12345)
        m = min(args.cpu_sinks, sp.n)
        sinks = np.sort(rng.choice(sp.n, m, replace=False))
        tc0 = time.perf_counter()
        ref, cnt = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, sinks=sinks, return_count=True)
        tc1 = time.perf_counter()
        ap = a_plain.cpu().numpy()[sinks]
        ac = a_comp.cpu().numpy()[sinks]
        result["cpu_baseline"] = {
            "value": round(cnt / (tc1 - tc0) / 1e9, 4), "unit": "G pair-interactions/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"FP64 oracle accelerations of {m} random sinks of {sp.name} "
                      f"({cnt} pair interactions, includes its binning of all {sp.n} particles), "
                      f"{tc1 - tc0:.2f} s",
        }
        result["err_vs_fp64"] = {"plain": err_stats(ap, ref), "compensated": err_stats(ac, ref),
                                 "sinks": m}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
