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
    ap.add_argument("--cpu-sinks", type=int, default=0,
                    help="sinks in the oracle's timed sample (0: every sink of the box)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def _code_tokens(text: str) -> str:
    """C++ source without comments and with whitespace runs collapsed, so
    that a comment-only edit leaves the hash unchanged (string and character
    literals are kept as written)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == "/" and text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif c == "/" and text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        elif c in "\"'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the HIP sources' code (comments and layout ignored), to tell
    whether stored counters are current."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1810_02916_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(f.encode() + b"\0" + _code_tokens(fh.read()).encode())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, kernel: str):
    """HBM bytes per launch from profiles/traffic_<workload>.txt, written from
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs and scaled by the copy-kernel
    calibration; None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    if vals.get("source_hash") != kernel_source_hash():
        return None
    v = vals.get(f"{kernel}_bytes")
    return float(v) if v is not None else None


def copy_calibration():
    import torch
    n = 1 << 28   # 2^28 float32 = 1 GiB read + 1 GiB written per copy
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 5}))


def bench_batched(args):
    """64 uneven boxes: per-box calls vs one batched call vs one graph replay
    (binning + compensated accelerations each time)."""
    import numpy as np
    import torch

    from paper_1810_02916_amd import nearfield as nfp
    from paper_1810_02916_amd.synth import batched_specs, make_box, occupancy_stats

    specs = batched_specs(64)
    dev = torch.device("cuda:0")
    boxes = [make_box(s) for s in specs]
    I = sum(occupancy_stats(p, s.K, s.L)["interactions"] for p, s in zip(boxes, specs))
    pos = [torch.from_numpy(p).to(dev) for p in boxes]
    Ks, Ls, Es = [s.K for s in specs], [s.L for s in specs], [s.eps_s for s in specs]

    def per_box():
        return [nfp.accel(nfp.bin_particles(p, K, L, e, check=False), 1.0, compensated=True)
                for p, K, L, e in zip(pos, Ks, Ls, Es)]

    def batched():
        return nfp.accel(nfp.bin_particles_batched(pos, Ks, Ls, Es, check=False), 1.0,
                         compensated=True)

    cf = nfp.CapturedForce(pos, Ks, Ls, Es, 1.0, compensated=True)

    def timeit(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / args.steps

    t_box, t_bat, t_graph = timeit(per_box), timeit(batched), timeit(cf.replay)
    ref = batched()
    got = cf.replay()
    torch.cuda.synchronize()
    same = all(torch.equal(a, b) for a, b in zip(ref, got))
    n = sum(s.n for s in specs)
    print(json.dumps({
        "metric": "G pair-interactions/s and particles/s (FP32 vs compensated, err vs FP64)",
        "value": round(I / (t_graph * 1e-3) / 1e9, 3), "unit": "G pair-interactions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_graph, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batched64", "boxes": len(specs), "n_total": n,
                   "interactions": I, "step": "bin + accel compensated, all boxes"},
        "ms": {"per_box_calls": round(t_box, 4), "one_batched_call": round(t_bat, 4),
               "graph_replay": round(t_graph, 4)},
        "gdips": {"per_box_calls": round(I / t_box / 1e6, 2),
                  "one_batched_call": round(I / t_bat / 1e6, 2),
                  "graph_replay": round(I / t_graph / 1e6, 2)},
        "graph_equals_eager": same,
    }), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU; multi-GPU runs are not part of this build",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calib:
        copy_calibration()
        return
    if args.workload == "batched64":
        bench_batched(args)
        return

    import numpy as np
    import torch

    from paper_1810_02916_amd import nearfield as nfp
    from paper_1810_02916_amd.synth import (WORKLOADS, make_box_device,
                                            occupancy_stats_device)

    sp = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pos = make_box_device(sp, dev)
    occ = occupancy_stats_device(pos, sp.K, sp.L)
    I = occ["interactions"]
    cot = torch.randn((sp.n, 3), generator=torch.Generator(device=dev).manual_seed(sp.seed * 10 + 2),
                      device=dev, dtype=torch.float32)
    print(f"[bench] {sp.name}: n={sp.n} K={sp.K} interactions={I}", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        b = nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s, check=False)
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

    # The widened rows, timed after the step (not part of value): the Plummer
    # law (plain accelerations), the p = 8 cell multipoles, the time-step
    # statistics and the kick/drift update.
    def timed(fn, reps=args.steps):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps
    t_plum = timed(lambda: nfp.accel(b, 1.0, plummer=True))
    t_full = timed(lambda: nfp.accel(b, 1.0, spline_everywhere=True))
    t_mom = timed(lambda: nfp.multipoles(b, 8))
    vel = torch.randn((sp.n, 3), generator=torch.Generator(device=dev).manual_seed(sp.seed * 10 + 3),
                      device=dev, dtype=torch.float32)
    t_stats = timed(lambda: nfp.step_stats(b, a_plain, vel))
    pos2, vel2 = pos.clone(), vel.clone()
    t_kd = timed(lambda: nfp.kick_drift(b, a_plain, vel2, pos2, 1e-6, 1e-6))
    stats_bytes = 28.0 * sp.n + 4.0 * (sp.K ** 3 + 1) + 8.0 * sp.K ** 3 + 24.0 * sp.K ** 3
    kd_bytes = 84.0 * sp.n
    mom_bytes = 16.0 * sp.n + 4.0 * nfp.multipole_terms(8) * sp.K ** 3 + 4.0 * (sp.K ** 3 + 1)
    extras = {
        "plummer_accel_plain": {"ms": round(t_plum, 4), "gdips": round(I / t_plum / 1e6, 2)},
        "accel_plain_shortcut_off": {"ms": round(t_full, 4), "gdips": round(I / t_full / 1e6, 2)},
        "multipoles_p8": {"ms": round(t_mom, 4), "terms": nfp.multipole_terms(8),
                          "algorithmic_bytes": int(mom_bytes),
                          "hbm_gbs": round(mom_bytes / (t_mom * 1e-3) / 1e9, 1),
                          "hbm_frac": round(mom_bytes / (t_mom * 1e-3) / PEAK_HBM, 4)},
        "step_stats": {"ms": round(t_stats, 4), "algorithmic_bytes": int(stats_bytes),
                       "hbm_gbs": round(stats_bytes / (t_stats * 1e-3) / 1e9, 1)},
        "kick_drift": {"ms": round(t_kd, 4), "algorithmic_bytes": int(kd_bytes),
                       "hbm_gbs": round(kd_bytes / (t_kd * 1e-3) / 1e9, 1),
                       "hbm_frac": round(kd_bytes / (t_kd * 1e-3) / PEAK_HBM, 4)},
    }
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
                     "frac": round(achieved / PEAK_FP32, 4),
                     "traffic": stored_traffic(sp.name, dom),
                     "flop_per_pair": fdom, "pairs_per_launch": I,
                     "timed": "HIP events around the library call on its stream: planner "
                              "kernels + dense, light and narrow force kernels"},
        "kernel_source_hash": kernel_source_hash(),
        "extras": extras,
    }

    if not args.no_cpu:
        import oracle
        from tests.errstats import err_stats
        rng = np.random.default_rng(12345)
        m = sp.n if args.cpu_sinks <= 0 else min(args.cpu_sinks, sp.n)
        sinks = np.sort(rng.choice(sp.n, m, replace=False))
        pos_np = pos.cpu().numpy()
        print(f"[bench] oracle on {m} sinks", file=sys.stderr, flush=True)
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
