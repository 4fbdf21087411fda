#!/usr/bin/env python3
"""Near-field force benchmark (one GPU).

A step is one pass of the whole hot path over one synthetic box already
resident in HBM:
    bin (cell offsets + stable sort)  ->  accel (plain FP32)
    ->  accel (compensated FP32)      ->  VJP (compensated FP32)
``value`` counts the pair interactions those three force passes evaluate
(3 x I per step, I = sum over sinks of the sources in their 5x5x5 block,
self pairs included) per second of step time, in G pair-interactions/s.

After the timed steps the same line carries, untimed by ``value``:
  * the error of every variant against the FP64 oracle, end to end and
    split into the floor set by rounding the offsets to float (e_repr) and
    the kernel's own error (against the oracle on the float offsets);
  * the oracle timed on the host (all threads, and one core);
  * the pair interactions each force kernel class (dense / light / narrow)
    evaluates;
  * nested records for the other workloads: uniform32k (plain method,
    small), clustered262k (differentiation through autograd), batched64 (64
    uneven boxes: per-box calls, one batched call, one graph replay, and the
    autotuned tiles) and clustered134m (512^3, the paper's mass resolution);
  * the widened rows (Plummer law, multipoles, step statistics and choice,
    kick/drift).

Prints one JSON line.  --gpus above 1 is refused: the benchmark runs on one GPU.
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
# the adjoint's operation list: r (3 sub), v_j - v_i (3 sub), r^2 (5), rsqrt
# (1), q^2 and q^3 (2), r.dv (5), h (2), t (1), accumulation (12), spline (2)
FLOP_VJP = 36
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12
METRIC = "G pair-interactions/s and particles/s (FP32 vs compensated, err vs FP64)"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clustered2m")
    ap.add_argument("--cpu-sinks", type=int, default=0,
                    help="sinks in the oracle's timed sample (0: every sink of the box)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (no errors, no baseline)")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the nested records of the other workloads")
    ap.add_argument("--serial", action="store_true",
                    help="force kernels one after another (per-kernel profiles); value is "
                         "then not the product configuration")
    ap.add_argument("--copy-calib", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _code_tokens(text: str) -> str:
    from paper_1810_02916_amd.srchash import code_tokens
    return code_tokens(text)


def kernel_source_hash() -> str:
    """Hash of the HIP sources' code (comments and layout ignored), to tell
    whether stored counters are current."""
    from paper_1810_02916_amd.srchash import kernel_source_hash as h
    return h()


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


def cpu_info() -> dict:
    """The host CPU as /proc/cpuinfo describes it, and the CPUs this process
    may run on."""
    model, phys, cores, logical = "unknown", set(), set(), 0
    cur = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in list(f) + [""]:
                if not line.strip():
                    if cur:
                        logical += 1
                        phys.add(cur.get("physical id", "0"))
                        cores.add((cur.get("physical id", "0"), cur.get("core id", str(logical))))
                        model = cur.get("model name", model)
                    cur = {}
                    continue
                k, _, v = line.partition(":")
                cur[k.strip()] = v.strip()
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 0
    return {"model": model, "sockets": len(phys), "physical_cores": len(cores),
            "logical_cpus": logical, "cpus_allowed": allowed}


# ---------------------------------------------------------------- helpers

def ev_time(stream, fn, reps: int, warm: int = 1) -> float:
    """Mean ms per call of fn(), bracketed by HIP events on ``stream``."""
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def pairs_by_class(b, dense_min: int = 41, narrow: int = 12) -> dict:
    """Pair interactions each force kernel evaluates, from the binning: a
    cell's sinks are cut into chunks of 64; full chunks and a last chunk of at
    least dense_min sinks go to the dense kernel, a smaller last chunk to the
    light kernel, or to the narrow one below 12 sinks.  Each sink of a cell
    pairs with every source of the cell's 5^3 block."""
    import torch
    out = {"dense": 0, "light": 0, "narrow": 0}
    for bx in b.boxes:
        K = bx.K
        n = (bx.cell_start[1:] - bx.cell_start[:-1]).to(torch.int64).reshape(K, K, K)
        S = n.clone()
        for ax in range(3):
            acc = torch.zeros_like(S)
            for d in range(-2, 3):
                acc += torch.roll(S, d, dims=ax)
            S = acc
        rem = n % 64
        lt = (rem > 0) & (rem < dense_min)
        dense_sinks = n - torch.where(lt, rem, torch.zeros_like(rem))
        out["dense"] += int((dense_sinks * S).sum())
        out["light"] += int((torch.where(lt & (rem >= narrow), rem, 0) * S).sum())
        out["narrow"] += int((torch.where(lt & (rem < narrow), rem, 0) * S).sum())
    return out


def err_block(got, exact, rounded) -> dict:
    """End-to-end error, the kernel's own error and the representation floor
    (Sec. 4.5 compares the single-precision pipeline with double precision)."""
    from tests.errstats import err_stats
    return {"e2e": err_stats(got, exact), "kernel": err_stats(got, rounded),
            "e_repr_rms": err_stats(rounded, exact)["rms"]}


def sample_sinks(b, n: int, n_random: int, n_dense_cells: int, per_cell: int, seed: int):
    """Random sinks plus sinks of the densest cells (caller indices, sorted)."""
    import numpy as np
    cs = b.boxes[0].cell_start.cpu().numpy().astype(np.int64)
    order = b.boxes[0].order.cpu().numpy()
    counts = np.diff(cs)
    dense = np.argsort(counts)[-n_dense_cells:]
    rng = np.random.default_rng(seed)
    pick = [rng.choice(order[cs[c]:cs[c + 1]], min(per_cell, int(counts[c])), replace=False)
            for c in dense]
    return np.unique(np.concatenate([rng.choice(n, min(n, n_random), replace=False)] + pick)
                     ).astype(np.int64), int(counts.max())


# ---------------------------------------------------------------- nested records

def rec_uniform32k(args, stream, with_cpu: bool) -> dict:
    """Plain method, small box: bin + plain accelerations vs the oracle."""
    import oracle
    import torch
    from paper_1810_02916_amd import nearfield as nfp
    from paper_1810_02916_amd.synth import WORKLOADS, make_box
    sp = WORKLOADS["uniform32k"]
    pos_np = make_box(sp)
    pos = torch.from_numpy(pos_np).to("cuda:0")
    b = nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s)
    I = sum(pairs_by_class(b).values())
    t_bin = ev_time(stream, lambda: nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s, check=False), 20)
    t_acc = ev_time(stream, lambda: nfp.accel(b, 1.0), 20)
    t_cmp = ev_time(stream, lambda: nfp.accel(b, 1.0, compensated=True), 20)
    rec = {"n": sp.n, "K": sp.K, "interactions": I,
           "ms": {"bin": round(t_bin, 4), "accel_plain": round(t_acc, 4),
                  "accel_compensated": round(t_cmp, 4)},
           "gdips": {"accel_plain": round(I / t_acc / 1e6, 2),
                     "accel_compensated": round(I / t_cmp / 1e6, 2)},
           "mparticles_per_s": {"bin_plus_accel_plain": round(sp.n / (t_bin + t_acc) / 1e3, 2)}}
    if with_cpu:
        ap = nfp.accel(b, 1.0).cpu().numpy()
        ac = nfp.accel(b, 1.0, compensated=True).cpu().numpy()
        ex = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s)
        rd = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, round_offsets=True)
        rec["err_vs_fp64"] = {"plain": err_block(ap, ex, rd), "compensated": err_block(ac, ex, rd),
                              "sinks": sp.n}
    return rec


def rec_clustered262k(args, stream, with_cpu: bool) -> dict:
    """Differentiation: compensated accelerations forward and the VJP
    backward through the autograd function, against the oracle's JVP (the
    Jacobian is symmetric; the oracle's JVP equals its VJP, pinned on the
    CPU, and both agree with FP64 central differences, pinned too)."""
    import numpy as np
    import oracle
    import torch
    from paper_1810_02916_amd import nearfield as nfp
    from paper_1810_02916_amd.synth import WORKLOADS, gaussian_cotangent, make_box
    sp = WORKLOADS["clustered262k"]
    pos_np = make_box(sp)
    pos = torch.from_numpy(pos_np).to("cuda:0")
    v = gaussian_cotangent(sp.n, sp.seed * 10 + 2).astype(np.float32)
    vt = torch.from_numpy(v).to("cuda:0")
    b = nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s)
    I = sum(pairs_by_class(b).values())

    def fwd_bwd():
        p = pos.clone().requires_grad_(True)
        a = nfp.nearfield_accel(p, sp.K, sp.L, sp.eps_s, 1.0, True)
        (a * vt).sum().backward()
        return p.grad

    t_fb = ev_time(stream, fwd_bwd, 10)
    t_vjp = ev_time(stream, lambda: nfp.accel_vjp(b, vt, 1.0, compensated=True), 10)
    rec = {"n": sp.n, "K": sp.K, "interactions": I,
           "ms": {"autograd_forward_backward": round(t_fb, 4), "vjp_compensated": round(t_vjp, 4)},
           "gdips": {"vjp_compensated": round(I / t_vjp / 1e6, 2)}}
    if with_cpu:
        g = fwd_bwd().cpu().numpy()
        v64 = v.astype(np.float64)
        ex = oracle.jvp(pos_np, sp.K, sp.L, sp.eps_s, v64)
        rd = oracle.jvp(pos_np, sp.K, sp.L, sp.eps_s, v64, round_offsets=True)
        rec["err_vs_fp64"] = {"vjp_compensated_autograd": err_block(g, ex, rd), "sinks": sp.n}
    return rec


def rec_batched64(args, stream, with_cpu: bool) -> dict:
    """64 uneven boxes: per-box calls vs one batched call vs one graph replay
    (binning + compensated accelerations each time), with the library default
    tiles and with the autotuner's tiles."""
    import numpy as np
    import oracle
    import torch
    from paper_1810_02916_amd import nearfield as nfp
    from paper_1810_02916_amd import tune
    from paper_1810_02916_amd.synth import batched_specs, make_box
    specs = batched_specs(64)
    dev = torch.device("cuda:0")
    boxes = [make_box(s) for s in specs]
    pos = [torch.from_numpy(p).to(dev) for p in boxes]
    Ks, Ls, Es = [s.K for s in specs], [s.L for s in specs], [s.eps_s for s in specs]
    bb = nfp.bin_particles_batched(pos, Ks, Ls, Es)
    I = sum(pairs_by_class(bb).values())
    n_total = sum(s.n for s in specs)

    def per_box():
        return [nfp.accel(nfp.bin_particles(p, K, L, e, check=False), 1.0, compensated=True)
                for p, K, L, e in zip(pos, Ks, Ls, Es)]

    def batched(tiles=None):
        b = nfp.bin_particles_batched(pos, Ks, Ls, Es, check=False, tiles=tiles)
        return nfp.accel(b, 1.0, compensated=True)

    def wall(fn, reps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    reps = max(3, min(args.steps, 10))
    t_box = wall(per_box, reps)
    t_bat = wall(batched, reps)
    cf = nfp.CapturedForce(pos, Ks, Ls, Es, 1.0, compensated=True)
    t_graph = wall(cf.replay, reps)
    tuned = tune.tune(bb, use_cache=False)
    cft = nfp.CapturedForce(pos, Ks, Ls, Es, 1.0, compensated=True, tiles=tuned.tiles)
    t_graph_t = wall(cft.replay, reps)
    ref = batched()
    got = cf.replay()
    got_t = [o.clone() for o in cft.replay()]
    torch.cuda.synchronize()
    rec = {"boxes": len(specs), "n_total": n_total, "interactions": I,
           "ms": {"per_box_calls": round(t_box, 4), "one_batched_call": round(t_bat, 4),
                  "graph_replay": round(t_graph, 4), "graph_replay_tuned": round(t_graph_t, 4)},
           "gdips": {"per_box_calls": round(I / t_box / 1e6, 2),
                     "one_batched_call": round(I / t_bat / 1e6, 2),
                     "graph_replay": round(I / t_graph / 1e6, 2),
                     "graph_replay_tuned": round(I / t_graph_t / 1e6, 2)},
           "graph_equals_eager": all(torch.equal(a, c) for a, c in zip(ref, got)),
           "tuned_tiles": tuned.tiles.as_dict(), "tuning_ms": tuned.times_ms,
           "timed": "wall clock around the calls (host launch included)"}
    if with_cpu:
        rng = np.random.default_rng(5)
        blocks = {"default": [], "tuned": []}
        for p, s, a, at in zip(boxes, specs, got, got_t):
            sinks = np.sort(rng.choice(len(p), 64, replace=False))
            ex = oracle.accel(p, s.K, s.L, s.eps_s, sinks=sinks)
            rd = oracle.accel(p, s.K, s.L, s.eps_s, sinks=sinks, round_offsets=True)
            blocks["default"].append((a.cpu().numpy()[sinks], ex, rd))
            blocks["tuned"].append((at.cpu().numpy()[sinks], ex, rd))
        rec["err_vs_fp64"] = {
            k: err_block(*[np.concatenate([x[i] for x in v]) for i in range(3)])
            for k, v in blocks.items()}
        rec["err_vs_fp64"]["sinks"] = 64 * len(specs)
    return rec


def rec_clustered134m(args, stream, with_cpu: bool) -> dict:
    """512^3 particles, 256^3 cells, sigma_ln 2: the three force passes and
    the binning, errors on sampled sinks, the oracle timed on that sample."""
    import numpy as np
    import oracle
    import torch
    from paper_1810_02916_amd import nearfield as nfp
    from paper_1810_02916_amd.synth import WORKLOADS, make_box_device
    sp = WORKLOADS["clustered134m"]
    dev = torch.device("cuda:0")
    pos = make_box_device(sp, dev)
    b = nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s)
    pairs = pairs_by_class(b)
    I = sum(pairs.values())
    cot = torch.randn((sp.n, 3), generator=torch.Generator(device=dev).manual_seed(sp.seed * 10 + 2),
                      device=dev, dtype=torch.float32)
    reps = 3
    t_bin = ev_time(stream, lambda: nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s, check=False), reps)
    t_p = ev_time(stream, lambda: nfp.accel(b, 1.0), reps)
    t_c = ev_time(stream, lambda: nfp.accel(b, 1.0, compensated=True), reps)
    t_v = ev_time(stream, lambda: nfp.accel_vjp(b, cot, 1.0, compensated=True), reps)
    t_s = ev_time(stream, lambda: nfp.accel(b, 1.0, compensated=True, symmetric=True), reps)
    step = t_bin + t_p + t_c + t_v
    rec = {"n": sp.n, "K": sp.K, "L": sp.L, "sigma_ln": sp.sigma_ln, "interactions": I,
           "pairs_by_kernel": pairs,
           "ms": {"bin": round(t_bin, 3), "accel_plain": round(t_p, 3),
                  "accel_compensated": round(t_c, 3), "vjp_compensated": round(t_v, 3),
                  "accel_compensated_symmetric": round(t_s, 3), "step": round(step, 3)},
           "value": round(3.0 * I / (step * 1e-3) / 1e9, 3),
           "gdips": {"accel_plain": round(I / t_p / 1e6, 2),
                     "accel_compensated": round(I / t_c / 1e6, 2),
                     "vjp_compensated": round(I / t_v / 1e6, 2)},
           "frac_fp32_peak": {"accel_compensated": round(FLOP_ACCEL * I / (t_c * 1e-3) / PEAK_FP32, 4),
                              "vjp_compensated": round(FLOP_VJP * I / (t_v * 1e-3) / PEAK_FP32, 4)},
           "bin_hbm_gbs": round(40.0 * sp.n / (t_bin * 1e-3) / 1e9, 1)}
    if with_cpu:
        sinks, maxc = sample_sinks(b, sp.n, 8192, 4, 512, 4)
        s_t = torch.from_numpy(sinks).to(dev)
        ap = nfp.accel(b, 1.0)[s_t].cpu().numpy()
        ac = nfp.accel(b, 1.0, compensated=True)[s_t].cpu().numpy()
        asym = nfp.accel(b, 1.0, compensated=True, symmetric=True)[s_t].cpu().numpy()
        gv = nfp.accel_vjp(b, cot, 1.0, compensated=True)[s_t].cpu().numpy()
        v = cot.cpu().numpy().astype(np.float64)
        del cot, b
        pos_np = pos.cpu().numpy()
        del pos
        torch.cuda.empty_cache()
        # the oracle bins all particles on every call: time that alone (one
        # sink) to separate it from the pair sums of the sample
        tb0 = time.perf_counter()
        oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, sinks=sinks[:1])
        tb1 = time.perf_counter()
        tc0 = time.perf_counter()
        ex, cnt = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, sinks=sinks, return_count=True)
        tc1 = time.perf_counter()
        rd = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, sinks=sinks, round_offsets=True)
        exg = oracle.jvp(pos_np, sp.K, sp.L, sp.eps_s, v, sinks=sinks)
        rdg = oracle.jvp(pos_np, sp.K, sp.L, sp.eps_s, v, sinks=sinks, round_offsets=True)
        rec["err_vs_fp64"] = {"plain": err_block(ap, ex, rd), "compensated": err_block(ac, ex, rd),
                              "compensated_symmetric": err_block(asym, ex, rd),
                              "vjp_compensated": err_block(gv, exg, rdg),
                              "sinks": int(len(sinks)),
                              "sample": f"{len(sinks)} sinks: 8192 random plus up to 512 from "
                                        f"each of the 4 densest cells (largest {maxc})"}
        t_obin = tb1 - tb0
        rate = cnt / max(1e-9, (tc1 - tc0) - t_obin)
        rec["cpu_oracle"] = {"value": round(rate / 1e9, 4), "unit": "G pair-interactions/s",
                             "threads": oracle.num_threads(), "sample_pairs": cnt,
                             "sample_s": round(tc1 - tc0, 2), "binning_s": round(t_obin, 2),
                             "extrapolated_full_box_s": round(t_obin + I / rate, 1),
                             "note": "pair rate of the sample with the oracle's own binning "
                                     "of all particles (timed alone) taken out; the full box "
                                     "extrapolated as that binning plus I at that rate"}
    return rec


# ---------------------------------------------------------------- main

def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU; multi-GPU runs are not supported",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calib:
        copy_calibration()
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
    log(f"{sp.name}: n={sp.n} K={sp.K} interactions={I}")
    stream = torch.cuda.current_stream(dev)

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        b = nfp.bin_particles(pos, sp.K, sp.L, sp.eps_s, check=False)
        if ev is not None:
            ev[1].record(stream)
        a0 = nfp.accel(b, 1.0, serial=args.serial)
        if ev is not None:
            ev[2].record(stream)
        a1 = nfp.accel(b, 1.0, compensated=True, serial=args.serial)
        if ev is not None:
            ev[3].record(stream)
        g = nfp.accel_vjp(b, cot, 1.0, compensated=True, serial=args.serial)
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
    log(f"{args.steps} steps timed")

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
    pairs = pairs_by_class(b)
    assert sum(pairs.values()) == I, (pairs, I)

    # The widened rows, timed after the step (not part of value): the Plummer
    # law (plain accelerations), the p = 8 cell multipoles, the time-step
    # statistics and choice and the kick/drift update.
    reps = args.steps
    t_plum = ev_time(stream, lambda: nfp.accel(b, 1.0, plummer=True), reps)
    t_full = ev_time(stream, lambda: nfp.accel(b, 1.0, spline_everywhere=True), reps)
    from paper_1810_02916_amd._lib import NfError
    try:   # the static scratch holds the planner of boxes up to a few million particles
        t_noalloc, noalloc_skip = ev_time(
            stream, lambda: nfp.accel_noalloc(b, 1.0, compensated=True), reps), None
    except NfError as exc:
        t_noalloc, noalloc_skip = None, str(exc)
    t_sym = ev_time(stream, lambda: nfp.accel(b, 1.0, compensated=True, symmetric=True), reps)
    a_sym = nfp.accel(b, 1.0, compensated=True, symmetric=True)
    t_mom = ev_time(stream, lambda: nfp.multipoles(b, 8), reps)
    vel = torch.randn((sp.n, 3), generator=torch.Generator(device=dev).manual_seed(sp.seed * 10 + 3),
                      device=dev, dtype=torch.float32)
    t_stats = ev_time(stream, lambda: nfp.step_stats(b, a_plain, vel), reps)
    amax, vrms, glob = nfp.step_stats(b, a_plain, vel)
    t_choose = ev_time(stream, lambda: nfp.step_bounds(b, amax, vrms, glob, dlna_max=0.03,
                                                       hubble=1.0, eta=0.15), reps)
    pos2, vel2 = pos.clone(), vel.clone()
    t_kd = ev_time(stream, lambda: nfp.kick_drift(b, a_plain, vel2, pos2, 1e-6, 1e-6), reps)
    stats_bytes = 28.0 * sp.n + 4.0 * (sp.K ** 3 + 1) + 8.0 * sp.K ** 3 + 24.0 * sp.K ** 3
    kd_bytes = 84.0 * sp.n
    mom_bytes = 16.0 * sp.n + 4.0 * nfp.multipole_terms(8) * sp.K ** 3 + 4.0 * (sp.K ** 3 + 1)
    extras = {
        "plummer_accel_plain": {"ms": round(t_plum, 4), "gdips": round(I / t_plum / 1e6, 2)},
        "accel_plain_shortcut_off": {"ms": round(t_full, 4), "gdips": round(I / t_full / 1e6, 2)},
        "accel_compensated_symmetric": {"ms": round(t_sym, 4), "gdips": round(I / t_sym / 1e6, 2),
                                        "engaged": not bool(torch.equal(a_sym, a_comp)),
                                        "vs_gather": round(t_comp / t_sym, 4),
                                        "note": "Newton's third law between dense cells"},
        "accel_compensated_noalloc": ({"ms": round(t_noalloc, 4),
                                       "gdips": round(I / t_noalloc / 1e6, 2),
                                       "note": "static scratch, the three kernels in turn"}
                                      if t_noalloc is not None else {"skipped": noalloc_skip}),
        "multipoles_p8": {"ms": round(t_mom, 4), "terms": nfp.multipole_terms(8),
                          "algorithmic_bytes": int(mom_bytes),
                          "hbm_gbs": round(mom_bytes / (t_mom * 1e-3) / 1e9, 1),
                          "hbm_frac": round(mom_bytes / (t_mom * 1e-3) / PEAK_HBM, 4)},
        "step_stats": {"ms": round(t_stats, 4), "algorithmic_bytes": int(stats_bytes),
                       "hbm_gbs": round(stats_bytes / (t_stats * 1e-3) / 1e9, 1)},
        "step_choice": {"ms": round(t_choose, 4)},
        "kick_drift": {"ms": round(t_kd, 4), "algorithmic_bytes": int(kd_bytes),
                       "hbm_gbs": round(kd_bytes / (t_kd * 1e-3) / 1e9, 1),
                       "hbm_frac": round(kd_bytes / (t_kd * 1e-3) / PEAK_HBM, 4)},
    }
    log("extras timed")
    result = {
        "metric": METRIC,
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
            "force_kernels": "one after another" if args.serial else "concurrent",
        },
        "breakdown_ms": {"bin": round(t_bin, 4), "accel_plain": round(t_plain, 4),
                         "accel_compensated": round(t_comp, 4), "vjp_compensated": round(t_vjp, 4)},
        "gdips": {"accel_plain": round(I / t_plain / 1e6, 2),
                  "accel_compensated": round(I / t_comp / 1e6, 2),
                  "vjp_compensated": round(I / t_vjp / 1e6, 2)},
        "pairs_by_kernel": pairs,
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

    with_cpu = not args.no_cpu
    if with_cpu:
        import oracle
        cinfo = cpu_info()
        rng = np.random.default_rng(12345)
        m = sp.n if args.cpu_sinks <= 0 else min(args.cpu_sinks, sp.n)
        sinks = np.sort(rng.choice(sp.n, m, replace=False))
        pos_np = pos.cpu().numpy()
        log(f"oracle on {m} sinks, {oracle.num_threads()} threads")
        tc0 = time.perf_counter()
        ref, cnt = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, sinks=sinks, return_count=True)
        tc1 = time.perf_counter()
        rnd = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, sinks=sinks, round_offsets=True)
        # one core, on a smaller sample
        threads = oracle.num_threads()
        sinks1 = np.sort(rng.choice(sp.n, min(sp.n, 1 << 16), replace=False))
        oracle.set_num_threads(1)
        tq0 = time.perf_counter()
        _, cnt1 = oracle.accel(pos_np, sp.K, sp.L, sp.eps_s, sinks=sinks1, return_count=True)
        tq1 = time.perf_counter()
        oracle.set_num_threads(threads)
        # the VJP on a sample of 2^18 sinks
        sv = np.sort(rng.choice(sp.n, min(sp.n, 1 << 18), replace=False))
        v64 = cot.cpu().numpy().astype(np.float64)
        refg = oracle.jvp(pos_np, sp.K, sp.L, sp.eps_s, v64, sinks=sv)
        rndg = oracle.jvp(pos_np, sp.K, sp.L, sp.eps_s, v64, sinks=sv, round_offsets=True)
        ap = a_plain.cpu().numpy()[sinks]
        ac = a_comp.cpu().numpy()[sinks]
        asym = a_sym.cpu().numpy()[sinks]
        gv = g.cpu().numpy()[sv]
        result["cpu_baseline"] = {
            "value": round(cnt / (tc1 - tc0) / 1e9, 4), "unit": "G pair-interactions/s",
            "cores": threads, "kind": "oracle",
            "sample": f"FP64 oracle accelerations of {m} random sinks of {sp.name} "
                      f"({cnt} pair interactions, includes its binning of all {sp.n} particles), "
                      f"{tc1 - tc0:.2f} s on {threads} OpenMP threads",
            "cpu": cinfo,
            "one_core": {"value": round(cnt1 / (tq1 - tq0) / 1e9, 4),
                         "unit": "G pair-interactions/s",
                         "sample": f"{len(sinks1)} random sinks ({cnt1} pair interactions), "
                                   f"{tq1 - tq0:.2f} s on 1 thread"},
        }
        result["err_vs_fp64"] = {
            "plain": err_block(ap, ref, rnd), "compensated": err_block(ac, ref, rnd),
            "compensated_symmetric": err_block(asym, ref, rnd),
            "vjp_compensated": err_block(gv, refg, rndg),
            "sinks": m, "vjp_sinks": int(len(sv)),
            "note": "e2e: against the oracle on exact offsets; kernel: against the oracle on "
                    "the float offsets the GPU reads; e_repr_rms: between the two oracles"}
        log("oracle done")

    if not args.no_configs:
        del out, b, a_plain, a_comp, g, pos2, vel2
        torch.cuda.empty_cache()
        configs = {}
        for name, fn in (("uniform32k", rec_uniform32k), ("clustered262k", rec_clustered262k),
                         ("batched64", rec_batched64), ("clustered134m", rec_clustered134m)):
            tq = time.perf_counter()
            configs[name] = fn(args, stream, with_cpu)
            configs[name]["record_s"] = round(time.perf_counter() - tq, 1)
            torch.cuda.empty_cache()
            log(f"config {name} done")
        result["configs"] = configs
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
