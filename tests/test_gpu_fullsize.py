"""Parity at the benchmark's full sizes, in the launch configuration that
bench.py times, on sinks the oracle evaluates one by one:

* clustered134m (512^3 particles, 256^3 cells): 8192 random sinks plus 512
  sinks from each of the 4 densest cells; plain and compensated
  accelerations and the compensated VJP (the oracle's JVP on the sampled
  sinks, the Jacobian being symmetric);
* batched64 (64 uneven boxes in one batched call): 256 random sinks per box,
  compensated accelerations.

Same gates as the small cases (tests/errstats.py): end to end against the
oracle on the exact offsets, the kernel's own error against the oracle on
the float offsets, and per-particle bounds."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1810_02916_amd import nearfield as nfp
from paper_1810_02916_amd.synth import WORKLOADS, batched_specs, make_box, make_box_device
from tests.errstats import gate, gate_vjp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _log(msg, t0):
    print(f"[fullsize] {msg} at {time.time() - t0:.1f}s", flush=True)


def test_clustered134m_sampled():
    t0 = time.time()
    sp = WORKLOADS["clustered134m"]
    pos_d = make_box_device(sp, DEV)
    _log("generated", t0)
    b = nfp.bin_particles(pos_d, sp.K, sp.L, sp.eps_s)
    a_plain = nfp.accel(b, 1.0)
    a_comp = nfp.accel(b, 1.0, compensated=True)
    gen = torch.Generator(device=DEV).manual_seed(sp.seed * 10 + 2)
    cot = torch.randn((sp.n, 3), generator=gen, device=DEV, dtype=torch.float32)
    g = nfp.accel_vjp(b, cot, 1.0, compensated=True)
    torch.cuda.synchronize()
    _log("gpu done", t0)
    cs = b.boxes[0].cell_start.cpu().numpy()
    order = b.boxes[0].order.cpu().numpy()
    counts = np.diff(cs.astype(np.int64))
    dense = np.argsort(counts)[-4:]
    rng = np.random.default_rng(4)
    pick = [rng.choice(order[cs[c]:cs[c + 1]], min(512, int(counts[c])), replace=False)
            for c in dense]
    sinks = np.unique(np.concatenate([rng.choice(sp.n, 8192, replace=False)] + pick)).astype(np.int64)
    s_t = torch.from_numpy(sinks).to(DEV)
    ap = a_plain[s_t].cpu().numpy().astype(np.float64)
    ac = a_comp[s_t].cpu().numpy().astype(np.float64)
    gv = g[s_t].cpu().numpy().astype(np.float64)
    v = cot.cpu().numpy().astype(np.float64)
    del a_plain, a_comp, g, cot, b
    pos = pos_d.cpu().numpy()
    del pos_d
    torch.cuda.empty_cache()
    _log(f"oracle on {len(sinks)} sinks (densest cell {int(counts.max())})", t0)
    ref = oracle.accel(pos, sp.K, sp.L, sp.eps_s, sinks=sinks)
    rnd = oracle.accel(pos, sp.K, sp.L, sp.eps_s, sinks=sinks, round_offsets=True)
    _log("oracle accel done", t0)
    refg = oracle.jvp(pos, sp.K, sp.L, sp.eps_s, v, sinks=sinks)
    rndg = oracle.jvp(pos, sp.K, sp.L, sp.eps_s, v, sinks=sinks, round_offsets=True)
    _log("oracle jvp done", t0)
    gate(ap, ref, rnd, False, tag="clustered134m plain")
    gate(ac, ref, rnd, True, tag="clustered134m compensated")
    gate_vjp(gv, refg, rndg, True, tag="clustered134m vjp")


def test_batched64_sampled():
    t0 = time.time()
    specs = batched_specs(64)
    boxes = [make_box(s) for s in specs]
    _log("generated", t0)
    b = nfp.bin_particles_batched([torch.from_numpy(p).to(DEV) for p in boxes],
                                  [s.K for s in specs], [s.L for s in specs],
                                  [s.eps_s for s in specs])
    acc = nfp.accel(b, 1.0, compensated=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    num = den = 0.0
    for p, s, a in zip(boxes, specs, acc):
        sinks = rng.choice(len(p), 256, replace=False).astype(np.int64)
        ref = oracle.accel(p, s.K, s.L, s.eps_s, sinks=sinks)
        got = a.cpu().numpy()[sinks].astype(np.float64)
        num += float(((got - ref) ** 2).sum())
        den += float((ref ** 2).sum())
        gate(got, ref, oracle.accel(p, s.K, s.L, s.eps_s, sinks=sinks, round_offsets=True), True,
             tag=f"box n={s.n}")
    _log(f"64 boxes, overall rms {np.sqrt(num / den):.3e}", t0)
