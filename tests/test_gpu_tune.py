"""Every tile choice the autotuner can pick gives the oracle's result within
the gates (tests/errstats.py), and the tuner itself: its pick, its table and
the captured graph that uses the pick."""
import dataclasses

import numpy as np
import pytest
import torch

import oracle
from paper_1810_02916_amd import nearfield as nfp
from paper_1810_02916_amd import tune
from paper_1810_02916_amd.synth import batched_specs, gaussian_cotangent, make_box
from tests.errstats import gate, gate_vjp

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
K, L = 9, 1.0
EPS = 0.05 * L / K


def _box_with_counts(counts, seed):
    rng = np.random.default_rng(seed)
    h = L / K
    parts = []
    for c in range(K ** 3):
        n = counts[c % len(counts)]
        if n:
            ijk = np.array([c // (K * K), (c // K) % K, c % K], dtype=np.float64)
            parts.append((ijk + rng.uniform(0.0, 1.0, size=(n, 3))) * h)
    pos = np.concatenate(parts)
    return pos[rng.permutation(len(pos))]


@pytest.fixture(scope="module")
def case():
    """Cells of 0-139 particles (remainders on both sides of every class
    boundary; 5x5x5 blocks of up to ~6000 sources, so the light and narrow
    kernels stage several windows) and the oracle's answers."""
    counts = [0, 1, 2, 3, 5, 7, 8, 10, 11, 12, 13, 16, 17, 23, 24, 25, 33, 40, 41, 49, 57,
              63, 64, 65, 75, 76, 129, 139]
    pos = _box_with_counts(counts, 77)
    v = gaussian_cotangent(len(pos), 78).astype(np.float32)
    v64 = v.astype(np.float64)
    return dict(
        pos=pos, v=torch.from_numpy(v).to(DEV),
        ref=oracle.accel(pos, K, L, EPS), rnd=oracle.accel(pos, K, L, EPS, round_offsets=True),
        refg=oracle.jvp(pos, K, L, EPS, v64),
        rndg=oracle.jvp(pos, K, L, EPS, v64, round_offsets=True))


CHOICES = [(k, v) for k in tune.ORDER for v in tune.CANDIDATES[k]]


@pytest.mark.parametrize("name,value", CHOICES, ids=[f"{k}={v}" for k, v in CHOICES])
def test_every_tile_choice_matches_the_oracle(case, name, value):
    t = dataclasses.replace(tune.DEFAULTS, **{name: value})
    print(f"[tiles] {t}", flush=True)
    b = nfp.bin_particles(torch.from_numpy(case["pos"]).to(DEV), K, L, EPS, tiles=t)
    for comp in (False, True):
        a = nfp.accel(b, 1.0, compensated=comp).cpu().numpy().astype(np.float64)
        gate(a, case["ref"], case["rnd"], comp, tag=f"{name}={value} comp={comp}")
    g = nfp.accel_vjp(b, case["v"], 1.0, compensated=True).cpu().numpy()
    gate_vjp(g, case["refg"], case["rndg"], True, tag=f"{name}={value} vjp")
    # the same choice through the allocation-free entry point: same kernels
    assert torch.equal(nfp.accel_noalloc(b, 1.0, compensated=True),
                       nfp.accel(b, 1.0, compensated=True))


def test_tune_picks_a_candidate_caches_it_and_the_graph_uses_it(case, tmp_path):
    path = str(tmp_path / "tune.json")
    specs = batched_specs(6, seed=31, lo=4000, hi=40000)
    poss = [torch.from_numpy(make_box(s)).to(DEV) for s in specs]
    args = ([s.K for s in specs], [s.L for s in specs], [s.eps_s for s in specs])
    b = nfp.bin_particles_batched(poss, *args)
    print("[tune] searching", flush=True)
    r = tune.tune(b, reps=2, path=path)
    assert not r.cached and r.tiles == b.tiles
    for k, v in r.tiles.as_dict().items():
        assert v in tune.CANDIDATES[k], (k, v)
    assert min(r.times_ms.values()) == r.times_ms[tune._label(r.tiles)]
    b2 = nfp.bin_particles_batched(poss, *args)
    r2 = tune.tune(b2, reps=2, path=path)
    assert r2.cached and r2.tiles == r.tiles and b2.tiles == r.tiles
    # a VJP entry is a different key
    assert tune.workload_key(b2, "vjp", True) != r.key
    # the graph built with the pick equals the eager calls with it, and the oracle
    cf = nfp.CapturedForce(poss, *args, 1.0, compensated=True, tiles=r.tiles)
    out = [o.clone() for o in cf.replay()]
    eager = nfp.accel(b, 1.0, compensated=True)
    torch.cuda.synchronize()
    for o, e in zip(out, eager):
        assert torch.equal(o, e)
    p0 = poss[0].cpu().numpy()
    s0 = specs[0]
    gate(out[0].cpu().numpy(), oracle.accel(p0, s0.K, s0.L, s0.eps_s),
         oracle.accel(p0, s0.K, s0.L, s0.eps_s, round_offsets=True), True, tag="tuned graph")


def test_tune_vjp_mode(case, tmp_path):
    b = nfp.bin_particles(torch.from_numpy(case["pos"]).to(DEV), K, L, EPS)
    r = tune.tune(b, mode="vjp", reps=1, path=str(tmp_path / "v.json"))
    g = nfp.accel_vjp(b, case["v"], 1.0, compensated=True).cpu().numpy()
    gate_vjp(g, case["refg"], case["rndg"], True, tag=f"vjp tuned {r.tiles}")
