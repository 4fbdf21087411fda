"""Newton's third law between dense cells (NF_PAIR_SYMMETRIC, Sec. 2.1: each
pair in one field; Eq. 2 odd in r): the symmetric path against the oracle
(the gates of tests/errstats.py), against the gather path, bitwise
reproducible, batched equal to single, and the fall-back to the gather form
when the symmetric plan outgrows its buffer."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_02916_amd import nearfield as nfp
from paper_1810_02916_amd.synth import WORKLOADS, batched_specs, make_box
from tests.errstats import err_stats, gate

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _gpu(pos):
    return torch.from_numpy(np.ascontiguousarray(pos)).to(DEV)


def _box(K, L, counts_of, seed):
    """Cell c holds counts_of(c) particles, uniform inside the cell."""
    rng = np.random.default_rng(seed)
    h = L / K
    parts = []
    for c in range(K ** 3):
        n = counts_of(c, rng)
        if n:
            ijk = np.array([c // (K * K), (c // K) % K, c % K], dtype=np.float64)
            parts.append((ijk + rng.uniform(0.0, 1.0, size=(n, 3))) * h)
    pos = np.concatenate(parts)
    return pos[rng.permutation(len(pos))]


def _mixed_counts(c, rng):
    # about one cell in six symmetric (41..1024 particles, partial last
    # chunks and up to 16 chunks), the rest sparse
    if rng.random() < 1 / 6:
        return int(rng.choice([41, 50, 63, 64, 65, 100, 128, 129, 200, 500, 1024]))
    return int(rng.integers(0, 12))


def _symmetric_cells(pos, K, L, dense_min=41):
    cs, _, _ = oracle.bin_particles(pos, K, L)
    n = np.diff(cs)
    rem = n % 64
    return ((n > 0) & (n <= 1024) & ((rem == 0) | (rem >= dense_min))).sum()


@pytest.mark.parametrize("K", [5, 7, 9])
def test_symmetric_matches_oracle(K):
    L = 1.0
    pos = _box(K, L, _mixed_counts, 500 + K)
    eps = 0.05 * L / K
    print(f"[pair] K={K} n={len(pos)} symmetric cells {_symmetric_cells(pos, K, L)}", flush=True)
    b = nfp.bin_particles(_gpu(pos), K, L, eps)
    ref = oracle.accel(pos, K, L, eps)
    rnd = oracle.accel(pos, K, L, eps, round_offsets=True)
    for comp in (False, True):
        sym = nfp.accel(b, 1.0, compensated=comp, symmetric=True)
        again = nfp.accel(b, 1.0, compensated=comp, symmetric=True)
        gat = nfp.accel(b, 1.0, compensated=comp)
        torch.cuda.synchronize()
        assert torch.equal(sym, again), "not bitwise reproducible"
        assert not torch.equal(sym, gat), "the symmetric path did not engage"
        s = sym.cpu().numpy().astype(np.float64)
        gate(s, ref, rnd, comp, tag=f"symmetric K={K} comp={comp}")
        st = err_stats(s, gat.cpu().numpy().astype(np.float64))
        assert st["rms"] <= (1e-6 if comp else 1e-5), st


def test_symmetric_on_clustered262k_and_plummer():
    sp = WORKLOADS["clustered262k"]
    pos = make_box(sp)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
    print(f"[pair] clustered262k symmetric cells {_symmetric_cells(pos, sp.K, sp.L)}", flush=True)
    ref = oracle.accel(pos, sp.K, sp.L, sp.eps_s)
    rnd = oracle.accel(pos, sp.K, sp.L, sp.eps_s, round_offsets=True)
    for comp in (False, True):
        a = nfp.accel(b, 1.0, compensated=comp, symmetric=True).cpu().numpy().astype(np.float64)
        gate(a, ref, rnd, comp, tag=f"clustered262k symmetric comp={comp}")
    eps_p = sp.eps_s / nfp.SPLINE_PER_PLUMMER
    bp = nfp.bin_particles(_gpu(pos), sp.K, sp.L, eps_p)
    a = nfp.accel(bp, 1.0, compensated=True, plummer=True, symmetric=True)
    gate(a.cpu().numpy().astype(np.float64), oracle.accel(pos, sp.K, sp.L, eps_p, law="plummer"),
         oracle.accel(pos, sp.K, sp.L, eps_p, law="plummer", round_offsets=True), True,
         tag="plummer symmetric")


def test_symmetric_batched_equals_single_and_serial():
    specs = batched_specs(4, seed=12, lo=20000, hi=60000)
    poss = [make_box(s) for s in specs]
    bb = nfp.bin_particles_batched([_gpu(p) for p in poss], [s.K for s in specs],
                                   [s.L for s in specs], [s.eps_s for s in specs])
    batched = nfp.accel(bb, 1.0, compensated=True, symmetric=True)
    serial = nfp.accel(bb, 1.0, compensated=True, symmetric=True, serial=True)
    for p, s, ab, asr in zip(poss, specs, batched, serial):
        single = nfp.accel(nfp.bin_particles(_gpu(p), s.K, s.L, s.eps_s), 1.0, compensated=True,
                           symmetric=True)
        torch.cuda.synchronize()
        assert torch.equal(single, ab)
        assert torch.equal(asr, ab)


def test_symmetric_plan_over_capacity_falls_back_to_the_gather_form():
    """Every cell of 64 particles: each sink needs 125 partial sums, more
    than the buffer's 16 per particle, so the call runs in the gather form and
    equals the call without the flag bitwise."""
    K, L = 8, 1.0
    pos = _box(K, L, lambda c, rng: 64, 9)
    b = nfp.bin_particles(_gpu(pos), K, L, 0.05 / K)
    for comp in (False, True):
        assert torch.equal(nfp.accel(b, 1.0, compensated=comp, symmetric=True),
                           nfp.accel(b, 1.0, compensated=comp))
