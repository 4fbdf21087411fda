"""The allocation-free accelerations (nf_accel_noalloc) against nf_accel.

The allocation-free entry point runs the same kernels with its scratch in the
library's static per-GPU array and the three force kernels in turn on the
caller's stream, so its results equal nf_accel's bitwise.  Two calls in a
row, the second on a smaller box, check that a call leaves nothing behind
that the next one depends on (the array keeps the last call's contents)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_02916_amd import _lib
from paper_1810_02916_amd import nearfield as nfp
from paper_1810_02916_amd.synth import WORKLOADS, batched_specs, make_box
from tests.errstats import err_stats

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _gpu(pos):
    return torch.from_numpy(np.ascontiguousarray(pos)).to(DEV)


@pytest.mark.parametrize("compensated", [False, True])
def test_noalloc_equals_accel_on_two_calls(compensated):
    refs, gots = [], []
    for name in ("clustered262k", "uniform32k"):   # the second input is smaller
        sp = WORKLOADS[name]
        pos = make_box(sp)
        print(f"[noalloc] {name} comp={compensated}", flush=True)
        b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
        out = torch.full((sp.n, 3), float("nan"), dtype=torch.float32, device=DEV)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated(DEV)
        got = nfp.accel_noalloc(b, 1.0, compensated=compensated, out=[out])
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated(DEV) == before
        ref = nfp.accel(b, 1.0, compensated=compensated)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), name
        st = err_stats(got.cpu().numpy().astype(np.float64), oracle.accel(pos, sp.K, sp.L, sp.eps_s))
        assert st["rms"] <= (1e-6 if compensated else 1e-5), (name, st)
        refs.append(ref)
        gots.append(got)


def test_noalloc_batched_boxes_and_plummer():
    specs = batched_specs(5, seed=9, lo=3000, hi=20000)
    poss = [make_box(s) for s in specs]
    bb = nfp.bin_particles_batched([_gpu(p) for p in poss], [s.K for s in specs],
                                   [s.L for s in specs], [s.eps_s for s in specs])
    print("[noalloc] batched", flush=True)
    for kw in (dict(compensated=True), dict(plummer=True)):
        got = nfp.accel_noalloc(bb, 1.0, **kw)
        ref = nfp.accel(bb, 1.0, **kw)
        torch.cuda.synchronize()
        for g, r in zip(got, ref):
            assert torch.equal(g, r), kw
    # then a smaller single box through the same scratch
    sp = WORKLOADS["uniform32k"]
    b = nfp.bin_particles(_gpu(make_box(sp)), sp.K, sp.L, sp.eps_s)
    assert torch.equal(nfp.accel_noalloc(b, 1.0), nfp.accel(b, 1.0))


def test_noalloc_rejects_a_call_beyond_its_scratch():
    """A grid of 160^3 cells needs about 80 MiB of scratch: the call fails on
    the host with NF_EUNSUPPORTED and leaves the output untouched."""
    pos = _gpu(np.random.default_rng(1).random((1000, 3)))
    b = nfp.bin_particles(pos, 160, 1.0, 1e-3)
    out = torch.full((1000, 3), 7.0, dtype=torch.float32, device=DEV)
    with pytest.raises(_lib.NfError) as ei:
        nfp.accel_noalloc(b, 1.0, out=[out])
    assert ei.value.code == _lib.NF_EUNSUPPORTED
    assert "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())
