"""The planner's work list (nf_plan_items) against the items the cell counts
define (the rule nf.h states: every cell's sinks cut into chunks of 64; full
chunks and a last chunk of at least dense_min sinks are dense, a smaller last
chunk light, or narrow below narrow_max sinks).  The set of (box, cell,
chunk, class) rows must be equal, bit for bit, and every class must sit in its
own range of the list; the order inside a class is free."""
import numpy as np
import pytest
import torch

from paper_1810_02916_amd import nearfield as nfp
from paper_1810_02916_amd.synth import WORKLOADS, batched_specs, make_box

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def expected_items(b):
    """Rows (box, cell, chunk, class) from the cell counts, as the rule
    states, in numpy."""
    rows = []
    for bi, bx in enumerate(b.boxes):
        t = bx.tiles
        dense_min = t.dense_min or 41
        narrow_max = t.narrow_max or 12
        n = np.diff(bx.cell_start.cpu().numpy().astype(np.int64))
        cells = np.nonzero(n)[0]
        n = n[cells]
        full, rem = n // 64, n % 64
        nd = full + (rem >= dense_min)
        dc = np.repeat(cells, nd)
        start = np.repeat(np.cumsum(nd) - nd, nd)
        dk = np.arange(int(nd.sum())) - start
        rows.append(np.stack([np.full_like(dc, bi), dc, dk, np.zeros_like(dc)], axis=1))
        lt = (rem > 0) & (rem < dense_min)
        cls = np.where(rem[lt] < narrow_max, 2, 1)
        rows.append(np.stack([np.full(int(lt.sum()), bi), cells[lt], full[lt], cls], axis=1))
    return np.concatenate(rows).astype(np.int64)


def check_plan(b):
    items, counts = nfp.plan_items(b)
    got = items.cpu().numpy().astype(np.int64)
    exp = expected_items(b)
    assert len(got) == len(exp) == sum(counts)
    nd, nl, nn = counts
    assert (got[:nd, 3] == 0).all() and (got[nd:nd + nl, 3] == 1).all()
    assert (got[nd + nl:, 3] == 2).all()
    assert [int((exp[:, 3] == c).sum()) for c in range(3)] == list(counts)
    key = lambda a: a[np.lexsort((a[:, 3], a[:, 2], a[:, 1], a[:, 0]))]
    np.testing.assert_array_equal(key(got), key(exp))
    return counts


@pytest.mark.parametrize("dense_min,narrow_max", [(0, 0), (2, 1), (17, 8), (65, 64), (41, 24)])
def test_plan_items_match_the_rule(dense_min, narrow_max):
    sp = WORKLOADS["clustered262k"]
    b = nfp.bin_particles(torch.from_numpy(make_box(sp)).to(DEV), sp.K, sp.L, sp.eps_s,
                          tiles=nfp.Tiles(dense_min=dense_min, narrow_max=narrow_max))
    counts = check_plan(b)
    print(f"[plan] dense_min={dense_min} narrow_max={narrow_max}: {counts}", flush=True)
    if dense_min == 65:
        assert counts[1] == 0   # every remainder below 64 < narrow_max 64 is narrow


def test_plan_items_batched_boxes_with_their_own_tiles():
    specs = batched_specs(5, seed=9, lo=3000, hi=40000)
    b = nfp.bin_particles_batched([torch.from_numpy(make_box(s)).to(DEV) for s in specs],
                                  [s.K for s in specs], [s.L for s in specs],
                                  [s.eps_s for s in specs])
    b.set_tiles([nfp.Tiles(dense_min=dm, narrow_max=nm)
                 for dm, nm in zip((17, 33, 41, 57, 65), (1, 8, 12, 16, 24))])
    counts = check_plan(b)
    print(f"[plan] batched: {counts}", flush=True)


def test_plan_items_empty_box():
    b = nfp.bin_particles(torch.empty((0, 3), dtype=torch.float64, device=DEV), 5, 1.0, 0.01)
    items, counts = nfp.plan_items(b)
    assert counts == (0, 0, 0) and items.shape[0] == 0
