"""GPU parity of the per-cell multipole moments against the FP64 oracle.

Both sides take the same float offsets, compute in double and round each
moment once to float; they may sum in a different rounding order, so the bar
is two float ulps of the moment plus 1e-12 of the sum of |terms| (the scale
of any cancellation), and the count moment M_000 is exact."""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_02916_amd import nearfield as nfp
from paper_1810_02916_amd.synth import WORKLOADS, clustered_box, make_box

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _check(pos, K, L, p):
    b = nfp.bin_particles(torch.from_numpy(np.ascontiguousarray(pos)).to(DEV), K, L, 0.01)
    got = nfp.multipoles(b, p).cpu().numpy().astype(np.float64)
    ref, ref32 = oracle.multipoles(pos, K, L, p)
    absm = oracle.abs_moments(pos, K, L, p)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got[:, 0], ref[:, 0])
    tol = 2.0 ** -22 * np.abs(ref32.astype(np.float64)) + 1e-12 * absm
    bad = np.abs(got - ref32.astype(np.float64)) > tol
    assert not bad.any(), (np.argwhere(bad)[:5], got[bad][:5], ref32[bad][:5])


@pytest.mark.parametrize("p", [0, 1, 4, 8])
@pytest.mark.parametrize("name", ["uniform32k", "clustered262k"])
def test_multipoles_match_oracle(name, p):
    sp = WORKLOADS[name]
    print(f"[multipoles] {name} p={p}", flush=True)
    _check(make_box(sp), sp.K, sp.L, p)


def test_multipoles_dense_cells_and_wrapping():
    """Cells with hundreds of particles (several 64-particle chunks inside one
    batch), empty batches, positions outside [0, L)."""
    K, L = 5, 2.0
    rng = np.random.default_rng(71)
    h = L / K
    base = clustered_box(600, 9, K, L, 1.5, 0.5, seed=71)
    dense = (np.array([1, 3, 4]) + rng.uniform(0, 1, size=(333, 3))) * h
    far = rng.uniform(-3 * L, 4 * L, size=(100, 3))
    pos = np.concatenate([base, dense, far])[rng.permutation(1033)]
    _check(pos, K, L, 8)


def test_multipoles_batched_and_empty_box():
    specs = [(clustered_box(5000, 16, 12, 1.0, 1.5, 0.5, seed=5), 12, 1.0),
             (np.zeros((0, 3)), 7, 1.0),
             (clustered_box(9000, 20, 9, 3.0, 1.0, 0.5, seed=6), 9, 3.0)]
    b = nfp.bin_particles_batched([torch.from_numpy(p).to(DEV) for p, _, _ in specs],
                                  [K for _, K, _ in specs], [L for _, _, L in specs],
                                  [0.01] * len(specs))
    got = nfp.multipoles(b, 6)
    for (pos, K, L), g in zip(specs, got):
        g = g.cpu().numpy().astype(np.float64)
        if len(pos) == 0:
            np.testing.assert_array_equal(g, 0.0)
            assert g.shape == (K ** 3, nfp.multipole_terms(6))
            continue
        ref, ref32 = oracle.multipoles(pos, K, L, 6)
        absm = oracle.abs_moments(pos, K, L, 6)
        tol = 2.0 ** -22 * np.abs(ref32.astype(np.float64)) + 1e-12 * absm
        assert (np.abs(g - ref32) <= tol).all()


@pytest.mark.parametrize("p", [1, 8])
def test_multipoles_big_cells_in_pieces(p):
    """Cells above the piece size are summed in pieces and combined: cells of
    exactly one piece (512), one past it (513), two pieces (1024), one past
    (1025) and many (5000), next to small and empty cells, in two boxes of
    one batch."""
    K, L = 6, 1.0
    h = L / K
    rng = np.random.default_rng(90 + p)
    sizes = {(0, 0, 0): 512, (0, 0, 1): 513, (2, 5, 5): 1024, (3, 3, 3): 1025, (5, 5, 4): 5000,
             (1, 1, 1): 7}
    parts = [(np.array(c) + rng.uniform(0, 1, size=(n, 3))) * h for c, n in sizes.items()]
    pos = np.concatenate(parts + [rng.uniform(0, L, size=(300, 3))])
    pos = pos[rng.permutation(len(pos))]
    _check(pos, K, L, p)
    other = clustered_box(4000, 12, 7, 1.0, 1.5, 0.5, seed=9)
    b = nfp.bin_particles_batched([torch.from_numpy(other).to(DEV), torch.from_numpy(pos).to(DEV)],
                                  [7, K], [1.0, L], [0.01, 0.01])
    got = nfp.multipoles(b, p)
    for (q, KK, LL), g in zip([(other, 7, 1.0), (pos, K, L)], got):
        ref, ref32 = oracle.multipoles(q, KK, LL, p)
        absm = oracle.abs_moments(q, KK, LL, p)
        tol = 2.0 ** -22 * np.abs(ref32.astype(np.float64)) + 1e-12 * absm
        g = g.cpu().numpy().astype(np.float64)
        np.testing.assert_array_equal(g[:, 0], ref[:, 0])
        assert (np.abs(g - ref32) <= tol).all()
