"""GPU parity of the HIP path against the FP64 oracle.

Forces are gated end to end (oracle on the exact offsets) and on the
kernel's own error (oracle on the float-rounded offsets), by rms, by the
per-particle maximum and by the fraction of particles above 1e-4 (the
table in tests/errstats.py: plain 1e-5 / 5e-6, compensated 1e-6 / 5e-7;
the VJP's end-to-end gate is max(that, 2 e_repr)).  In the test of the
item classes every class (dense, light, narrow) is gated on its own.
Binning is bit-exact: cell_start and order equal the oracle's, and every
offset equals the oracle's double offset rounded to float.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1810_02916_amd import nearfield as nfp
from paper_1810_02916_amd.synth import (WORKLOADS, batched_specs, clustered_box,
                                        gaussian_cotangent, make_box, uniform_box)
from tests.errstats import err_stats, gate, gate_vjp

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _gpu(pos):
    return torch.from_numpy(np.ascontiguousarray(pos)).to(DEV)


def _bin_check(pos, K, L, eps=0.01):
    b = nfp.bin_particles(_gpu(pos), K, L, eps)
    torch.cuda.synchronize()
    cs, order, off = oracle.bin_particles(pos, K, L)
    bx = b.boxes[0]
    np.testing.assert_array_equal(bx.cell_start.cpu().numpy(), cs)
    np.testing.assert_array_equal(bx.order.cpu().numpy(), order)
    got = bx.off.cpu().numpy()
    assert got.view(np.uint32).tobytes() == off.view(np.uint32).tobytes(), "offsets differ bitwise"
    return b


# ------------------------------------------------------------------ binning

@pytest.mark.parametrize("name", ["uniform32k", "clustered262k"])
def test_bin_bit_exact(name):
    sp = WORKLOADS[name]
    print(f"[bin] {name}", flush=True)
    _bin_check(make_box(sp), sp.K, sp.L)


def test_bin_faces_and_wrapping():
    """Particles on cell faces, at x = 0 and x = L, slightly negative, and
    many box lengths away all bin exactly as the oracle does."""
    K, L = 7, 3.0
    h = L / K
    rng = np.random.default_rng(7)
    faces = np.array([[i * h, j * h, k * h] for i in range(K + 1) for j in (0, 3) for k in (1, K)],
                     dtype=np.float64)
    pos = np.concatenate([
        faces,
        np.array([[0.0, 0.0, 0.0], [L, L, L], [-1e-17, -1e-300, -0.0], [L - 1e-16, 1e-16, 0.5 * h],
                  [-7.25 * L, 13.5 * L, 1e6 * L + 0.1], [-h / 2, h / 2, -h]]),
        rng.uniform(-2 * L, 3 * L, size=(500, 3)),
    ])
    _bin_check(pos, K, L)


def test_bin_ragged_and_empty_cells():
    """Tiles with a ragged tail: n not a multiple of the 4096-key sort tile,
    many empty cells, one very dense cell."""
    rng = np.random.default_rng(11)
    K, L = 24, 1.0
    dense = 0.5 + 0.001 * rng.random((5001, 3))
    sparse = rng.random((777, 3))
    pos = np.concatenate([dense, sparse])[rng.permutation(5778)]
    _bin_check(pos, K, L)


def test_bin_empty_box_and_nonfinite():
    K, L = 5, 1.0
    b = nfp.bin_particles(torch.empty((0, 3), dtype=torch.float64, device=DEV), K, L, 0.01)
    torch.cuda.synchronize()
    assert (b.boxes[0].cell_start.cpu().numpy() == 0).all()
    pos = np.array([[0.1, 0.2, 0.3], [np.nan, 0.5, 0.5], [0.7, np.inf, 0.1], [0.4, 0.4, 4e62]])
    with pytest.raises(ValueError, match="non-finite"):
        nfp.bin_particles(_gpu(pos), K, L, 0.01)
    with pytest.raises(ValueError, match="non-finite"):
        nfp.nearfield_accel(_gpu(pos), K, L, 0.01)
    b = nfp.bin_particles(_gpu(pos), K, L, 0.01, check=False)
    torch.cuda.synchronize()
    assert b.nbad() == [3]
    order = b.boxes[0].order.cpu().numpy()
    assert sorted(order.tolist()) == [0, 1, 2, 3]


@pytest.mark.parametrize("K,n", [(8, 4096 * 3), (50, 200003), (64, 4096 * 50), (81, 300001)])
def test_bin_digit_widths(K, n):
    """Key ranges that take one 9-bit pass (K=8), two 9-bit passes (K=50,
    K=64: 17 and 18 bits) and three 8-bit passes (K=81: 20 bits), over many
    sort tiles, a full last tile and a ragged one; half the particles in a
    few dense clusters, the rest uniform, in shuffled order."""
    rng = np.random.default_rng(K * 1000 + 3)
    L = 2.0
    nc = n // 2
    centres = rng.uniform(0, L, size=(7, 3))
    clus = centres[rng.integers(0, 7, nc)] + 0.004 * L * rng.standard_normal((nc, 3))
    pos = np.concatenate([clus, rng.uniform(0, L, size=(n - nc, 3))])[rng.permutation(n)]
    print(f"[bin] K={K} n={n}", flush=True)
    _bin_check(pos, K, L)


def test_bin_batched_matches_single():
    specs = batched_specs(4, seed=5, lo=4000, hi=9000)
    poss = [make_box(s) for s in specs]
    bb = nfp.bin_particles_batched([_gpu(p) for p in poss], [s.K for s in specs],
                                   [s.L for s in specs], [s.eps_s for s in specs])
    torch.cuda.synchronize()
    for p, s, bx in zip(poss, specs, bb.boxes):
        cs, order, off = oracle.bin_particles(p, s.K, s.L)
        np.testing.assert_array_equal(bx.cell_start.cpu().numpy(), cs)
        np.testing.assert_array_equal(bx.order.cpu().numpy(), order)
        assert bx.off.cpu().numpy().tobytes() == off.tobytes()


# ------------------------------------------------------------------ accel

def _accel(pos, K, L, eps, gm=1.0, **kw):
    b = nfp.bin_particles(_gpu(pos), K, L, eps)
    a = nfp.accel(b, gm, **kw)
    torch.cuda.synchronize()
    return a.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("simple", [False, True])
@pytest.mark.parametrize("compensated", [False, True])
@pytest.mark.parametrize("name", ["uniform32k", "clustered262k"])
def test_accel_parity(name, compensated, simple):
    sp = WORKLOADS[name]
    pos = make_box(sp)
    print(f"[accel] {name} comp={compensated} simple={simple}", flush=True)
    got = _accel(pos, sp.K, sp.L, sp.eps_s, compensated=compensated, simple=simple)
    ref = oracle.accel(pos, sp.K, sp.L, sp.eps_s)
    rnd = oracle.accel(pos, sp.K, sp.L, sp.eps_s, round_offsets=True)
    gate(got, ref, rnd, compensated, tag=f"{name} comp={compensated} simple={simple}")


def test_accel_clustered2m_sampled():
    """Full-size clustered box (128^3 particles, 64^3 cells) in the launch
    configuration of the benchmark, checked on sampled sinks: 4096 random
    sinks plus every sink of the 4 densest cells."""
    sp = WORKLOADS["clustered2m"]
    pos = make_box(sp)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
    a_plain = nfp.accel(b, 1.0).cpu().numpy()
    a_comp = nfp.accel(b, 1.0, compensated=True).cpu().numpy()
    cs = b.boxes[0].cell_start.cpu().numpy()
    order = b.boxes[0].order.cpu().numpy()
    counts = np.diff(cs)
    dense = np.argsort(counts)[-4:]
    rng = np.random.default_rng(3)
    sinks = np.unique(np.concatenate(
        [rng.choice(pos.shape[0], 4096, replace=False)] +
        [order[cs[c]:cs[c + 1]] for c in dense]))
    ref = oracle.accel(pos, sp.K, sp.L, sp.eps_s, sinks=sinks)
    rnd = oracle.accel(pos, sp.K, sp.L, sp.eps_s, sinks=sinks, round_offsets=True)
    gate(a_plain[sinks], ref, rnd, False, tag="clustered2m plain")
    gate(a_comp[sinks], ref, rnd, True, tag="clustered2m compensated")


def test_accel_deterministic():
    sp = WORKLOADS["clustered262k"]
    pos = make_box(sp)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
    r = [nfp.accel(b, 1.0, compensated=c).cpu().numpy() for c in (False, True, False, True)]
    assert r[0].tobytes() == r[2].tobytes()
    assert r[1].tobytes() == r[3].tobytes()


def test_accel_two_body_and_coincident():
    """Two particles inside, at and outside eps, across a periodic face, and a
    coincident pair (zero force)."""
    K, L, gm = 8, 1.0, 2.5
    eps = 0.05
    cases = [
        [[0.30, 0.30, 0.30], [0.32, 0.30, 0.30]],   # inside eps
        [[0.30, 0.30, 0.30], [0.30, 0.35, 0.30]],   # at eps
        [[0.30, 0.30, 0.30], [0.30, 0.30, 0.45]],   # outside
        [[0.01, 0.50, 0.50], [0.99, 0.50, 0.50]],   # across the face x = 0
        [[0.60, 0.60, 0.60], [0.60, 0.60, 0.60]],   # coincident
    ]
    for pos in cases:
        pos = np.array(pos)
        got = _accel(pos, K, L, eps, gm, compensated=True)
        ref = oracle.accel(pos, K, L, eps, gm)
        scale = max(np.abs(ref).max(), 1e-30)
        assert np.abs(got - ref).max() <= 2e-6 * scale, (pos, got, ref)


def test_accel_K5_whole_box():
    """K = 5: the 5x5x5 block is the whole box, every pair interacts once."""
    pos = uniform_box(1500, 2.0, 21)
    got = _accel(pos, 5, 2.0, 0.05, compensated=True)
    ref = oracle.brute_accel(pos, 5, 2.0, 0.05)
    gate(got, ref, oracle.accel(pos, 5, 2.0, 0.05, round_offsets=True), True, tag="K=5")


def test_accel_batched_bitwise_equals_single():
    specs = batched_specs(5, seed=9, lo=3000, hi=20000)
    poss = [make_box(s) for s in specs]
    bb = nfp.bin_particles_batched([_gpu(p) for p in poss], [s.K for s in specs],
                                   [s.L for s in specs], [s.eps_s for s in specs])
    for comp in (False, True):
        batched = [a.cpu().numpy() for a in nfp.accel(bb, 1.0, compensated=comp)]
        for p, s, ab in zip(poss, specs, batched):
            single = _accel(p, s.K, s.L, s.eps_s, compensated=comp).astype(np.float32)
            assert single.tobytes() == ab.tobytes()
            gate(ab, oracle.accel(p, s.K, s.L, s.eps_s),
                 oracle.accel(p, s.K, s.L, s.eps_s, round_offsets=True), comp, tag=f"box n={s.n}")


# ------------------------------------------------------------------ vjp

@pytest.mark.parametrize("compensated", [False, True])
def test_vjp_matches_oracle(compensated):
    sp = WORKLOADS["clustered262k"]
    pos = make_box(sp)
    v = gaussian_cotangent(sp.n, 1815 * 10 + 2)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
    g = nfp.accel_vjp(b, torch.from_numpy(v.astype(np.float32)).to(DEV), 1.0,
                      compensated=compensated).cpu().numpy()
    # the cotangent the kernel sees is float32; feed the oracle the same values
    v64 = v.astype(np.float32).astype(np.float64)
    ref = oracle.jvp(pos, sp.K, sp.L, sp.eps_s, v64)
    rnd = oracle.jvp(pos, sp.K, sp.L, sp.eps_s, v64, round_offsets=True)
    gate_vjp(g, ref, rnd, compensated, tag=f"vjp comp={compensated}")


def test_autograd_backward_is_vjp():
    sp = WORKLOADS["clustered262k"]
    pos = _gpu(make_box(sp)).requires_grad_(True)
    a = nfp.nearfield_accel(pos, sp.K, sp.L, sp.eps_s, 1.0)
    v = torch.from_numpy(gaussian_cotangent(sp.n, 77).astype(np.float32)).to(DEV)
    (a * v).sum().backward()
    b = nfp.bin_particles(pos.detach(), sp.K, sp.L, sp.eps_s)
    g = nfp.accel_vjp(b, v, 1.0)
    assert pos.grad.dtype == torch.float64
    assert torch.equal(pos.grad.float(), g)


@pytest.mark.parametrize("K", [5, 6, 7, 9, 13])
def test_tile_paths_small_K_dense_and_sparse(K):
    """Pencils that wrap around z = 0 and z = K-1, planning groups of 1..4
    cells, cells above and below 64 particles, empty cells."""
    rng = np.random.default_rng(100 + K)
    L = 1.0
    h = L / K
    base = clustered_box(K ** 3 * 6, 2 * K, K, L, 1.5, 0.5, seed=K)
    dense = (np.array([1, K - 1, 0]) + rng.uniform(0, 1, size=(300, 3))) * h   # a >64 cell at z = 0
    dense2 = (np.array([2, 2, K - 1]) + rng.uniform(0, 1, size=(150, 3))) * h  # at z = K-1
    pos = np.concatenate([base, dense, dense2])[rng.permutation(len(base) + 450)]
    eps = 0.03 * h
    ref = oracle.accel(pos, K, L, eps)
    rnd = oracle.accel(pos, K, L, eps, round_offsets=True)
    for comp in (False, True):
        got = _accel(pos, K, L, eps, compensated=comp)
        gate(got, ref, rnd, comp, tag=f"K={K} comp={comp}")
    v = gaussian_cotangent(len(pos), 7 * K).astype(np.float32)
    b = nfp.bin_particles(_gpu(pos), K, L, eps)
    refg = oracle.jvp(pos, K, L, eps, v.astype(np.float64))
    rndg = oracle.jvp(pos, K, L, eps, v.astype(np.float64), round_offsets=True)
    for comp in (False, True):
        g = nfp.accel_vjp(b, torch.from_numpy(v).to(DEV), 1.0, compensated=comp).cpu().numpy()
        gate_vjp(g, refg, rndg, comp, tag=f"K={K} vjp comp={comp}")


def _box_with_counts(K, L, counts, seed):
    """Cell c (linear order) holds counts[c % len(counts)] particles, uniform
    inside the cell."""
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


def _item_class(b, dense_min, narrow=12):
    """Per caller index: the class of the work item that sums it (0 dense,
    1 light, 2 narrow).  A cell's sinks are cut into chunks of 64; a last
    chunk of fewer than dense_min sinks is one light item, a narrow one below
    12 sinks."""
    bx = b.boxes[0]
    cs = bx.cell_start.cpu().numpy()
    order = bx.order.cpu().numpy()
    cls = np.zeros(len(order), dtype=np.int64)
    n = np.diff(cs)
    for c in np.nonzero(n)[0]:
        rem = int(n[c]) % 64
        if 0 < rem < dense_min:
            cls[order[cs[c + 1] - rem:cs[c + 1]]] = 2 if rem < narrow else 1
    return cls


@pytest.mark.parametrize("dense_min", [41, 2])
def test_tile_item_classes_by_cell_count(dense_min):
    """Cells of every size around the item-class boundaries: remainders of
    1..13 sinks (narrow items below 12, light items from 12), 40 and 41
    (the default split between light and dense), and cells of 64 k plus such
    a remainder, so one call mixes dense, light and narrow items.  Each
    class is gated on its own sinks."""
    K, L = 9, 1.0
    counts = [0, 1, 2, 3, 5, 7, 10, 11, 12, 13, 40, 41, 63, 64, 65, 75, 76, 129, 139]
    pos = _box_with_counts(K, L, counts, seed=dense_min)
    eps = 0.05 * L / K
    b = nfp.bin_particles(_gpu(pos), K, L, eps)
    b.set_dense_min(dense_min)
    cls = _item_class(b, dense_min)
    print(f"[classes] dense_min {dense_min} n {len(pos)} per class {np.bincount(cls)}", flush=True)
    assert (np.bincount(cls, minlength=3) > (0 if dense_min > 12 else -1)).all()
    ref = oracle.accel(pos, K, L, eps)
    rnd = oracle.accel(pos, K, L, eps, round_offsets=True)
    v = gaussian_cotangent(len(pos), 11 + dense_min).astype(np.float32)
    refg = oracle.jvp(pos, K, L, eps, v.astype(np.float64))
    rndg = oracle.jvp(pos, K, L, eps, v.astype(np.float64), round_offsets=True)
    for comp in (False, True):
        got = nfp.accel(b, 1.0, compensated=comp).cpu().numpy().astype(np.float64)
        g = nfp.accel_vjp(b, torch.from_numpy(v).to(DEV), 1.0, compensated=comp).cpu().numpy()
        gate(got, ref, rnd, comp, tag=f"dense_min {dense_min} comp={comp}")
        gate_vjp(g, refg, rndg, comp, tag=f"vjp comp={comp}")
        for k in range(3):
            m = cls == k
            if m.any():
                gate(got[m], ref[m], rnd[m], comp, tag=f"class {k} comp={comp}")
                gate_vjp(g[m], refg[m], rndg[m], comp,
                     tag=f"class {k} vjp comp={comp}")


def test_tile_all_items_narrow():
    """A sparse box (at most 11 particles per cell): every item is narrow and
    the dense and light kernels find empty queues."""
    K, L = 16, 1.0
    counts = [1, 4, 0, 11, 2, 7, 3, 9, 0, 5, 6, 10, 8]
    pos = _box_with_counts(K, L, counts, seed=3)
    eps = 0.05 * L / K
    ref = oracle.accel(pos, K, L, eps)
    rnd = oracle.accel(pos, K, L, eps, round_offsets=True)
    print(f"[narrow] n {len(pos)}", flush=True)
    for comp in (False, True):
        got = _accel(pos, K, L, eps, compensated=comp)
        gate(got, ref, rnd, comp, tag=f"narrow comp={comp}")
    v = gaussian_cotangent(len(pos), 12).astype(np.float32)
    b = nfp.bin_particles(_gpu(pos), K, L, eps)
    assert (_item_class(b, 41) == 2).all()
    g = nfp.accel_vjp(b, torch.from_numpy(v).to(DEV), 1.0, compensated=True).cpu().numpy()
    refg = oracle.jvp(pos, K, L, eps, v.astype(np.float64))
    rndg = oracle.jvp(pos, K, L, eps, v.astype(np.float64), round_offsets=True)
    gate_vjp(g, refg, rndg, True, tag="narrow vjp")


@pytest.mark.parametrize("dense_min", [2, 17, 65])
def test_tile_choice_dense_min(dense_min):
    """Every split between the two tile kernels gives the oracle's result:
    dense_min 2 (almost every chunk dense), 17, and 65 (only full 64-sink
    chunks dense, every remainder light).  The binning is reused and the
    workspace regrown by set_dense_min."""
    sp = WORKLOADS["clustered262k"]
    pos = make_box(sp)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
    b.set_dense_min(dense_min)
    print(f"[dense_min] {dense_min}", flush=True)
    ref = oracle.accel(pos, sp.K, sp.L, sp.eps_s)
    rnd = oracle.accel(pos, sp.K, sp.L, sp.eps_s, round_offsets=True)
    for comp in (False, True):
        got = nfp.accel(b, 1.0, compensated=comp).cpu().numpy().astype(np.float64)
        gate(got, ref, rnd, comp, tag=f"dense_min {dense_min} comp={comp}")
    v = gaussian_cotangent(sp.n, 5 + dense_min).astype(np.float32)
    g = nfp.accel_vjp(b, torch.from_numpy(v).to(DEV), 1.0, compensated=True).cpu().numpy()
    refg = oracle.jvp(pos, sp.K, sp.L, sp.eps_s, v.astype(np.float64))
    rndg = oracle.jvp(pos, sp.K, sp.L, sp.eps_s, v.astype(np.float64), round_offsets=True)
    gate_vjp(g, refg, rndg, True, tag=f"dense_min {dense_min} vjp")


@pytest.mark.parametrize("simple", [False, True])
@pytest.mark.parametrize("name", ["uniform32k", "clustered262k"])
def test_plummer_accel_and_vjp(name, simple):
    """The Plummer law (Sec. 4.3) on both kernel paths: plain and compensated
    accelerations and the compensated VJP against the oracle's Plummer law,
    with eps_p = eps_s / 2.16 (the paper's equal-dynamical-time length)."""
    sp = WORKLOADS[name]
    pos = make_box(sp)
    eps_p = sp.eps_s / nfp.SPLINE_PER_PLUMMER
    print(f"[plummer] {name} simple={simple}", flush=True)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, eps_p)
    ref = oracle.accel(pos, sp.K, sp.L, eps_p, law="plummer")
    rnd = oracle.accel(pos, sp.K, sp.L, eps_p, law="plummer", round_offsets=True)
    for comp in (False, True):
        got = nfp.accel(b, 1.0, compensated=comp, simple=simple, plummer=True)
        gate(got.cpu().numpy().astype(np.float64), ref, rnd, comp,
             tag=f"plummer {name} simple={simple} comp={comp}")
    v = gaussian_cotangent(sp.n, 91).astype(np.float32)
    g = nfp.accel_vjp(b, torch.from_numpy(v).to(DEV), 1.0, compensated=True, simple=simple,
                      plummer=True).cpu().numpy()
    refg = oracle.jvp(pos, sp.K, sp.L, eps_p, v.astype(np.float64), law="plummer")
    rndg = oracle.jvp(pos, sp.K, sp.L, eps_p, v.astype(np.float64), law="plummer",
                      round_offsets=True)
    gate_vjp(g, refg, rndg, True, tag=f"plummer {name} vjp")


def test_plummer_large_softening_and_autograd():
    """eps_p above a cell width (the Plummer law has no branch to skip) and
    the autograd path with plummer=True."""
    K, L = 8, 1.0
    pos = clustered_box(4000, 16, K, L, 1.5, 0.5, seed=78)
    eps = 1.3 * L / K
    ref = oracle.accel(pos, K, L, eps, law="plummer")
    rnd = oracle.accel(pos, K, L, eps, law="plummer", round_offsets=True)
    p = _gpu(pos).requires_grad_(True)
    a = nfp.nearfield_accel(p, K, L, eps, 1.0, compensated=True, plummer=True)
    gate(a.detach().cpu().numpy().astype(np.float64), ref, rnd, True, tag="plummer 1.3 cells")
    v = gaussian_cotangent(len(pos), 79).astype(np.float32)
    (a * torch.from_numpy(v).to(DEV)).sum().backward()
    refg = oracle.jvp(pos, K, L, eps, v.astype(np.float64), law="plummer")
    rndg = oracle.jvp(pos, K, L, eps, v.astype(np.float64), law="plummer", round_offsets=True)
    gate_vjp(p.grad.cpu().numpy(), refg, rndg, True, tag="plummer vjp")


def test_spline_everywhere_matches_the_shortcut():
    """The outer-shell shortcut takes the branch the min form would take, so
    switching it off changes only the FP32 summation order (and the cost);
    both agree with the oracle."""
    sp = WORKLOADS["clustered262k"]
    pos = make_box(sp)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
    ref = oracle.accel(pos, sp.K, sp.L, sp.eps_s)
    rnd = oracle.accel(pos, sp.K, sp.L, sp.eps_s, round_offsets=True)
    for comp in (False, True):
        a = nfp.accel(b, 1.0, compensated=comp).cpu().numpy().astype(np.float64)
        f = nfp.accel(b, 1.0, compensated=comp, spline_everywhere=True).cpu().numpy()
        assert err_stats(f.astype(np.float64), a)["rms"] <= (1e-7 if comp else 2e-6)
        gate(f.astype(np.float64), ref, rnd, comp, tag=f"spline everywhere comp={comp}")


def test_tile_large_softening_uses_spline_everywhere():
    """eps above one cell width: the outer-shell Newton shortcut must be off."""
    K, L = 8, 1.0
    pos = clustered_box(4000, 16, K, L, 1.5, 0.5, seed=77)
    eps = 1.7 * L / K
    ref = oracle.accel(pos, K, L, eps)
    got = _accel(pos, K, L, eps, compensated=True)
    gate(got, ref, oracle.accel(pos, K, L, eps, round_offsets=True), True, tag="eps 1.7 cells")


def test_captured_graph_replays_match_eager():
    """Binning + accelerations of several uneven boxes captured once in a HIP
    graph: every replay, with eager work and synchronisations between
    replays and positions changed in place, matches the eager result
    bitwise."""
    specs = batched_specs(6, seed=21, lo=2000, hi=30000)
    poss = [_gpu(make_box(s)) for s in specs]
    cf = nfp.CapturedForce(poss, [s.K for s in specs], [s.L for s in specs],
                           [s.eps_s for s in specs], 1.0, compensated=True)
    rng = np.random.default_rng(4)
    for rep in range(4):
        if rep:
            for s, p in zip(specs, cf.positions):   # move the particles, in place
                p.add_(torch.from_numpy(rng.normal(0.0, 0.3 * s.L / s.K, size=tuple(p.shape))).to(DEV))
        out = [o.clone() for o in cf.replay()]
        torch.cuda.synchronize()
        eager = nfp.accel(nfp.bin_particles_batched([p.clone() for p in cf.positions],
                                                    [s.K for s in specs], [s.L for s in specs],
                                                    [s.eps_s for s in specs]),
                          1.0, compensated=True)
        torch.cuda.synchronize()
        for a, e in zip(out, eager):
            assert torch.equal(a, e), rep
    p0 = cf.positions[0].cpu().numpy()
    s0 = specs[0]
    gate(cf.out[0].cpu().numpy(), oracle.accel(p0, s0.K, s0.L, s0.eps_s),
         oracle.accel(p0, s0.K, s0.L, s0.eps_s, round_offsets=True), True, tag="graph box 0")


def test_concurrent_callers_on_two_streams():
    """Two host threads, each on a stream of its own, bin and evaluate
    different boxes over and over (the library's side streams and events are
    shared by the device's calls): every result equals, bitwise, the same
    call made alone."""
    import threading
    names = ["uniform32k", "clustered262k"]
    poss = [_gpu(make_box(WORKLOADS[n])) for n in names]
    cots = [torch.from_numpy(gaussian_cotangent(WORKLOADS[n].n, 31).astype(np.float32)).to(DEV)
            for n in names]

    def run(i):
        sp = WORKLOADS[names[i]]
        b = nfp.bin_particles(poss[i], sp.K, sp.L, sp.eps_s)
        return (nfp.accel(b, 1.0), nfp.accel(b, 1.0, compensated=True),
                nfp.accel_vjp(b, cots[i], 1.0, compensated=True))

    alone = [run(i) for i in range(2)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(device=DEV) for _ in range(2)]
    results = [[], []]
    errors = []

    def worker(i):
        try:
            with torch.cuda.stream(streams[i]):
                for _ in range(4):
                    results[i].append(run(i))
                streams[i].synchronize()
        except Exception as e:   # surfaced below
            errors.append(e)

    print("[concurrent] two threads", flush=True)
    ts = [threading.Thread(target=worker, args=(i,)) for i in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i in range(2):
        assert len(results[i]) == 4
        for r in results[i]:
            for got, ref in zip(r, alone[i]):
                assert torch.equal(got, ref), names[i]


def test_serial_kernels_equal_concurrent_bitwise():
    """NF_SERIAL runs the three force kernels one after another on the
    caller's stream; each item's result depends only on its inputs, so the
    outputs equal the concurrent launch bitwise."""
    sp = WORKLOADS["clustered262k"]
    pos = make_box(sp)
    b = nfp.bin_particles(_gpu(pos), sp.K, sp.L, sp.eps_s)
    v = torch.from_numpy(gaussian_cotangent(sp.n, 55).astype(np.float32)).to(DEV)
    for comp in (False, True):
        assert torch.equal(nfp.accel(b, 1.0, compensated=comp, serial=True),
                           nfp.accel(b, 1.0, compensated=comp))
        assert torch.equal(nfp.accel_vjp(b, v, 1.0, compensated=comp, serial=True),
                           nfp.accel_vjp(b, v, 1.0, compensated=comp))
