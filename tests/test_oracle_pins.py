"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each test would fail for a plausible slip in the oracle (a dropped term, a
wrong sign, a wrong neighbour set, a transposed Jacobian):
  * Eq. 2's coefficients re-derived from the construction the paper states
    (Sec. 4.3: Taylor series in r of the softened law, joined to r^-2 with
    continuous value, first and second derivative) and compared with the
    printed coefficients (tests/golden/eq2_constants.txt);
  * the Newtonian two-body force outside the softening radius;
  * C^2 continuity at the spline radius;
  * Newton's third law; the zero force of a one-particle-per-cell lattice;
  * an independent O(N^2) brute force, and textbook minimum-image and
    open-boundary direct sums in the cases where the 5x5x5 block reduces to
    them;
  * invariances (permutation, whole-cell translation, scaling, gm);
  * derivative pins: central finite differences, J = J^T, sum rules and the
    closed-form two-body Jacobian;
  * the Plummer law of Sec. 4.3: two-body closed form, open and minimum-image
    direct sums, its Jacobian, and the equal-minimum-dynamical-time relation
    behind the printed eps_s = 2.16 eps_p.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1810_02916_amd.synth import clustered_box, gaussian_cotangent, uniform_box

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "eq2_constants.txt")


def _golden():
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                out[k] = float(v)
    return out


def _construction_coefficients(eps):
    """F(r) = r (a + b r + c r^2) joined to 1/r^2 at r = eps with matching
    value, slope and curvature; returns (a, b, c)."""
    # F(r) = a r + b r^2 + c r^3 ; F' = a + 2 b r + 3 c r^2 ; F'' = 2 b + 6 c r
    e = eps
    M = np.array([[e, e ** 2, e ** 3], [1.0, 2 * e, 3 * e ** 2], [0.0, 2.0, 6 * e]])
    rhs = np.array([e ** -2, -2.0 * e ** -3, 6.0 * e ** -4])
    return np.linalg.solve(M, rhs)


def _two_body(r, eps, K=16, L=1.0, gm=1.0, axis=0, x0=0.37):
    p = np.full((2, 3), 0.41)
    p[0, axis] = x0
    p[1, axis] = x0 + r
    return oracle.accel(p, K, L, eps, gm)


def test_spline_coefficients_match_construction():
    g = _golden()
    for eps in (0.013, 0.05, 0.3):
        a, b, c = _construction_coefficients(eps)
        np.testing.assert_allclose([a * eps ** 3, b * eps ** 4, c * eps ** 5],
                                   [g["c0"], g["c1"], g["c2"]], rtol=1e-9)


@pytest.mark.parametrize("u", [0.05, 0.3, 0.5, 0.77, 0.999])
def test_two_body_inside_eps(u):
    eps = 0.01  # physical units; K=16, L=1 -> cell width 1/16
    a, b, c = _construction_coefficients(eps)
    r = u * eps
    acc = _two_body(r, eps)
    F = r * (a + b * r + c * r * r)
    np.testing.assert_allclose(acc[0], [F, 0, 0], rtol=1e-12, atol=1e-9 * F)
    np.testing.assert_allclose(acc[1], [-F, 0, 0], rtol=1e-12, atol=1e-9 * F)


@pytest.mark.parametrize("r", [0.011, 0.02, 0.06, 0.09])
def test_two_body_outside_is_newton(r):
    eps = 0.01
    for axis in range(3):
        acc = _two_body(r, eps, axis=axis)
        expect = np.zeros(3)
        expect[axis] = 1.0 / r ** 2
        np.testing.assert_allclose(acc[0], expect, rtol=1e-12, atol=1e-12 / r ** 2)
        np.testing.assert_allclose(acc[1], -expect, rtol=1e-12, atol=1e-12 / r ** 2)


def test_two_body_across_periodic_face_and_gm():
    K, L, gm = 16, 1.0, 3.5
    p = np.array([[0.01, 0.5, 0.5], [0.99, 0.5, 0.5]])
    acc = oracle.accel(p, K, L, 0.001, gm)
    d = 0.02   # particle 1 sits 0.02 below particle 0 through the face
    np.testing.assert_allclose(acc[0], [-gm / d ** 2, 0, 0], rtol=1e-9)
    np.testing.assert_allclose(acc[1], [gm / d ** 2, 0, 0], rtol=1e-9)


def test_beyond_two_cells_no_force():
    """A pair three cells apart on one axis is far field: zero near force."""
    K, L = 16, 1.0
    h = L / K
    p = np.array([[0.5 * h, 0.5, 0.5], [3.5 * h, 0.5, 0.5]])
    np.testing.assert_array_equal(oracle.accel(p, K, L, 1e-3), 0.0)
    p = np.array([[0.5 * h, 0.5, 0.5], [2.5 * h, 0.5, 0.5]])
    assert np.abs(oracle.accel(p, K, L, 1e-3)).max() > 0


def test_c2_continuity_at_eps():
    eps = 0.02
    h = 1e-5 * eps

    def F(r):
        return _two_body(r, eps)[0, 0]

    lo = [F(eps - k * h) for k in (0, 1, 2)]
    hi = [F(eps + k * h) for k in (0, 1, 2)]
    np.testing.assert_allclose(lo[0], 1.0 / eps ** 2, rtol=1e-12)
    np.testing.assert_allclose(hi[0], 1.0 / eps ** 2, rtol=1e-12)
    d1_lo = (lo[0] - lo[1]) / h
    d1_hi = (hi[1] - hi[0]) / h
    np.testing.assert_allclose(d1_lo, -2.0 / eps ** 3, rtol=1e-4)
    np.testing.assert_allclose(d1_hi, -2.0 / eps ** 3, rtol=1e-4)
    d2_lo = (lo[0] - 2 * lo[1] + lo[2]) / h ** 2
    d2_hi = (hi[2] - 2 * hi[1] + hi[0]) / h ** 2
    np.testing.assert_allclose(d2_lo, 6.0 / eps ** 4, rtol=2e-3)
    np.testing.assert_allclose(d2_hi, 6.0 / eps ** 4, rtol=2e-3)


def test_min_form_is_branch_form():
    """The ratio spline/Newton, g(u) = u^3 (10 - 15u + 6u^2), rises
    monotonically to 1 at u = 1, so one min() selects the right branch
    (Sec. 4.3 footnote)."""
    g = _golden()
    u = np.linspace(1e-4, 3.0, 30001)
    ratio = u ** 3 * (g["c0"] + g["c1"] * u + g["c2"] * u * u)
    assert np.all(np.diff(ratio) >= 0)
    assert np.all(ratio[u < 1] <= 1 + 1e-15)
    assert np.all(ratio[u > 1] >= 1 - 1e-15)


def test_coincident_pair_zero_force():
    p = np.array([[0.3, 0.3, 0.3], [0.3, 0.3, 0.3], [0.31, 0.3, 0.3]])
    acc = oracle.accel(p, 8, 1.0, 0.05)
    np.testing.assert_allclose(acc[0], acc[1])
    np.testing.assert_allclose(acc[0] + acc[1], -acc[2], rtol=1e-12)


@pytest.mark.parametrize("K", [5, 7, 12])
def test_newton_third_law(K):
    pos = clustered_box(3000, 12, K, 2.0, 1.5, 0.5, seed=K)
    acc = oracle.accel(pos, K, 2.0, 0.01)
    assert np.abs(acc.sum(axis=0)).max() <= 1e-12 * np.abs(acc).sum()


@pytest.mark.parametrize("shift", [(0.0, 0.0, 0.0), (0.13, -0.31, 0.47), (0.5, 0.5, 0.5)])
def test_lattice_one_per_cell_zero_force(shift):
    K, L = 9, 1.0
    h = L / K
    g = (np.arange(K) + 0.5) * h
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + np.array(shift) * h
    acc = oracle.accel(pos, K, L, 0.3 * h)
    assert np.abs(acc).max() <= 1e-10 / h ** 2


def test_lattice_sublattice_slot_symmetry():
    """m^3 particles per cell on a regular sub-lattice: the force depends only
    on the slot within the cell, and sums to zero."""
    K, L, m = 7, 1.0, 2
    h = L / K
    g = (np.arange(K * m) + 0.5) * (h / m)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    acc = oracle.accel(pos, K, L, 0.1 * h)
    slot = (np.floor(pos / (h / m)).astype(int) % m) @ np.array([m * m, m, 1])
    for s in range(m ** 3):
        a = acc[slot == s]
        assert np.abs(a - a[0]).max() <= 1e-9 * np.abs(acc).max()
    assert np.abs(acc.sum(0)).max() <= 1e-10 * np.abs(acc).sum()


@pytest.mark.parametrize("K,kind", [(5, "u"), (6, "u"), (8, "c"), (11, "c")])
def test_brute_force(K, kind):
    L = 1.7
    pos = uniform_box(1200, L, 100 + K) if kind == "u" else clustered_box(1331, 11, K, L, 1.5, 0.5, 3)
    eps = 0.2 * L / K
    a = oracle.accel(pos, K, L, eps, 0.7)
    b = oracle.brute_accel(pos, K, L, eps, 0.7)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_K5_equals_minimum_image_sum():
    """For K = 5 with every particle within a quarter cell of its cell centre,
    all per-axis separations are below half the box, so the near field is the
    textbook minimum-image all-pairs sum."""
    K, L = 5, 1.0
    h = L / K
    rng = np.random.default_rng(5)
    c = rng.integers(0, K, size=(600, 3))
    pos = (c + 0.5 + rng.uniform(-0.25, 0.25, size=(600, 3))) * h
    eps = 1e-3 * h
    ref = np.zeros_like(pos)
    for i in range(len(pos)):
        d = pos - pos[i]
        d -= L * np.round(d / L)
        r = np.linalg.norm(d, axis=1)
        r[i] = np.inf
        assert r.min() > eps
        ref[i] = (d / r[:, None] ** 3).sum(0)
    np.testing.assert_allclose(oracle.accel(pos, K, L, eps), ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_compact_cluster_equals_open_direct_sum():
    """All particles inside one cell of a large grid: no periodic images and
    every pair interacts, so the near field is the open-boundary direct sum."""
    K, L = 20, 4.0
    h = L / K
    rng = np.random.default_rng(9)
    pos = 7 * h + h * rng.uniform(0.05, 0.95, size=(300, 3))
    eps = 1e-4
    d = pos[None, :, :] - pos[:, None, :]
    r = np.linalg.norm(d, axis=2)
    np.fill_diagonal(r, np.inf)
    ref = (d / r[:, :, None] ** 3).sum(1)
    np.testing.assert_allclose(oracle.accel(pos, K, L, eps), ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_invariances():
    K, L, eps = 8, 1.0, 0.004
    pos = clustered_box(2000, 12, K, L, 1.5, 0.5, seed=2)
    a = oracle.accel(pos, K, L, eps)
    perm = np.random.default_rng(1).permutation(len(pos))
    np.testing.assert_allclose(oracle.accel(pos[perm], K, L, eps), a[perm], rtol=1e-11,
                               atol=1e-13 * np.abs(a).max())
    h = L / K
    # whole-cell translation (exactly representable shift)
    np.testing.assert_allclose(oracle.accel(pos + np.array([3, -2, 5]) * h, K, L, eps), a,
                               rtol=1e-9, atol=1e-12 * np.abs(a).max())
    # (L, eps) scaled by lam: a scales by lam^-2
    lam = 4.0
    np.testing.assert_allclose(oracle.accel(pos * lam, K, L * lam, eps * lam), a / lam ** 2,
                               rtol=1e-12, atol=1e-14 * np.abs(a).max())
    np.testing.assert_allclose(oracle.accel(pos, K, L, eps, 2.5), 2.5 * a, rtol=1e-15)


def test_binning_is_stable_sort_by_cell():
    K, L = 6, 1.0
    rng = np.random.default_rng(4)
    pos = rng.uniform(-0.5, 1.5, size=(3000, 3))
    cs, order, off = oracle.bin_particles(pos, K, L)
    cell, o = oracle.cells(pos, K, L)
    lin = (cell[:, 0] * K + cell[:, 1]) * K + cell[:, 2]
    np.testing.assert_array_equal(order, np.argsort(lin, kind="stable"))
    np.testing.assert_array_equal(cs, np.searchsorted(lin[order], np.arange(K ** 3 + 1)))
    # offsets reconstruct the positions modulo the box
    x = ((cell + 0.5 + o) * (L / K))
    np.testing.assert_allclose(np.mod(x - pos + L / 2, L) - L / 2, 0, atol=1e-12)
    assert np.all(np.abs(o) <= 0.5)
    np.testing.assert_array_equal(off[:, :3], o[order].astype(np.float32))


def test_float_offsets_representation_floor():
    """Rounding the offsets to float changes each coordinate by at most
    2^-25 cell widths, so the accelerations move by a correspondingly small
    relative amount (the floor any FP32 kernel inherits)."""
    K, L = 16, 1.0
    pos = uniform_box(8000, L, 8)
    a = oracle.accel(pos, K, L, 2.16 * 0.04 / 20)
    b = oracle.accel(pos, K, L, 2.16 * 0.04 / 20, round_offsets=True)
    rms = np.sqrt(((a - b) ** 2).sum() / (a ** 2).sum())
    assert 0 < rms < 2e-6


def test_interaction_count():
    K, L = 7, 1.0
    pos = clustered_box(2000, 12, K, L, 1.5, 0.5, seed=6)
    _, cnt = oracle.accel(pos, K, L, 0.01, return_count=True)
    assert cnt == oracle.interactions(pos, K, L)
    cell, _ = oracle.cells(pos, K, L)
    d = cell[None, :, :] - cell[:, None, :]
    d = np.mod(d + 2, K) - 2
    assert cnt == int(np.all(np.abs(d) <= 2, axis=2).sum())


# ------------------------------------------------------------------ derivatives

def _frozen_tangent(pos, K, L, h, seed):
    """Seeded tangent that is zero for particles within 10 h of a cell face
    (so that x +- h t keeps every cell assignment)."""
    t = gaussian_cotangent(len(pos), seed)
    s = pos * (K / L)
    frac = s - np.floor(s)
    margin = 10 * h * (K / L) * np.abs(t).max()
    near = np.any((frac < margin) | (frac > 1 - margin), axis=1)
    t[near] = 0.0
    return t


def test_jvp_matches_central_differences():
    K, L = 8, 1.0
    pos = clustered_box(2000, 12, K, L, 1.5, 0.5, seed=12)
    eps = 0.01
    h = 1e-6 * (L / 12)
    t = _frozen_tangent(pos, K, L, h, 31)
    fd = (oracle.accel(pos + h * t, K, L, eps) - oracle.accel(pos - h * t, K, L, eps)) / (2 * h)
    jt = oracle.jvp(pos, K, L, eps, t)
    err = np.sqrt(((fd - jt) ** 2).sum() / (jt ** 2).sum())
    assert err < 1e-6, err


def test_vjp_scatter_equals_jvp_gather():
    """The Jacobian of a conservative force is symmetric: the chain-rule VJP
    (scatter form) equals the gather-form JVP on the same vector."""
    K, L = 7, 1.0
    pos = clustered_box(1500, 12, K, L, 1.5, 0.5, seed=13)
    v = gaussian_cotangent(len(pos), 5)
    a = oracle.vjp(pos, K, L, 0.02, v, 1.3)
    b = oracle.jvp(pos, K, L, 0.02, v, 1.3)
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


def test_vjp_directional_identity_and_sum_rules():
    K, L = 8, 1.0
    pos = clustered_box(2000, 12, K, L, 1.5, 0.5, seed=14)
    eps = 0.01
    h = 1e-6 * (L / 12)
    t = _frozen_tangent(pos, K, L, h, 41)
    v = gaussian_cotangent(len(pos), 42)
    xbar = oracle.vjp(pos, K, L, eps, v)
    fd = (oracle.accel(pos + h * t, K, L, eps) - oracle.accel(pos - h * t, K, L, eps)) / (2 * h)
    lhs = float((v * fd).sum())
    rhs = float((xbar * t).sum())
    assert abs(lhs - rhs) <= 1e-6 * (np.abs(v * fd).sum())
    # translation invariance: sum_k xbar_k = 0; constant cotangent gives zero
    assert np.abs(xbar.sum(0)).max() <= 1e-10 * np.abs(xbar).sum()
    c = oracle.vjp(pos, K, L, eps, np.tile([0.3, -1.0, 2.0], (len(pos), 1)))
    assert np.abs(c).max() <= 1e-9 * np.abs(xbar).max()


def test_two_body_jacobian_closed_form():
    K, L, eps = 16, 1.0, 0.01
    rng = np.random.default_rng(3)
    for r in (0.02, 0.05):
        dvec = rng.normal(size=3)
        dvec *= r / np.linalg.norm(dvec)
        p = np.array([[0.5, 0.5, 0.5], 0.5 + dvec])
        v = np.array([[0.0, 0.0, 0.0], [1.0, -2.0, 0.5]])
        xbar = oracle.vjp(p, K, L, eps, v)
        rh = dvec / r
        J = (np.eye(3) - 3 * np.outer(rh, rh)) / r ** 3
        np.testing.assert_allclose(xbar[0], J @ v[1], rtol=1e-10)
        np.testing.assert_allclose(xbar[1], -J @ v[1], rtol=1e-10)
    # coincident pair: only the isotropic 10/eps^3 term
    p = np.array([[0.3, 0.3, 0.3], [0.3, 0.3, 0.3]])
    v = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 3.0]])
    xbar = oracle.vjp(p, K, L, eps, v)
    np.testing.assert_allclose(xbar[0], _golden()["c0"] / eps ** 3 * v[1], rtol=1e-12)


# ------------------------------------------------------------------ Plummer law (Sec. 4.3)

def _plummer_two_body(r, eps, K=16, L=1.0, gm=1.0, x0=0.37):
    p = np.full((2, 3), 0.41)
    p[0, 0] = x0
    p[1, 0] = x0 + r
    return oracle.accel(p, K, L, eps, gm, law="plummer")


@pytest.mark.parametrize("r", [0.001, 0.004, 0.01, 0.03, 0.09])
def test_plummer_two_body_closed_form(r):
    """a = gm d / (|d|^2 + eps_p^2)^(3/2), inside and outside eps_p."""
    eps, gm = 0.01, 1.7
    acc = _plummer_two_body(r, eps, gm=gm)
    F = gm * r / (r * r + eps * eps) ** 1.5
    np.testing.assert_allclose(acc[0], [F, 0, 0], rtol=1e-12, atol=1e-12 * F)
    np.testing.assert_allclose(acc[1], [-F, 0, 0], rtol=1e-12, atol=1e-12 * F)


def test_plummer_coincident_pair_and_far_limit():
    p = np.array([[0.3, 0.3, 0.3], [0.3, 0.3, 0.3]])
    np.testing.assert_array_equal(oracle.accel(p, 8, 1.0, 0.05, law="plummer"), 0.0)
    # far from eps_p the law tends to Newton with relative deviation ~ 1.5 (eps/r)^2
    r, eps = 0.1, 1e-4
    a = _plummer_two_body(r, eps)[0, 0]
    assert abs(a * r * r - 1.0) < 2 * 1.5 * (eps / r) ** 2


def test_plummer_compact_cluster_equals_open_direct_sum():
    K, L = 20, 4.0
    h = L / K
    rng = np.random.default_rng(19)
    pos = 7 * h + h * rng.uniform(0.05, 0.95, size=(300, 3))
    eps = 0.01
    d = pos[None, :, :] - pos[:, None, :]
    w = (d ** 2).sum(2) + eps * eps
    ref = (d / w[:, :, None] ** 1.5).sum(1)
    np.testing.assert_allclose(oracle.accel(pos, K, L, eps, law="plummer"), ref, rtol=1e-10,
                               atol=1e-12 * np.abs(ref).max())


def test_plummer_K5_equals_minimum_image_sum():
    K, L = 5, 1.0
    h = L / K
    rng = np.random.default_rng(15)
    c = rng.integers(0, K, size=(500, 3))
    pos = (c + 0.5 + rng.uniform(-0.25, 0.25, size=(500, 3))) * h
    eps = 0.05 * h
    ref = np.zeros_like(pos)
    for i in range(len(pos)):
        d = pos - pos[i]
        d -= L * np.round(d / L)
        w = (d ** 2).sum(1) + eps * eps
        ref[i] = (d / w[:, None] ** 1.5).sum(0)
    np.testing.assert_allclose(oracle.accel(pos, K, L, eps, law="plummer"), ref, rtol=1e-11,
                               atol=1e-11 * np.abs(ref).max())


def test_plummer_jacobian_pins():
    """Central differences, J = J^T (scatter VJP = gather JVP) and the closed
    two-body Jacobian (I w - 3 d d^T) / w^(5/2), w = |d|^2 + eps_p^2."""
    K, L = 8, 1.0
    pos = clustered_box(2000, 12, K, L, 1.5, 0.5, seed=22)
    eps = 0.004
    h = 1e-6 * (L / 12)
    t = _frozen_tangent(pos, K, L, h, 51)
    fd = (oracle.accel(pos + h * t, K, L, eps, law="plummer")
          - oracle.accel(pos - h * t, K, L, eps, law="plummer")) / (2 * h)
    jt = oracle.jvp(pos, K, L, eps, t, law="plummer")
    assert np.sqrt(((fd - jt) ** 2).sum() / (jt ** 2).sum()) < 1e-6
    v = gaussian_cotangent(len(pos), 52)
    a = oracle.vjp(pos, K, L, eps, v, 1.3, law="plummer")
    b = oracle.jvp(pos, K, L, eps, v, 1.3, law="plummer")
    assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()
    rng = np.random.default_rng(4)
    for r in (0.003, 0.05):
        dvec = rng.normal(size=3)
        dvec *= r / np.linalg.norm(dvec)
        p = np.array([[0.5, 0.5, 0.5], 0.5 + dvec])
        v = np.array([[0.0, 0.0, 0.0], [1.0, -2.0, 0.5]])
        xbar = oracle.vjp(p, 16, 1.0, 0.01, v, law="plummer")
        w = r * r + 1e-4
        J = (np.eye(3) * w - 3 * np.outer(dvec, dvec)) / w ** 2.5
        np.testing.assert_allclose(xbar[0], J @ v[1], rtol=1e-10)


def test_spline_plummer_equal_minimum_dynamical_time():
    """Sec. 4.3 converts a Plummer length to the spline radius giving the same
    minimum pairwise dynamical time, which is set by the largest F/r: 1/eps_p^3
    for Plummer (at r = 0) and 10/eps_s^3 for Eq. 2 (also at r -> 0).  Equal
    at eps_s = 10^(1/3) eps_p = 2.154 eps_p; the printed 2.16 is that root to
    three digits."""
    eps_p = 0.004
    r = 1e-9   # F/r at r -> 0: the spline's leading correction is 1.5 r/eps_s ~ 2e-7
    gp = _plummer_two_body(r, eps_p)[0, 0] / r
    g_exact = _two_body(r, 10 ** (1 / 3) * eps_p)[0, 0] / r
    g_paper = _two_body(r, _golden()["spline_per_plummer"] * eps_p)[0, 0] / r
    assert abs(g_exact / gp - 1) < 1e-6
    assert abs(g_paper / gp - 1) < 1e-2
    # the spline's F/r is largest at r -> 0 (it decreases on (0, eps_s))
    eps_s = 2.16 * eps_p
    gs = [_two_body(u * eps_s, eps_s)[0, 0] / (u * eps_s) for u in (1e-6, 0.2, 0.5, 0.9, 1.5)]
    assert all(a > b for a, b in zip(gs, gs[1:]))


# ------------------------------------------------------------------ rounded offsets and sink subsets

def _snapped_box(n, K, seed):
    """Positions in a box of side 1 with K a power of two, so that x * K is
    exact; offsets drawn in [-0.49, 0.49] (a float-rounded offset then stays
    inside its cell)."""
    rng = np.random.default_rng(seed)
    c = rng.integers(0, K, size=(n, 3)).astype(np.float64)
    o = rng.uniform(-0.49, 0.49, size=(n, 3))
    return (c + 0.5 + o) / K


def test_round_offsets_mode_equals_exact_oracle_on_snapped_positions():
    """The rounded-offset mode (Sec. 4.5: the single-precision state judged
    against double precision) evaluates the exact oracle on positions moved
    to (c + 1/2 + fl32(o)) / kappa, which are representable exactly when
    kappa is a power of two: accelerations, JVP and VJP agree bitwise with
    the exact mode run on those moved positions, and differ from the exact
    mode on the original ones."""
    K, L, eps = 16, 1.0, 0.05 / 16
    pos = _snapped_box(3000, K, 41)
    cell, o = oracle.cells(pos, K, L)
    snapped = (cell + 0.5 + o.astype(np.float32).astype(np.float64)) / K
    c2, o2 = oracle.cells(snapped, K, L)
    np.testing.assert_array_equal(c2, cell)
    np.testing.assert_array_equal(o2, o.astype(np.float32).astype(np.float64))
    t = gaussian_cotangent(len(pos), 42)
    for law, e in (("spline", eps), ("plummer", eps / 2.16)):
        r = oracle.accel(pos, K, L, e, law=law, round_offsets=True)
        assert r.tobytes() == oracle.accel(snapped, K, L, e, law=law).tobytes()
        assert not np.array_equal(r, oracle.accel(pos, K, L, e, law=law))
        rj = oracle.jvp(pos, K, L, e, t, law=law, round_offsets=True)
        assert rj.tobytes() == oracle.jvp(snapped, K, L, e, t, law=law).tobytes()
        rv = oracle.vjp(pos, K, L, e, t, law=law, round_offsets=True)
        assert rv.tobytes() == oracle.vjp(snapped, K, L, e, t, law=law).tobytes()
        assert not np.array_equal(rj, oracle.jvp(pos, K, L, e, t, law=law))


def test_sink_subset_equals_full_evaluation():
    """The sink-subset path that the full-size parity tests and the benchmark
    use returns, bitwise, the rows of the full evaluation (any order,
    repeats allowed), for both laws and both offset modes."""
    K, L, eps = 7, 1.0, 0.03 / 7
    pos = clustered_box(3000, 14, K, L, 1.5, 0.5, seed=17)
    t = gaussian_cotangent(len(pos), 18)
    rng = np.random.default_rng(19)
    sinks = np.concatenate([rng.choice(len(pos), 200, replace=False), [5, 5, 0, len(pos) - 1]])
    for law in ("spline", "plummer"):
        for ro in (False, True):
            full = oracle.accel(pos, K, L, eps, law=law, round_offsets=ro)
            sub, cnt = oracle.accel(pos, K, L, eps, law=law, round_offsets=ro, sinks=sinks,
                                    return_count=True)
            assert sub.tobytes() == full[sinks].tobytes()
            fullj = oracle.jvp(pos, K, L, eps, t, law=law, round_offsets=ro)
            subj = oracle.jvp(pos, K, L, eps, t, law=law, round_offsets=ro, sinks=sinks)
            assert subj.tobytes() == fullj[sinks].tobytes()
    # the subset's interaction count is the sum of its sinks' block counts
    cell, _ = oracle.cells(pos, K, L)
    d = np.mod(cell[None, :, :] - cell[sinks][:, None, :] + 2, K) - 2
    assert cnt == int(np.all(np.abs(d) <= 2, axis=2).sum())
    with pytest.raises(oracle.OracleError):
        oracle.accel(pos, K, L, eps, sinks=[len(pos)])


def _tile_box(K):
    """The boxes of the GPU tile tests: a clustered box of 6 particles per
    cell plus two cells of 300 and 150 particles at z = 0 and z = K-1."""
    rng = np.random.default_rng(100 + K)
    L, h = 1.0, 1.0 / K
    base = clustered_box(K ** 3 * 6, 2 * K, K, L, 1.5, 0.5, seed=K)
    dense = (np.array([1, K - 1, 0]) + rng.uniform(0, 1, size=(300, 3))) * h
    dense2 = (np.array([2, 2, K - 1]) + rng.uniform(0, 1, size=(150, 3))) * h
    pos = np.concatenate([base, dense, dense2])[rng.permutation(len(base) + 450)]
    return pos, L, 0.03 * h


def _floor(a_exact, a_round):
    return float(np.sqrt(((a_round - a_exact) ** 2).sum() / (a_exact ** 2).sum()))


@pytest.mark.parametrize("K", [5, 6, 7, 9, 13])
def test_vjp_representation_floor_band(K):
    """Reading of the VJP tolerance: rounding the offsets to float alone
    (no FP32 arithmetic at all) moves the VJP by 0.4-3e-6 rms on these
    boxes, more than it moves the accelerations, because the Jacobian of
    Eq. 2 carries one more power of 1/r than the force.  An end-to-end VJP
    gate at 1e-6 is therefore below what any kernel on float offsets can
    reach; the GPU tests gate the kernel's own error against the oracle on
    the same float offsets, and the end-to-end error at max(1e-6, 2 x floor)."""
    pos, L, eps = _tile_box(K)
    t = gaussian_cotangent(len(pos), 7 * K).astype(np.float32).astype(np.float64)
    fv = _floor(oracle.jvp(pos, K, L, eps, t), oracle.jvp(pos, K, L, eps, t, round_offsets=True))
    fa = _floor(oracle.accel(pos, K, L, eps), oracle.accel(pos, K, L, eps, round_offsets=True))
    print(K, "vjp floor", fv, "accel floor", fa)
    assert 4e-7 <= fv <= 3e-6
    assert fv > fa


def test_vjp_representation_floor_clustered262k():
    """The same floor on the 64^3 clustered box the VJP parity tests use:
    0.4-1.5e-6 rms for the VJP, an order of magnitude above the
    accelerations' floor on that box."""
    from paper_1810_02916_amd.synth import WORKLOADS, make_box
    sp = WORKLOADS["clustered262k"]
    pos = make_box(sp)
    t = gaussian_cotangent(sp.n, 1815 * 10 + 2).astype(np.float32).astype(np.float64)
    fv = _floor(oracle.jvp(pos, sp.K, sp.L, sp.eps_s, t),
                oracle.jvp(pos, sp.K, sp.L, sp.eps_s, t, round_offsets=True))
    fa = _floor(oracle.accel(pos, sp.K, sp.L, sp.eps_s),
                oracle.accel(pos, sp.K, sp.L, sp.eps_s, round_offsets=True))
    print("clustered262k vjp floor", fv, "accel floor", fa)
    assert 4e-7 <= fv <= 1.5e-6
    assert fv > 5 * fa
