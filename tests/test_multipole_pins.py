"""Pins of the multipole oracle (Sec. 2.1: per-cell multipole moments of the
particle positions, double precision inside, float storage, p = 8 usual) to
facts of the definition: counts, single-particle closed form, reflection
parity, the binomial shift theorem, and the term count."""
from math import comb

import numpy as np
import pytest

import oracle
from paper_1810_02916_amd.synth import clustered_box


@pytest.mark.parametrize("p", [0, 1, 3, 8])
def test_term_count_and_order(p):
    t = oracle.terms(p)
    assert len(t) == comb(p + 3, 3)
    assert len(set(t)) == len(t) and all(a + b + c <= p for a, b, c in t)
    deg = [a + b + c for a, b, c in t]
    assert deg == sorted(deg)
    if p >= 1:
        assert t[:4] == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_counts_and_single_particle_closed_form():
    K, L = 6, 1.0
    pos = clustered_box(3000, 12, K, L, 1.5, 0.5, seed=61)
    m, m32 = oracle.multipoles(pos, K, L, 8)
    cs, order, off = oracle.bin_particles(pos, K, L)
    np.testing.assert_array_equal(m[:, 0], np.diff(cs.astype(np.int64)))
    # one particle alone in a cell: every moment is its monomial
    h = L / K
    q = np.array([[2.3, 4.1, 0.7]]) * h
    mm, _ = oracle.multipoles(q, K, L, 8)
    c = (2 * K + 4) * K + 0
    o = (q[0] / h) - np.floor(q[0] / h) - 0.5
    o32 = o.astype(np.float32).astype(np.float64)
    want = [o32[0] ** a * o32[1] ** b * o32[2] ** cc for a, b, cc in oracle.terms(8)]
    np.testing.assert_allclose(mm[c], want, rtol=1e-14, atol=1e-300)
    assert np.count_nonzero(mm.sum(1)) == 1


def test_reflection_parity():
    """Reflecting every particle through its cell's centre plane x -> -x
    flips the sign of exactly the moments with odd a."""
    K, L = 5, 1.0
    h = L / K
    rng = np.random.default_rng(3)
    c = rng.integers(0, K, size=(800, 3))
    u = rng.uniform(-0.45, 0.45, size=(800, 3))
    u = np.round(u * 2 ** 20) / 2 ** 20          # exactly representable, so -u is exact too
    pos = (c + 0.5 + u) * h
    ref = pos.copy()
    ref[:, 0] = (c[:, 0] + 0.5 - u[:, 0]) * h
    m, _ = oracle.multipoles(pos, K, L, 6)
    mr, _ = oracle.multipoles(ref, K, L, 6)
    sign = np.array([(-1.0) ** a for a, b, cc in oracle.terms(6)])
    np.testing.assert_allclose(mr, m * sign, rtol=1e-12, atol=1e-12 * np.abs(m).max())


def test_binomial_shift_theorem():
    """Moments about a point s follow from those about the centre:
    sum (x-sx)^a (y-sy)^b (z-sz)^c = sum_ijk C(a,i)C(b,j)C(c,k) (-s)^(a-i,b-j,c-k) M_ijk."""
    K, L, p = 5, 1.0, 5
    pos = clustered_box(2000, 12, K, L, 1.2, 0.4, seed=8)
    m, _ = oracle.multipoles(pos, K, L, p)
    cs, order, off = oracle.bin_particles(pos, K, L)
    s = np.array([0.21, -0.13, 0.34])
    idx = {t: k for k, t in enumerate(oracle.terms(p))}
    x = off[:, :3].astype(np.float64) - s
    cell = np.repeat(np.arange(K ** 3), np.diff(cs.astype(np.int64)))
    for (a, b, c), k in idx.items():
        direct = np.bincount(cell, weights=x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c,
                             minlength=K ** 3)
        shifted = np.zeros(K ** 3)
        for i in range(a + 1):
            for j in range(b + 1):
                for kk in range(c + 1):
                    shifted += (comb(a, i) * comb(b, j) * comb(c, kk)
                                * (-s[0]) ** (a - i) * (-s[1]) ** (b - j) * (-s[2]) ** (c - kk)
                                * m[:, idx[(i, j, kk)]])
        np.testing.assert_allclose(shifted, direct, rtol=1e-9, atol=1e-11 * np.abs(direct).max())
