"""FP64 oracle of the per-cell multipole moments (test infrastructure only).

Sec. 2.1 of the paper computes the multipole moments of the particle
positions of every cell right after the near-field binning, storing them as
32-bit floats while computing in double precision; order p = 8 is its usual
choice.  The paper does not fix the basis; this oracle (and the library) use
complete Cartesian moments about the cell centre,

    M_abc(cell) = sum over particles i in the cell of x_i^a y_i^b z_i^c,
    a + b + c <= p,

with (x, y, z) the particle's offset from its cell centre in cell widths,
taken from the float offsets of the binning, widened to double.  Terms are
ordered by degree n = a + b + c, then a descending, then b descending.
"""
from __future__ import annotations

import numpy as np

from .oracle import bin_particles


def terms(p: int):
    """[(a, b, c)] in storage order for order p."""
    out = []
    for n in range(p + 1):
        for a in range(n, -1, -1):
            for b in range(n - a, -1, -1):
                out.append((a, b, n - a - b))
    return out


def multipoles(pos, K: int, L: float, p: int = 8):
    """(moments [K^3, T] float64, moments rounded to float32) of the binned
    box, T = (p+1)(p+2)(p+3)/6."""
    cs, order, off = bin_particles(pos, K, L)
    x = off[:, 0].astype(np.float64)
    y = off[:, 1].astype(np.float64)
    z = off[:, 2].astype(np.float64)
    ncell = int(K) ** 3
    cell = np.repeat(np.arange(ncell), np.diff(cs.astype(np.int64)))
    tt = terms(p)
    m = np.zeros((ncell, len(tt)), dtype=np.float64)
    for k, (a, b, c) in enumerate(tt):
        m[:, k] = np.bincount(cell, weights=(x ** a) * (y ** b) * (z ** c), minlength=ncell)
    return m, m.astype(np.float32)


def abs_moments(pos, K: int, L: float, p: int = 8):
    """sum over the cell of |x^a y^b z^c| (the scale of each moment's rounding)."""
    cs, order, off = bin_particles(pos, K, L)
    x, y, z = (np.abs(off[:, k].astype(np.float64)) for k in range(3))
    ncell = int(K) ** 3
    cell = np.repeat(np.arange(ncell), np.diff(cs.astype(np.int64)))
    tt = terms(p)
    m = np.zeros((ncell, len(tt)), dtype=np.float64)
    for k, (a, b, c) in enumerate(tt):
        m[:, k] = np.bincount(cell, weights=(x ** a) * (y ** b) * (z ** c), minlength=ncell)
    return m
