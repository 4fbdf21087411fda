"""O(N^2) NumPy brute force of the near-field sum (test infrastructure only).

Independent of the C oracle: no binning, no sorting, no neighbour loops.  For
every ordered pair (i, j) it computes both cells from scratch, keeps the pair
when the periodically wrapped cell difference lies in [-2, 2] on every axis
(the R = 2 near-field block of Sec. 2.1), and applies Eq. 2 of Sec. 4.3 in
the single-min form of the paper's footnote (the C oracle uses the branching
form), so the two implementations agree only if both are right.
Meant for N up to a few thousand.
"""
from __future__ import annotations

import numpy as np


def brute_accel(pos, K: int, L: float, eps_s: float, gm: float = 1.0,
                block: int = 512) -> np.ndarray:
    pos = np.asarray(pos, dtype=np.float64)
    n = pos.shape[0]
    kappa = K / L
    s = pos * kappa
    fl = np.floor(s)
    cell = np.mod(fl.astype(np.int64), K)
    off = (s - fl) - 0.5
    eps = eps_s * kappa
    out = np.zeros((n, 3), dtype=np.float64)
    for i0 in range(0, n, block):
        i1 = min(n, i0 + block)
        dc = cell[None, :, :] - cell[i0:i1, None, :]            # (bi, n, 3)
        dw = np.mod(dc + 2, K) - 2                                # wrapped to [-2, K-3]
        near = np.all(np.abs(dw) <= 2, axis=2)                    # (bi, n)
        r = (off[None, :, :] - off[i0:i1, None, :]) + dw          # cell widths
        r2 = np.einsum("ijk,ijk->ij", r, r)
        rho = np.sqrt(r2)
        with np.errstate(divide="ignore", invalid="ignore"):
            newton = np.where(rho > 0, 1.0 / (rho * rho * rho), np.inf)
        poly = (10.0 - 15.0 * rho / eps + 6.0 * (rho / eps) ** 2) / eps ** 3
        g = np.minimum(poly, newton)
        g = np.where(near & (rho > 0), g, 0.0)
        out[i0:i1] = np.einsum("ij,ijk->ik", g, r)
    return gm * kappa * kappa * out
