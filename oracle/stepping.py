"""FP64 oracle of the time-step inputs and the kick/drift update (test
infrastructure only).

Sec. 4.2: all particles share one step, chosen at the start of each step as
the smallest of three bounds: a largest step in ln(a); eta times a ratio
v_rms / a_max evaluated per cell (taken here as the smallest ratio over the
non-empty cells, then raised to the global ratio when that is larger, which
is the protection against cold cells the section describes); and the step
at which the fastest particle moves 80% of a cell width.  The step's CPU
work lists a Kick and a Drift stage (the performance tables of Sec. 2.3); the
update here is the kick then drift form: v <- v + kick * a, x <- x + drift * v
with the kicked v.

Precision as in the library: velocities are float, positions double; the
kick is evaluated in double and rounded once to float, the drift in double
without contraction.  Per-cell v_rms is the root mean square of |v| over the
cell's particles (the mean velocity is not removed).
"""
from __future__ import annotations

import numpy as np

from .oracle import cells


def kick_drift(pos, vel, acc, kick: float, drift: float):
    """(new positions float64 [n,3], new velocities float32 [n,3])."""
    v = np.asarray(vel, dtype=np.float32).astype(np.float64)
    a = np.asarray(acc, dtype=np.float32).astype(np.float64)
    vnew = (v + float(kick) * a).astype(np.float32)
    xnew = np.asarray(pos, dtype=np.float64) + float(drift) * vnew.astype(np.float64)
    return xnew, vnew


def step_stats(pos, K: int, L: float, acc, vel):
    """Per-cell (a_max, v_rms) as float64 [K^3] each (0 for empty cells) and
    the box's global (a_max, v_rms, v_max) as float64."""
    c, _ = cells(pos, K, L)
    K = int(K)
    lin = (c[:, 0] * K + c[:, 1]) * K + c[:, 2]
    a = np.asarray(acc, dtype=np.float32).astype(np.float64)
    v = np.asarray(vel, dtype=np.float32).astype(np.float64)
    amag = np.sqrt((a[:, 0] * a[:, 0] + a[:, 1] * a[:, 1]) + a[:, 2] * a[:, 2])
    v2 = (v[:, 0] * v[:, 0] + v[:, 1] * v[:, 1]) + v[:, 2] * v[:, 2]
    ncell = K ** 3
    cnt = np.bincount(lin, minlength=ncell)
    amax = np.zeros(ncell)
    np.maximum.at(amax, lin, amag)
    s2 = np.bincount(lin, weights=v2, minlength=ncell)
    vrms = np.where(cnt > 0, np.sqrt(s2 / np.maximum(cnt, 1)), 0.0)
    n = len(v)
    glob = np.array([amag.max() if n else 0.0, np.sqrt(v2.sum() / n) if n else 0.0,
                     np.sqrt(v2.max()) if n else 0.0])
    return amax, vrms, glob


def step_bounds(amax, vrms, glob, *, dlna_max: float, hubble: float, eta: float,
                cell_width: float):
    """The three bounds of Sec. 4.2 (time units of 1/hubble): the largest
    step in ln a, eta times the per-cell ratio (raised to the global ratio
    when that is larger), and 80% of a cell at the fastest particle's speed;
    +inf for a ratio whose denominator is zero."""
    amax = np.asarray(amax, dtype=np.float64)
    vrms = np.asarray(vrms, dtype=np.float64)
    dt1 = dlna_max / hubble
    ok = amax > 0
    cell_ratio = float(np.min(vrms[ok] / amax[ok])) if ok.any() else np.inf
    glob_ratio = glob[1] / glob[0] if glob[0] > 0 else np.inf
    dt2 = eta * max(cell_ratio, glob_ratio)
    dt3 = 0.8 * cell_width / glob[2] if glob[2] > 0 else np.inf
    return float(dt1), float(dt2), float(dt3)


def choose_step(amax, vrms, glob, *, dlna_max: float, hubble: float, eta: float,
                cell_width: float) -> float:
    """The smallest of the three bounds of Sec. 4.2."""
    return min(step_bounds(amax, vrms, glob, dlna_max=dlna_max, hubble=hubble, eta=eta,
                           cell_width=cell_width))
