"""Seeded synthetic particle boxes.

This module only *draws inputs*: it holds none of the near-field arithmetic
(no cell offsets, no neighbour enumeration, no force law).  Both the FP64
oracle and the HIP path receive the arrays it returns.

The paper's own workload (the 2048^3 Euclid comparison initial conditions and
their late-time clustered states, Sec. 2.3) is not available, so seeded boxes
of the same character stand in for it:

* ``uniform_box``   -- iid uniform positions (the unclustered limit).
* ``clustered_box`` -- a lattice displaced with the Zel'dovich approximation by
  a Gaussian field with a power-law spectrum (the paper sets up its initial
  conditions with the ordinary ZA, Sec. 2.1 and 4.1), followed by a lognormal
  re-weighting of cell occupancies that produces the heavy-tailed cell counts
  of late-time halos (largest cell above 2e5 particles, Sec. 2.2).

Every stage draws from its own child stream of ``numpy.random.SeedSequence``
so that changing one stage never shifts another.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "uniform_box",
    "clustered_box",
    "gaussian_cotangent",
    "BoxSpec",
    "WORKLOADS",
    "make_box",
    "make_box_device",
    "clustered_box_device",
    "batched_specs",
    "occupancy_stats",
    "occupancy_stats_device",
]


def _streams(seed: int, k: int):
    return [np.random.Generator(np.random.PCG64(s))
            for s in np.random.SeedSequence(int(seed)).spawn(k)]


def uniform_box(n: int, L: float, seed: int) -> np.ndarray:
    """``n`` iid uniform positions in ``[0, L)^3`` as an ``(n, 3)`` float64 array."""
    (g,) = _streams(seed, 1)
    return g.uniform(0.0, L, size=(int(n), 3))


def _gaussian_field_k(side: int, g: np.random.Generator, spectral_index: float):
    """Fourier modes (rfftn layout) of a Gaussian field with P(k) ~ k^index.

    White noise is drawn in real space, so the modes are Hermitian by
    construction.  The k=0 mode and every Nyquist plane are zeroed.
    Returns (field_k, kx, ky, kz, k2) with integer wavenumbers.
    """
    w = g.standard_normal((side, side, side))
    wk = np.fft.rfftn(w)
    del w
    kx = np.fft.fftfreq(side, d=1.0 / side)[:, None, None]
    ky = np.fft.fftfreq(side, d=1.0 / side)[None, :, None]
    kz = np.fft.rfftfreq(side, d=1.0 / side)[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (spectral_index / 4.0), 0.0)
    if side % 2 == 0:
        nyq = side // 2
        amp = amp * (np.abs(kx) != nyq) * (np.abs(ky) != nyq) * (np.abs(kz) != nyq)
    return wk * amp, kx, ky, kz, k2


def clustered_box(n: int, side: int, K: int, L: float, sigma_ln: float,
                  psi_rms_cells: float, seed: int,
                  spectral_index: float = -2.0) -> np.ndarray:
    """Clustered box of exactly ``n`` particles, returned as ``(n, 3)`` float64.

    1. lattice of ``side^3`` points at (i+1/2) L/side;
    2. Gaussian density field delta on that lattice, P(k) ~ k^spectral_index;
    3. ZA displacement psi(k) = i k delta(k) / k^2, scaled to an rms 3-D
       length of ``psi_rms_cells`` widths of the K^3 grid;
    4. m_c = displaced-lattice counts on the K^3 grid;
    5. G_c = delta averaged over the lattice points of each K^3 cell,
       standardised to zero mean and unit variance;
    6. cell counts n_c ~ Multinomial(n, w / sum w) with w_c = m_c exp(sigma_ln G_c);
    7. positions uniform inside their cell;
    8. a seeded permutation, so the input is not ordered by cell.
    """
    n = int(n)
    side = int(side)
    K = int(K)
    g_field, g_counts, g_pos, g_perm = _streams(seed, 4)
    dk, kx, ky, kz, k2 = _gaussian_field_k(side, g_field, spectral_index)
    spacing = L / side
    cell = L / K

    # lattice coordinates and their K-cell index
    lat1 = (np.arange(side, dtype=np.float64) + 0.5) * spacing

    # displaced lattice -> counts on K^3
    with np.errstate(divide="ignore", invalid="ignore"):
        inv_k2 = np.where(k2 > 0, 1.0 / k2, 0.0)
    psi = []
    for ka in (kx, ky, kz):
        psi.append(np.fft.irfftn(1j * ka * inv_k2 * dk, s=(side, side, side), axes=(0, 1, 2)))
    rms = math.sqrt(float(sum(np.mean(p * p) for p in psi)))
    scale = (psi_rms_cells * cell / rms) if rms > 0 else 0.0
    cidx = np.zeros((side, side, side), dtype=np.int64)
    for a, p in enumerate(psi):
        shape = [1, 1, 1]
        shape[a] = side
        x = (lat1.reshape(shape) + scale * p) % L
        ca = np.minimum((x * (K / L)).astype(np.int64), K - 1)
        cidx = cidx * K + ca
    del psi
    m = np.bincount(cidx.ravel(), minlength=K ** 3).astype(np.float64)
    del cidx

    # delta averaged onto the K^3 grid by undisplaced lattice position
    delta = np.fft.irfftn(dk, s=(side, side, side), axes=(0, 1, 2))
    del dk
    c1 = np.minimum((lat1 * (K / L)).astype(np.int64), K - 1)
    lat_cell = (c1[:, None, None] * K + c1[None, :, None]) * K + c1[None, None, :]
    ssum = np.bincount(lat_cell.ravel(), weights=delta.ravel(), minlength=K ** 3)
    cnt = np.bincount(lat_cell.ravel(), minlength=K ** 3)
    del delta, lat_cell
    G = np.where(cnt > 0, ssum / np.maximum(cnt, 1), 0.0)
    sd = G.std()
    G = (G - G.mean()) / (sd if sd > 0 else 1.0)

    logw = np.where(m > 0, np.log(np.maximum(m, 1.0)) + sigma_ln * G, -np.inf)
    w = np.exp(logw - logw[np.isfinite(logw)].max())
    counts = g_counts.multinomial(n, w / w.sum())

    cells = np.repeat(np.arange(K ** 3, dtype=np.int64), counts)
    cz = cells % K
    cy = (cells // K) % K
    cx = cells // (K * K)
    del cells
    u = g_pos.random((n, 3))
    pos = np.empty((n, 3), dtype=np.float64)
    pos[:, 0] = (cx + u[:, 0]) * cell
    pos[:, 1] = (cy + u[:, 1]) * cell
    pos[:, 2] = (cz + u[:, 2]) * cell
    del u, cx, cy, cz
    perm = g_perm.permutation(n)
    return np.ascontiguousarray(pos[perm])


def clustered_box_device(n: int, side: int, K: int, L: float, sigma_ln: float,
                         psi_rms_cells: float, seed: int, device="cuda:0",
                         spectral_index: float = -2.0):
    """The clustered recipe of ``clustered_box`` drawn with torch on a device,
    for boxes too large for host-side generation.  Returns an ``(n, 3)``
    float64 tensor on ``device``.  The multinomial cell counts are sampled
    exactly by locating n uniform draws in the cumulative cell weights; the
    draws are independent, so the particles come out in random order.  Its
    random stream differs from ``clustered_box`` (same recipe, other
    generator)."""
    import torch
    dev = torch.device(device)
    g = torch.Generator(device=dev)
    g.manual_seed(int(seed))
    side, K, n = int(side), int(K), int(n)
    w = torch.randn((side, side, side), generator=g, device=dev, dtype=torch.float64)
    wk = torch.fft.rfftn(w)
    del w
    f = torch.fft.fftfreq(side, d=1.0 / side, device=dev, dtype=torch.float64)
    fz = torch.fft.rfftfreq(side, d=1.0 / side, device=dev, dtype=torch.float64)
    kx, ky, kz = f[:, None, None], f[None, :, None], fz[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    amp = torch.where(k2 > 0, k2.clamp_min(1e-300) ** (spectral_index / 4.0), torch.zeros_like(k2))
    if side % 2 == 0:
        nyq = side // 2
        amp = amp * (kx.abs() != nyq) * (ky.abs() != nyq) * (kz.abs() != nyq)
    dk = wk * amp
    del wk, amp
    inv_k2 = torch.where(k2 > 0, 1.0 / k2.clamp_min(1e-300), torch.zeros_like(k2))
    spacing, cell = L / side, L / K
    lat1 = (torch.arange(side, device=dev, dtype=torch.float64) + 0.5) * spacing
    psi = [torch.fft.irfftn(1j * ka * inv_k2 * dk, s=(side, side, side)) for ka in (kx, ky, kz)]
    rms = float(torch.sqrt(sum((p * p).mean() for p in psi)))
    scale = psi_rms_cells * cell / rms if rms > 0 else 0.0
    cidx = torch.zeros((side, side, side), dtype=torch.int64, device=dev)
    for a, p in enumerate(psi):
        shape = [1, 1, 1]
        shape[a] = side
        x = torch.remainder(lat1.reshape(shape) + scale * p, L)
        ca = torch.clamp((x * (K / L)).to(torch.int64), max=K - 1)
        cidx = cidx * K + ca
    del psi
    m = torch.bincount(cidx.reshape(-1), minlength=K ** 3).to(torch.float64)
    del cidx
    delta = torch.fft.irfftn(dk, s=(side, side, side))
    del dk
    c1 = torch.clamp((lat1 * (K / L)).to(torch.int64), max=K - 1)
    lat_cell = ((c1[:, None, None] * K + c1[None, :, None]) * K + c1[None, None, :]).reshape(-1)
    ssum = torch.bincount(lat_cell, weights=delta.reshape(-1), minlength=K ** 3)
    cnt = torch.bincount(lat_cell, minlength=K ** 3)
    del delta, lat_cell
    G = torch.where(cnt > 0, ssum / cnt.clamp_min(1), torch.zeros_like(ssum))
    G = (G - G.mean()) / (G.std() if float(G.std()) > 0 else 1.0)
    logw = torch.where(m > 0, torch.log(m.clamp_min(1.0)) + sigma_ln * G,
                       torch.full_like(m, -float("inf")))
    wts = torch.exp(logw - logw[torch.isfinite(logw)].max())
    cdf = torch.cumsum(wts, 0)
    u = torch.rand(n, generator=g, device=dev, dtype=torch.float64) * cdf[-1]
    cells = torch.clamp(torch.searchsorted(cdf, u, right=True), max=K ** 3 - 1)
    del u, cdf
    cz = cells % K
    cy = (cells // K) % K
    cx = cells // (K * K)
    del cells
    pos = torch.rand((n, 3), generator=g, device=dev, dtype=torch.float64)
    pos[:, 0] += cx
    pos[:, 1] += cy
    pos[:, 2] += cz
    pos *= cell
    return pos


def gaussian_cotangent(n: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) cotangent / tangent vectors, ``(n, 3)`` float64."""
    (g,) = _streams(seed, 1)
    return g.standard_normal((int(n), 3))


# --------------------------------------------------------------------------
# Workload registry.  Softening lengths are Plummer-equivalent (Sec. 4.3):
# eps_p is a fraction of the mean inter-particle spacing, and the spline
# radius is eps_s = 2.16 eps_p.
# --------------------------------------------------------------------------

SPLINE_PER_PLUMMER = 2.16


@dataclasses.dataclass(frozen=True)
class BoxSpec:
    name: str
    n: int
    K: int
    L: float
    eps_p: float
    kind: str              # "uniform" | "clustered"
    side: int = 0
    sigma_ln: float = 0.0
    psi_rms_cells: float = 0.0
    seed: int = 0

    @property
    def eps_s(self) -> float:
        return SPLINE_PER_PLUMMER * self.eps_p


def make_box(spec: BoxSpec) -> np.ndarray:
    if spec.kind == "clustered_device":
        return make_box_device(spec).cpu().numpy()
    if spec.kind == "uniform":
        return uniform_box(spec.n, spec.L, spec.seed)
    return clustered_box(spec.n, spec.side, spec.K, spec.L, spec.sigma_ln,
                         spec.psi_rms_cells, spec.seed)


def make_box_device(spec: BoxSpec, device="cuda:0"):
    """Positions as a float64 tensor on ``device``."""
    import torch
    if spec.kind == "clustered_device":
        return clustered_box_device(spec.n, spec.side, spec.K, spec.L, spec.sigma_ln,
                                    spec.psi_rms_cells, spec.seed, device)
    return torch.from_numpy(make_box(spec)).to(device)


WORKLOADS = {
    # 32^3 uniform particles, unit box, 16^3 cells, eps_p = 0.04 x spacing
    "uniform32k": BoxSpec("uniform32k", 32 ** 3, 16, 1.0, 0.04 / 32, "uniform", seed=1811),
    # 128^3 clustered particles, 64^3 cells, sigma_ln = 1.5, eps_p = 0.041 x spacing
    "clustered2m": BoxSpec("clustered2m", 128 ** 3, 64, 1.0, 0.041 / 128, "clustered",
                           side=128, sigma_ln=1.5, psi_rms_cells=0.5, seed=1812),
    # 512^3 clustered particles in a 125 Mpc/h box, 256^3 cells, sigma_ln = 2.0
    # (drawn on the device: host-side generation of 512^3 takes minutes)
    "clustered134m": BoxSpec("clustered134m", 512 ** 3, 256, 125.0, 0.041 * 125.0 / 512,
                             "clustered_device", side=512, sigma_ln=2.0, psi_rms_cells=0.5,
                             seed=1814),
    # 64^3 clustered particles, 32^3 cells (differentiation workload)
    "clustered262k": BoxSpec("clustered262k", 64 ** 3, 32, 1.0, 0.041 / 64, "clustered",
                             side=64, sigma_ln=1.5, psi_rms_cells=0.5, seed=1815),
}


def batched_specs(nbox: int = 64, seed: int = 1813, lo: int = 32 ** 3,
                  hi: int = 96 ** 3) -> list:
    """Uneven boxes: counts uniform in [lo, hi], K_b = max(5, round((n_b/8)^(1/3)))."""
    (g,) = _streams(seed, 1)
    ns = g.integers(lo, hi + 1, size=nbox)
    out = []
    for b, nb in enumerate(ns):
        nb = int(nb)
        side = int(math.ceil(nb ** (1.0 / 3.0) - 1e-9))
        K = max(5, int(round((nb / 8.0) ** (1.0 / 3.0))))
        out.append(BoxSpec(f"batch{b}", nb, K, 1.0, 0.041 / nb ** (1.0 / 3.0), "clustered",
                           side=side, sigma_ln=1.5, psi_rms_cells=0.5,
                           seed=seed * 1000 + b))
    return out


def occupancy_stats_device(pos, K: int, L: float) -> dict:
    """``occupancy_stats`` for a float64 torch tensor, computed on its device."""
    import torch
    c = torch.remainder(torch.floor(pos * (K / L)).to(torch.int64), K)
    cnt = torch.bincount((c[:, 0] * K + c[:, 1]) * K + c[:, 2], minlength=K ** 3).reshape(K, K, K)
    del c
    s = cnt.clone()
    for ax in range(3):
        acc = torch.zeros_like(s)
        for d in range(-2, 3):
            acc += torch.roll(s, d, dims=ax)
        s = acc
    nz = cnt[cnt > 0].to(torch.float64)
    I = int((cnt * s).sum())
    return {
        "n": int(pos.shape[0]),
        "cells": int(K ** 3),
        "max_cell": int(cnt.max()),
        "empty_frac": float((cnt == 0).to(torch.float64).mean()),
        "std_ln_count": float(torch.log(nz).std()) if nz.numel() else 0.0,
        "interactions": I,
        "interactions_per_particle": I / max(1, int(pos.shape[0])),
    }


def occupancy_stats(pos: np.ndarray, K: int, L: float) -> dict:
    """Cell-occupancy diagnostics: max count, log-count spread and the
    interaction count I = sum_c n_c S_c (S_c = particles in the 5^3 block
    around c, self-pairs included).  Uses the plain floor-based cell of each
    particle; it is a diagnostic of the input, not part of the method."""
    c = np.floor(pos * (K / L)).astype(np.int64) % K
    lin = (c[:, 0] * K + c[:, 1]) * K + c[:, 2]
    cnt = np.bincount(lin, minlength=K ** 3).reshape(K, K, K)
    s = cnt.astype(np.int64)
    for ax in range(3):
        acc = np.zeros_like(s)
        for d in range(-2, 3):
            acc += np.roll(s, d, axis=ax)
        s = acc
    I = int((cnt.astype(np.int64) * s).sum())
    nz = cnt[cnt > 0]
    return {
        "n": int(pos.shape[0]),
        "cells": int(K ** 3),
        "max_cell": int(cnt.max()),
        "empty_frac": float((cnt == 0).mean()),
        "std_ln_count": float(np.log(nz).std()) if nz.size else 0.0,
        "interactions": I,
        "interactions_per_particle": I / max(1, pos.shape[0]),
    }
