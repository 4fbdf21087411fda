"""Python binding of the near-field library: argument marshalling only.

Every step runs in libnf.so's HIP kernels; torch supplies device memory and
the current stream.

    b = bin_particles(pos, K, L, eps_s)        # Sec. 2.1 binning
    a = accel(b, gm)                            # Sec. 2.1 + Eq. 2 sum
    a = accel(b, gm, plummer=True)              # Plummer law (eps read as eps_p)
    g = accel_vjp(b, cot, gm)                   # VJP w.r.t. positions
    a = nearfield_accel(pos, K, L, eps_s, gm)   # autograd-enabled
"""
from __future__ import annotations

import ctypes
import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import torch

from . import _lib
from ._lib import (NF_COMPENSATED, NF_PAIR_SYMMETRIC, NF_PLUMMER, NF_SERIAL, NF_SIMPLE,
                   NF_SPLINE_EVERYWHERE, NfBox)

__all__ = [
    "SPLINE_PER_PLUMMER",
    "Tiles",
    "eps_spline_from_plummer",
    "Binned",
    "bin_particles",
    "bin_particles_batched",
    "rebin",
    "accel",
    "accel_noalloc",
    "accel_vjp",
    "multipole_terms",
    "step_stats",
    "kick_drift",
    "step_bounds",
    "choose_step",
    "multipoles",
    "NearFieldAccel",
    "nearfield_accel",
    "CapturedForce",
]

# Sec. 4.3: spline radius with the same minimum pairwise dynamical time as a
# Plummer softening eps_p.
SPLINE_PER_PLUMMER = 2.16


def eps_spline_from_plummer(eps_p: float) -> float:
    return SPLINE_PER_PLUMMER * float(eps_p)


@dataclass(frozen=True)
class Tiles:
    """Tile choices of the force kernels (nf_box's tile fields; 0 picks the
    library default).  A cell's sinks are cut into chunks of 64: a chunk of at
    least ``dense_min`` sinks is dense, a smaller last chunk light, or narrow
    below ``narrow_max`` sinks; ``light_window`` / ``narrow_window`` are the
    sources staged per round (512/1024/2048 and 128/256/512); ``flush`` is
    the length of the plain partial sums of the compensated mode.  They change
    speed and FP32 summation order only."""
    dense_min: int = 0
    narrow_max: int = 0
    light_window: int = 0
    narrow_window: int = 0
    flush: int = 0

    def as_dict(self) -> dict:
        return {"dense_min": self.dense_min, "narrow_max": self.narrow_max,
                "light_window": self.light_window, "narrow_window": self.narrow_window,
                "flush": self.flush}


DEFAULT_TILES = Tiles()


def _stream_handle(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


@dataclass
class _BoxBuffers:
    pos: torch.Tensor          # [n,3] float64 (kept alive)
    K: int
    L: float
    eps_s: float
    off: torch.Tensor          # [n,4] float32, sorted
    cell_start: torch.Tensor   # [K^3+1] int32
    order: torch.Tensor        # [n] int32
    nbad: torch.Tensor         # [1] int32
    tiles: Tiles = DEFAULT_TILES

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])

    def cstruct(self) -> NfBox:
        t = self.tiles
        return NfBox(self.n, self.K, t.dense_min, self.L, self.eps_s, self.pos.data_ptr(),
                     self.off.data_ptr(), self.cell_start.data_ptr(), self.order.data_ptr(),
                     self.nbad.data_ptr(), t.narrow_max, t.light_window, t.narrow_window,
                     t.flush)


@dataclass
class Binned:
    """Binned boxes (one or many) plus a workspace sized for all calls."""
    boxes: List[_BoxBuffers]
    workspace: torch.Tensor
    device: torch.device
    _arr: object = field(default=None, repr=False)

    def carray(self):
        if self._arr is None:
            arr = (NfBox * len(self.boxes))()
            for i, b in enumerate(self.boxes):
                arr[i] = b.cstruct()
            self._arr = arr
        return self._arr

    @property
    def nbox(self) -> int:
        return len(self.boxes)

    def nbad(self) -> List[int]:
        return [int(b.nbad.item()) for b in self.boxes]

    @property
    def tiles(self) -> Tiles:
        return self.boxes[0].tiles

    def set_tiles(self, tiles) -> None:
        """Change the force kernels' tile choices: one ``Tiles`` for all
        boxes, or a sequence of one per box (the windows must agree); the
        workspace grows if the new choices need more."""
        per_box = [tiles] * self.nbox if isinstance(tiles, Tiles) else list(tiles)
        if len(per_box) != self.nbox:
            raise ValueError("one Tiles per box is required")
        for bx, t in zip(self.boxes, per_box):
            bx.tiles = t
        self._arr = None
        need = _lib.load().nf_workspace_bytes(self.nbox, self.carray(), 0)
        if need == 0:
            _lib.check(_lib.NF_EINVAL)
        if need > self.workspace.numel():
            self.workspace = torch.empty(int(need), dtype=torch.uint8, device=self.device)

    def ensure_workspace(self, flags: int) -> None:
        """Grow the workspace to what a call with ``flags`` needs (the pair
        symmetry flag needs more than binning and the gather form)."""
        need = _lib.load().nf_workspace_bytes(self.nbox, self.carray(), int(flags))
        if need == 0:
            _lib.check(_lib.NF_EINVAL)
        if need > self.workspace.numel():
            self.workspace = torch.empty(int(need), dtype=torch.uint8, device=self.device)

    def set_dense_min(self, v: int) -> None:
        """Change only the dense / light boundary (0: library default)."""
        self.set_tiles(dataclasses.replace(self.tiles, dense_min=int(v)))


def _prep_pos(pos: torch.Tensor) -> torch.Tensor:
    if not isinstance(pos, torch.Tensor) or not pos.is_cuda:
        raise ValueError("positions must be a CUDA (HIP) tensor")
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("positions must have shape (n, 3)")
    return pos.detach().to(torch.float64).contiguous()


def _alloc_box(pos: torch.Tensor, K: int, L: float, eps_s: float) -> _BoxBuffers:
    dev = pos.device
    n = pos.shape[0]
    K = int(K)
    if K < 5:
        raise ValueError("K must be >= 5")
    return _BoxBuffers(
        pos=pos, K=K, L=float(L), eps_s=float(eps_s),
        off=torch.empty((n, 4), dtype=torch.float32, device=dev),
        cell_start=torch.empty(K ** 3 + 1, dtype=torch.int32, device=dev),
        order=torch.empty(n, dtype=torch.int32, device=dev),
        nbad=torch.zeros(1, dtype=torch.int32, device=dev),
    )


def _check_nbad(b: Binned) -> None:
    bad = b.nbad()
    if any(bad):
        raise ValueError(f"non-finite or out-of-range positions: {bad} per box (such particles "
                         "are binned into cell 0 and every force of their box is meaningless)")


def bin_particles_batched(positions: Sequence[torch.Tensor], Ks: Sequence[int],
                          Ls: Sequence[float], eps: Sequence[float],
                          dense_min: int = 0, check: bool = True,
                          tiles: Optional[Tiles] = None) -> Binned:
    """Bin several boxes in one call (one radix sort over all of them).
    ``tiles`` are the force kernels' tile choices (default: the library's);
    ``dense_min``, if given, overrides theirs.
    ``check``: read back the library's count of non-finite positions and raise
    ValueError if any box has one (one device synchronisation; pass False to
    skip it and inspect ``Binned.nbad()`` yourself)."""
    lib = _lib.load()
    if not (len(positions) == len(Ks) == len(Ls) == len(eps)) or len(positions) == 0:
        raise ValueError("positions, Ks, Ls and eps must be non-empty and of equal length")
    ps = [_prep_pos(p) for p in positions]
    dev = ps[0].device
    if any(p.device != dev for p in ps):
        raise ValueError("all boxes must live on one device")
    boxes = [_alloc_box(p, K, L, e) for p, K, L, e in zip(ps, Ks, Ls, eps)]
    t = tiles if tiles is not None else DEFAULT_TILES
    if dense_min:
        t = dataclasses.replace(t, dense_min=int(dense_min))
    for bx in boxes:
        bx.tiles = t
    arr = (NfBox * len(boxes))()
    for i, b in enumerate(boxes):
        arr[i] = b.cstruct()
    nbytes = lib.nf_workspace_bytes(len(boxes), arr, 0)
    if nbytes == 0:
        _lib.check(_lib.NF_EINVAL)
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=dev)
    with torch.cuda.device(dev):
        rc = lib.nf_bin_particles(len(boxes), arr, ctypes.c_void_p(ws.data_ptr()), int(nbytes),
                                  _stream_handle(dev))
    _lib.check(rc)
    out = Binned(boxes=boxes, workspace=ws, device=dev)
    out._arr = arr
    if check:
        _check_nbad(out)
    return out


def rebin(b: Binned, check: bool = True) -> Binned:
    """Bin again into the same buffers (positions updated in place);
    ``check`` as in ``bin_particles_batched``."""
    lib = _lib.load()
    with torch.cuda.device(b.device):
        rc = lib.nf_bin_particles(b.nbox, b.carray(), ctypes.c_void_p(b.workspace.data_ptr()),
                                  b.workspace.numel(), _stream_handle(b.device))
    _lib.check(rc)
    if check:
        _check_nbad(b)
    return b


def bin_particles(pos: torch.Tensor, K: int, L: float, eps_s: float,
                  dense_min: int = 0, check: bool = True,
                  tiles: Optional[Tiles] = None) -> Binned:
    """Bin one box: cell offsets (FP64 -> FP32) and a stable sort by cell."""
    return bin_particles_batched([pos], [K], [L], [eps_s], dense_min, check, tiles)


def _flags(compensated: bool, simple: bool, plummer: bool = False,
           spline_everywhere: bool = False, serial: bool = False,
           symmetric: bool = False) -> int:
    return ((NF_COMPENSATED if compensated else 0) | (NF_SIMPLE if simple else 0)
            | (NF_PLUMMER if plummer else 0)
            | (NF_SPLINE_EVERYWHERE if spline_everywhere else 0)
            | (NF_SERIAL if serial else 0)
            | (NF_PAIR_SYMMETRIC if symmetric else 0))


def _ptr_array(tensors: Sequence[torch.Tensor]):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = t.data_ptr()
    return arr


def accel(b: Binned, gm: float = 1.0, *, compensated: bool = False, simple: bool = False,
          plummer: bool = False, spline_everywhere: bool = False, serial: bool = False,
          symmetric: bool = False, out: Optional[List[torch.Tensor]] = None):
    """Near-field accelerations, float32 [n,3] in input order (a list for
    several boxes).  ``plummer``: the Plummer law of Sec. 4.3 with each box's
    softening length read as eps_p, instead of Eq. 2.  ``spline_everywhere``:
    the outer-shell shortcut off (same results, for measurement).
    ``serial``: the three force kernels one after another (same results, for
    measuring each kernel alone).  ``symmetric``: Newton's third law between
    dense cells (each pair of two such cells evaluated once; the workspace
    grows on the first such call)."""
    lib = _lib.load()
    flags = _flags(compensated, simple, plummer, spline_everywhere, serial, symmetric)
    if symmetric:
        b.ensure_workspace(flags)
    if out is None:
        out = [torch.empty((bx.n, 3), dtype=torch.float32, device=b.device) for bx in b.boxes]
    ptrs = _ptr_array(out)
    with torch.cuda.device(b.device):
        rc = lib.nf_accel(b.nbox, b.carray(), float(gm), flags, ptrs,
                          ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel(),
                          _stream_handle(b.device))
    _lib.check(rc)
    return out[0] if b.nbox == 1 else out


def accel_noalloc(b: Binned, gm: float = 1.0, *, compensated: bool = False,
                  simple: bool = False, plummer: bool = False,
                  spline_everywhere: bool = False, out: Optional[List[torch.Tensor]] = None):
    """``accel`` through the allocation-free entry point (nf_accel_noalloc):
    the library's static per-GPU scratch instead of the boxes' workspace.
    With ``out`` given, the call itself allocates nothing."""
    lib = _lib.load()
    if out is None:
        out = [torch.empty((bx.n, 3), dtype=torch.float32, device=b.device) for bx in b.boxes]
    with torch.cuda.device(b.device):
        rc = lib.nf_accel_noalloc(b.nbox, b.carray(), float(gm),
                                  _flags(compensated, simple, plummer, spline_everywhere),
                                  _ptr_array(out), _stream_handle(b.device))
    _lib.check(rc)
    return out[0] if b.nbox == 1 else out


def plan_items(b: Binned):
    """The work list of the force calls (nf_plan_items): an int32 tensor
    [m, 4] of (box, cell, chunk, class) on the device, dense items (class 0)
    first, then light (1), then narrow (2), and the three class counts."""
    lib = _lib.load()
    # a cell of n sinks gives at most n / 64 + 1 items
    cap = sum(bx.n // 64 + bx.K ** 3 for bx in b.boxes)
    items = torch.empty((max(cap, 1), 4), dtype=torch.int32, device=b.device)
    counts = torch.zeros(3, dtype=torch.int64, device=b.device)
    with torch.cuda.device(b.device):
        rc = lib.nf_plan_items(b.nbox, b.carray(), ctypes.c_void_p(items.data_ptr()), cap,
                               ctypes.c_void_p(counts.data_ptr()),
                               ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel(),
                               _stream_handle(b.device))
    _lib.check(rc)
    c = [int(x) for x in counts.cpu()]
    return items[:sum(c)], tuple(c)


def accel_vjp(b: Binned, cot, gm: float = 1.0, *, compensated: bool = False,
              simple: bool = False, plummer: bool = False, serial: bool = False):
    """Vector-Jacobian product of the accelerations w.r.t. positions
    (cell assignment held fixed); float32 [n,3] per box."""
    lib = _lib.load()
    cots = [cot] if isinstance(cot, torch.Tensor) else list(cot)
    if len(cots) != b.nbox:
        raise ValueError("one cotangent per box is required")
    cots = [c.detach().to(device=b.device, dtype=torch.float32).contiguous() for c in cots]
    for c, bx in zip(cots, b.boxes):
        if tuple(c.shape) != (bx.n, 3):
            raise ValueError("cotangent must have shape (n, 3)")
    grads = [torch.empty((bx.n, 3), dtype=torch.float32, device=b.device) for bx in b.boxes]
    with torch.cuda.device(b.device):
        rc = lib.nf_accel_vjp(b.nbox, b.carray(), float(gm),
                              _flags(compensated, simple, plummer, serial=serial),
                              _ptr_array(cots), _ptr_array(grads),
                              ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel(),
                              _stream_handle(b.device))
    _lib.check(rc)
    return grads[0] if b.nbox == 1 else grads


def multipole_terms(order: int) -> int:
    """Moments per cell at this order: (p+1)(p+2)(p+3)/6."""
    p = int(order)
    return (p + 1) * (p + 2) * (p + 3) // 6


def multipoles(b: Binned, order: int = 8):
    """Per-cell Cartesian multipole moments about the cell centres (cell
    widths), float32 [K^3, T] per box (a list for several boxes); terms by
    degree, then a descending, then b descending."""
    lib = _lib.load()
    T = multipole_terms(order)
    out = [torch.empty((bx.K ** 3, T), dtype=torch.float32, device=b.device) for bx in b.boxes]
    with torch.cuda.device(b.device):
        rc = lib.nf_multipoles(b.nbox, b.carray(), int(order), _ptr_array(out),
                               ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel(),
                               _stream_handle(b.device))
    _lib.check(rc)
    return out[0] if b.nbox == 1 else out


def _f32_list(xs, b: Binned, what: str):
    xs = [xs] if isinstance(xs, torch.Tensor) else list(xs)
    if len(xs) != b.nbox:
        raise ValueError(f"one {what} tensor per box is required")
    for x, bx in zip(xs, b.boxes):
        if x.dtype != torch.float32 or not x.is_contiguous() or tuple(x.shape) != (bx.n, 3) \
                or x.device != b.device:
            raise ValueError(f"{what} must be contiguous float32 (n, 3) tensors on the boxes' device")
    return xs


def step_stats(b: Binned, acc, vel):
    """Per-cell a_max and v_rms (float32 [K^3] per box) and the global
    (a_max, v_rms, v_max) per box (float64 [nbox, 3]), the inputs of the
    step choice of Sec. 4.2."""
    lib = _lib.load()
    accs, vels = _f32_list(acc, b, "acc"), _f32_list(vel, b, "vel")
    amax = [torch.empty(bx.K ** 3, dtype=torch.float32, device=b.device) for bx in b.boxes]
    vrms = [torch.empty(bx.K ** 3, dtype=torch.float32, device=b.device) for bx in b.boxes]
    glob = torch.empty((b.nbox, 3), dtype=torch.float64, device=b.device)
    with torch.cuda.device(b.device):
        rc = lib.nf_step_stats(b.nbox, b.carray(), _ptr_array(accs), _ptr_array(vels),
                               _ptr_array(amax), _ptr_array(vrms), ctypes.c_void_p(glob.data_ptr()),
                               ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel(),
                               _stream_handle(b.device))
    _lib.check(rc)
    if b.nbox == 1:
        return amax[0], vrms[0], glob[0]
    return amax, vrms, glob


def kick_drift(b: Binned, acc, vel, pos, kick: float, drift: float) -> None:
    """In place: vel <- vel + kick * acc (float), pos <- pos + drift * vel
    (float64, kicked vel).  ``pos`` may be the tensor the boxes were binned
    from; bin again (rebin) before the next force call."""
    lib = _lib.load()
    accs, vels = _f32_list(acc, b, "acc"), _f32_list(vel, b, "vel")
    poss = [pos] if isinstance(pos, torch.Tensor) else list(pos)
    if len(poss) != b.nbox:
        raise ValueError("one position tensor per box is required")
    for p, bx in zip(poss, b.boxes):
        if p.dtype != torch.float64 or not p.is_contiguous() or tuple(p.shape) != (bx.n, 3) \
                or p.device != b.device:
            raise ValueError("pos must be contiguous float64 (n, 3) tensors on the boxes' device")
    with torch.cuda.device(b.device):
        rc = lib.nf_kick_drift(b.nbox, b.carray(), _ptr_array(accs), _ptr_array(vels),
                               _ptr_array(poss), float(kick), float(drift),
                               ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel(),
                               _stream_handle(b.device))
    _lib.check(rc)


def step_bounds(b: Binned, amax, vrms, glob, *, dlna_max: float, hubble: float,
                eta: float) -> torch.Tensor:
    """The three step bounds of Sec. 4.2 and the step, per box, from
    ``step_stats`` output, computed by the library (nf_step_choose): float64
    [nbox, 4] on the device = (dlna_max / hubble, eta * max(smallest per-cell
    v_rms / a_max, global v_rms / a_max), 0.8 cell width / v_max, step)."""
    lib = _lib.load()
    am = [amax] if isinstance(amax, torch.Tensor) else list(amax)
    vr = [vrms] if isinstance(vrms, torch.Tensor) else list(vrms)
    if len(am) != b.nbox or len(vr) != b.nbox:
        raise ValueError("one amax and one vrms tensor per box is required")
    for x, bx in zip(am + vr, b.boxes + b.boxes):
        if x.dtype != torch.float32 or not x.is_contiguous() or x.numel() != bx.K ** 3 \
                or x.device != b.device:
            raise ValueError("amax and vrms must be contiguous float32 [K^3] tensors on the "
                             "boxes' device")
    g = glob.reshape(-1, 3)
    if g.dtype != torch.float64 or not g.is_contiguous() or g.shape[0] != b.nbox \
            or g.device != b.device:
        raise ValueError("glob must be a contiguous float64 [nbox, 3] tensor on the boxes' device")
    out = torch.empty((b.nbox, 4), dtype=torch.float64, device=b.device)
    with torch.cuda.device(b.device):
        rc = lib.nf_step_choose(b.nbox, b.carray(), _ptr_array(am), _ptr_array(vr),
                                ctypes.c_void_p(g.data_ptr()), float(dlna_max), float(hubble),
                                float(eta), ctypes.c_void_p(out.data_ptr()),
                                ctypes.c_void_p(b.workspace.data_ptr()), b.workspace.numel(),
                                _stream_handle(b.device))
    _lib.check(rc)
    return out


def choose_step(b: Binned, amax, vrms, glob, *, dlna_max: float, hubble: float,
                eta: float) -> float:
    """The step of Sec. 4.2 for one box (``step_bounds``' last column)."""
    return float(step_bounds(b, amax, vrms, glob, dlna_max=dlna_max, hubble=hubble,
                             eta=eta)[0, 3])


class NearFieldAccel(torch.autograd.Function):
    """acc = near-field acceleration of positions ``pos`` (float64 [n,3]).

    The backward pass is the hand-written VJP kernel with the binning of the
    forward pass held fixed."""

    @staticmethod
    def forward(ctx, pos, K, L, eps_s, gm, compensated, plummer=False):
        b = bin_particles(pos, K, L, eps_s)
        a = accel(b, gm, compensated=compensated, plummer=plummer)
        ctx.binned = b
        ctx.gm = gm
        ctx.compensated = compensated
        ctx.plummer = plummer
        ctx.pos_dtype = pos.dtype
        return a

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_acc):
        g = accel_vjp(ctx.binned, grad_acc, ctx.gm, compensated=ctx.compensated,
                      plummer=ctx.plummer)
        return g.to(ctx.pos_dtype), None, None, None, None, None, None


def nearfield_accel(pos: torch.Tensor, K: int, L: float, eps_s: float, gm: float = 1.0,
                    compensated: bool = False, plummer: bool = False) -> torch.Tensor:
    return NearFieldAccel.apply(pos, K, L, eps_s, gm, compensated, plummer)


class CapturedForce:
    """Binning + accelerations of a fixed set of boxes captured once into a
    HIP graph; ``replay()`` recomputes both from the current contents of the
    position buffers ``self.positions`` (update them in place).

    Every library call is a pure sequence of kernel launches (descriptors go
    through kernel arguments, buffers are filled by kernels), so the whole
    step is one graph launch.  A replay cannot stop on bad input: check
    ``nbad()`` (the binning's count of non-finite positions per box, as of
    the last replay) before trusting its forces."""

    def __init__(self, positions: Sequence[torch.Tensor], Ks, Ls, eps, gm: float = 1.0,
                 compensated: bool = False, plummer: bool = False,
                 tiles: Optional[Tiles] = None):
        """``tiles``: the force kernels' tile choices, e.g. the autotuner's
        (``tune.tune(...).tiles``); default: the library's."""
        self.positions = [_prep_pos(p) for p in positions]
        self.gm = float(gm)
        self.compensated = bool(compensated)
        self.plummer = bool(plummer)
        self.binned = bin_particles_batched(self.positions, Ks, Ls, eps, tiles=tiles)
        self.out = [torch.empty((bx.n, 3), dtype=torch.float32, device=self.binned.device)
                    for bx in self.binned.boxes]
        accel(self.binned, self.gm, compensated=self.compensated, plummer=self.plummer,
                  out=self.out)   # warm up
        torch.cuda.synchronize(self.binned.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            rebin(self.binned, check=False)
            accel(self.binned, self.gm, compensated=self.compensated, plummer=self.plummer,
                  out=self.out)

    def replay(self) -> List[torch.Tensor]:
        self.graph.replay()
        return self.out

    def nbad(self) -> List[int]:
        """Per box, the positions of the last replay that were not finite
        (their box's forces are then meaningless)."""
        return self.binned.nbad()
