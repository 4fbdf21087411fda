"""Autotuner of the force kernels' tile choices.

The force kernels cut the sinks of every cell into chunks of 64 and sort the
chunks into three occupancy classes (dense, light, narrow), each summed by its
own kernel; five tile choices set the class boundaries and the kernels'
shapes (``nearfield.Tiles``):

  dense_min      the dense / light boundary (sinks in a cell's last chunk)
  narrow_max     the light / narrow boundary
  light_window   sources a light item stages in LDS per round
  narrow_window  the same for narrow items
  flush          compensated mode: terms per plain FP32 partial sum

None of them changes which pairs are summed; they change speed and the FP32
summation order.  The best choice depends on the workload's occupancy
distribution, so ``tune`` times candidates on the caller's own binned boxes
by coordinate descent (each choice in turn, the others held at their current
best, repeated until a pass changes nothing) and keeps the winner in a JSON
table keyed by the device architecture, the HIP version, a hash of the kernel
sources, a coarse signature of the occupancy classes, the call (accelerations
or VJP) and the compensation flag.  ``NF_TUNE_TABLE`` names the table
(default ``~/.cache/nearfield_tune.json``).
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Callable, Dict, Iterable, Optional, Sequence, Tuple

import numpy as np

from .nearfield import Tiles

CANDIDATES: Dict[str, Tuple[int, ...]] = {
    "dense_min": (17, 25, 33, 41, 49, 57, 65),
    "narrow_max": (1, 8, 12, 16, 24),
    "light_window": (512, 1024, 2048),
    "narrow_window": (128, 256, 512),
    "flush": (16, 32, 64),
}
ORDER = ("dense_min", "narrow_max", "light_window", "narrow_window", "flush")
# the library's defaults, written out (a 0 field means the same choice)
DEFAULTS = Tiles(dense_min=41, narrow_max=12, light_window=1024, narrow_window=256, flush=32)
# cell-count bins of the occupancy signature: [lo, hi) sinks per cell
COUNT_BINS = (1, 4, 8, 16, 32, 64, 128, 256, 1024, 1 << 62)


def table_path() -> str:
    return os.environ.get("NF_TUNE_TABLE",
                          os.path.join(os.path.expanduser("~"), ".cache", "nearfield_tune.json"))


# ------------------------------------------------------------------ search

def search(timer: Callable[[Tiles], float], candidates: Dict[str, Sequence[int]] = CANDIDATES,
           start: Tiles = DEFAULTS, order: Iterable[str] = ORDER,
           max_passes: int = 3) -> Tuple[Tiles, Dict[Tiles, float]]:
    """Coordinate descent over the tile choices.  ``timer(tiles)`` returns
    the cost (ms) of one call with those choices; each distinct choice is
    timed once.  Returns (best, {tiles: ms})."""
    order = [k for k in order if k in candidates]
    times: Dict[Tiles, float] = {}

    def cost(t: Tiles) -> float:
        if t not in times:
            times[t] = float(timer(t))
        return times[t]

    best = start
    cost(best)
    for _ in range(max_passes):
        changed = False
        for name in order:
            for v in candidates[name]:
                t = dataclasses.replace(best, **{name: int(v)})
                if cost(t) < cost(best):
                    best, changed = t, True
        if not changed:
            break
    return best, times


# ------------------------------------------------------------------ table

def occupancy_signature(counts: Sequence[np.ndarray]) -> str:
    """Coarse signature of a workload's occupancy classes: the number of
    boxes (1, up to 8, up to 64, more) and, over the cells of all boxes, the
    share of sinks in cells of 1-3, 4-7, 8-15, ..., 256-1023 and 1024 or more
    particles, each rounded to eighths."""
    allc = np.concatenate([np.asarray(c, dtype=np.int64).ravel() for c in counts])
    total = max(1, int(allc.sum()))
    shares = []
    for lo, hi in zip(COUNT_BINS[:-1], COUNT_BINS[1:]):
        m = (allc >= lo) & (allc < hi)
        shares.append(int(round(8.0 * float(allc[m].sum()) / total)))
    nb = len(counts)
    nbox = "1" if nb == 1 else ("8" if nb <= 8 else ("64" if nb <= 64 else "many"))
    return f"boxes{nbox}:" + "-".join(str(s) for s in shares)


def table_key(arch: str, hip: str, source_hash: str, occupancy: str, mode: str,
              compensated: bool) -> str:
    return "|".join([arch, f"hip{hip}", f"src{source_hash}", occupancy, mode,
                     "comp" if compensated else "plain"])


def load_table(path: Optional[str] = None) -> dict:
    path = path or table_path()
    try:
        with open(path) as f:
            t = json.load(f)
        return t if isinstance(t, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: Optional[str] = None) -> None:
    path = path or table_path()
    table = load_table(path)
    table[key] = entry
    try:
        os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def tiles_from(d: dict) -> Tiles:
    return Tiles(**{k: int(d[k]) for k in Tiles().as_dict()})


# ------------------------------------------------------------------ tune

@dataclasses.dataclass
class TuneResult:
    tiles: Tiles
    times_ms: Dict[str, float]      # tried choices ("dense_min=41,...") -> ms
    key: str
    cached: bool


def _label(t: Tiles) -> str:
    return ",".join(f"{k}={v}" for k, v in t.as_dict().items())


def workload_key(b, mode: str, compensated: bool) -> str:
    import torch

    from .srchash import kernel_source_hash
    props = torch.cuda.get_device_properties(b.device)
    arch = getattr(props, "gcnArchName", props.name).split(":")[0]
    counts = [(bx.cell_start[1:] - bx.cell_start[:-1]).cpu().numpy() for bx in b.boxes]
    return table_key(arch, str(torch.version.hip), kernel_source_hash(),
                     occupancy_signature(counts), mode, compensated)


def tune(b, mode: str = "accel", compensated: bool = True, reps: int = 3,
         use_cache: bool = True, candidates: Dict[str, Sequence[int]] = CANDIDATES,
         path: Optional[str] = None) -> TuneResult:
    """Pick the tile choices for binned boxes ``b`` (applied to ``b``).
    ``mode``: "accel" or "vjp" (the call being tuned)."""
    import torch

    from . import nearfield as nfp
    if mode not in ("accel", "vjp"):
        raise ValueError("mode must be 'accel' or 'vjp'")
    key = workload_key(b, mode, compensated)
    if use_cache:
        hit = load_table(path).get(key)
        if hit is not None:
            t = tiles_from(hit["tiles"])
            b.set_tiles(t)
            return TuneResult(t, dict(hit.get("ms", {})), key, True)
    if not compensated:
        candidates = {k: v for k, v in candidates.items() if k != "flush"}
    out = [torch.empty((bx.n, 3), dtype=torch.float32, device=b.device) for bx in b.boxes]
    cot = [torch.zeros((bx.n, 3), dtype=torch.float32, device=b.device) for bx in b.boxes]
    stream = torch.cuda.current_stream(b.device)

    def call():
        if mode == "accel":
            nfp.accel(b, 1.0, compensated=compensated, out=out)
        else:
            nfp.accel_vjp(b, cot if b.nbox > 1 else cot[0], 1.0, compensated=compensated)

    def timer(t: Tiles) -> float:
        b.set_tiles(t)
        call()                       # first launch of an instance, untimed
        torch.cuda.synchronize(b.device)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            call()
        e1.record(stream)
        torch.cuda.synchronize(b.device)
        return e0.elapsed_time(e1) / reps

    # a few untimed calls first: the first candidate timed is otherwise
    # measured while the clocks still ramp up, which biases the search
    # against it
    b.set_tiles(DEFAULTS)
    for _ in range(4 * reps):
        call()
    torch.cuda.synchronize(b.device)
    best, times = search(timer, candidates)
    b.set_tiles(best)
    ms = {_label(t): round(v, 5) for t, v in times.items()}
    if use_cache:
        store(key, {"tiles": best.as_dict(), "ms": ms}, path)
    return TuneResult(best, ms, key, False)
