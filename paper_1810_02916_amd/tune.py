"""Autotuner for the force kernels' tile choice.

The one tunable is ``dense_min``: the sinks of a cell are cut into chunks of
64, and a chunk of at least ``dense_min`` sinks is summed one sink per lane
with broadcast sources, a smaller one is spread over (sink, source-slice)
lanes with LDS-staged sources.  The best split
depends on the occupancy distribution of the workload, so the tuner times
the compensated acceleration pass for a few candidates on the caller's own
binned boxes and keeps the fastest.  Results are cached per workload
signature in a JSON table (``NF_TUNE_TABLE``, default
``~/.cache/nearfield_tune.json``).
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Tuple

import torch

from . import nearfield as nfp

CANDIDATES = (9, 17, 25, 33, 41, 49, 57, 65)


def _table_path() -> str:
    return os.environ.get("NF_TUNE_TABLE",
                          os.path.join(os.path.expanduser("~"), ".cache", "nearfield_tune.json"))


def signature(b: nfp.Binned) -> str:
    """Workload signature: device arch, box count, sizes and coarse occupancy."""
    props = torch.cuda.get_device_properties(b.device)
    arch = getattr(props, "gcnArchName", props.name)
    parts = [arch.split(":")[0], str(b.nbox)]
    for bx in b.boxes:
        n, ncell = bx.n, bx.K ** 3
        parts.append(f"{n}/{ncell}")
    return "|".join(parts)


def _set_dense_min(b: nfp.Binned, v: int) -> None:
    b.set_dense_min(v)


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_dense_min(b: nfp.Binned, candidates: Iterable[int] = CANDIDATES, reps: int = 3,
                   use_cache: bool = True) -> Tuple[int, Dict[int, float]]:
    """Pick ``dense_min`` for binned boxes ``b`` (applied to ``b``); returns
    (best, {candidate: ms})."""
    key = signature(b)
    path = _table_path()
    table = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                table = json.load(f)
        except (OSError, ValueError):
            table = {}
    if use_cache and key in table:
        best = int(table[key]["dense_min"])
        _set_dense_min(b, best)
        return best, {int(k): v for k, v in table[key]["ms"].items()}
    out = [torch.empty((bx.n, 3), dtype=torch.float32, device=b.device) for bx in b.boxes]
    times: Dict[int, float] = {}
    for v in candidates:
        _set_dense_min(b, v)
        times[int(v)] = _time(lambda: nfp.accel(b, 1.0, compensated=True, out=out), reps)
    best = min(times, key=times.get)
    _set_dense_min(b, best)
    if use_cache:
        table[key] = {"dense_min": best, "ms": times}
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            with open(path, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        except OSError:
            pass
    return best, times
