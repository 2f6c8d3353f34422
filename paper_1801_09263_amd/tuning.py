"""Autotuning results cached on disk.

The autotuner itself is ``lace_autotune`` in the library: it times every
pipeline candidate of a cell (pairs per batch; pencil, whole-plane or
half-plane xy schedule) on real orbitals and keeps the fastest.  This module stores the winners in a
JSON file keyed by precision, grid size and orbital count, and applies them
to new plans, so later runs skip the timing.
"""
from __future__ import annotations

import json
import os

from . import lace


def cache_path(path: str | None = None) -> str:
    if path:
        return path
    env = os.environ.get("LACE_TUNE_FILE")
    if env:
        return env
    return os.path.join(os.path.expanduser("~"), ".cache", "lace",
                        "tuning.json")


def tune_key(n: int, n_orb: int, precision: int) -> str:
    prec = "fp64" if precision == lace.LACE_FP64 else "fp32"
    return f"{prec}-n{int(n)}-orb{int(n_orb)}"


def load(path: str | None = None) -> dict:
    p = cache_path(path)
    if not os.path.exists(p):
        return {}
    with open(p) as fh:
        return json.load(fh)


def store(entries: dict, path: str | None = None) -> None:
    p = cache_path(path)
    os.makedirs(os.path.dirname(p), exist_ok=True)
    data = load(p)
    data.update(entries)
    tmp = p + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def apply_cached(plan, cell_index: int, n: int, n_orb: int, precision: int,
                 path: str | None = None) -> bool:
    """Set the cached tuning on a plan cell; False if there is none."""
    ent = load(path).get(tune_key(n, n_orb, precision))
    if not ent:
        return False
    lace.lace_set_tuning(plan, cell_index, ent["pairs_per_batch"],
                         ent["use_plane"])
    return True


def autotune(plan, cell_index: int, n: int, psi_g, n_orb: int, ws,
             precision: int, path: str | None = None, stream=None) -> dict:
    """Run the library autotuner on one cell and cache the winner."""
    cands = lace.lace_autotune(plan, cell_index, psi_g, n_orb, ws, stream)
    ppb, plane = lace.lace_get_tuning(plan, cell_index)
    ent = dict(pairs_per_batch=ppb, use_plane=plane,
               candidates=[dict(pairs_per_batch=a, use_plane=b, us_per_pair=c)
                           for a, b, c in cands])
    store({tune_key(n, n_orb, precision): ent}, path)
    return ent
