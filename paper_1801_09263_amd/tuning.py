"""Autotuning results cached on disk.

The autotuner itself is ``lace_autotune`` in the library: it times the
pipeline candidates of a cell (pairs per batch; pencil, whole-plane or
half-plane xy schedule; then the z-pass tile width and the radix order of
the transforms) on real orbitals and keeps the fastest.  This module stores the winners in a
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


PRECISION_NAMES = {lace.LACE_FP64: "fp64", lace.LACE_FP32: "fp32",
                   lace.LACE_FP64_GAMMA: "fp64g", lace.LACE_FP32_GAMMA: "fp32g"}


def tune_key(n: int, n_orb: int, precision: int) -> str:
    """Cache key: the exact plan precision (a tuning of one precision, e.g.
    the whole-plane schedule of an FP32 plan, may not exist for another),
    the grid size and the orbital count."""
    if precision not in PRECISION_NAMES:
        raise ValueError(f"unknown precision {precision}")
    return f"{PRECISION_NAMES[precision]}-n{int(n)}-orb{int(n_orb)}"


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
                         ent["use_plane"], ent.get("z_tile", 0),
                         ent.get("radix_order", 0))
    return True


def autotune(plan, cell_index: int, n: int, psi_g, n_orb: int, ws,
             precision: int, path: str | None = None, stream=None,
             s_thr: float = 0.0) -> dict:
    """Run the library autotuner on one cell (the pairs S keeps at s_thr)
    and cache the winner."""
    cands = lace.lace_autotune(plan, cell_index, psi_g, n_orb, ws, stream,
                               s_thr=s_thr)
    ppb, plane, ztile, radix = lace.lace_get_tuning(plan, cell_index)
    ent = dict(pairs_per_batch=ppb, use_plane=plane, z_tile=ztile,
               radix_order=radix,
               candidates=[dict(pairs_per_batch=a, use_plane=b, z_tile=z,
                                radix_order=r, us_per_pair=c)
                           for a, b, z, r, c in cands])
    store({tune_key(n, n_orb, precision): ent}, path)
    return ent
