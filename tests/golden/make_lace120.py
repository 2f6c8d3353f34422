"""Write lace120_screening.txt: the oracle's screening of the lace-120
workload and its screened exchange energy.

Calls only ``oracle`` (the CPU FP64 oracle) and ``synth`` (the seeded input
generator).  The stored values are the oracle's:

* the kept set of Eq. (6) (a pair (i, j), i <= j, is kept when
  S_ij >= S_thr) as one 256-bit mask per column j,
* the pairs whose S_ij lies within an absolute band of S_thr (S is
  dimensionless with S_ii = 1; a path that screens from single-precision
  grids carries errors of that order and may decide those either way),
* E_x = -(1/2) sum over the kept ordered pairs of (ij|ji) (Eq. (2) truncated
  as in Eqs. (7)-(8)).

Run from the repository root: ``python tests/golden/make_lace120.py``
(about 6,000 core-seconds of FFTs, spread over the host's cores; 12 GB of
memory).
"""
from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                   "lace120_screening.txt")
BAND = 1e-6   # absolute half-width of the borderline band around S_thr

_STATE = {}


def _columns(cols):
    st = _STATE
    return cols, O.exchange_integrals_columns(st["psi"], st["v"], st["L"],
                                              st["pairs"], cols)


def main():
    t0 = time.time()
    inp = synth.make_inputs("lace-120")
    L, n, s_thr = inp["L"], inp["n"], inp["s_thr"]
    coeffs, miller = inp["coeffs"], inp["miller"]
    n_orb = coeffs.shape[0]
    psi = O.orbitals_on_grid(coeffs, miller, L, n)
    print(f"grid orbitals {time.time() - t0:.0f} s", flush=True)
    s = O.overlap_of_moduli(psi, L)
    print(f"overlap of moduli {time.time() - t0:.0f} s", flush=True)
    pairs = O.kept_pairs(s, s_thr)
    v = O.coulomb_kernel(L, n)
    _STATE.update(psi=psi, v=v, L=L, pairs=pairs)
    chunks = [list(range(c, n_orb, 64)) for c in range(64)]
    total = np.zeros(n_orb)
    workers = int(os.environ.get("GOLDEN_WORKERS", os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        done = 0
        for cols, vals in pool.imap_unordered(_columns, chunks):
            total[cols] = vals
            done += 1
            print(f"columns: {done}/{len(chunks)} chunks, "
                  f"{time.time() - t0:.0f} s", flush=True)
    ex = -0.5 * float(np.sum(total))
    band = [(i, j, s[i, j]) for j in range(n_orb) for i in range(j + 1)
            if abs(s[i, j] - s_thr) <= BAND]
    with open(OUT, "w") as f:
        f.write("# Screening of the lace-120 workload (synth.make_inputs('lace-120'),\n"
                "# seed 0) by the CPU FP64 oracle, written by make_lace120.py.\n"
                "# Eq. (6): pair (i, j), i <= j, kept when S_ij >= S_thr.\n"
                "# ex_pairs: -(1/2) sum over kept ordered pairs of (ij|ji) (Eq. (2)\n"
                "# truncated as in Eqs. (7)-(8)), Hartree.\n"
                "# borderline: pairs with |S_ij - S_thr| <= band, as i j S_ij.\n"
                "# mask: line j holds the kept i <= j as a 256-bit number (bit i),\n"
                "# 64 hex digits, most significant first.\n")
        f.write(f"n_orb {n_orb}\n")
        f.write(f"s_thr {s_thr!r}\n")
        f.write(f"n_kept {len(pairs)}\n")
        f.write(f"ex_pairs {ex!r}\n")
        f.write(f"band {BAND!r}\n")
        f.write(f"borderline {len(band)}\n")
        for i, j, sv in band:
            f.write(f"{i} {j} {float(sv)!r}\n")
        f.write("mask\n")
        kept = np.zeros((n_orb, n_orb), dtype=bool)
        for i, j in pairs:
            kept[i, j] = True
        for j in range(n_orb):
            word = 0
            for i in range(j + 1):
                if kept[i, j]:
                    word |= 1 << i
            f.write(f"{word:064x}\n")
    print(f"wrote {OUT}: {len(pairs)} kept, E_x {ex!r}, "
          f"{len(band)} borderline, {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
