#!/usr/bin/env python3
"""Throughput of the L-ACE exchange path on one MI355X.

One step is the whole hot path on the localized 120^3 workload (L = 23.5
bohr, 256 Loewdin-orthonormalized Gaussian orbitals on 128 random centres,
S_thr = 1e-3, FP32 pair densities and FFTs, FP64 screening sums, M,
Cholesky and xi): orbitals to the grid, screening, the kept pair FFTs with
the kernel multiply and accumulation into W, W back to plane waves, M,
symmetrization, Cholesky, xi, E_x, and ACE applied to the 256 orbitals.

Prints one JSON line: value = kept pair-FFTs per second over the whole step,
plus the roofline of the dominant pair-pipeline kernel (HIP-event timing
inside the library, algorithmic bytes), the plain unscreened FP64 path on
the 120^3 random-orbital workload for comparison, and the CPU oracle timed on
a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E peak
FP64_MFMA_PEAK_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_of(text: str) -> str:
    """C++ source without comments, blank lines and trailing blanks."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())


def kernel_source_hash() -> str:
    """Hash of the pass kernels' code (comments left out): the stored HBM
    counter figures hold for exactly this code."""
    h = hashlib.sha256()
    for f in ("fft_core.hpp", "fft_kernels.hip", "internal.hpp"):
        with open(os.path.join(ROOT, "paper_1801_09263_amd", "csrc", f)) as fh:
            h.update(code_of(fh.read()).encode())
    return h.hexdigest()[:16]


# Two byte counts per pass.
# Algorithmic (per pair, the minimal fused three-pass schedule taking each
# pair alone): in units of one orbital grid s N_g (s = 4 B for the real
# grids of real-orbital FP32 plans, 8 B complex FP32, 16 B complex FP64), an
# off-diagonal pair moves 3 in pass A (read psi_i, psi_j, write its pair
# density), 2 in pass B (read and write it), 7 in pass C (read it, re-read
# psi_i and psi_j, read and write W_i and W_j): 12 per pair; a diagonal pair
# 2, 2 and 4.
# Moved (from the library, lace_profile_read): per transform slot with o
# distinct orbitals, pass A moves o G + U (read the orbitals, write the pair
# buffer), pass B 2 U, pass C U + 3 o G (read the buffer and the orbitals,
# read and write their W); U = one complex grid, G = one orbital grid (U, or
# U / 2 for real orbitals).  A star slot's two pairs share an orbital, so the
# kernels move fewer bytes than the per-pair count.
PASS_NAMES = ("pair-product+xy-forward", "z-forward*v*z-backward",
              "xy-backward+accumulate")
PAIR_GRIDS = ((3, 2), (2, 2), (7, 4))   # (off-diagonal, diagonal) per pass


def pass_alg_bytes(k, n_off, n_diag, s, ng):
    off, dia = PAIR_GRIDS[k]
    return (off * n_off + dia * n_diag) * s * ng


def pass_roofline(prof):
    rows = []
    for k in range(3):
        ms = prof["ms"][k]
        nbytes = prof["alg_bytes"][k]
        launches = max(prof["launches"][k], 1)
        gbs = nbytes / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        rows.append(dict(name=PASS_NAMES[k], ms_total=ms,
                         launches=prof["launches"][k],
                         avg_launch_us=1e3 * ms / launches,
                         bytes_per_launch=nbytes / launches,
                         achieved_GBs=gbs))
    return rows


def copy_bandwidth(torch, nbytes=4 << 30, reps=5):
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    x.fill_(1.0)
    y.copy_(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del x, y
    return 2 * nbytes * reps / dt / 1e9


def add_bandwidth(torch, nbytes=2 << 30, reps=5):
    """c = a + b over float32 tensors: two streams read, one written (pass
    C's mix is 7 grids read to 3 written)."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.ones_like(a)
    c = torch.empty_like(a)
    torch.add(a, b, out=c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        torch.add(a, b, out=c)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del a, b, c
    return 3 * nbytes * reps / dt / 1e9


def run_step(sess, s_thr, y):
    sess.apply_exchange(s_thr)
    sess.build_ace("avg")
    sess.apply_ace(sess.psi, y)


def time_steps(torch, sess, s_thr, steps, warmup, profile=False):
    from paper_1801_09263_amd import lace
    y = torch.empty_like(sess.psi)
    for _ in range(warmup):
        run_step(sess, s_thr, y)
    torch.cuda.synchronize()
    if profile:
        lace.lace_profile_enable(sess.plan, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run_step(sess, s_thr, y)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n_kept = sess.n_kept
    prof = None
    if profile:
        prof = lace.lace_profile_read(sess.plan)
        lace.lace_profile_enable(sess.plan, False)
    return n_kept, (t1 - t0) / steps, prof


def time_exchange(torch, sess, s_thr):
    sess.apply_exchange(s_thr)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sess.apply_exchange(s_thr)
    torch.cuda.synchronize()
    return sess.n_kept, time.perf_counter() - t0


def ace_rows(torch, lace, sess, inp, seed, n_calls=8):
    """FP64 matrix-core rows: apply_ace on n_b = 256 (16 N N_pw n_b flop per
    call), build_ace (M = psi^H W and xi = W Z, 8 N^2 N_pw flop each, plus
    the Cholesky and triangular inverse of N x N), lace_align (30 polar steps on
    N x N plus two N_pw x N x N products), and the SCDM localization of a
    perturbed outer step's orbitals."""
    import numpy as np
    import synth
    n, n_pw = sess.n_orb, sess.n_pw
    x = sess.psi
    y = torch.empty_like(x)
    sess.apply_ace(x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_calls):
        sess.apply_ace(x, y)
    torch.cuda.synchronize()
    t_ace = (time.perf_counter() - t0) / n_calls
    f_ace = 16.0 * n * n_pw * x.shape[0]
    t0 = time.perf_counter()
    for _ in range(n_calls):
        sess.build_ace("avg")
    torch.cuda.synchronize()
    t_build = (time.perf_counter() - t0) / n_calls
    f_build = 2 * 8.0 * n * n * n_pw   # the two GEMMs of the build
    pos, wid = synth.gaussian_params(inp["L"], n, 128, synth.rng_for(2, 0, 0, 0, seed))
    p2, w2 = synth.perturb_gaussian_params(pos, wid, synth.rng_for(2, 0, 0, 1, seed))
    new = torch.tensor(synth.orbitals_from_params(inp["miller"], inp["L"], p2, w2),
                       device="cuda")
    out = torch.empty_like(new)
    resid = torch.zeros(1, dtype=torch.float64, device="cuda")
    lace.lace_align(sess.plan, 0, new, sess.psi, n, out, resid, sess.ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n_calls):
        lace.lace_align(sess.plan, 0, new, sess.psi, n, out, resid, sess.ws)
    torch.cuda.synchronize()
    t_align = (time.perf_counter() - t0) / n_calls
    moved = float(torch.linalg.norm(new - sess.psi) / np.sqrt(n))
    left = float(torch.linalg.norm(out - sess.psi) / np.sqrt(n))
    # SCDM localization of the 256 orbitals (n_orb passes over the grids)
    pts = torch.empty(n, dtype=torch.int32, device="cuda")
    lace.lace_scdm(sess.plan, 0, new, n, out, pts, resid, sess.ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lace.lace_scdm(sess.plan, 0, new, n, out, pts, resid, sess.ws)
    torch.cuda.synchronize()
    t_scdm = time.perf_counter() - t0
    return dict(
        apply_ace_n_b=int(x.shape[0]), apply_ace_ms=round(t_ace * 1e3, 3),
        apply_ace_tflops=round(f_ace / t_ace / 1e12, 2),
        apply_ace_frac_fp64_mfma=round(f_ace / t_ace / 1e12 / FP64_MFMA_PEAK_TFLOPS, 4),
        build_ace_ms=round(t_build * 1e3, 3),
        build_ace_tflops_two_gemms=round(f_build / t_build / 1e12, 2),
        align_ms=round(t_align * 1e3, 3), align_resid=resid.item(),
        align_rms_distance_before=round(moved, 4),
        align_rms_distance_after=round(left, 4),
        scdm_ms=round(t_scdm * 1e3, 2), scdm_resid=resid.item())


# (psi, v, pairs) of the CPU sample, inherited by the forked workers
_ORACLE_SAMPLE = None


def _oracle_columns(cols):
    """One worker's share of the CPU sample: W_j for the columns `cols`,
    reduced to sum_j Re <psi_j, W_j> so that little crosses the pipe."""
    import numpy as np
    import oracle
    psi, v, pairs = _ORACLE_SAMPLE
    w = oracle.apply_exchange_columns(psi, v, pairs, cols)
    return sum(float(np.vdot(psi[j], w[c]).real) for c, j in enumerate(cols))


def host_cores() -> int:
    """Cores this process may use, at most 16 (one GPU's share of a host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(inp, n_sample_orb=32):
    """The oracle, as it stands, on a bounded sample of the same workload,
    on the host's cores: grid orbitals of `n_sample_orb` orbitals spread over
    the cell and screening among them in this process, then the W columns
    of the kept pairs dealt to forked worker processes (balanced by their
    number of ordered Poisson solves).  Must run before the GPU is touched:
    the workers are forked."""
    import multiprocessing as mp
    import numpy as np
    import oracle
    global _ORACLE_SAMPLE
    cores = host_cores()
    idx = np.linspace(0, inp["coeffs"].shape[0] - 1, n_sample_orb).astype(int)
    coeffs = inp["coeffs"][idx]
    t0 = time.perf_counter()
    psi = oracle.orbitals_on_grid(coeffs, inp["miller"], inp["L"], inp["n"])
    v = oracle.coulomb_kernel(inp["L"], inp["n"])
    s = oracle.overlap_of_moduli(psi, inp["L"])
    pairs = oracle.kept_pairs(s, inp["s_thr"])
    load = np.zeros(n_sample_orb, dtype=int)
    for i, j in pairs:
        load[j] += 1
        if i != j:
            load[i] += 1
    shares = [[] for _ in range(cores)]
    acc = [0] * cores
    for j in sorted(range(n_sample_orb), key=lambda c: -load[c]):
        k = acc.index(min(acc))
        shares[k].append(j)
        acc[k] += load[j]
    shares = [sh for sh in shares if sh]
    _ORACLE_SAMPLE = (psi, v, pairs)
    with mp.get_context("fork").Pool(len(shares)) as pool:
        pool.map(_oracle_columns, shares, chunksize=1)
    dt = time.perf_counter() - t0
    _ORACLE_SAMPLE = None
    return dict(value=len(pairs) / dt, unit="pair-FFTs/s", cores=len(shares),
                kind="oracle",
                sample=(f"{n_sample_orb} of the 256 orbitals of the lace-120 "
                        f"workload: grid orbitals and screening in one "
                        f"process, then the {len(pairs)} kept pairs (each as "
                        f"two ordered Poisson solves, {int(load.sum())} in "
                        f"all) dealt by W column to {len(shares)} worker "
                        f"processes, numpy FFT; {dt:.1f} s wall"))


def batched_rows(torch, seed, steps):
    """The 16-cell batched workload: 4 cells of each of 48^3/32, 64^3/64,
    80^3/96, 96^3/128 localized orbitals, S_thr = 1e-3, all in one call;
    autotuned per class; eager streams and the replayed HIP graph."""
    import synth
    from paper_1801_09263_amd import lace
    from paper_1801_09263_amd.batch import MultiCell
    cells = synth.make_batch_cells(seed)
    mc = MultiCell(cells, [c["coeffs"].shape[0] for c in cells],
                   lace.LACE_FP32_GAMMA)
    for k, c in enumerate(cells):
        mc.set_orbitals(k, c["coeffs"])
    tuned = {}
    for k, c in enumerate(cells):
        key = (c["n"], c["coeffs"].shape[0])
        if key not in tuned:
            cands = mc.autotune(k)
            tuned[key] = lace.lace_get_tuning(mc.plan, k) + (
                min(cd[4] for cd in cands),)
        lace.lace_set_tuning(mc.plan, k, *tuned[key][:4])
    st = torch.cuda.Stream()
    out = {}
    for mode in ("eager", "graph"):
        with torch.cuda.stream(st):
            mc.run(graph=(mode == "graph"), stream=st)
            st.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                mc.run(graph=(mode == "graph"), stream=st)
            st.synchronize()
            out[mode] = (time.perf_counter() - t0) / steps
    kept = sum(mc.n_kept)
    total = sum(n * (n + 1) // 2 for n in mc.n_orbs)
    res = dict(
        cells=len(cells), kept_pairs=kept, total_pairs=total,
        ms_eager=round(out["eager"] * 1e3, 1),
        ms_graph=round(out["graph"] * 1e3, 1),
        pair_ffts_per_s_eager=round(kept / out["eager"], 1),
        pair_ffts_per_s_graph=round(kept / out["graph"], 1),
        tuning={f"{n}^3/{no}": dict(pairs_per_batch=t[0], use_plane=t[1],
                                   z_tile=t[2], radix_order=t[3],
                                   us_per_pair=round(t[4], 2))
                for (n, no), t in tuned.items()},
        kept_fraction_by_class={})
    for k, c in enumerate(cells[:4]):
        n = mc.n_orbs[k]
        res["kept_fraction_by_class"][f"{c['n']}^3/{n}"] = round(
            mc.n_kept[k] / (n * (n + 1) / 2), 3)
    mc.close()
    return res


def serving_rows(torch, seed, n_jobs, rate=None, inner=4):
    """Poisson stream (40 jobs/s by default): 95% of jobs from the four
    batched cell classes, 5% localized 120^3 cells, 4 outer iterations each;
    every iteration aligns the orbitals to the previous ones, applies the
    exchange, rebuilds ACE and applies it `inner` times."""
    rate = synth_rate(rate)
    import synth
    from paper_1801_09263_amd import lace
    from paper_1801_09263_amd.serving import Job, JobClass, Server, summarize
    raw = synth.serving_classes(seed)
    classes = []
    for c in raw:
        pool = [torch.tensor(v, device="cuda") for v in c["variants"]]
        cell = {k: c[k] for k in ("L", "n", "miller", "s_thr", "rc")}
        classes.append(JobClass(c["name"], cell, c["n_orb"], pool))
    spec = synth.serving_stream(n_jobs, 4, [len(c.pool) for c in classes],
                                rate=rate, seed=seed)
    # warm-up on one slot first, so every kernel is loaded by one thread
    warm = Server(classes, lace.LACE_FP32_GAMMA, n_slots=1)
    warm.run([Job(-1 - k, 0.0, k, [0]) for k in range(len(classes))])
    warm.close()
    srv = Server(classes, lace.LACE_FP32_GAMMA, n_slots=4, inner=inner,
                 align=True)
    jobs = srv.run([Job(j, t, c, v) for j, t, c, v in spec])
    srv.close()
    res = summarize(jobs, rate)
    res = {k: (round(v, 4) if isinstance(v, float) else v)
           for k, v in res.items()}
    res["slots"] = 4
    res["inner_ace_applications"] = inner
    res["large_jobs"] = sum(1 for j in jobs if j.cls == 4)
    if res["offered_load"] > 4:
        res["note"] = ("finite stream of J jobs; one GPU is oversubscribed "
                       "at this rate, so latency grows with J")
    del classes
    torch.cuda.empty_cache()
    return res


def synth_rate(rate):
    import synth
    return synth.SERVE_RATE if rate is None else float(rate)


def pmc_sample(torch, seed, tuning=(64, 2)):
    """Fixed run for hardware-counter passes: a plain 1 GiB device copy
    (the calibration of FETCH_SIZE / WRITE_SIZE), then one screened
    exchange application of the localized 120^3 workload in the
    real-orbital mode (by default 64 pairs per batch, half-plane xy passes)
    with the pass profiler on, so that only the schedule's batches are
    launched, one at a time.  Prints the launches, kept pairs and the
    library's moved bytes per pass for the comparison with the counters."""
    import synth
    from paper_1801_09263_amd import lace
    from paper_1801_09263_amd.session import CellSession
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    del x, y
    inp = synth.make_inputs("lace-120", seed=seed)
    n_orb = inp["coeffs"].shape[0]
    sess = CellSession(inp, n_orb, lace.LACE_FP32_GAMMA)
    sess.set_orbitals(inp["coeffs"])
    lace.lace_set_tuning(sess.plan, 0, *tuning)
    lace.lace_profile_enable(sess.plan, True)
    sess.apply_exchange(inp["s_thr"])
    torch.cuda.synchronize()
    prof = lace.lace_profile_read(sess.plan)
    print(json.dumps({"pmc_sample": "ok", "tuning": list(tuning),
                      "n_kept": sess.n_kept,
                      "n_orb": n_orb, "n": int(inp["n"]),
                      "launches": prof["launches"],
                      "alg_bytes": prof["alg_bytes"]}), flush=True)


PASS_MATCH = ("ProQuad", "k_zconv", "EpiAccQuad")   # pass A, B, C kernels


def counter_sums(db_path):
    """Per kernel name: dispatches and the sum of the counter's value over
    them (rocprofv3 SQLite output of one --pmc pass)."""
    import sqlite3
    db = sqlite3.connect(db_path)
    rows = db.execute("select kernel_name, dispatch_id, sum(value) from "
                      "counters_collection group by dispatch_id").fetchall()
    db.close()
    return rows


def write_traffic(fetch_db, write_db, sample_log, out_path):
    """profiles/traffic.json from the FETCH_SIZE and WRITE_SIZE passes of
    --pmc-sample: each counter is scaled by what it reads for the 1 GiB
    device copy (the largest copy dispatch of the run), summed over every
    dispatch of each pass kernel and divided by the launches."""
    with open(sample_log) as fh:
        sample = [json.loads(ln) for ln in fh if ln.startswith('{"pmc_sample"')][-1]
    copy_bytes = float(1 << 30)
    res = {"kernel_source_hash": kernel_source_hash()}
    per = {}
    for tag, path in (("fetch", fetch_db), ("write", write_db)):
        rows = counter_sums(path)
        copy_kib = max(v for name, _, v in rows if "copyBuffer" in name)
        scale = copy_bytes / (copy_kib * 1024.0)
        res[tag + "_scale"] = scale
        res["copy_" + tag + "_kib"] = copy_kib
        for k, key in enumerate(PASS_MATCH):
            sel = [(name, v) for name, _, v in rows if key in name]
            d = per.setdefault(str(k), {})
            d["kernel"] = re.sub(r"\s+", " ", sel[0][0]).split("(")[0]
            d["launches"] = len(sel)
            d[tag + "_kib"] = sum(v for _, v in sel) / len(sel)
            d[tag + "_bytes"] = d[tag + "_kib"] * 1024.0 * scale
    res["copy_kernel"] = "__amd_rocclr_copyBuffer"
    res["copy_bytes"] = copy_bytes
    n_orb, n_kept, n = sample["n_orb"], sample["n_kept"], sample["n"]
    for k in range(3):
        d = per[str(k)]
        launches = sample["launches"][k]
        assert d["launches"] == launches, (k, d["launches"], launches)
        d["bytes_per_launch"] = d["fetch_bytes"] + d["write_bytes"]
        d["moved_bytes_per_launch"] = sample["alg_bytes"][k] / launches
        d["alg_bytes_per_launch"] = pass_alg_bytes(
            k, n_kept - n_orb, n_orb, 4, n ** 3) / launches
        d["ratio"] = d["bytes_per_launch"] / d["moved_bytes_per_launch"]
        d["ratio_alg"] = d["bytes_per_launch"] / d["alg_bytes_per_launch"]
    res["passes"] = per
    res["sample"] = ("one screened exchange of the localized %d^3 workload, "
                     "%d kept pairs of %d orbitals, tuning %s (pairs per "
                     "batch, xy schedule, z tile, radix order), launches one "
                     "at a time" % (n, n_kept, n_orb,
                                    sample.get("tuning", [64, 2])))
    with open(out_path, "w") as fh:
        json.dump(res, fh, indent=1)
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain 120^3 comparison rows")
    ap.add_argument("--no-cpu", action="store_true",
                    help="skip the CPU oracle baseline")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 16-cell batched row")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving stream row")
    ap.add_argument("--serve-jobs", type=int, default=48,
                    help="jobs in the serving stream")
    ap.add_argument("--serve-light-rate", type=float, default=5.0,
                    help="arrival rate (jobs/s) of the second, sustainable "
                         "serving stream")
    ap.add_argument("--tuning", default=None, metavar="PPB,MODE[,ZT,RO]",
                    help="fixed pipeline tuning (pairs per batch, xy schedule "
                         "0 pencil / 1 plane / 2 half plane, optionally the z "
                         "tile 0 default / 1 half / 2 twice and the radix "
                         "order 0 / 1) instead of autotuning the main "
                         "workload")
    ap.add_argument("--pmc-sample", action="store_true",
                    help="fixed run for hardware-counter passes: a 1 GiB "
                         "copy (calibration) and one profiled screened "
                         "exchange of the localized workload")
    ap.add_argument("--write-traffic", nargs=3,
                    metavar=("FETCH_DB", "WRITE_DB", "SAMPLE_LOG"),
                    help="no GPU work: write profiles/traffic.json from the "
                         "rocprofv3 databases of the FETCH_SIZE and "
                         "WRITE_SIZE passes of --pmc-sample and its output")
    args = ap.parse_args()
    if args.write_traffic:
        res = write_traffic(*args.write_traffic,
                            os.path.join(ROOT, "profiles", "traffic.json"))
        print(json.dumps(res["passes"], indent=1))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU layout is described, not built", file=sys.stderr)
        sys.exit(2)

    import synth

    inp = cpu = None
    if not args.pmc_sample:
        log("generating the localized 120^3 workload")
        inp = synth.make_inputs("lace-120", seed=args.seed)
        if not args.no_cpu:
            # before torch and the GPU: the oracle's workers are forked
            log("CPU oracle sample")
            cpu = cpu_baseline(inp)
            log("CPU oracle", cpu)

    import torch

    from paper_1801_09263_amd import lace
    from paper_1801_09263_amd.session import CellSession

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    lace.load()

    if args.pmc_sample:
        pmc_sample(torch, args.seed,
                   tuple(int(v) for v in args.tuning.split(","))
                   if args.tuning else (64, 2))
        return

    n_orb = inp["coeffs"].shape[0]
    sess = CellSession(inp, n_orb, lace.LACE_FP32_GAMMA, n_vec=n_orb)
    sess.set_orbitals(inp["coeffs"])
    real_dev = sess.check_real()
    if args.tuning:
        lace.lace_set_tuning(sess.plan, 0,
                             *(int(v) for v in args.tuning.split(",")))
        log(f"orbitals real to {real_dev:.1e}; fixed tuning")
    else:
        log(f"orbitals real to {real_dev:.1e}; autotuning the pair pipeline")
        cands = lace.lace_autotune(sess.plan, 0, sess.psi, n_orb, sess.ws,
                                   s_thr=inp["s_thr"])
        log("candidates", cands)
    tuning = lace.lace_get_tuning(sess.plan, 0)
    log("tuning", tuning)
    log(f"timing {args.steps} steps after {args.warmup} warmup")
    n_kept, t_step, _ = time_steps(torch, sess, inp["s_thr"], args.steps,
                                   args.warmup, profile=False)
    n_total = n_orb * (n_orb + 1) // 2
    e_x = sess.e_x.item()
    ex_tr = sess.ex_tr.item()
    info = sess.info()
    _, t_exch = time_exchange(torch, sess, inp["s_thr"])
    value = n_kept / t_step
    log(f"step {t_step * 1e3:.1f} ms, kept {n_kept}/{n_total}, "
        f"exchange {t_exch * 1e3:.1f} ms")
    # Per-pass kernel figures: the same steps again with the library's pass
    # events on, which run the batches on the caller's stream one launch at a
    # time (the timed steps let consecutive batches overlap on two streams),
    # so each launch's duration is that kernel's own.  These are the last
    # pair-pipeline launches of the run.
    log(f"profiling {args.steps} more steps, launches serialized")
    _, t_step_prof, prof = time_steps(torch, sess, inp["s_thr"], args.steps, 0,
                                      profile=True)
    log(f"profiled step {t_step_prof * 1e3:.1f} ms")

    # roofline of the dominant kernel of the pair pipeline
    rows = pass_roofline(prof)
    dom = max(range(3), key=lambda k: rows[k]["ms_total"])
    # algorithmic bytes: every diagonal pair is kept (S_ii = 1 > S_thr)
    n_diag = n_orb
    n_off = n_kept - n_diag
    s_bytes, ng = 4, int(inp["n"]) ** 3     # real FP32 grids
    launches_per_step = rows[dom]["launches"] / args.steps
    alg_launch = pass_alg_bytes(dom, n_off, n_diag, s_bytes, ng) / launches_per_step
    achieved = alg_launch / (rows[dom]["avg_launch_us"] * 1e-6) / 1e9
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as fh:
            tr = json.load(fh)
        ps = tr.get("passes", {}).get(str(dom))
        if tr.get("kernel_source_hash") == kernel_source_hash() and ps:
            # counter-measured bytes / the library's moved bytes of this
            # kernel in the counter sample, applied to this run's mean launch
            traffic = round(ps["ratio"] * rows[dom]["bytes_per_launch"], 0)
    pipe_ms = sum(prof["ms"])
    pipe_bytes = sum(prof["alg_bytes"])
    roofline = dict(
        bound="hbm", kernel=rows[dom]["name"],
        achieved=round(achieved, 1), peak=HBM_PEAK_GBS,
        unit="GB/s", frac=round(achieved / HBM_PEAK_GBS, 4),
        traffic=traffic,
        avg_launch_us=round(rows[dom]["avg_launch_us"], 2),
        bytes_per_launch=round(alg_launch, 0),
        bytes_model=("per kept pair, in orbital grids of s N_g (s = 4 B real "
                     "FP32 grids, N_g = %d): pass A 3 (diagonal 2), pass B 2 "
                     "(2), pass C 7 (4); %d off-diagonal and %d diagonal "
                     "pairs over %.0f launches per step" %
                     (ng, n_off, n_diag, launches_per_step)),
        moved_bytes_per_launch=round(rows[dom]["bytes_per_launch"], 0),
        moved_GBs=round(rows[dom]["achieved_GBs"], 1),
        moved_frac=round(rows[dom]["achieved_GBs"] / HBM_PEAK_GBS, 4),
        passes=[{k: (round(v, 3) if isinstance(v, float) else v)
                 for k, v in r.items()} for r in rows],
        durations=("HIP events around each launch on the library's stream, "
                   "in a profiled repeat of the timed steps that runs the "
                   "launches one at a time (the batches of the schedule only); "
                   "the timed steps overlap consecutive batches on two "
                   "streams"),
        exchange_GBs_overlapped=round(pipe_bytes / args.steps / t_exch / 1e9, 1),
        pipeline_GBs=round(pipe_bytes / (pipe_ms * 1e-3) / 1e9, 1),
        pipeline_frac=round(pipe_bytes / (pipe_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
    )
    # ACE algebra on the FP64 matrix cores: an inner loop of ACE
    # applications to blocks of 256 functions (a Davidson-like solver's use
    # of the operator between two exchange builds), the M = psi^H W product,
    # and the alignment of a perturbed outer step's orbitals
    ace = ace_rows(torch, lace, sess, inp, args.seed)
    log("ace", ace)
    sess.close()
    del sess
    torch.cuda.empty_cache()

    compare = None
    if not args.no_compare:
        compare = {}
        log("same localized workload on the complex FP32 path")
        s2 = CellSession(inp, n_orb, lace.LACE_FP32, n_vec=n_orb)
        s2.set_orbitals(inp["coeffs"])
        n2, t2 = time_exchange(torch, s2, inp["s_thr"])
        _, ts2, _ = time_steps(torch, s2, inp["s_thr"], 1, 0)
        compare["lace_fp32_complex"] = dict(
            pairs=n2, exchange_ms=round(t2 * 1e3, 1),
            step_ms=round(ts2 * 1e3, 1), pair_ffts_per_s=round(n2 / ts2, 1))
        s2.close()
        del s2
        torch.cuda.empty_cache()
        log("localized workload plus 10 virtual orbitals (real-orbital FP32)")
        import numpy as np
        n_v = 10
        virt = synth.virtual_orbitals(inp["miller"], inp["L"], inp["coeffs"],
                                      n_v, synth.rng_for(2, 0, 0, 1, args.seed))
        s3 = CellSession(inp, n_orb + n_v, lace.LACE_FP32_GAMMA,
                         n_vec=n_orb + n_v)
        s3.set_orbitals(np.concatenate([inp["coeffs"], virt]))
        lace.lace_set_tuning(s3.plan, 0, *tuning)
        y3 = torch.empty_like(s3.psi)
        s3.apply_exchange(inp["s_thr"], n_occ=n_orb)
        s3.build_ace("avg")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s3.apply_exchange(inp["s_thr"], n_occ=n_orb)
        torch.cuda.synchronize()
        t_ex3 = time.perf_counter() - t0
        s3.build_ace("avg")
        s3.apply_ace(s3.psi, y3)
        torch.cuda.synchronize()
        t_st3 = time.perf_counter() - t0
        compare["lace_fp32_gamma_virtual10"] = dict(
            occupied=n_orb, virtual=n_v, pairs=s3.n_kept,
            occupied_pairs=s3.n_kept - n_orb * n_v,
            exchange_ms=round(t_ex3 * 1e3, 1), step_ms=round(t_st3 * 1e3, 1),
            pair_ffts_per_s=round(s3.n_kept / t_st3, 1),
            cholesky_info=s3.info())
        log("lace_fp32_gamma_virtual10", compare["lace_fp32_gamma_virtual10"])
        s3.close()
        del s3
        torch.cuda.empty_cache()
        log("plain unscreened 120^3 random orbitals (FP64 and FP32 pairs)")
        inp1 = synth.make_inputs("plain-ace-120", seed=args.seed)
        for name, prec in (("plain_fp64", lace.LACE_FP64),
                           ("plain_fp32", lace.LACE_FP32)):
            s1 = CellSession(inp1, n_orb, prec, n_vec=n_orb)
            s1.set_orbitals(inp1["coeffs"])
            n1, t1 = time_exchange(torch, s1, 0.0)
            _, ts1, _ = time_steps(torch, s1, 0.0, 1, 0)
            compare[name] = dict(pairs=n1, exchange_ms=round(t1 * 1e3, 1),
                                 step_ms=round(ts1 * 1e3, 1),
                                 pair_ffts_per_s=round(n1 / ts1, 1),
                                 exchange_pair_ffts_per_s=round(n1 / t1, 1))
            log(name, compare[name])
            s1.close()
            del s1
            torch.cuda.empty_cache()
        compare["lace_fp32_vs_plain_fp64_step_speedup"] = round(
            compare["plain_fp64"]["step_ms"] / (t_step * 1e3), 3)
    copy_gbs = copy_bandwidth(torch)
    add_gbs = add_bandwidth(torch)
    batched = None
    if not args.no_batched:
        log("16-cell batched workload")
        batched = batched_rows(torch, args.seed, max(1, args.steps))
        log("batched", batched)
    serving = None
    if not args.no_serve:
        log(f"serving stream of {args.serve_jobs} jobs")
        serving = serving_rows(torch, args.seed, args.serve_jobs)
        log("serving", serving)
        # the same stream at a rate one GPU sustains: service-time latency
        light = serving_rows(torch, args.seed, args.serve_jobs,
                             rate=args.serve_light_rate)
        serving = dict(oversubscribed=serving, sustained=light)
        log("serving at a sustained rate", light)

    out = {
        "metric": "pair-FFTs/s + HBM roofline %, L-ACE vs plain FP64; "
                  "p50/p99 job latency",
        "value": round(value, 1),
        "unit": "pair-FFTs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_step * 1e3, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "lace-120: L=23.5 bohr cubic cell, 120^3 grid, "
                        "Ecut=40 Ha (156795 plane waves), 256 Gaussian "
                        "orbitals on 128 centres, Loewdin, S_thr=1e-3; FP32 "
                        "pairs/FFTs (real-orbital packing), FP64 screening "
                        "sums, energies, M, Cholesky, xi",
            "kept_pairs": n_kept, "total_pairs": n_total,
            "kept_fraction": round(n_kept / n_total, 4),
            "exchange_ms": round(t_exch * 1e3, 1),
            "exchange_pair_ffts_per_s": round(n_kept / t_exch, 1),
            "e_x": e_x, "e_x_trace": ex_tr, "cholesky_info": info,
            "orbitals": "real (Gamma point), checked to %.1e; two pair "
                        "densities per complex FFT" % real_dev,
            "tuning": {"pairs_per_batch": tuning[0], "use_plane": tuning[1],
                       "z_tile": tuning[2], "radix_order": tuning[3]},
            "parallelism": "1 GPU",
        },
        "roofline": roofline,
        "copy_GBs_measured": round(copy_gbs, 1),
        "add_GBs_measured": round(add_gbs, 1),
        "compare": compare,
        "ace": ace,
        "batched": batched,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
