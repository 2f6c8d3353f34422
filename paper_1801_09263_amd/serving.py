"""Continuous-batching request loop for exchange jobs.

A job is one set of orbitals on one cell size class that runs several outer
iterations of the hybrid SCF loop (the double loop of Sec. 2 of the paper,
with the inner KS solve replaced by a precomputed orbital update): at each
iteration the new orbitals are aligned to the previous iteration's (the
convergence aid at the end of Sec. 2), the exchange is applied to them, the
ACE projector is rebuilt, and ACE is applied `inner` times to the orbitals,
as the inner solver would between two exchange builds.

Requests arrive over time.  The admission controller admits them in arrival
order while a worker slot is free and the sum of the admitted jobs' device
footprints stays within the memory budget.  Each slot owns a HIP stream and
a plan and runs one job at a time.  Slots run concurrently, so the work of
different jobs overlaps on the GPU.  A job's W, xi, M and workspace stay
allocated (resident) across its outer iterations.  Every device step runs in
the HIP library; this module only schedules.
"""
from __future__ import annotations

import dataclasses
import queue
import threading
import time

import numpy as np
import torch

from . import lace


@dataclasses.dataclass
class JobClass:
    """One cell size: the cell (L, n, miller, s_thr), the orbital count and
    a pool of orbital sets resident on the device (read-only inputs)."""
    name: str
    cell: dict
    n_orb: int
    pool: list            # device tensors (n_orb, n_pw) complex128
    footprint: int = 0    # device bytes one job of this class holds


@dataclasses.dataclass
class Job:
    jid: int
    arrival: float        # seconds after the stream starts
    cls: int
    variants: list        # pool index of the orbitals at each outer step
    admit: float = -1.0
    done: float = -1.0
    slot: int = -1
    e_x: list = dataclasses.field(default_factory=list)
    kept: list = dataclasses.field(default_factory=list)
    info: list = dataclasses.field(default_factory=list)
    xi_host: object = None


def job_footprint(plan, cell_index, n_orb, n_pw) -> int:
    ws = lace.lace_workspace_size(plan, cell_index, n_orb, n_orb)
    return int(ws + 3 * n_orb * n_pw * 16 + n_orb * n_orb * 16 + 64)


class Server:
    def __init__(self, classes, precision=lace.LACE_FP32, n_slots=4,
                 hbm_budget=None, keep_xi=False, device="cuda", inner=1,
                 align=False):
        self.classes = classes
        self.precision = precision
        self.inner = int(inner)
        self.align = bool(align)
        self.n_slots = int(n_slots)
        self.keep_xi = keep_xi
        self.device = device
        cells = [c.cell for c in classes]
        self.plans = [lace.lace_plan_create(cells, precision)
                      for _ in range(self.n_slots)]
        self.streams = [torch.cuda.Stream() for _ in range(self.n_slots)]
        for k, c in enumerate(classes):
            n_pw = int(np.asarray(c.cell["miller"]).shape[0])
            c.footprint = job_footprint(self.plans[0], k, c.n_orb, n_pw)
            if self.align:   # two more orbital sets: aligned, ping-pong
                c.footprint += 2 * c.n_orb * n_pw * 16
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.8 * free)
        self.hbm_budget = int(hbm_budget)
        biggest = max(c.footprint for c in classes)
        if biggest > self.hbm_budget:
            raise ValueError("a job class does not fit the memory budget")

    # ---------------------------------------------------------- worker
    def _run_job(self, slot, job, t0):
        c = self.classes[job.cls]
        plan = self.plans[slot]
        st = self.streams[slot]
        n, cell = c.n_orb, job.cls
        n_pw = c.pool[0].shape[1]
        with torch.cuda.stream(st):
            z = dict(dtype=torch.complex128, device=self.device)
            w = torch.empty((n, n_pw), **z)
            xi = torch.empty((n, n_pw), **z)
            y = torch.empty((n, n_pw), **z)
            m = torch.empty((n, n), **z)
            ex = torch.zeros(len(job.variants), dtype=torch.float64,
                             device=self.device)
            ex_tr = torch.empty(1, dtype=torch.float64, device=self.device)
            # Cholesky info word of each outer step's ACE build, and the
            # pairs each step runs
            info = torch.zeros(len(job.variants), dtype=torch.int32,
                               device=self.device)
            kept = torch.zeros(len(job.variants), dtype=torch.int64,
                               device=self.device)
            ws = torch.empty(lace.lace_workspace_size(plan, cell, n, n),
                             dtype=torch.uint8, device=self.device)
            prev = None
            if self.align and len(job.variants) > 1:
                cur = torch.empty((n, n_pw), **z)
                nxt = torch.empty((n, n_pw), **z)
            for step, v in enumerate(job.variants):
                psi = c.pool[v]
                if self.align and prev is not None:
                    lace.lace_align(plan, cell, psi, prev, n, nxt, None, ws, st)
                    psi = nxt
                    cur, nxt = nxt, cur
                lace.lace_apply_exchange(
                    plan, cell, psi, n, c.cell.get("s_thr", 0.0), None, w,
                    ex[step:step + 1], ws, st, n_kept=kept[step:step + 1])
                lace.lace_build_ace(plan, cell, psi, w, n, "avg", xi, m,
                                    ex_tr, ws, st, info=info[step:step + 1])
                for _ in range(self.inner):
                    lace.lace_apply_ace(plan, cell, xi, n, psi, n, y, ws, st)
                prev = psi
            st.synchronize()
        job.done = time.perf_counter() - t0
        job.e_x = ex.cpu().tolist()
        job.info = info.cpu().tolist()
        job.kept = kept.cpu().tolist()
        if self.keep_xi:
            job.xi_host = xi.cpu().numpy()
        del w, xi, y, m, ex, ex_tr, ws, info, kept
        if any(job.info):
            raise lace.LaceError(lace.LACE_ENOTPD,
                                 f"job {job.jid}: ACE build (info {job.info})")

    def _worker(self, slot, inbox, outbox, t0):
        while True:
            job = inbox.get()
            if job is None:
                return
            try:
                self._run_job(slot, job, t0)
                outbox.put((slot, job, None))
            except Exception as exc:  # reported by the admission loop
                outbox.put((slot, job, exc))

    # ------------------------------------------------------- admission
    def run(self, jobs):
        """Serve `jobs` (sorted by arrival).  Returns the jobs with admit
        and completion times filled in."""
        jobs = sorted(jobs, key=lambda j: j.arrival)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        inboxes = [queue.Queue() for _ in range(self.n_slots)]
        outbox = queue.Queue()
        threads = [threading.Thread(target=self._worker,
                                    args=(s, inboxes[s], outbox, t0),
                                    daemon=True)
                   for s in range(self.n_slots)]
        for th in threads:
            th.start()
        free = list(range(self.n_slots))
        used = 0
        nxt = 0
        waiting = []
        finished = 0
        errors = []
        try:
            while finished < len(jobs):
                now = time.perf_counter() - t0
                while nxt < len(jobs) and jobs[nxt].arrival <= now:
                    waiting.append(jobs[nxt])
                    nxt += 1
                while waiting and free:
                    j = waiting[0]
                    fp = self.classes[j.cls].footprint
                    if used + fp > self.hbm_budget:
                        break
                    waiting.pop(0)
                    used += fp
                    j.slot = free.pop(0)
                    j.admit = time.perf_counter() - t0
                    inboxes[j.slot].put(j)
                timeout = 0.05
                if nxt < len(jobs) and not waiting:
                    timeout = max(0.0, min(timeout, jobs[nxt].arrival - now))
                try:
                    slot, j, exc = outbox.get(timeout=timeout)
                except queue.Empty:
                    continue
                if exc is not None:
                    errors.append(exc)
                used -= self.classes[j.cls].footprint
                free.append(slot)
                finished += 1
        finally:
            for q in inboxes:
                q.put(None)
            for th in threads:
                th.join()
        if errors:
            raise errors[0]
        return jobs

    def close(self):
        for p in self.plans:
            p.close()


def summarize(jobs, rate):
    lat = np.array([j.done - j.arrival for j in jobs])
    wait = np.array([j.admit - j.arrival for j in jobs])
    serv = np.array([j.done - j.admit for j in jobs])
    span = max(j.done for j in jobs) - min(j.arrival for j in jobs)
    return dict(
        jobs=len(jobs), arrival_rate=rate,
        p50_latency_s=float(np.percentile(lat, 50)),
        p99_latency_s=float(np.percentile(lat, 99)),
        mean_wait_s=float(wait.mean()), mean_service_s=float(serv.mean()),
        jobs_per_s=len(jobs) / span, makespan_s=span,
        offered_load=float(rate * serv.mean()))
