"""Device buffers of a set of cells handled together.

``MultiCell`` owns one plan over several cells (any mix of grid sizes),
one workspace and one set of plane-wave arrays per job, and calls the
batched entry point.  It does no arithmetic of its own.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lace


class MultiCell:
    def __init__(self, cells, n_orbs, precision=lace.LACE_FP32,
                 device="cuda"):
        self.cells = cells
        self.n_orbs = [int(n) for n in n_orbs]
        self.plan = lace.lace_plan_create(cells, precision)
        self.device = device
        self.jobs = []
        for k, (cell, n) in enumerate(zip(cells, self.n_orbs)):
            n_pw = int(np.asarray(cell["miller"]).shape[0])
            nbytes = lace.lace_workspace_size(self.plan, k, n, n)
            z = dict(dtype=torch.complex128, device=device)
            self.jobs.append(dict(
                cell=k, n_orb=n, s_thr=float(cell.get("s_thr", 0.0)),
                psi_g=torch.zeros((n, n_pw), **z),
                w_g=torch.zeros((n, n_pw), **z),
                xi_g=torch.zeros((n, n_pw), **z),
                m_out=torch.zeros((n, n), **z),
                e_x=torch.zeros(1, dtype=torch.float64, device=device),
                n_kept=torch.zeros(1, dtype=torch.int64, device=device),
                ex_tr=torch.zeros(1, dtype=torch.float64, device=device),
                ws=torch.empty(nbytes, dtype=torch.uint8, device=device),
                sym="avg"))

    def set_orbitals(self, k, coeffs):
        self.jobs[k]["psi_g"].copy_(torch.as_tensor(
            np.ascontiguousarray(coeffs), dtype=torch.complex128))

    def run(self, graph=False, stream=None, build_ace=True):
        jobs = self.jobs if build_ace else [
            {k: v for k, v in j.items() if k not in ("xi_g", "m_out", "ex_tr")}
            for j in self.jobs]
        lace.lace_apply_exchange_batched(self.plan, jobs, graph=graph,
                                         stream=stream)
        return self.n_kept

    @property
    def n_kept(self):
        """Pairs run per job by the last call (synchronizes the device)."""
        torch.cuda.synchronize()
        return [int(j["n_kept"].item()) for j in self.jobs]

    def autotune(self, k, stream=None):
        j = self.jobs[k]
        return lace.lace_autotune(self.plan, k, j["psi_g"], j["n_orb"],
                                  j["ws"], stream, s_thr=j["s_thr"])

    def close(self):
        self.plan.close()
