"""Device buffers of one cell around the C ABI.

``CellSession`` owns a plan, a workspace and the plane-wave arrays of one
cell (orbitals, W = K psi, xi, M) as torch tensors, and calls the library.
It does no arithmetic of its own.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lace


class CellSession:
    def __init__(self, cell: dict, n_orb: int, precision=lace.LACE_FP32,
                 n_vec: int = 0, device: str = "cuda"):
        self.cell = cell
        self.n_orb = int(n_orb)
        self.n_pw = int(np.asarray(cell["miller"]).shape[0])
        self.plan = lace.lace_plan_create([cell], precision)
        self.precision = precision
        self.device = device
        self.n_vec = max(int(n_vec), self.n_orb)
        nbytes = lace.lace_workspace_size(self.plan, 0, self.n_orb, self.n_vec)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        shape = (self.n_orb, self.n_pw)
        self.psi = torch.zeros(shape, dtype=torch.complex128, device=device)
        self.w = torch.zeros(shape, dtype=torch.complex128, device=device)
        self.xi = torch.zeros(shape, dtype=torch.complex128, device=device)
        self.m = torch.zeros((self.n_orb, self.n_orb), dtype=torch.complex128,
                             device=device)
        self.s = torch.zeros((self.n_orb, self.n_orb), dtype=torch.float64,
                             device=device)
        self.e_x = torch.zeros(1, dtype=torch.float64, device=device)
        self.ex_tr = torch.zeros(1, dtype=torch.float64, device=device)
        # pairs run by the last exchange call, written on the device
        self.n_kept_t = torch.zeros(1, dtype=torch.int64, device=device)
        self.kept = None

    def set_orbitals(self, coeffs):
        c = torch.as_tensor(np.ascontiguousarray(coeffs), dtype=torch.complex128)
        assert tuple(c.shape) == (self.n_orb, self.n_pw)
        self.psi.copy_(c.to(self.device))

    def screen(self, stream=None):
        lace.lace_screen(self.plan, 0, self.psi, self.n_orb, self.s, self.ws,
                         stream)
        return self.s

    @property
    def n_kept(self) -> int:
        """Pairs run by the last exchange call (synchronizes the device)."""
        torch.cuda.synchronize()
        return int(self.n_kept_t.item())

    def apply_exchange(self, s_thr=0.0, pairs=None, stream=None, n_occ=None,
                       want_kept=False):
        """W = K psi.  With n_occ < n_orb the first n_occ orbitals are the
        occupied ones and the rest virtual (pairs must then be None).
        want_kept: the screened call also writes the kept pair list to
        self.kept (int32, (n, 2) after n_kept rows)."""
        if n_occ is not None and n_occ < self.n_orb:
            if pairs is not None:
                raise ValueError("explicit pairs with virtual orbitals")
            lace.lace_apply_exchange_virtual(
                self.plan, 0, self.psi, n_occ, self.n_orb - n_occ, s_thr,
                self.w, self.e_x, self.ws, stream, n_kept=self.n_kept_t)
        else:
            if want_kept and self.kept is None:
                self.kept = torch.zeros(self.n_orb * (self.n_orb + 1),
                                        dtype=torch.int32, device=self.device)
            lace.lace_apply_exchange(
                self.plan, 0, self.psi, self.n_orb, s_thr, pairs, self.w,
                self.e_x, self.ws, stream, n_kept=self.n_kept_t,
                kept=self.kept if want_kept else None)
        return self.w

    def kept_pairs(self):
        """The kept pairs of the last screened call with want_kept, as an
        (n_kept, 2) numpy array (synchronizes the device)."""
        n = self.n_kept
        return self.kept[: 2 * n].cpu().numpy().reshape(n, 2)

    def build_ace(self, sym="avg", stream=None):
        lace.lace_build_ace(self.plan, 0, self.psi, self.w, self.n_orb, sym,
                            self.xi, self.m, self.ex_tr, self.ws, stream)
        return self.xi

    def check_real(self, stream=None) -> float:
        return lace.lace_check_real(self.plan, 0, self.psi, self.n_orb,
                                    self.ws, stream)

    def info(self, stream=None) -> int:
        """Cholesky info word of the last build_ace (synchronizes the
        stream)."""
        return lace.lace_get_info(self.ws, stream)

    def apply_ace(self, x, y=None, stream=None):
        n_vec = x.shape[0]
        if n_vec > self.n_vec:
            raise ValueError("more functions than the workspace was sized for")
        if y is None:
            y = torch.empty_like(x)
        lace.lace_apply_ace(self.plan, 0, self.xi, self.n_orb, x, n_vec, y,
                            self.ws, stream)
        return y

    def close(self):
        self.plan.close()
