"""Thin ctypes binding of liblace (include/lace.h).

Argument marshalling only: every step of the exchange path runs in the HIP
library.  Device buffers are torch tensors on the GPU (PyTorch provides the
memory and the stream); pair lists are host arrays.  When the library has not
been built, every entry point raises ``LaceUnavailable``: there is no
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblace.so")

LACE_OK = 0
LACE_EINVAL = -1
LACE_ENOMEM = -2
LACE_ENOTPD = -3
LACE_EUNSUPPORTED = -4
LACE_EHIP = -5

LACE_FP64 = 0
LACE_FP32 = 1
LACE_FP64_GAMMA = 2
LACE_FP32_GAMMA = 3
LACE_SYM_AVG = 0
LACE_SYM_UPPER = 1
LACE_SYM_LOWER = 2
SYM_MODES = {"avg": LACE_SYM_AVG, "upper": LACE_SYM_UPPER,
             "lower": LACE_SYM_LOWER}

# Every entry point declared in include/lace.h.
SYMBOLS = (
    "lace_plan_create", "lace_plan_destroy", "lace_workspace_size",
    "lace_screen", "lace_apply_exchange", "lace_build_ace", "lace_apply_ace",
    "lace_fft3d", "lace_get_info", "lace_status_string",
    "lace_profile_enable", "lace_profile_read", "lace_schedule_pairs",
    "lace_schedule_slots", "lace_apply_exchange_virtual", "lace_align",
    "lace_scdm",
    "lace_apply_exchange_batched", "lace_set_tuning", "lace_get_tuning",
    "lace_autotune", "lace_check_real", "lace_read_schedule",
    "lace_apply_ace_noalloc",
)
LACE_BATCH_GRAPH = 1


class LaceUnavailable(RuntimeError):
    pass


class LaceError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {lace_status_string(code)} ({code})")


class CellDesc(ctypes.Structure):
    _fields_ = [("L", ctypes.c_double), ("n", ctypes.c_int32),
                ("rc", ctypes.c_double), ("n_pw", ctypes.c_int64),
                ("miller", ctypes.POINTER(ctypes.c_int32)),
                ("omega", ctypes.c_double)]


class LaceJob(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int32), ("psi_g", ctypes.c_void_p),
                ("n_orb", ctypes.c_int32), ("s_thr", ctypes.c_double),
                ("w_g", ctypes.c_void_p), ("e_x", ctypes.c_void_p),
                ("n_kept", ctypes.c_void_p), ("sym", ctypes.c_int32),
                ("xi_g", ctypes.c_void_p), ("m_out", ctypes.c_void_p),
                ("ex_tr", ctypes.c_void_p), ("info", ctypes.c_void_p),
                ("ws", ctypes.c_void_p),
                ("ws_bytes", ctypes.c_size_t)]


_LIB = None


def load(path: str = LIB_PATH):
    """Load liblace.so and declare the signatures (no GPU work)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise LaceUnavailable(
            f"{path} is not built; run python -m paper_1801_09263_amd.build")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, sz = (ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                             ctypes.c_double, ctypes.c_size_t)
    p_i32 = ctypes.POINTER(ctypes.c_int32)
    lib.lace_plan_create.argtypes = [ctypes.POINTER(CellDesc), i32, i32,
                                     ctypes.POINTER(vp)]
    lib.lace_plan_destroy.argtypes = [vp]
    lib.lace_workspace_size.argtypes = [vp, i32, i32, i32,
                                        ctypes.POINTER(sz)]
    lib.lace_screen.argtypes = [vp, i32, vp, i32, vp, vp, sz, vp]
    lib.lace_apply_exchange.argtypes = [vp, i32, vp, i32, dbl, vp, vp, i64,
                                        vp, vp, vp, vp, vp, sz, vp]
    lib.lace_apply_exchange_virtual.argtypes = [
        vp, i32, vp, i32, i32, dbl, vp, vp, vp, vp, sz, vp]
    lib.lace_align.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, sz, vp]
    lib.lace_scdm.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, sz, vp]
    lib.lace_build_ace.argtypes = [vp, i32, vp, vp, i32, i32, vp, vp, vp, vp,
                                   vp, sz, vp]
    lib.lace_apply_ace.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp, sz, vp]
    lib.lace_apply_ace_noalloc.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp]
    lib.lace_fft3d.argtypes = [vp, i32, i32, vp, i32, vp]
    lib.lace_get_info.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int32)]
    lib.lace_profile_enable.argtypes = [vp, i32]
    p_i64 = ctypes.POINTER(ctypes.c_int64)
    lib.lace_profile_read.argtypes = [vp, ctypes.POINTER(ctypes.c_double),
                                      p_i64, p_i64,
                                      ctypes.POINTER(ctypes.c_double)]
    lib.lace_check_real.argtypes = [vp, i32, vp, i32, vp, sz, vp,
                                    ctypes.POINTER(ctypes.c_double)]
    lib.lace_schedule_pairs.argtypes = [p_i32, p_i32, i64, i32, i32, p_i32,
                                        p_i64]
    lib.lace_schedule_slots.argtypes = [p_i32, p_i32, i64, i32, i32, p_i32,
                                        p_i32, p_i64]
    lib.lace_read_schedule.argtypes = [vp, i32, i32, vp, vp, p_i32, p_i32, i64,
                                       p_i32, p_i32, p_i64]
    lib.lace_apply_exchange_batched.argtypes = [vp, ctypes.POINTER(LaceJob),
                                                i32, i32, vp]
    lib.lace_set_tuning.argtypes = [vp, i32, i32, i32, i32, i32]
    p_int = ctypes.POINTER(ctypes.c_int)
    lib.lace_get_tuning.argtypes = [vp, i32, p_int, p_int, p_int, p_int]
    lib.lace_autotune.argtypes = [vp, i32, vp, i32, dbl, vp, sz, vp,
                                  p_int, p_int, p_int, p_int,
                                  ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_int)]
    lib.lace_status_string.argtypes = [i32]
    lib.lace_status_string.restype = ctypes.c_char_p
    for name in SYMBOLS:
        if name != "lace_status_string":
            getattr(lib, name).restype = i32
    _LIB = lib
    return lib


def lace_status_string(code: int) -> str:
    return load().lace_status_string(int(code)).decode()


def _check(code: int, what: str):
    if code != LACE_OK:
        raise LaceError(code, what)


def _ptr(t, dtype=None, what="buffer"):
    """Raw device pointer of a contiguous torch CUDA tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _n_pw(plan, cell):
    if not 0 <= int(cell) < len(plan.cells):
        return 0     # the library rejects the cell index itself
    return int(np.asarray(plan.cells[int(cell)]["miller"]).shape[0])


def _need(t, count, what):
    """The C ABI receives raw pointers and cannot see a tensor's size: an
    undersized buffer is rejected here, before the call."""
    if t is not None and t.numel() < count:
        raise ValueError(f"{what} holds {t.numel()} elements, needs {count}")


def _stream_obj(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return stream


def _stream(stream):
    return ctypes.c_void_p(_stream_obj(stream).cuda_stream)


def _count(t, stream):
    """A one-element int64 device tensor for a count the library writes:
    the caller's, or a new one kept alive for the stream."""
    import torch
    if t is not None:
        return t, False
    st = _stream_obj(stream)
    with torch.cuda.stream(st):
        t = torch.zeros(1, dtype=torch.int64, device="cuda")
    return t, True


def _read_count(t, own, stream):
    """The count as an int when the binding made the tensor (synchronizes
    the stream), else the caller's tensor."""
    if not own:
        return t
    _stream_obj(stream).synchronize()
    return int(t.item())


def pair_tensors(pairs, n_orb, device="cuda", stream=None):
    """An explicit pair list as two device int32 tensors (i, j) and its
    length, checked on the host first: 0 <= i <= j < n_orb and no repeats.
    An empty list still gets (one-element) tensors, so that the library sees
    a list and not a request to screen."""
    import torch
    if isinstance(pairs, tuple) and len(pairs) == 2 and hasattr(pairs[0], "is_cuda"):
        return pairs[0], pairs[1], pairs[0].numel()
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int64).reshape(-1, 2))
    if pr.size:
        i, j = pr[:, 0], pr[:, 1]
        if (i < 0).any() or (j < i).any() or (j >= n_orb).any():
            raise ValueError("pairs must satisfy 0 <= i <= j < n_orb")
        if np.unique(i * n_orb + j).size != pr.shape[0]:
            raise ValueError("repeated pair")
    st = _stream_obj(stream)
    count = pr.shape[0]
    if count == 0:
        pr = np.zeros((1, 2), np.int64)
    with torch.cuda.stream(st):
        pi = torch.tensor(pr[:, 0].astype(np.int32), device=device)
        pj = torch.tensor(pr[:, 1].astype(np.int32), device=device)
    return pi, pj, count


class Plan:
    """Owner of a ``lace_plan*``; destroyed on ``close()`` or collection."""

    def __init__(self, handle, cells, precision):
        self.handle = handle
        self.cells = cells
        self.precision = precision

    def close(self):
        if self.handle:
            load().lace_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):  # pragma: no cover - interpreter shutdown order
        try:
            self.close()
        except Exception:
            pass


def lace_plan_create(cells, precision=LACE_FP64) -> Plan:
    """``cells``: list of dicts with L, n, miller (n_pw x 3 int array) and
    optional rc (Coulomb truncation) or omega (> 0: the short-range
    erfc(omega r) / r interaction)."""
    lib = load()
    keep = []
    arr = (CellDesc * len(cells))()
    for k, c in enumerate(cells):
        m = np.ascontiguousarray(c["miller"], dtype=np.int32)
        keep.append(m)
        arr[k].L = float(c["L"])
        arr[k].n = int(c["n"])
        arr[k].rc = float(c.get("rc", 0.0) or 0.0)
        arr[k].omega = float(c.get("omega", 0.0) or 0.0)
        arr[k].n_pw = int(m.shape[0])
        arr[k].miller = m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    h = ctypes.c_void_p()
    _check(lib.lace_plan_create(arr, len(cells), int(precision),
                                ctypes.byref(h)), "lace_plan_create")
    return Plan(h, cells, precision)


def lace_workspace_size(plan: Plan, cell: int, n_orb: int, n_vec: int = 0):
    out = ctypes.c_size_t()
    _check(load().lace_workspace_size(plan.handle, cell, n_orb, n_vec,
                                      ctypes.byref(out)),
           "lace_workspace_size")
    return out.value


def lace_screen(plan, cell, psi_g, n_orb, s_out, ws, stream=None):
    import torch
    _need(psi_g, n_orb * _n_pw(plan, cell), "psi_g")
    _need(s_out, n_orb * n_orb, "s_out")
    _check(load().lace_screen(plan.handle, cell,
                              _ptr(psi_g, torch.complex128, "psi_g"), n_orb,
                              _ptr(s_out, torch.float64, "s_out"),
                              _ptr(ws, None, "ws"), ws.numel() * ws.element_size(),
                              _stream(stream)), "lace_screen")


def lace_apply_exchange_virtual(plan, cell, psi_g, n_occ, n_virt, s_thr, w_g,
                                e_x, ws, stream=None, n_kept=None):
    """W for n_occ occupied and n_virt virtual orbitals (occupied first).
    Returns the number of pair transforms run (an int, after synchronizing
    the stream), or the caller's n_kept tensor, which receives it."""
    import torch
    n = (int(n_occ) + int(n_virt)) * _n_pw(plan, cell)
    _need(psi_g, n, "psi_g")
    _need(w_g, n, "w_g")
    _need(e_x, 1, "e_x")
    nk, own = _count(n_kept, stream)
    _check(load().lace_apply_exchange_virtual(
        plan.handle, cell, _ptr(psi_g, torch.complex128, "psi_g"), int(n_occ),
        int(n_virt), float(s_thr), _ptr(w_g, torch.complex128, "w_g"),
        _ptr(e_x, torch.float64, "e_x"), _ptr(nk, torch.int64, "n_kept"),
        _ptr(ws, None, "ws"), ws.numel() * ws.element_size(), _stream(stream)),
        "lace_apply_exchange_virtual")
    return _read_count(nk, own, stream)


def lace_align(plan, cell, psi_new, psi_old, n_orb, psi_out, resid, ws,
               stream=None):
    """psi_out = psi_new U, U the unitary closest to psi_new^H psi_old."""
    import torch
    n = n_orb * _n_pw(plan, cell)
    for t, name in ((psi_new, "psi_new"), (psi_old, "psi_old"),
                    (psi_out, "psi_out")):
        _need(t, n, name)
    _need(resid, 1, "resid")
    _check(load().lace_align(
        plan.handle, cell, _ptr(psi_new, torch.complex128, "psi_new"),
        _ptr(psi_old, torch.complex128, "psi_old"), int(n_orb),
        _ptr(psi_out, torch.complex128, "psi_out"),
        _ptr(resid, torch.float64, "resid"), _ptr(ws, None, "ws"),
        ws.numel() * ws.element_size(), _stream(stream)), "lace_align")


def lace_scdm(plan, cell, psi_g, n_orb, phi_g, points, resid, ws,
              stream=None):
    """phi = SCDM-localized psi; points (int32 device tensor or None)."""
    import torch
    n = n_orb * _n_pw(plan, cell)
    _need(psi_g, n, "psi_g")
    _need(phi_g, n, "phi_g")
    _need(points, n_orb, "points")
    _need(resid, 1, "resid")
    _check(load().lace_scdm(
        plan.handle, cell, _ptr(psi_g, torch.complex128, "psi_g"), int(n_orb),
        _ptr(phi_g, torch.complex128, "phi_g"),
        _ptr(points, torch.int32, "points"), _ptr(resid, torch.float64, "resid"),
        _ptr(ws, None, "ws"), ws.numel() * ws.element_size(), _stream(stream)),
        "lace_scdm")


def lace_apply_exchange(plan, cell, psi_g, n_orb, s_thr, pairs, w_g, e_x, ws,
                        stream=None, n_kept=None, kept=None):
    """``pairs``: None (screen with s_thr), an (n, 2) int array of
    unordered pairs i <= j (checked here, then copied to the device), or a
    tuple of two device int32 tensors.  ``kept``: optional int32 device
    tensor of n_orb (n_orb + 1) elements that receives the kept pairs when
    the call screens.  Returns the number of pairs run (an int, after
    synchronizing the stream), or the caller's n_kept tensor, which
    receives it."""
    import torch
    _need(psi_g, n_orb * _n_pw(plan, cell), "psi_g")
    _need(w_g, n_orb * _n_pw(plan, cell), "w_g")
    _need(e_x, 1, "e_x")
    _need(kept, n_orb * (n_orb + 1), "kept")
    st = _stream_obj(stream)
    if pairs is None:
        pi = pj = None
        npairs = 0
    else:
        pi, pj, npairs = pair_tensors(pairs, n_orb, stream=st)
        if pj.numel() < npairs:
            raise ValueError("pair_i and pair_j differ in length")
        pi.record_stream(st)
        pj.record_stream(st)
    nk, own = _count(n_kept, st)
    _check(load().lace_apply_exchange(
        plan.handle, cell, _ptr(psi_g, torch.complex128, "psi_g"), n_orb,
        float(s_thr), _ptr(pi, torch.int32, "pair_i"),
        _ptr(pj, torch.int32, "pair_j"), npairs,
        _ptr(w_g, torch.complex128, "w_g"), _ptr(e_x, torch.float64, "e_x"),
        _ptr(nk, torch.int64, "n_kept"), _ptr(kept, torch.int32, "kept"),
        _ptr(ws, None, "ws"), ws.numel() * ws.element_size(), _stream(st)),
        "lace_apply_exchange")
    return _read_count(nk, own, st)


def lace_read_schedule(plan, cell, n_orb, ws, pairs, stream=None):
    """The batch and slot of each of ``pairs`` in the schedule the last
    exchange call on ``ws`` built on the device (synchronizes the stream).
    Returns (batch_of, slot_of, n_batches)."""
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    pi = np.ascontiguousarray(pr[:, 0])
    pj = np.ascontiguousarray(pr[:, 1])
    bo = np.empty(pr.shape[0], dtype=np.int32)
    so = np.empty(pr.shape[0], dtype=np.int32)
    nb = ctypes.c_int64(0)
    P = ctypes.POINTER(ctypes.c_int32)
    _check(load().lace_read_schedule(plan.handle, cell, int(n_orb),
                                     _ptr(ws, None, "ws"), _stream(stream),
                                     pi.ctypes.data_as(P), pj.ctypes.data_as(P),
                                     pr.shape[0], bo.ctypes.data_as(P),
                                     so.ctypes.data_as(P), ctypes.byref(nb)),
           "lace_read_schedule")
    return bo, so, nb.value


def lace_build_ace(plan, cell, psi_g, w_g, n_orb, sym, xi_g, m_out, ex_tr, ws,
                   stream=None, info=None):
    """``info``: optional int32 device tensor (one element) that receives
    the Cholesky info word of this call; None keeps it in the workspace
    (read with ``lace_get_info(ws, stream)``)."""
    import torch
    n = n_orb * _n_pw(plan, cell)
    for t, name in ((psi_g, "psi_g"), (w_g, "w_g"), (xi_g, "xi_g")):
        _need(t, n, name)
    _need(m_out, n_orb * n_orb, "m_out")
    _need(ex_tr, 1, "ex_tr")
    _need(info, 1, "info")
    mode = SYM_MODES[sym] if isinstance(sym, str) else int(sym)
    _check(load().lace_build_ace(
        plan.handle, cell, _ptr(psi_g, torch.complex128, "psi_g"),
        _ptr(w_g, torch.complex128, "w_g"), n_orb, mode,
        _ptr(xi_g, torch.complex128, "xi_g"),
        _ptr(m_out, torch.complex128, "m_out"),
        _ptr(ex_tr, torch.float64, "ex_tr"),
        _ptr(info, torch.int32, "info"), _ptr(ws, None, "ws"),
        ws.numel() * ws.element_size(), _stream(stream)), "lace_build_ace")


def lace_apply_ace(plan, cell, xi_g, n_orb, x_g, n_vec, y_g, ws, stream=None):
    import torch
    n_pw = _n_pw(plan, cell)
    _need(xi_g, n_orb * n_pw, "xi_g")
    _need(x_g, n_vec * n_pw, "x_g")
    _need(y_g, n_vec * n_pw, "y_g")
    _check(load().lace_apply_ace(
        plan.handle, cell, _ptr(xi_g, torch.complex128, "xi_g"), n_orb,
        _ptr(x_g, torch.complex128, "x_g"), n_vec,
        _ptr(y_g, torch.complex128, "y_g"), _ptr(ws, None, "ws"),
        ws.numel() * ws.element_size(), _stream(stream)), "lace_apply_ace")


def lace_apply_ace_noalloc(plan, cell, xi_g, n_orb, x_g, n_vec, y_g,
                           stream=None):
    """lace_apply_ace with the library's fixed per-GPU scratch instead of a
    workspace: no device memory is allocated by the call."""
    import torch
    n_pw = _n_pw(plan, cell)
    _need(xi_g, n_orb * n_pw, "xi_g")
    _need(x_g, n_vec * n_pw, "x_g")
    _need(y_g, n_vec * n_pw, "y_g")
    _check(load().lace_apply_ace_noalloc(
        plan.handle, cell, _ptr(xi_g, torch.complex128, "xi_g"), n_orb,
        _ptr(x_g, torch.complex128, "x_g"), n_vec,
        _ptr(y_g, torch.complex128, "y_g"), _stream(stream)),
        "lace_apply_ace_noalloc")


def lace_fft3d(plan, cell, direction, grids, count, stream=None):
    if 0 <= int(cell) < len(plan.cells) and grids is not None:
        n = int(plan.cells[int(cell)]["n"])
        point = 16 if plan.precision in (LACE_FP64, LACE_FP64_GAMMA) else 8
        need = int(count) * n ** 3 * point
        if grids.numel() * grids.element_size() < need:
            raise ValueError(f"grids holds {grids.numel() * grids.element_size()}"
                             f" bytes, needs {need}")
    _check(load().lace_fft3d(plan.handle, cell, int(direction),
                             _ptr(grids, None, "grids"), int(count),
                             _stream(stream)), "lace_fft3d")


def lace_get_info(ws, stream=None) -> int:
    """Cholesky info word of the last ACE build that used workspace ``ws``
    without an info tensor (synchronizes ``stream``)."""
    info = ctypes.c_int32(0)
    code = load().lace_get_info(_ptr(ws, None, "ws"), _stream(stream),
                                ctypes.byref(info))
    if code not in (LACE_OK, LACE_ENOTPD):
        _check(code, "lace_get_info")
    return info.value


def lace_profile_enable(plan, enable=True):
    _check(load().lace_profile_enable(plan.handle, 1 if enable else 0),
           "lace_profile_enable")


def lace_profile_read(plan):
    """Per-pass totals of the pair pipeline since profiling was enabled:
    dict of lists (index 0 pass A, 1 pass B, 2 pass C): milliseconds,
    launches, pairs and algorithmic HBM bytes."""
    ms = (ctypes.c_double * 3)()
    la = (ctypes.c_int64 * 3)()
    pr = (ctypes.c_int64 * 3)()
    by = (ctypes.c_double * 3)()
    _check(load().lace_profile_read(plan.handle, ms, la, pr, by),
           "lace_profile_read")
    return dict(ms=list(ms), launches=list(la), pairs=list(pr),
                alg_bytes=list(by))


def lace_check_real(plan, cell, psi_g, n_orb, ws, stream=None) -> float:
    """Relative deviation of the orbitals from C_{-G} = conj(C_G)."""
    import torch
    _need(psi_g, n_orb * _n_pw(plan, cell), "psi_g")
    out = ctypes.c_double(0.0)
    _check(load().lace_check_real(plan.handle, cell,
                                  _ptr(psi_g, torch.complex128, "psi_g"),
                                  n_orb, _ptr(ws, None, "ws"),
                                  ws.numel() * ws.element_size(),
                                  _stream(stream), ctypes.byref(out)),
           "lace_check_real")
    return out.value


def lace_schedule_pairs(pairs, n_orb, per_batch):
    """Batch index of every pair (host only).  Returns (batch_of, n)."""
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    pi = np.ascontiguousarray(pr[:, 0])
    pj = np.ascontiguousarray(pr[:, 1])
    out = np.empty(pr.shape[0], dtype=np.int32)
    nb = ctypes.c_int64(0)
    P = ctypes.POINTER(ctypes.c_int32)
    _check(load().lace_schedule_pairs(pi.ctypes.data_as(P), pj.ctypes.data_as(P),
                                      pr.shape[0], int(n_orb), int(per_batch),
                                      out.ctypes.data_as(P), ctypes.byref(nb)),
           "lace_schedule_pairs")
    return out, nb.value


def lace_schedule_slots(pairs, n_orb, per_batch):
    """Batch and slot of every pair for plans of real orbitals (host only).
    Returns (batch_of, slot_of, n)."""
    pr = np.ascontiguousarray(np.asarray(pairs, dtype=np.int32).reshape(-1, 2))
    pi = np.ascontiguousarray(pr[:, 0])
    pj = np.ascontiguousarray(pr[:, 1])
    bo = np.empty(pr.shape[0], dtype=np.int32)
    so = np.empty(pr.shape[0], dtype=np.int32)
    nb = ctypes.c_int64(0)
    P = ctypes.POINTER(ctypes.c_int32)
    _check(load().lace_schedule_slots(pi.ctypes.data_as(P), pj.ctypes.data_as(P),
                                      pr.shape[0], int(n_orb), int(per_batch),
                                      bo.ctypes.data_as(P), so.ctypes.data_as(P),
                                      ctypes.byref(nb)),
           "lace_schedule_slots")
    return bo, so, nb.value


def _vp(t):
    return None if t is None else t.data_ptr()


def lace_apply_exchange_batched(plan, jobs, graph=False, stream=None):
    """``jobs``: list of dicts with cell, psi_g, n_orb, s_thr, w_g and
    optional e_x, n_kept (int64 device tensor), sym, xi_g, m_out, ex_tr,
    info, plus ws (torch tensors).  Returns the kept pair count of each job:
    ints (after synchronizing the stream) when no job brings an n_kept
    tensor, else the n_kept tensors (None for a job without one)."""
    import torch
    arr = (LaceJob * len(jobs))()
    st = _stream_obj(stream)
    any_count = any(j.get("n_kept") is not None for j in jobs)
    counts = []
    for k, j in enumerate(jobs):
        n_orb, n_pw = int(j["n_orb"]), _n_pw(plan, j.get("cell", 0))
        for name in ("psi_g", "w_g", "xi_g"):
            _need(j.get(name), n_orb * n_pw, name)
        _need(j.get("m_out"), n_orb * n_orb, "m_out")
        for name in ("e_x", "ex_tr", "info", "n_kept"):
            _need(j.get(name), 1, name)
        for name in ("psi_g", "w_g", "xi_g", "m_out"):
            t = j.get(name)
            if t is not None:
                _ptr(t, torch.complex128, name)
        for name in ("e_x", "ex_tr"):
            t = j.get(name)
            if t is not None:
                _ptr(t, torch.float64, name)
        if j.get("info") is not None:
            _ptr(j["info"], torch.int32, "info")
        _ptr(j["ws"], None, "ws")
        arr[k].cell = int(j.get("cell", 0))
        arr[k].psi_g = _vp(j["psi_g"])
        arr[k].n_orb = int(j["n_orb"])
        arr[k].s_thr = float(j.get("s_thr", 0.0))
        arr[k].w_g = _vp(j["w_g"])
        arr[k].e_x = _vp(j.get("e_x"))
        if any_count:
            nk = j.get("n_kept")
        else:
            nk, _ = _count(None, st)
        if nk is not None:
            _ptr(nk, torch.int64, "n_kept")
        counts.append(nk)
        arr[k].n_kept = _vp(nk)
        arr[k].sym = SYM_MODES.get(j.get("sym", "avg"), 0) \
            if isinstance(j.get("sym", "avg"), str) else int(j["sym"])
        arr[k].xi_g = _vp(j.get("xi_g"))
        arr[k].m_out = _vp(j.get("m_out"))
        arr[k].ex_tr = _vp(j.get("ex_tr"))
        arr[k].info = _vp(j.get("info"))
        arr[k].ws = _vp(j["ws"])
        arr[k].ws_bytes = j["ws"].numel() * j["ws"].element_size()
    _check(load().lace_apply_exchange_batched(
        plan.handle, arr, len(jobs), LACE_BATCH_GRAPH if graph else 0,
        _stream(st)), "lace_apply_exchange_batched")
    if any_count:
        return counts
    st.synchronize()
    return [int(t.item()) for t in counts]


def lace_set_tuning(plan, cell, pairs_per_batch, use_plane, z_tile=0,
                    radix_order=0):
    _check(load().lace_set_tuning(plan.handle, cell, int(pairs_per_batch),
                                  int(use_plane), int(z_tile),
                                  int(radix_order)), "lace_set_tuning")


def lace_get_tuning(plan, cell):
    """(pairs_per_batch, use_plane, z_tile, radix_order) of the cell."""
    v = [ctypes.c_int() for _ in range(4)]
    _check(load().lace_get_tuning(plan.handle, cell, *[ctypes.byref(x) for x in v]),
           "lace_get_tuning")
    return tuple(x.value for x in v)


def lace_autotune(plan, cell, psi_g, n_orb, ws, stream=None, s_thr=0.0):
    """Time the pipeline candidates on this cell for the pairs S keeps at
    s_thr, keep the fastest.  Returns a list of (pairs_per_batch,
    use_plane, z_tile, radix_order, us_per_pair)."""
    import torch
    _need(psi_g, n_orb * _n_pw(plan, cell), "psi_g")
    cap = 64
    cols = [(ctypes.c_int * cap)() for _ in range(4)]
    us = (ctypes.c_double * cap)()
    n = ctypes.c_int(cap)
    _check(load().lace_autotune(plan.handle, cell,
                                _ptr(psi_g, torch.complex128, "psi_g"), n_orb,
                                float(s_thr), _ptr(ws, None, "ws"),
                                ws.numel() * ws.element_size(),
                                _stream(stream), *cols, us,
                                ctypes.byref(n)), "lace_autotune")
    return [(cols[0][k], cols[1][k], cols[2][k], cols[3][k], us[k])
            for k in range(min(n.value, cap))]
