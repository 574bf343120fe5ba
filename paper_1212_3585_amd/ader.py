"""Thin Python binding of the C ABI in include/ader.h (ctypes).

Argument marshalling only: every stage of the step runs in the HIP kernels of
libaderweno.so.  PyTorch provides device memory and the current stream.  The
module fails loudly when the library has not been built; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libaderweno.so")

OK, EINVAL, EUNSUPPORTED, EHIP, EWORKSPACE = 0, -1, -2, -3, -4
SYS_LINADV, SYS_EULER, SYS_MHD_GLM = 0, 1, 2
PREC_FP64, PREC_FP32_PREDICTOR = 0, 1
BC_PERIODIC, BC_TRANSMISSIVE = 0, 1
FLUX_RUSANOV, FLUX_OSHER = 0, 1
FLAG_NAN, FLAG_NONPHYSICAL, FLAG_NOCONV, FLAG_BADINDEX = 1, 2, 4, 8

# every symbol declared in include/ader.h
EXPORTS = [
    "ader_plan_create", "ader_plan_destroy", "ader_plan_nvar",
    "ader_workspace_bytes", "ader_clear_status", "ader_compute_dt", "ader_step",
    "ader_step_static",
    "ader_debug_reconstruct", "ader_debug_predict", "ader_debug_traces", "ader_read_status",
    "ader_debug_constants", "ader_profile_begin", "ader_profile_end", "ader_tune",
    "ader_set_tile_rows",
    "ader_level_workspace_bytes", "ader_step_level",
    "ader_server_create", "ader_server_destroy", "ader_server_footprint",
    "ader_server_submit", "ader_server_progress", "ader_server_request",
    "ader_server_stats_get",
    "ader_amr_create", "ader_amr_destroy", "ader_amr_level_cells", "ader_amr_set_level",
    "ader_amr_set_flags", "ader_amr_build", "ader_amr_regrid", "ader_amr_step", "ader_amr_clock",
    "ader_amr_tune",
    "ader_amr_get_level", "ader_amr_counts", "ader_amr_stats",
    "ader_status_string", "ader_last_error",
]
AMR_ABSENT, AMR_VMOTHER, AMR_ACTIVE, AMR_VCHILD = -2, -1, 0, 1
REQ_QUEUED, REQ_RESIDENT, REQ_DONE, REQ_FAILED = 0, 1, 2, 3
STAGES = ["dt", "weno", "predict", "flux", "update"]


class AderError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class CProblem(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("M", ctypes.c_int), ("system", ctypes.c_int),
        ("gamma", ctypes.c_double), ("ch", ctypes.c_double), ("adv", ctypes.c_double * 3),
        ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
        ("hi", ctypes.c_double * 3), ("bc", ctypes.c_int * 3),
        ("cfl", ctypes.c_double), ("flux", ctypes.c_int), ("precision", ctypes.c_int),
        ("picard_tol", ctypes.c_double), ("picard_max", ctypes.c_int),
    ]


class CLevelView(ctypes.Structure):
    _fields_ = [
        ("level", ctypes.c_int), ("dx", ctypes.c_double * 3),
        ("npred", ctypes.c_int64), ("pred_cells", ctypes.c_void_p),
        ("pred_patch", ctypes.c_void_p), ("nupd", ctypes.c_int64),
        ("upd", ctypes.c_void_p), ("upd_nbr", ctypes.c_void_p),
    ]


class CServerConfig(ctypes.Structure):
    _fields_ = [("hbm_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int),
                ("streams", ctypes.c_int), ("rounds_ahead", ctypes.c_int)]


class CRequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("flags", ctypes.c_uint32),
                ("steps", ctypes.c_uint64), ("picard_iterations", ctypes.c_uint64),
                ("t", ctypes.c_double), ("submit_s", ctypes.c_double),
                ("admit_s", ctypes.c_double), ("done_s", ctypes.c_double)]


class CServerStats(ctypes.Structure):
    _fields_ = [("arena_bytes", ctypes.c_size_t), ("bytes_in_use", ctypes.c_size_t),
                ("peak_bytes_in_use", ctypes.c_size_t), ("resident", ctypes.c_int),
                ("peak_resident", ctypes.c_int), ("queued", ctypes.c_int),
                ("rounds", ctypes.c_int64), ("launches", ctypes.c_int64),
                ("completed", ctypes.c_int64)]


class CAmrConfig(ctypes.Structure):
    _fields_ = [("r", ctypes.c_int), ("max_level", ctypes.c_int),
                ("indicator_var", ctypes.c_int), ("chi_ref", ctypes.c_double),
                ("chi_rec", ctypes.c_double), ("eps", ctypes.c_double), ("buffer", ctypes.c_int),
                ("use_graph", ctypes.c_int)]


_lib = None


def load_library():
    """Load libaderweno.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} not found: build it first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
    sig = {
        "ader_plan_create": [ctypes.POINTER(CProblem), ctypes.POINTER(vp)],
        "ader_plan_destroy": [vp],
        "ader_plan_nvar": [vp, ctypes.POINTER(ctypes.c_int)],
        "ader_workspace_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
        "ader_clear_status": [vp, vp, vp],
        "ader_compute_dt": [vp, vp, i64, dbl, dbl, vp, vp, vp],
        "ader_step": [vp, vp, vp, i64, vp, vp, vp],
        "ader_step_static": [vp, vp, vp, i64, vp, vp, vp],
        "ader_debug_reconstruct": [vp, vp, i64, vp, vp, vp],
        "ader_debug_predict": [vp, vp, i64, vp, vp, vp, vp],
        "ader_debug_traces": [vp, vp, i64, vp, vp, vp, vp],
        "ader_read_status": [vp, vp, ctypes.POINTER(ctypes.c_uint32),
                             ctypes.POINTER(ctypes.c_uint64), vp],
        "ader_debug_constants": [vp, vp, vp, vp, vp],
        "ader_profile_begin": [vp],
        "ader_tune": [vp, vp, i64, vp, vp, vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), vp],
        "ader_set_tile_rows": [vp, ctypes.c_int],
        "ader_profile_end": [vp, vp, vp],
        "ader_level_workspace_bytes": [vp, i64, ctypes.POINTER(ctypes.c_size_t)],
        "ader_step_level": [vp, ctypes.POINTER(CLevelView), vp, vp, i64, vp, vp, vp],
        "ader_server_create": [ctypes.POINTER(CServerConfig), ctypes.POINTER(vp)],
        "ader_server_destroy": [vp],
        "ader_server_footprint": [ctypes.POINTER(CProblem), ctypes.POINTER(ctypes.c_size_t)],
        "ader_server_submit": [vp, ctypes.POINTER(CProblem), vp, dbl, vp,
                               ctypes.POINTER(i64)],
        "ader_server_progress": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                 ctypes.POINTER(ctypes.c_int)],
        "ader_server_request": [vp, i64, ctypes.POINTER(CRequestInfo)],
        "ader_server_stats_get": [vp, ctypes.POINTER(CServerStats)],
        "ader_amr_create": [ctypes.POINTER(CProblem), ctypes.POINTER(CAmrConfig),
                            ctypes.POINTER(vp)],
        "ader_amr_destroy": [vp],
        "ader_amr_level_cells": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
        "ader_amr_set_level": [vp, ctypes.c_int, vp],
        "ader_amr_set_flags": [vp, ctypes.c_int, vp],
        "ader_amr_build": [vp],
        "ader_amr_regrid": [vp, ctypes.POINTER(ctypes.c_int)],
        "ader_amr_tune": [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                          ctypes.POINTER(ctypes.c_int), vp],
        "ader_amr_step": [vp, dbl, vp],
        "ader_amr_clock": [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), ctypes.POINTER(dbl)],
        "ader_amr_get_level": [vp, ctypes.c_int, vp, vp],
        "ader_amr_counts": [vp, ctypes.c_int, ctypes.POINTER(i64)],
        "ader_amr_stats": [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64),
                           ctypes.POINTER(ctypes.c_uint64)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.ader_status_string.argtypes = [ctypes.c_int]
    lib.ader_status_string.restype = ctypes.c_char_p
    lib.ader_last_error.argtypes = []
    lib.ader_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != OK:
        msg = load_library().ader_last_error().decode()
        raise AderError(status, where, msg)


def require_gpu():
    """Raise unless a HIP device and the built library are both present."""
    import torch
    load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device visible")


@dataclass
class Problem:
    dim: int = 2
    M: int = 2
    system: int = SYS_EULER
    gamma: float = 1.4
    ch: float = 2.0
    adv: tuple = (1.0, 1.0, 1.0)
    n: tuple = (20, 20, 1)
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc: tuple = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    cfl: float = 0.9
    flux: int = FLUX_RUSANOV
    precision: int = PREC_FP64
    picard_tol: float = 1e-14
    picard_max: int = 64

    def to_c(self) -> CProblem:
        c = CProblem()
        c.dim, c.M, c.system = self.dim, self.M, self.system
        c.gamma = self.gamma
        c.ch = self.ch
        c.adv[:] = list(self.adv)[:3] + [0.0] * (3 - len(self.adv))
        c.n[:] = list(self.n)[:3] + [1] * (3 - len(self.n))
        c.lo[:] = list(self.lo)[:3] + [0.0] * (3 - len(self.lo))
        c.hi[:] = list(self.hi)[:3] + [1.0] * (3 - len(self.hi))
        c.bc[:] = list(self.bc)[:3] + [0] * (3 - len(self.bc))
        c.cfl = self.cfl
        c.flux = self.flux
        c.precision = self.precision
        c.picard_tol = self.picard_tol
        c.picard_max = self.picard_max
        return c

    @property
    def ncells(self) -> int:
        return int(np.prod(list(self.n)[:self.dim]))


def _ptr(t) -> int:
    return t.data_ptr()


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """A plan plus its device workspace.  Tensors are fp64 on the HIP device."""

    def __init__(self, problem: Problem, device="cuda"):
        import torch
        self.lib = load_library()
        self.problem = problem
        self._plan = ctypes.c_void_p()
        cp = problem.to_c()
        _check(self.lib.ader_plan_create(ctypes.byref(cp), ctypes.byref(self._plan)),
               "ader_plan_create")
        nv = ctypes.c_int()
        _check(self.lib.ader_plan_nvar(self._plan, ctypes.byref(nv)), "ader_plan_nvar")
        self.nvar = nv.value
        nb = ctypes.c_size_t()
        _check(self.lib.ader_workspace_bytes(self._plan, ctypes.byref(nb)),
               "ader_workspace_bytes")
        self.workspace_bytes = nb.value
        self.device = torch.device(device)
        # torch's caching allocator returns 256-byte aligned blocks
        self.ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=self.device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.clear_status()

    def __del__(self):
        try:
            if self._plan:
                self.lib.ader_plan_destroy(self._plan)
                self._plan = ctypes.c_void_p()
        except Exception:
            pass

    @property
    def ncells(self) -> int:
        return self.problem.ncells

    def empty_state(self, ld=None):
        import torch
        ld = self.ncells if ld is None else ld
        return torch.zeros((self.nvar, ld), dtype=torch.float64, device=self.device)

    def clear_status(self, stream=None):
        _check(self.lib.ader_clear_status(self._plan, _ptr(self.ws), _stream(stream)),
               "ader_clear_status")

    def compute_dt(self, u, t=0.0, t_end=float("inf"), dt_out=None, stream=None):
        dt_out = self.dt if dt_out is None else dt_out
        _check(self.lib.ader_compute_dt(self._plan, _ptr(u), u.shape[1], t, t_end,
                                        _ptr(dt_out), _ptr(self.ws), _stream(stream)),
               "ader_compute_dt")
        return dt_out

    def step(self, u_in, u_out, dt=None, stream=None):
        dt = self.dt if dt is None else dt
        _check(self.lib.ader_step(self._plan, _ptr(u_in), _ptr(u_out), u_in.shape[1],
                                  _ptr(dt), _ptr(self.ws), _stream(stream)), "ader_step")
        return u_out

    def step_static(self, u_in, u_out, dt=None, status=None, stream=None):
        """ader_step_static: the step on the library's static device workspace
        (no workspace argument); status: None or a device int32/uint32 tensor
        of two entries (status bits, Picard sweeps of this call)."""
        dt = self.dt if dt is None else dt
        _check(self.lib.ader_step_static(self._plan, _ptr(u_in), _ptr(u_out), u_in.shape[1],
                                         _ptr(dt), None if status is None else _ptr(status),
                                         _stream(stream)), "ader_step_static")
        return u_out

    def reconstruct(self, u, stream=None):
        import torch
        n = self.problem.M + 1
        wh = torch.empty(self.ncells * self.nvar * n ** self.problem.dim,
                         dtype=torch.float64, device=self.device)
        _check(self.lib.ader_debug_reconstruct(self._plan, _ptr(u), u.shape[1], _ptr(wh),
                                               _ptr(self.ws), _stream(stream)),
               "ader_debug_reconstruct")
        return wh

    def predict(self, wh, ncells, dt=None, stream=None):
        import torch
        n = self.problem.M + 1
        dt = self.dt if dt is None else dt
        qh = torch.empty(max(ncells, 1) * self.nvar * n ** (self.problem.dim + 1),
                         dtype=torch.float64, device=self.device)
        _check(self.lib.ader_debug_predict(self._plan, _ptr(wh), ncells, _ptr(qh), _ptr(dt),
                                           _ptr(self.ws), _stream(stream)),
               "ader_debug_predict")
        return qh

    def traces(self, u, dt=None, stream=None):
        """Face traces of the fused 2D cell kernel: [4 faces, cells, nvar, s, b]
        (faces x-low, x-high, y-low, y-high; s time node, b transverse node)."""
        import torch
        n = self.problem.M + 1
        dt = self.dt if dt is None else dt
        tr = torch.empty((4, self.ncells, self.nvar, n, n), dtype=torch.float64,
                         device=self.device)
        _check(self.lib.ader_debug_traces(self._plan, _ptr(u), u.shape[1], _ptr(dt), _ptr(tr),
                                          _ptr(self.ws), _stream(stream)),
               "ader_debug_traces")
        return tr

    def read_status(self, stream=None):
        flags = ctypes.c_uint32()
        iters = ctypes.c_uint64()
        _check(self.lib.ader_read_status(self._plan, _ptr(self.ws), ctypes.byref(flags),
                                         ctypes.byref(iters), _stream(stream)),
               "ader_read_status")
        return flags.value, iters.value

    def constants(self):
        n = self.problem.M + 1
        arrs = [np.zeros(n), np.zeros(n), np.zeros(n * n), np.zeros(n * n)]
        _check(self.lib.ader_debug_constants(
            self._plan, *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs]),
            "ader_debug_constants")
        return {"nodes": arrs[0], "weights": arrs[1], "dmat": arrs[2].reshape(n, n),
                "time_inv_w": arrs[3].reshape(n, n)}

    def tune(self, u, dt=None, reps=5, stream=None):
        """Pick the fused 2D cell kernel's tile height on this state; returns
        (rows, {rows: mean ms per launch})."""
        dt = self.dt if dt is None else dt
        rows = ctypes.c_int()
        ms = np.zeros(4)
        _check(self.lib.ader_tune(self._plan, _ptr(u), u.shape[1], _ptr(dt), _ptr(self.ws),
                                  _stream(stream), int(reps), ctypes.byref(rows),
                                  ms.ctypes.data_as(ctypes.c_void_p)), "ader_tune")
        return rows.value, {r: float(m) for r, m in zip((2, 4, 8, 16), ms) if m >= 0}

    def set_tile_rows(self, rows):
        _check(self.lib.ader_set_tile_rows(self._plan, int(rows)), "ader_set_tile_rows")

    def profile_begin(self):
        _check(self.lib.ader_profile_begin(self._plan), "ader_profile_begin")

    def profile_end(self):
        """{stage: (total milliseconds, launches)} since profile_begin."""
        ms = np.zeros(len(STAGES))
        cnt = np.zeros(len(STAGES), dtype=np.int64)
        _check(self.lib.ader_profile_end(self._plan, ms.ctypes.data_as(ctypes.c_void_p),
                                         cnt.ctypes.data_as(ctypes.c_void_p)),
               "ader_profile_end")
        return {name: (float(ms[i]), int(cnt[i])) for i, name in enumerate(STAGES)}

    def step_level(self, pred_cells, pred_patch, upd, upd_nbr, dx, u_in, u_out, dt=None,
                   level=0, stream=None):
        """One step over a level's cell lists (int32 device tensors; see
        ader_step_level).  Allocates the level workspace on first use."""
        import torch
        npred = int(pred_cells.numel())
        nb = ctypes.c_size_t()
        _check(self.lib.ader_level_workspace_bytes(self._plan, npred, ctypes.byref(nb)),
               "ader_level_workspace_bytes")
        if getattr(self, "_lws", None) is None or self._lws.numel() < nb.value:
            self._lws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
            self._lws[:1024].zero_()
        view = CLevelView()
        view.level = level
        view.dx[:] = list(dx)[:3] + [1.0] * (3 - len(dx))
        view.npred = npred
        view.pred_cells = _ptr(pred_cells) if npred else None
        view.pred_patch = _ptr(pred_patch) if npred else None
        view.nupd = int(upd.numel())
        view.upd = _ptr(upd) if view.nupd else None
        view.upd_nbr = _ptr(upd_nbr) if view.nupd else None
        dt = self.dt if dt is None else dt
        _check(self.lib.ader_step_level(self._plan, ctypes.byref(view), _ptr(u_in), _ptr(u_out),
                                        u_in.shape[1], _ptr(dt), _ptr(self._lws),
                                        _stream(stream)), "ader_step_level")
        return u_out

    def read_level_status(self, stream=None):
        flags = ctypes.c_uint32()
        iters = ctypes.c_uint64()
        _check(self.lib.ader_read_status(self._plan, _ptr(self._lws), ctypes.byref(flags),
                                         ctypes.byref(iters), _stream(stream)),
               "ader_read_status")
        return flags.value, iters.value

    def run(self, u, t_end, max_steps=10**9, stream=None):
        """Advance u to t_end; returns (u, t, steps).  Reads dt back each step."""
        import torch
        t = 0.0
        steps = 0
        a, b = u.clone(), torch.empty_like(u)
        while t < t_end and steps < max_steps:
            self.compute_dt(a, t, t_end, stream=stream)
            self.step(a, b, stream=stream)
            dt = float(self.dt.item())
            t += dt
            steps += 1
            a, b = b, a
        return a, t, steps


class Server:
    """Solve server (ader_server_*): queue independent 2D solves, drive them
    with progress(), read results and per-request timings.

    Initial averages are numpy arrays [nvar, cells] or [nvar, nx, ny]
    (x fastest in the flat form); results come back in the same shape."""

    def __init__(self, hbm_bytes=8 << 30, max_slots=256, streams=4, rounds_ahead=2):
        self.lib = load_library()
        cfg = CServerConfig(hbm_bytes, max_slots, streams, rounds_ahead)
        h = ctypes.c_void_p()
        _check(self.lib.ader_server_create(ctypes.byref(cfg), ctypes.byref(h)),
               "ader_server_create")
        self._h = h
        self._out = {}

    def close(self):
        if getattr(self, "_h", None):
            self.lib.ader_server_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @staticmethod
    def footprint(problem: Problem) -> int:
        b = ctypes.c_size_t()
        cp = problem.to_c()
        _check(load_library().ader_server_footprint(ctypes.byref(cp), ctypes.byref(b)),
               "ader_server_footprint")
        return b.value

    def submit(self, problem: Problem, u0: np.ndarray, t_end: float) -> int:
        u0c = np.ascontiguousarray(u0, dtype=np.float64)
        shape = u0c.shape
        flat = u0c.reshape(shape[0], -1)
        if shape[1:] and len(shape) == 3:   # [nv, nx, ny] -> x fastest
            flat = np.ascontiguousarray(np.transpose(u0c, (0, 2, 1))).reshape(shape[0], -1)
        out = np.empty_like(flat)
        cp = problem.to_c()
        rid = ctypes.c_int64()
        _check(self.lib.ader_server_submit(self._h, ctypes.byref(cp),
                                           flat.ctypes.data_as(ctypes.c_void_p), float(t_end),
                                           out.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.byref(rid)), "ader_server_submit")
        self._out[rid.value] = (out, shape)
        return rid.value

    def progress(self, wait=False):
        r, q = ctypes.c_int(), ctypes.c_int()
        _check(self.lib.ader_server_progress(self._h, int(bool(wait)), ctypes.byref(r),
                                             ctypes.byref(q)), "ader_server_progress")
        return r.value, q.value

    def info(self, rid: int) -> dict:
        inf = CRequestInfo()
        _check(self.lib.ader_server_request(self._h, rid, ctypes.byref(inf)),
               "ader_server_request")
        return {f: getattr(inf, f) for f, _ in CRequestInfo._fields_}

    def result(self, rid: int) -> np.ndarray:
        out, shape = self._out[rid]
        if len(shape) == 3:
            return np.transpose(out.reshape(shape[0], shape[2], shape[1]), (0, 2, 1)).copy()
        return out.reshape(shape)

    def stats(self) -> dict:
        st = CServerStats()
        _check(self.lib.ader_server_stats_get(self._h, ctypes.byref(st)),
               "ader_server_stats_get")
        return {f: getattr(st, f) for f, _ in CServerStats._fields_}

    def drain(self, ids=None):
        """Drive progress() until the given requests (default: all) are done
        or failed."""
        ids = list(self._out) if ids is None else list(ids)
        while True:
            self.progress(wait=True)
            if all(self.info(i)["state"] >= REQ_DONE for i in ids):
                return


def _flat_x_fastest(U):
    """[nv, nx, ny(, nz)] -> [nv, cells] with x fastest."""
    nv = U.shape[0]
    d = U.ndim - 1
    return np.ascontiguousarray(np.transpose(U, (0,) + tuple(range(d, 0, -1)))).reshape(nv, -1)


def _unflat_x_fastest(F, shape):
    d = len(shape)
    G = F.reshape((F.shape[0],) + tuple(reversed(shape)))
    return np.ascontiguousarray(np.transpose(G, (0,) + tuple(range(d, 0, -1))))


class Amr:
    """AMR mesh with local time stepping (ader_amr_*).  Level data are numpy
    arrays [nvar, nx, ny(, nz)] over each level's whole index space."""

    def __init__(self, problem: Problem, r=3, max_level=1, indicator_var=0, chi_ref=0.2,
                 eps=0.01, buffer=1, use_graph=True, chi_rec=None):
        self.lib = load_library()
        self.problem = problem
        self.L = max_level
        chi_rec = chi_ref if chi_rec is None else chi_rec
        cfg = CAmrConfig(r, max_level, indicator_var, chi_ref, chi_rec, eps, buffer,
                         int(bool(use_graph)))
        h = ctypes.c_void_p()
        _check(self.lib.ader_amr_create(ctypes.byref(problem.to_c()), ctypes.byref(cfg),
                                        ctypes.byref(h)), "ader_amr_create")
        self._h = h
        self.shapes = []
        for l in range(max_level + 1):
            n = (ctypes.c_int * 3)()
            _check(self.lib.ader_amr_level_cells(h, l, n), "ader_amr_level_cells")
            self.shapes.append(tuple(n[:problem.dim]))

    def close(self):
        if getattr(self, "_h", None):
            self.lib.ader_amr_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def set_level(self, level, U):
        F = np.ascontiguousarray(_flat_x_fastest(np.asarray(U, dtype=np.float64)))
        _check(self.lib.ader_amr_set_level(self._h, level, F.ctypes.data_as(ctypes.c_void_p)),
               "ader_amr_set_level")

    def set_flags(self, level, flags):
        f = np.ascontiguousarray(_flat_x_fastest(np.asarray(flags, dtype=np.uint8)[None])[0])
        _check(self.lib.ader_amr_set_flags(self._h, level, f.ctypes.data_as(ctypes.c_void_p)),
               "ader_amr_set_flags")

    def build(self):
        _check(self.lib.ader_amr_build(self._h), "ader_amr_build")

    def regrid(self):
        """Refine and recoarsen at the current time; True when the mesh changed."""
        ch = ctypes.c_int()
        _check(self.lib.ader_amr_regrid(self._h, ctypes.byref(ch)), "ader_amr_regrid")
        return bool(ch.value)

    def tune(self, reps=3):
        """Pick the AMR kernels' block shapes (after a step); returns
        (pred_block, flux_block, {"predict": {block: ms}, "flux": {...}})."""
        pb, fb = ctypes.c_int(), ctypes.c_int()
        ms = np.zeros(6)
        _check(self.lib.ader_amr_tune(self._h, int(reps), ctypes.byref(pb), ctypes.byref(fb),
                                      ms.ctypes.data_as(ctypes.c_void_p)), "ader_amr_tune")
        sizes = (128, 256, 512)
        return pb.value, fb.value, {
            "predict": {b: float(m) for b, m in zip(sizes, ms[:3]) if m >= 0},
            "flux": {b: float(m) for b, m in zip(sizes, ms[3:]) if m >= 0}}

    def step(self, t_end, stream=None):
        _check(self.lib.ader_amr_step(self._h, float(t_end), _stream(stream)), "ader_amr_step")

    def clock(self):
        t, dt0 = ctypes.c_double(), ctypes.c_double()
        steps = ctypes.c_int64()
        _check(self.lib.ader_amr_clock(self._h, ctypes.byref(t), ctypes.byref(steps),
                                       ctypes.byref(dt0)), "ader_amr_clock")
        return t.value, steps.value, dt0.value

    def run(self, t_end, max_steps=10 ** 9, regrid_every=0):
        """Level-0 steps until t_end (reads the clock after each step); with
        regrid_every = k > 0 a regrid follows every k-th step."""
        t, steps, _ = self.clock()
        while t < t_end and steps < max_steps:
            self.step(t_end)
            t, steps, _ = self.clock()
            if regrid_every > 0 and steps % regrid_every == 0:
                self.regrid()
        return t, steps

    def level(self, level):
        """(U[nvar, *shape], status[*shape]) of a level."""
        nv = self.nvar
        N = int(np.prod(self.shapes[level]))
        F = np.empty((nv, N))
        st = np.empty(N, dtype=np.int8)
        _check(self.lib.ader_amr_get_level(self._h, level, F.ctypes.data_as(ctypes.c_void_p),
                                           st.ctypes.data_as(ctypes.c_void_p)),
               "ader_amr_get_level")
        return (_unflat_x_fastest(F, self.shapes[level]),
                _unflat_x_fastest(st[None], self.shapes[level])[0])

    @property
    def nvar(self):
        s = self.problem.system
        return 1 if s == SYS_LINADV else (self.problem.dim + 2 if s == SYS_EULER else 9)

    def counts(self, level):
        c = (ctypes.c_int64 * 3)()
        _check(self.lib.ader_amr_counts(self._h, level, c), "ader_amr_counts")
        return {"active": c[0], "vchild": c[1], "vmother": c[2]}

    def stats(self):
        f, it, cu = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(self.lib.ader_amr_stats(self._h, ctypes.byref(f), ctypes.byref(it),
                                       ctypes.byref(cu)), "ader_amr_stats")
        return {"flags": f.value, "picard_iterations": it.value, "cell_updates": cu.value}
