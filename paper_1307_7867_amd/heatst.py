"""Python binding of libheatst (include/heatst.h): argument marshalling only.

Every step of the solver runs in the HIP kernels of libheatst.so; PyTorch
provides device memory (the plan workspace and user tensors) and streams.
If the shared library has not been built, importing the binding works but
any use raises RuntimeError -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libheatst.so")
TUNE_CACHE = os.path.join(HERE, "tune_cache.json")

HS_OK, HS_EINVAL, HS_ENOMEM, HS_ENOCONV, HS_ENONFINITE, HS_EDEVICE, HS_ESTATE, HS_PENDING = \
    0, -1, -2, -3, -4, -5, -6, 1
HS_FP64, HS_MIXED = 0, 1
HS_ORDER_COMPACT = -4   # level order code of the compact fourth-order pair


class HeatstError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} ({status})")


class LevelDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("order", C.c_int32), ("nnodes", C.c_int32)]


class MgDesc(C.Structure):
    _fields_ = [("nu1", C.c_int32), ("nu2", C.c_int32), ("omega", C.c_double),
                ("n_coarsest", C.c_int32), ("tol", C.c_double), ("max_cycles", C.c_int32),
                ("fixed_cycles", C.c_int32), ("precision", C.c_int32), ("inner_nu1", C.c_int32),
                ("inner_nu2", C.c_int32), ("fused_sweeps", C.c_int32), ("cycle_graphs", C.c_int32)]


class ProblemDesc(C.Structure):
    _fields_ = [("nu", C.c_double), ("t0", C.c_double), ("dt", C.c_double),
                ("forcing_c", C.c_double), ("nsteps", C.c_int32), ("nlevels", C.c_int32),
                ("lev", LevelDesc * 3), ("mg", MgDesc), ("sweeps", C.c_int32),
                ("sdc_tol", C.c_double), ("max_sweeps", C.c_int32), ("batch", C.c_int32),
                ("nslices", C.c_int32), ("h_lane_n", C.POINTER(C.c_int32)),
                ("pfasst_pred_sweeps", C.c_int32), ("lane_memory", C.c_int32),
                ("sdc_node_parallel", C.c_int32), ("pfasst_groups", C.c_int32),
                ("fas_interp", C.c_int32)]


class LaneStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("steps_done", C.c_int32), ("total_sweeps", C.c_int32),
                ("total_solves", C.c_int32), ("total_cycles", C.c_int64),
                ("max_cycles", C.c_int32), ("failed_solves", C.c_int32),
                ("last_rho", C.c_double), ("last_sdc_res", C.c_double),
                ("level_cycles", C.c_int64 * 3)]


class ServerDesc(C.Structure):
    _fields_ = [("order", C.c_int32), ("nnodes", C.c_int32), ("mg", MgDesc), ("sweeps", C.c_int32),
                ("sdc_tol", C.c_double), ("max_sweeps", C.c_int32), ("forcing_c", C.c_double),
                ("nclasses", C.c_int32), ("class_n", C.c_int32 * 8), ("class_slots", C.c_int32 * 8)]


class RequestInfo(C.Structure):
    _fields_ = [("state", C.c_int32), ("status", C.c_int32), ("cls", C.c_int32), ("lane", C.c_int32),
                ("t_submit", C.c_double), ("t_admit", C.c_double), ("t_done", C.c_double),
                ("stats", LaneStats)]


_lib = None
_V = C.c_void_p
_P = C.POINTER


def lib():
    """Load libheatst.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "or python paper_1307_7867_amd/build.py")
    L = C.CDLL(LIB_PATH)
    S = C.c_int
    L.hs_status_string.restype = C.c_char_p
    L.hs_status_string.argtypes = [S]
    sig = {
        "hs_collocation": [C.c_int32, _V, _V],
        "hs_workspace_bytes": [_P(ProblemDesc), _P(C.c_size_t)],
        "hs_plan_create": [_P(ProblemDesc), _P(_V)],
        "hs_plan_bind": [_V, _V, C.c_size_t, _V],
        "hs_plan_destroy": [_V],
        "hs_plan_lanes": [_V, _P(C.c_int32), _V],
        "hs_set_lane": [_V, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_int32, _V],
        "hs_lap_apply": [_V, C.c_int32, C.c_double, C.c_double, _V, _V, _V],
        "hs_heat_rhs": [_V, C.c_int32, _V, _V, _V, _V, _V],
        "hs_mg_vcycle": [_V, C.c_int32, _V, _V, _V, _V],
        "hs_smooth": [_V, C.c_int32, _V, _V, _V, _V, C.c_int32, _V],
        "hs_mg_solve_static": [C.c_int32, C.c_int32, C.c_double, _V, _V, _V, _V],
        "hs_compact_apply": [C.c_int32, C.c_int32, C.c_double, C.c_double, _V, _V, _V],
        "hs_plan_timer": [_V, C.c_int32, C.c_int32],
        "hs_plan_timer_read": [_V, _P(C.c_int32), _P(C.c_double)],
        "hs_tune_set": [C.c_int32] * 6,
        "hs_tune_clear": [],
        "hs_tune_load": [C.c_char_p, _P(C.c_int32)],
        "hs_tune_lookup": [C.c_int32] * 4 + [_P(C.c_int32), _P(C.c_int32)],
        "hs_set_state": [_V, _V, _V],
        "hs_get_state": [_V, _V, _V],
        "hs_get_nodes": [_V, C.c_int32, _V, _V, _V, _V, _V],
        "hs_set_nodes": [_V, C.c_int32, _V, _V, _V],
        "hs_begin_step": [_V, _V],
        "hs_sdc_sweep": [_V, C.c_int32, _V],
        "hs_fas_restrict": [_V, _V],
        "hs_fas_interp": [_V, _V],
        "hs_mlsdc_iter": [_V, _V],
        "hs_end_step": [_V, _V],
        "hs_step": [_V, _V],
        "hs_solve": [_V, _V],
        "hs_pfasst_run": [_V, _V],
        "hs_solve_graph": [_V, _V],
        "hs_stats_read": [_V, _V, _V],
        "hs_set_lane_state": [_V, C.c_int32, _V, _V],
        "hs_get_lane_state": [_V, C.c_int32, _V, _V],
        "hs_server_pool_bytes": [_P(ServerDesc), _P(C.c_size_t), _P(C.c_size_t)],
        "hs_server_request_bytes": [_P(ServerDesc), C.c_int32, _P(C.c_size_t)],
        "hs_server_resident": [_V, _P(C.c_size_t), _P(C.c_size_t)],
        "hs_lane_bytes": [_P(ProblemDesc), C.c_int32, _P(C.c_size_t)],
        "hs_plan_bind_lane": [_V, C.c_int32, _V, C.c_size_t, _V],
        "hs_plan_unbind_lane": [_V, C.c_int32],
        "hs_server_create": [_P(ServerDesc), _V, C.c_size_t, C.c_size_t, _P(_V)],
        "hs_server_submit": [_V, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_int32, _V, _V,
                             _P(C.c_uint64)],
        "hs_server_poll": [_V, C.c_uint64, _P(RequestInfo)],
        "hs_server_drain": [_V],
        "hs_server_destroy": [_V],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.restype = S
        f.argtypes = args
    _lib = L
    # launch shapes tuned on this GPU model (paper_1307_7867_amd/tune.py), unless
    # HEATST_TUNE_CACHE names another file or is empty (built-in shapes)
    path = os.environ.get("HEATST_TUNE_CACHE", TUNE_CACHE)
    if path and os.path.exists(path):
        cnt = C.c_int32(0)
        check(L.hs_tune_load(os.fsencode(path), C.byref(cnt)), "hs_tune_load")
    return L


def status_string(s: int) -> str:
    try:
        return lib().hs_status_string(s).decode()
    except RuntimeError:
        return "libheatst not loaded"


def check(status: int, where: str, allow=()) -> int:
    if status < 0 and status not in allow:
        raise HeatstError(status, where)
    return status


def collocation(M: int):
    """Nodes tau[M] and collocation matrix Q[M, M] (eq. (6)) used by the GPU path."""
    tau = np.zeros(M)
    Q = np.zeros((M, M))
    check(lib().hs_collocation(M, tau.ctypes.data_as(_V), Q.ctypes.data_as(_V)), "hs_collocation")
    return tau, Q


HS_STATIC_MAX_N = 63


HS_TIMER_PJAC, HS_TIMER_RESID_FW, HS_TIMER_SWEEP1, HS_TIMER_SWEEP2, HS_TIMER_FP32 = 1, 2, 3, 4, 16


def tune_set(n, order, precision, batch, zb, zb_rfw):
    check(lib().hs_tune_set(n, order, precision, batch, zb, zb_rfw), "hs_tune_set")


def tune_clear():
    check(lib().hs_tune_clear(), "hs_tune_clear")


def tune_load(path) -> int:
    cnt = C.c_int32(0)
    check(lib().hs_tune_load(os.fsencode(path), C.byref(cnt)), "hs_tune_load")
    return cnt.value


def tune_lookup(n, order, precision, batch):
    zb, zr = C.c_int32(0), C.c_int32(0)
    check(lib().hs_tune_lookup(n, order, precision, batch, C.byref(zb), C.byref(zr)), "hs_tune_lookup")
    return zb.value, zr.value


def mg_solve_static(u, b, a, n, order, nu1=2, nu2=1, omega=6.0 / 7.0, n_coarsest=3, tol=1e-12,
                    max_cycles=60, fixed_cycles=0, precision=HS_FP64, inner=(2, 2), stream=None,
                    allow=()):
    """hs_mg_solve_static: solve (I - a L_h) u = b on one n^3 grid in place on
    the device tensor u, with no plan and no device allocation (the library's
    static scratch holds everything else).  Returns the status."""
    d = MgDesc(nu1, nu2, omega, n_coarsest, tol, max_cycles, fixed_cycles, precision, inner[0], inner[1], 1, 0)
    s = lib().hs_mg_solve_static(n, order, a, C.byref(d), _ptr(u), _ptr(b), _stream(stream))
    return check(s, "hs_mg_solve_static", allow=allow)


def compact_apply(u, y, n, batch, alpha, beta, stream=None):
    """hs_compact_apply: y = alpha B_h u + beta A_h u (the compact pair) on
    `batch` packed n^3 grids of the device tensors u and y."""
    check(lib().hs_compact_apply(n, batch, alpha, beta, _ptr(u), _ptr(y), _stream(stream)), "hs_compact_apply")


@dataclass
class Problem:
    """Python mirror of hs_problem (see include/heatst.h)."""
    n: int = 15
    order: int = 2
    nnodes: int = 3
    nu: float = 0.1
    t0: float = 0.0
    dt: float = 0.125
    forcing_c: float = 3.0
    nsteps: int = 1
    coarse: tuple | None = None          # (n, order, nnodes) of the coarse MLSDC level
    coarse2: tuple | None = None         # (n, order, nnodes) of a third, coarsest level
    nu1: int = 2
    nu2: int = 1
    omega: float = 6.0 / 7.0
    n_coarsest: int = 3
    tol: float = 1e-12
    max_cycles: int = 60
    fixed_cycles: int = 0
    precision: int = HS_FP64
    inner_nu1: int = 2
    inner_nu2: int = 2
    fused_sweeps: int = 1
    cycle_graphs: int = 0
    sweeps: int = 4
    sdc_tol: float = 1e-10
    max_sweeps: int = 20
    batch: int = 1
    nslices: int = 1
    lane_n: list | None = None
    pfasst_pred_sweeps: int = 0
    sdc_node_parallel: int = 0
    pfasst_groups: int = 0
    fas_interp: int = 0

    def desc(self):
        d = ProblemDesc()
        d.nu, d.t0, d.dt, d.forcing_c = self.nu, self.t0, self.dt, self.forcing_c
        d.nsteps = self.nsteps
        d.nlevels = (3 if self.coarse2 else 2) if self.coarse else 1
        d.lev[0] = LevelDesc(self.n, self.order, self.nnodes)
        if self.coarse:
            d.lev[1] = LevelDesc(*self.coarse)
        if self.coarse and self.coarse2:
            d.lev[2] = LevelDesc(*self.coarse2)
        d.mg = MgDesc(self.nu1, self.nu2, self.omega, self.n_coarsest, self.tol, self.max_cycles,
                      self.fixed_cycles, self.precision, self.inner_nu1, self.inner_nu2,
                      self.fused_sweeps, self.cycle_graphs)
        d.sweeps, d.sdc_tol, d.max_sweeps = self.sweeps, self.sdc_tol, self.max_sweeps
        d.batch, d.nslices = self.batch, self.nslices
        d.pfasst_pred_sweeps = self.pfasst_pred_sweeps
        d.sdc_node_parallel = self.sdc_node_parallel
        d.pfasst_groups = self.pfasst_groups
        d.fas_interp = self.fas_interp
        keep = None
        if self.lane_n is not None:
            keep = (C.c_int32 * len(self.lane_n))(*self.lane_n)
            d.h_lane_n = C.cast(keep, _P(C.c_int32))
        return d, keep

    def workspace_bytes(self) -> int:
        d, keep = self.desc()
        out = C.c_size_t(0)
        check(lib().hs_workspace_bytes(C.byref(d), C.byref(out)), "hs_workspace_bytes")
        return out.value


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A bound plan: owns its workspace tensor on the current CUDA (HIP) device."""

    def __init__(self, problem: Problem, stream=None):
        import torch
        self.problem = problem
        L = lib()
        self._desc, self._keep = problem.desc()
        size = C.c_size_t(0)
        check(L.hs_workspace_bytes(C.byref(self._desc), C.byref(size)), "hs_workspace_bytes")
        self.bytes = size.value
        self._h = C.c_void_p()
        check(L.hs_plan_create(C.byref(self._desc), C.byref(self._h)), "hs_plan_create")
        self.ws = torch.empty(self.bytes + 256, dtype=torch.uint8, device="cuda")
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        self.stream = stream
        check(L.hs_plan_bind(self._h, C.c_void_p(aligned), self.bytes, _stream(stream)), "hs_plan_bind")
        lanes = C.c_int32(0)
        check(L.hs_plan_lanes(self._h, C.byref(lanes), None), "hs_plan_lanes")
        self.lanes = lanes.value
        ln = (C.c_int32 * self.lanes)()
        check(L.hs_plan_lanes(self._h, None, C.cast(ln, _V)), "hs_plan_lanes")
        self.lane_n = list(ln)
        self.nlevels = 2 if problem.coarse else 1

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                lib().hs_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass

    # geometry -----------------------------------------------------------
    def level_n(self, level):
        return [n if level == 0 else (n - 1) // 2 for n in self.lane_n]

    def level_M(self, level):
        return self.problem.nnodes if level == 0 else self.problem.coarse[2]

    def field_len(self, level=0):
        return sum(n ** 3 for n in self.level_n(level))

    def _s(self):
        return _stream(self.stream)

    # kernel-level calls -------------------------------------------------
    def lap_apply(self, u, alpha, beta, level=0, out=None):
        import torch
        y = torch.empty_like(u) if out is None else out
        check(lib().hs_lap_apply(self._h, level, alpha, beta, _ptr(u), _ptr(y), self._s()), "hs_lap_apply")
        return y

    def heat_rhs(self, u, t, level=0):
        import torch
        tt = (C.c_double * self.lanes)(*([t] * self.lanes if np.isscalar(t) else list(t)))
        fi = torch.empty_like(u)
        fe = torch.empty_like(u)
        check(lib().hs_heat_rhs(self._h, level, _ptr(u), C.cast(tt, _V), _ptr(fi), _ptr(fe), self._s()),
              "hs_heat_rhs")
        return fi, fe

    def mg_vcycle(self, u, b, a, level=0, allow_noconv=False):
        aa = (C.c_double * self.lanes)(*([a] * self.lanes if np.isscalar(a) else list(a)))
        s = lib().hs_mg_vcycle(self._h, level, C.cast(aa, _V), _ptr(u), _ptr(b), self._s())
        return check(s, "hs_mg_vcycle", allow=(HS_ENOCONV,) if allow_noconv else ())

    def smooth(self, u, b, tmp, a, nsweeps, level=0):
        aa = (C.c_double * self.lanes)(*([a] * self.lanes if np.isscalar(a) else list(a)))
        check(lib().hs_smooth(self._h, level, C.cast(aa, _V), _ptr(u), _ptr(b), _ptr(tmp), nsweeps,
                              self._s()), "hs_smooth")

    # state and nodes ----------------------------------------------------
    def set_lane(self, lane, nu, dt, t0, nsteps, active=True):
        check(lib().hs_set_lane(self._h, lane, nu, dt, t0, nsteps, 1 if active else 0, self._s()),
              "hs_set_lane")

    def set_lane_state(self, lane, u0):
        check(lib().hs_set_lane_state(self._h, lane, _ptr(u0), self._s()), "hs_set_lane_state")

    def get_lane_state(self, lane):
        import torch
        out = torch.empty(self.lane_n[lane] ** 3, dtype=torch.float64, device="cuda")
        check(lib().hs_get_lane_state(self._h, lane, _ptr(out), self._s()), "hs_get_lane_state")
        return out

    def set_state(self, u0):
        check(lib().hs_set_state(self._h, _ptr(u0), self._s()), "hs_set_state")

    def get_state(self):
        import torch
        n = self.lane_n[-1] ** 3 if self.problem.nslices > 1 else self.field_len(0)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        check(lib().hs_get_state(self._h, _ptr(out), self._s()), "hs_get_state")
        return out

    def get_nodes(self, level=0):
        import torch
        M = self.level_M(level)
        U = torch.empty(M * self.field_len(level), dtype=torch.float64, device="cuda")
        FI = torch.empty_like(U)
        Ut = tau = None
        if level == 1:
            Ut = torch.empty_like(U)
            tau = torch.empty_like(U)
        check(lib().hs_get_nodes(self._h, level, _ptr(U), _ptr(FI), _ptr(Ut), _ptr(tau), self._s()),
              "hs_get_nodes")
        return U, FI, Ut, tau

    def set_nodes(self, level, U, FI):
        check(lib().hs_set_nodes(self._h, level, _ptr(U), _ptr(FI), self._s()), "hs_set_nodes")

    # step-level calls ---------------------------------------------------
    def begin_step(self):
        check(lib().hs_begin_step(self._h, self._s()), "hs_begin_step")

    def sdc_sweep(self, level=0):
        check(lib().hs_sdc_sweep(self._h, level, self._s()), "hs_sdc_sweep")

    def fas_restrict(self):
        check(lib().hs_fas_restrict(self._h, self._s()), "hs_fas_restrict")

    def fas_interp(self):
        check(lib().hs_fas_interp(self._h, self._s()), "hs_fas_interp")

    def mlsdc_iter(self):
        check(lib().hs_mlsdc_iter(self._h, self._s()), "hs_mlsdc_iter")

    def end_step(self):
        check(lib().hs_end_step(self._h, self._s()), "hs_end_step")

    def step(self):
        check(lib().hs_step(self._h, self._s()), "hs_step")

    def solve(self):
        check(lib().hs_solve(self._h, self._s()), "hs_solve")

    def solve_graph(self):
        check(lib().hs_solve_graph(self._h, self._s()), "hs_solve_graph")

    def pfasst_run(self):
        check(lib().hs_pfasst_run(self._h, self._s()), "hs_pfasst_run")

    def stats(self):
        arr = (LaneStats * self.lanes)()
        st = lib().hs_stats_read(self._h, C.cast(arr, _V), self._s())
        out = []
        for a in arr:
            d = dict((f, getattr(a, f)) for f, _ in LaneStats._fields_)
            d["level_cycles"] = list(a.level_cycles)
            out.append(d)
        return st, out

    # measurement aid ----------------------------------------------------
    def timer(self, kind, max_launches=4096):
        check(lib().hs_plan_timer(self._h, kind, max_launches), "hs_plan_timer")

    def timer_read(self):
        n, ms = C.c_int32(0), C.c_double(0.0)
        check(lib().hs_plan_timer_read(self._h, C.byref(n), C.byref(ms)), "hs_plan_timer_read")
        return n.value, ms.value
