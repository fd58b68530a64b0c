"""CPU FP64 oracle for the space-time heat solver -- TEST INFRASTRUCTURE ONLY.

This package wraps ``heat_oracle.c`` (plain serial C, built with gcc and
``-ffp-contract=off``) through ctypes.  It is the reference the GPU library
is checked against; only the tests, the smoke check and the benchmark's CPU
baseline may import it.  It does not import the GPU package and the GPU
package does not import it.

All arrays are float64 numpy arrays in [z][y][x] order (x fastest), n
interior points per axis, h = 1/(n+1) (section 1, eqs. (1)-(2)).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "heat_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_heat.so")

OK, EINVAL, ENOCONV, ENONFINITE = 0, -1, -3, -4
COMPACT = -4   # level order code of the compact 4th-order scheme (or_compact_apply)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fPIC",
             "-shared", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class MG(C.Structure):
    _fields_ = [("nu1", C.c_int32), ("nu2", C.c_int32), ("omega", C.c_double),
                ("n_coarsest", C.c_int32), ("tol", C.c_double), ("max_cycles", C.c_int32),
                ("fixed_cycles", C.c_int32)]


class Level(C.Structure):
    _fields_ = [("n", C.c_int32), ("order", C.c_int32), ("M", C.c_int32)]


class Problem(C.Structure):
    _fields_ = [("nu", C.c_double), ("t0", C.c_double), ("dt", C.c_double),
                ("forcing_c", C.c_double), ("nsteps", C.c_int32), ("sweeps", C.c_int32),
                ("sdc_tol", C.c_double), ("max_sweeps", C.c_int32), ("nlevels", C.c_int32),
                ("lev", Level * 3), ("mg", MG), ("node_parallel", C.c_int32), ("fas_interp", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("status", C.c_int32), ("sweeps", C.c_int32), ("total_sweeps", C.c_int32),
                ("total_solves", C.c_int32), ("total_cycles", C.c_int64),
                ("max_cycles_seen", C.c_int32), ("last_residual", C.c_double)]


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        L = _lib
        L.or_grid_h.restype = C.c_double
        L.or_grid_h.argtypes = [C.c_int]
        L.or_laplacian.argtypes = [C.c_int, C.c_int, _D, _D]
        L.or_lap_apply.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _D, _D]
        L.or_heat_op.argtypes = [C.c_int, C.c_int, C.c_double, _D, _D]
        L.or_compact_apply.argtypes = [C.c_int, C.c_double, C.c_double, _D, _D]
        L.or_sdc_residual_compact.restype = C.c_double
        L.or_sdc_residual_compact.argtypes = [C.POINTER(Level), C.c_double, C.c_double, C.c_double, C.c_double,
                                              _D, _D]
        L.or_spread_compact.argtypes = [C.POINTER(Level), C.c_double, _D, _D, _D]
        L.or_compact_binv.argtypes = [C.c_int, _D, _D]
        L.or_mlsdc_iter_compact.argtypes = [C.POINTER(Problem), C.c_double, _D, _D, _D, _D, _D, _D, _D,
                                            C.POINTER(Stats)]
        L.or_sdc_sweep_compact.argtypes = [C.POINTER(Level), C.POINTER(MG), C.c_double, C.c_double, C.c_double,
                                           C.c_double, _D, _D, C.POINTER(Stats)]
        L.or_residual.argtypes = [C.c_int, C.c_int, C.c_double, _D, _D, _D]
        L.or_jacobi.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, _D, _D, _D]
        L.or_restrict_fw.argtypes = [C.c_int, _D, _D]
        L.or_prolong_add.argtypes = [C.c_int, _D, _D]
        L.or_prolong_add_cubic.argtypes = [C.c_int, _D, _D]
        L.or_inject.argtypes = [C.c_int, _D, _D]
        L.or_dense_solve.argtypes = [C.c_int, C.c_int, C.c_double, _D, _D]
        L.or_mg_solve.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(MG), _D, _D,
                                  C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_lobatto_nodes.argtypes = [C.c_int, _D]
        L.or_collocation_matrix.argtypes = [C.c_int, _D]
        L.or_forcing.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _D]
        L.or_heat_rhs.argtypes = [C.c_int, C.c_int, C.c_double, C.c_double, C.c_double, _D, _D, _D]
        L.or_spread.argtypes = [C.POINTER(Level), C.c_double, _D, _D, _D]
        L.or_sdc_residual.restype = C.c_double
        L.or_sdc_residual.argtypes = [C.POINTER(Level), C.c_double, C.c_double, C.c_double,
                                      C.c_double, _D, _D, _D]
        L.or_sdc_sweep.argtypes = [C.POINTER(Level), C.POINTER(MG), C.c_double, C.c_double,
                                   C.c_double, C.c_double, _D, _D, _D, C.POINTER(Stats)]
        L.or_sdc_sweep_nodes.argtypes = [C.POINTER(Level), C.POINTER(MG), C.c_double, C.c_double,
                                         C.c_double, C.c_double, _D, _D, C.POINTER(Stats)]
        L.or_fas_restrict.argtypes = [C.POINTER(Level), C.POINTER(Level), C.c_double, C.c_double,
                                      C.c_double, C.c_double, _D, _D, _D, _D, _D, _D]
        L.or_fas_restrict_tau.argtypes = [C.POINTER(Level), C.POINTER(Level), C.c_double, C.c_double,
                                          C.c_double, C.c_double, _D, _D, _D, _D, _D, _D, _D]
        L.or_fas_interp.argtypes = [C.POINTER(Level), C.POINTER(Level), C.c_double, _D, _D, _D, _D, C.c_int]
        L.or_mlsdc_iter.argtypes = [C.POINTER(Problem), C.c_double, _D, _D, _D, _D, _D, _D,
                                    C.POINTER(Stats)]
        L.or_run.argtypes = [C.POINTER(Problem), _D, C.POINTER(Stats)]
        L.or_pfasst_run.argtypes = [C.POINTER(Problem), C.c_int, _D, C.POINTER(Stats)]
        L.or_pfasst.argtypes = [C.POINTER(Problem), C.c_int, C.c_int, _D, C.POINTER(Stats)]
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def mg_params(nu1=2, nu2=1, omega=6.0 / 7.0, n_coarsest=3, tol=1e-12, max_cycles=60,
              fixed_cycles=0) -> MG:
    return MG(nu1, nu2, omega, n_coarsest, tol, max_cycles, fixed_cycles)


def level(n, order, M) -> Level:
    return Level(n, order, M)


def problem(levels, nu=0.1, t0=0.0, dt=0.1, nsteps=1, forcing_c=3.0, sweeps=4, sdc_tol=1e-10,
            max_sweeps=20, mg=None, node_parallel=0, fas_interp=1) -> Problem:
    pb = Problem()
    pb.node_parallel = node_parallel
    pb.fas_interp = fas_interp
    pb.nu, pb.t0, pb.dt, pb.forcing_c = nu, t0, dt, forcing_c
    pb.nsteps, pb.sweeps, pb.sdc_tol, pb.max_sweeps = nsteps, sweeps, sdc_tol, max_sweeps
    pb.nlevels = len(levels)
    for i, lv in enumerate(levels):
        pb.lev[i] = lv if isinstance(lv, Level) else Level(*lv)
    pb.mg = mg if mg is not None else mg_params()
    return pb


def grid_h(n):
    return lib().or_grid_h(n)


def laplacian(u, order):
    u = _f(u); n = u.shape[0]; out = np.empty_like(u)
    lib().or_laplacian(n, order, _p(u), _p(out))
    return out


def lap_apply(u, order, alpha, beta):
    u = _f(u); n = u.shape[0]; out = np.empty_like(u)
    lib().or_lap_apply(n, order, alpha, beta, _p(u), _p(out))
    return out


def heat_op(u, order, a):
    u = _f(u); n = u.shape[0]; out = np.empty_like(u)
    lib().or_heat_op(n, order, a, _p(u), _p(out))
    return out


def residual(u, b, order, a):
    u = _f(u); b = _f(b); out = np.empty_like(u)
    lib().or_residual(u.shape[0], order, a, _p(u), _p(b), _p(out))
    return out


def jacobi(u, b, order, a, omega=6.0 / 7.0):
    u = _f(u); b = _f(b); out = np.empty_like(u)
    lib().or_jacobi(u.shape[0], order, a, omega, _p(u), _p(b), _p(out))
    return out


def compact_apply(u, alpha, beta):
    """alpha B_h u + beta A_h u with the compact pair (or_compact_apply)."""
    u = _f(u)
    n = u.shape[-1]
    y = np.empty_like(u)
    lib().or_compact_apply(n, alpha, beta, _p(u), _p(y))
    return y


def compact_binv(y):
    """B_h^{-1} y, exactly, in the sine basis (or_compact_binv)."""
    y = _f(y)
    x = np.empty_like(y)
    lib().or_compact_binv(y.shape[-1], _p(y), _p(x))
    return x


def mlsdc_iter_compact(pb, tn, Uf, G, Uc, FIc, Ut, tau):
    """One two-level MLSDC iteration with the compact fine level, in place
    (or_mlsdc_iter_compact); returns (status, B^{-1} G used for the FAS restriction)."""
    FIf = np.empty_like(Uf)
    st = Stats()
    s = lib().or_mlsdc_iter_compact(C.byref(pb), tn, _p(Uf), _p(G), _p(FIf), _p(Uc), _p(FIc), _p(Ut), _p(tau),
                                    C.byref(st))
    return s, FIf


def spread_compact(lv, nu, u0):
    n, M = lv.n, lv.M
    U = np.empty((M, n, n, n)); G = np.empty_like(U)
    lib().or_spread_compact(C.byref(lv), nu, _p(_f(u0)), _p(U), _p(G))
    return U, G


def sdc_residual_compact(lv, nu, tn, dt, c, U, G):
    return lib().or_sdc_residual_compact(C.byref(lv), nu, tn, dt, c, _p(_f(U)), _p(_f(G)))


def sdc_sweep_compact(lv, mg, nu, tn, dt, c, U, G):
    """In-place compact sweep on U, G (G = nu A_h U at every node)."""
    st = Stats()
    s = lib().or_sdc_sweep_compact(C.byref(lv), C.byref(mg), nu, tn, dt, c, _p(U), _p(G), C.byref(st))
    return s, st


def restrict_fw(rf):
    rf = _f(rf); nf = rf.shape[0]; nc = (nf - 1) // 2
    out = np.empty((nc, nc, nc))
    lib().or_restrict_fw(nf, _p(rf), _p(out))
    return out


def prolong_add(ec, uf):
    ec = _f(ec); out = _f(uf).copy()
    lib().or_prolong_add(ec.shape[0], _p(ec), _p(out))
    return out


def prolong_add_cubic(ec, uf):
    """uf + tricubic interpolation of ec (the FAS correction transfer with fas_interp = 3)."""
    ec = _f(ec); out = _f(uf).copy()
    lib().or_prolong_add_cubic(ec.shape[0], _p(ec), _p(out))
    return out


def inject(uf):
    uf = _f(uf); nf = uf.shape[0]; nc = (nf - 1) // 2
    out = np.empty((nc, nc, nc))
    lib().or_inject(nf, _p(uf), _p(out))
    return out


def dense_solve(b, order, a):
    b = _f(b); out = np.zeros_like(b)
    s = lib().or_dense_solve(b.shape[0], order, a, _p(b), _p(out))
    if s != OK:
        raise ValueError("dense_solve: grid too large")
    return out


def mg_solve(b, order, a, u0=None, mg=None):
    """Returns (u, status, cycles, rho)."""
    b = _f(b)
    u = np.zeros_like(b) if u0 is None else _f(u0).copy()
    cyc = C.c_int(0); rho = C.c_double(0)
    mg = mg if mg is not None else mg_params()
    s = lib().or_mg_solve(b.shape[0], order, a, C.byref(mg), _p(u), _p(b), C.byref(cyc),
                          C.byref(rho))
    return u, s, cyc.value, rho.value


def lobatto_nodes(M):
    out = np.empty(M)
    assert lib().or_lobatto_nodes(M, _p(out)) == OK
    return out


def collocation_matrix(M):
    out = np.empty((M, M))
    assert lib().or_collocation_matrix(M, _p(out)) == OK
    return out


def forcing(n, nu, c, t):
    out = np.empty((n, n, n))
    lib().or_forcing(n, nu, c, t, _p(out))
    return out


def heat_rhs(u, order, nu, c, t):
    u = _f(u); fi = np.empty_like(u); fe = np.empty_like(u)
    lib().or_heat_rhs(u.shape[0], order, nu, c, t, _p(u), _p(fi), _p(fe))
    return fi, fe


def spread(lv: Level, nu, u0):
    u0 = _f(u0); n = lv.n
    U = np.empty((lv.M, n, n, n)); FI = np.empty_like(U)
    lib().or_spread(C.byref(lv), nu, _p(u0), _p(U), _p(FI))
    return U, FI


def sdc_residual(lv, nu, tn, dt, c, U, FI, tau=None):
    return lib().or_sdc_residual(C.byref(lv), nu, tn, dt, c, _p(_f(U)), _p(_f(FI)),
                                 _p(_f(tau)) if tau is not None else None)


def sdc_sweep(lv, mg, nu, tn, dt, c, U, FI, tau=None):
    """In-place sweep on U, FI (float64 C-contiguous).  Returns (status, Stats)."""
    st = Stats()
    s = lib().or_sdc_sweep(C.byref(lv), C.byref(mg), nu, tn, dt, c, _p(U), _p(FI),
                           _p(tau) if tau is not None else None, C.byref(st))
    return s, st


def sdc_sweep_nodes(lv, mg, nu, tn, dt, c, U, FI):
    """In-place node-parallel sweep on U, FI.  Returns (status, Stats)."""
    st = Stats()
    s = lib().or_sdc_sweep_nodes(C.byref(lv), C.byref(mg), nu, tn, dt, c, _p(U), _p(FI), C.byref(st))
    return s, st


def fas_restrict(lf, lc, nu, tn, dt, c, Uf, FIf, tauf=None):
    """Restriction + FAS correction to the next coarser level; tauf is the
    fine level's own FAS correction (None on the finest level)."""
    nc, Mc = lc.n, lc.M
    Uc = np.empty((Mc, nc, nc, nc)); FIc = np.empty_like(Uc)
    Ut = np.empty_like(Uc); tau = np.empty_like(Uc)
    if tauf is None:
        lib().or_fas_restrict(C.byref(lf), C.byref(lc), nu, tn, dt, c, _p(_f(Uf)), _p(_f(FIf)),
                              _p(Uc), _p(FIc), _p(Ut), _p(tau))
    else:
        lib().or_fas_restrict_tau(C.byref(lf), C.byref(lc), nu, tn, dt, c, _p(_f(Uf)), _p(_f(FIf)),
                                  _p(_f(tauf)), _p(Uc), _p(FIc), _p(Ut), _p(tau))
    return Uc, FIc, Ut, tau


def fas_interp(lf, lc, nu, Uf, FIf, Uc, Ut, interp=1):
    """In-place on Uf, FIf; interp 1 trilinear, 3 tricubic in space."""
    lib().or_fas_interp(C.byref(lf), C.byref(lc), nu, _p(Uf), _p(FIf), _p(_f(Uc)), _p(_f(Ut)), interp)


def mlsdc_iter(pb, tn, Uf, FIf, Uc, FIc, Ut, tau):
    st = Stats()
    s = lib().or_mlsdc_iter(C.byref(pb), tn, _p(Uf), _p(FIf), _p(Uc), _p(FIc), _p(Ut), _p(tau),
                            C.byref(st))
    return s, st


def run(pb, u0):
    """SDC (nlevels=1) or MLSDC (nlevels=2, 3) over pb.nsteps steps.  Returns (u, status, Stats)."""
    u = _f(u0).copy()
    st = Stats()
    s = lib().or_run(C.byref(pb), _p(u), C.byref(st))
    return u, s, st


def pfasst_run(pb, P, u0):
    u = _f(u0).copy()
    st = Stats()
    s = lib().or_pfasst_run(C.byref(pb), P, _p(u), C.byref(st))
    return u, s, st


def pfasst(pb, P, u0, pred_sweeps=0):
    """PFASST with an optional serial coarse predictor (pred_sweeps coarse
    sweeps per slice) and, with pb.sweeps == 0, iterations until every
    slice's collocation residual is <= pb.sdc_tol.  Returns (u, status, Stats);
    Stats.sweeps is the number of iterations of the last block."""
    u = _f(u0).copy()
    st = Stats()
    s = lib().or_pfasst(C.byref(pb), P, pred_sweeps, _p(u), C.byref(st))
    return u, s, st
