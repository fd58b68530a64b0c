"""Host-side checks of libheatst that need no GPU: the shared library loads
and exports every entry point of include/heatst.h, the problem validation
and workspace sizing behave, and the collocation data the GPU path uses
(computed independently of the oracle) matches the exact values."""
import ctypes as C
import json
import math
import os
import re
import subprocess

import numpy as np
import pytest
import sympy as sp

from paper_1307_7867_amd import heatst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "heatst.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 25
    out = subprocess.run(["nm", "-D", "--defined-only", heatst.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(hs_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    L = heatst.lib()
    for n in names:
        assert hasattr(L, n)


def test_library_has_gfx950_code_object():
    # the device code object bundled into the library targets gfx950
    blob = open(heatst.LIB_PATH, "rb").read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_status_strings():
    assert heatst.status_string(0) == "ok"
    assert "invalid" in heatst.status_string(-1)


def test_no_device_allocation_symbols_used():
    # the library only uses caller-owned device memory
    out = subprocess.run(["nm", "-D", "--undefined-only", heatst.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for sym in ("hipMalloc", "hipMallocAsync", "hipMallocManaged", "hipExtMallocWithFlags"):
        assert not re.search(rf"\s{sym}(@|$)", out, flags=re.M), sym


@pytest.mark.parametrize("M", [2, 3, 4, 5])
def test_collocation_data_exact(M):
    tau, Q = heatst.collocation(M)
    s = sp.Symbol("s")
    r = {2: [], 3: [sp.Rational(1, 2)], 4: [sp.Rational(1, 2) - sp.sqrt(5) / 10, sp.Rational(1, 2) + sp.sqrt(5) / 10],
         5: [sp.Rational(1, 2) - sp.sqrt(21) / 14, sp.Rational(1, 2), sp.Rational(1, 2) + sp.sqrt(21) / 14]}[M]
    t = [sp.Integer(0)] + r + [sp.Integer(1)]
    for m in range(M):
        assert abs(tau[m] - float(t[m])) < 2e-16
    for j in range(M):
        lj = sp.Integer(1)
        for i in range(M):
            if i != j:
                lj *= (s - t[i]) / (t[j] - t[i])
        for m in range(M):
            ex = float(sp.integrate(sp.expand(lj), (s, 0, t[m])).evalf(30))
            assert abs(Q[m, j] - ex) < 3e-16


def base_problem(**kw):
    p = heatst.Problem(n=15, order=2, nnodes=3)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("kw", [dict(n=16), dict(n=0), dict(n=1023), dict(order=3), dict(nnodes=6),
                                dict(nnodes=1), dict(nu=0.0), dict(dt=-1.0), dict(batch=0),
                                dict(nu1=0), dict(omega=1.5), dict(n_coarsest=7),
                                dict(precision=7), dict(sweeps=0, sdc_tol=0.0),
                                dict(fixed_cycles=0, tol=0.0),
                                dict(coarse=(8, 2, 3)), dict(coarse=(7, 2, 4), nnodes=5, n=15),
                                dict(nslices=4, batch=4), dict(lane_n=[15, 17], batch=2),
                                dict(fused_sweeps=3), dict(fused_sweeps=-1), dict(cycle_graphs=2)])
def test_invalid_problems_rejected(kw):
    p = base_problem(**kw)
    with pytest.raises(heatst.HeatstError) as e:
        p.workspace_bytes()
    assert e.value.status == heatst.HS_EINVAL


def test_workspace_bytes_accounts_for_fields():
    n, M = 63, 5
    p = base_problem(n=n, nnodes=M)
    b = p.workspace_bytes()
    N = n ** 3
    # node values, F, quadrature (M-1), rhs, tmp; plus the multigrid hierarchy
    fields = (M + M + (M - 1) + 2) * N * 8
    hier = sum(3 * k ** 3 * 8 for k in (31, 15, 7, 3))
    assert fields + hier <= b <= fields + hier + (1 << 20)
    p2 = base_problem(n=n, nnodes=M, batch=3)
    assert 3 * fields < p2.workspace_bytes() <= 3 * (fields + hier) + (1 << 20)


def test_workspace_mixed_precision_adds_fp32_hierarchy():
    p64 = base_problem(n=31, nnodes=5)
    p32 = base_problem(n=31, nnodes=5, precision=heatst.HS_MIXED)
    extra = p32.workspace_bytes() - p64.workspace_bytes()
    # an FP32 copy (u, t, b) of every grid, the finest included; the FP64
    # correction grids stay, so the difference is the FP32 hierarchy plus its
    # segment tables (a few KB)
    fp32 = sum(3 * k ** 3 * 4 for k in (31, 15, 7, 3))
    assert fp32 <= extra <= fp32 + 64 * 1024


def test_uneven_and_two_level_sizes():
    p = base_problem(n=31, nnodes=5, batch=3, lane_n=[31, 15, 63])
    assert p.workspace_bytes() > (63 ** 3) * 16 * 8
    # a coarse MLSDC level adds its node data (U, F_I: 3 nodes each; 2
    # quadrature fields; rhs, tmp; the restricted values and tau: 3 each) and
    # its own hierarchy below 31^3, plus tables
    p2 = base_problem(n=63, order=4, nnodes=5, coarse=(31, 2, 3))
    one = base_problem(n=63, order=4, nnodes=5)
    coarse = (3 + 3 + 2 + 2 + 3 + 3) * 31 ** 3 * 8 + sum(3 * k ** 3 * 8 for k in (15, 7, 3))
    assert coarse <= p2.workspace_bytes() - one.workspace_bytes() <= coarse + 64 * 1024
    p3 = base_problem(n=31, order=4, nnodes=5, coarse=(15, 2, 3), batch=4, nslices=4, nsteps=4)
    assert p3.workspace_bytes() > 4 * (31 ** 3) * 5 * 16


def test_product_path_has_no_cpu_fallback(monkeypatch, tmp_path):
    monkeypatch.setattr(heatst, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(heatst, "_lib", None)
    with pytest.raises(RuntimeError):
        heatst.Problem().workspace_bytes()


def test_static_solve_rejects_before_launching():
    """hs_mg_solve_static validates on the host: grids above HS_STATIC_MAX_N
    get HS_ENOMEM and graph capture HS_EINVAL before any device call (the
    pointers are never touched)."""
    import ctypes as C
    L = heatst.lib()
    d = heatst.MgDesc(2, 1, 6.0 / 7.0, 3, 1e-12, 60, 0, heatst.HS_FP64, 2, 2, 1, 0)
    fake = C.c_void_p(0x1000)
    assert L.hs_mg_solve_static(127, 2, 0.01, C.byref(d), fake, fake, None) == heatst.HS_ENOMEM
    assert L.hs_mg_solve_static(heatst.HS_STATIC_MAX_N + 2, 2, 0.01, C.byref(d), fake, fake,
                                None) == heatst.HS_EINVAL   # 65 is not 2^k - 1
    g = heatst.MgDesc(2, 1, 6.0 / 7.0, 3, 1e-12, 60, 0, heatst.HS_FP64, 2, 2, 1, 1)
    assert L.hs_mg_solve_static(31, 2, 0.01, C.byref(g), fake, fake, None) == heatst.HS_EINVAL
    assert L.hs_mg_solve_static(31, 2, -1.0, C.byref(d), fake, fake, None) == heatst.HS_EINVAL
    assert L.hs_mg_solve_static(31, 2, 0.01, C.byref(d), None, fake, None) == heatst.HS_EINVAL


def test_tune_table_parse_lookup_and_fallback(tmp_path):
    """The launch-shape table: built-in rule without entries, the entry of the
    largest batch <= the launch's count (else the smallest), JSON loading
    (extra fields and nested objects ignored), invalid entries rejected."""
    heatst.tune_clear()
    try:
        assert heatst.tune_lookup(127, 4, 0, 16) == (8, 8)     # built-in: 8 planes at 127^3
        assert heatst.tune_lookup(63, 2, 0, 1) == (2, 2)       # 2 planes at 63^3
        path = tmp_path / "tune.json"
        path.write_text(json.dumps({
            "device": "gfx950", "meta": {"note": "x, y", "n": 5},
            "entries": [
                {"n": 127, "order": 4, "precision": 0, "batch": 1, "zb": 8, "zb_rfw": 8, "us": 1.5},
                {"n": 127, "order": 4, "precision": 0, "batch": 16, "zb": 16, "zb_rfw": 32},
                {"n": 63, "order": 2, "precision": 1, "batch": 4, "zb": 4, "zb_rfw": 4, "note": "a,b"},
            ]}))
        assert heatst.tune_load(str(path)) == 3
        assert heatst.tune_lookup(127, 4, 0, 16) == (16, 32)
        assert heatst.tune_lookup(127, 4, 0, 40) == (16, 32)   # largest batch <= 40
        assert heatst.tune_lookup(127, 4, 0, 8) == (8, 8)      # largest batch <= 8 is 1
        assert heatst.tune_lookup(63, 2, 1, 1) == (4, 4)       # none <= 1: the smallest batch
        assert heatst.tune_lookup(63, 2, 0, 4) == (2, 2)       # other precision: built-in rule
        assert heatst.tune_lookup(127, 2, 0, 16) == (8, 8)     # other order: built-in rule
        heatst.tune_set(127, 4, 0, 16, 4, 4)                    # replaces the entry
        assert heatst.tune_lookup(127, 4, 0, 16) == (4, 4)
        for bad in [(127, 4, 0, 16, 0, 8), (127, 4, 0, 16, 8, 3), (100, 4, 0, 1, 8, 8), (127, 3, 0, 1, 8, 8),
                    (127, 4, 2, 1, 8, 8), (127, 4, 0, 0, 8, 8), (127, 4, 0, 1, 65, 8)]:
            with pytest.raises(heatst.HeatstError):
                heatst.tune_set(*bad)
        with pytest.raises(heatst.HeatstError):
            heatst.tune_load(str(tmp_path / "missing.json"))
        # a plan takes the shape at creation: its workspace holds the same bytes either way
        p = base_problem(n=31, nnodes=3)
        b0 = p.workspace_bytes()
        heatst.tune_set(31, 2, 0, 1, 1, 2)
        assert p.workspace_bytes() >= b0
    finally:
        heatst.tune_clear()


def test_pfasst_predictor_needs_slices():
    with pytest.raises(heatst.HeatstError) as e:
        base_problem(n=31, nnodes=3, pfasst_pred_sweeps=1).workspace_bytes()
    assert e.value.status == heatst.HS_EINVAL
    p = base_problem(n=31, order=4, nnodes=5, coarse=(15, 2, 3), batch=4, nslices=4, nsteps=4, sweeps=0,
                     pfasst_pred_sweeps=2)
    assert p.workspace_bytes() > 0


@pytest.mark.parametrize("kw", [
    dict(pfasst_groups=3),                                   # does not divide 4 slices
    dict(pfasst_groups=8),                                   # more groups than slices
    dict(pfasst_groups=-1),
    dict(pfasst_groups=2, sweeps=0),                         # groups need fixed iterations
    dict(pfasst_groups=2, cycle_graphs=1),
])
def test_pfasst_groups_validated(kw):
    args = dict(n=31, order=4, nnodes=5, coarse=(15, 2, 3), batch=4, nslices=4, nsteps=4, sweeps=2)
    args.update(kw)
    with pytest.raises(heatst.HeatstError) as e:
        base_problem(**args).workspace_bytes()
    assert e.value.status == heatst.HS_EINVAL


def test_pfasst_groups_add_snapshots_only():
    """Two groups of two slices: the group tables, one fine and one coarse
    end-value copy and a second block of partial maxima, nothing per slice."""
    args = dict(n=31, order=4, nnodes=5, coarse=(15, 2, 3), batch=4, nslices=4, nsteps=4, sweeps=2)
    b0 = base_problem(**args).workspace_bytes()
    b2 = base_problem(pfasst_groups=2, **args).workspace_bytes()
    snaps = (31 ** 3 + 15 ** 3) * 8
    assert b0 + snaps <= b2 <= b0 + snaps + (1 << 20)
    assert base_problem(pfasst_groups=1, **args).workspace_bytes() == b0


def test_fas_interp_validated_and_sized():
    """The tricubic transfer takes scratch of M_c n_c n_f (n_c + n_f) values per lane."""
    args = dict(n=31, order=4, nnodes=5, coarse=(15, 2, 3), batch=2)
    b1 = base_problem(**args).workspace_bytes()
    b3 = base_problem(fas_interp=3, **args).workspace_bytes()
    scratch = 2 * 3 * 15 * 31 * (15 + 31) * 8
    assert b1 + scratch <= b3 <= b1 + scratch + 4 * 256
    with pytest.raises(heatst.HeatstError) as e:
        base_problem(fas_interp=2, **args).workspace_bytes()
    assert e.value.status == heatst.HS_EINVAL


def test_three_levels_validated_and_sized():
    """A third level adds its node arrays (U, FI, P, rhs, Ut, tau), its
    multigrid hierarchy and its tables; the pipelined order is two-level only;
    level sizes and node counts must nest."""
    args = dict(n=31, order=4, nnodes=5, coarse=(15, 2, 3), batch=2, sweeps=2)
    b2 = base_problem(**args).workspace_bytes()
    b3 = base_problem(coarse2=(7, 2, 2), **args).workspace_bytes()
    nodes = 2 * (2 + 2 + 1 + 1 + 2 + 2) * 7 ** 3 * 8   # per lane: U, FI (M), P (M-1), rhs, tmp, Ut, tau (M)
    assert b2 + nodes <= b3 <= b2 + nodes + (1 << 20)
    for bad in (dict(coarse2=(5, 2, 2)), dict(coarse2=(7, 2, 4)), dict(coarse2=(7, 3, 2))):
        with pytest.raises(heatst.HeatstError) as e:
            base_problem(**{**args, **bad}).workspace_bytes()
        assert e.value.status == heatst.HS_EINVAL
    pf = dict(args, batch=4, nslices=4, nsteps=4, coarse2=(7, 2, 2))
    assert base_problem(**pf).workspace_bytes() > 0
    with pytest.raises(heatst.HeatstError) as e:
        base_problem(pfasst_groups=2, **pf).workspace_bytes()
    assert e.value.status == heatst.HS_EINVAL


def test_compact_apply_rejects_invalid_arguments():
    """hs_compact_apply validates on the host before any launch."""
    L = heatst.lib()
    one = C.c_void_p(1)
    for n, batch, u, y in ((4, 1, one, one), (0, 1, one, one), (513, 1, one, one), (15, 0, one, one),
                           (15, 1, None, one), (15, 1, one, None)):
        assert L.hs_compact_apply(n, batch, 1.0, 0.0, u, y, None) == heatst.HS_EINVAL


@pytest.mark.parametrize("kw", [
    dict(coarse=(7, 2, 3), coarse2=(3, 2, 2)),              # one or two levels only
    dict(precision=heatst.HS_MIXED),                         # FP64 only
    dict(sdc_node_parallel=1),
    dict(batch=2, nslices=2, nsteps=2, coarse=(7, 2, 3)),
])
def test_compact_plans_validated(kw):
    args = dict(n=15, order=heatst.HS_ORDER_COMPACT, nnodes=3)
    args.update(kw)
    with pytest.raises(heatst.HeatstError) as e:
        base_problem(**args).workspace_bytes()
    assert e.value.status == heatst.HS_EINVAL


def test_compact_plan_sized_and_coarse_level_rejected():
    """A compact single-level plan lays out like the order-2 one of the same
    grids; the compact code is not accepted below the finest level."""
    b = base_problem(n=31, order=heatst.HS_ORDER_COMPACT, nnodes=3).workspace_bytes()
    assert b == base_problem(n=31, order=2, nnodes=3).workspace_bytes()
    with pytest.raises(heatst.HeatstError) as e:
        base_problem(n=31, order=4, nnodes=3, coarse=(15, heatst.HS_ORDER_COMPACT, 3)).workspace_bytes()
    assert e.value.status == heatst.HS_EINVAL


def test_compact_mlsdc_plan_adds_the_sine_table():
    """Two-level MLSDC with the compact fine level lays out like the order-2
    plan of the same levels plus one table for B_h^{-1}: the DST-I matrix and
    the cosines, n (n + 1) values."""
    n = 31
    b = base_problem(n=n, order=heatst.HS_ORDER_COMPACT, nnodes=5, coarse=(15, 2, 3)).workspace_bytes()
    b2 = base_problem(n=n, order=2, nnodes=5, coarse=(15, 2, 3)).workspace_bytes()
    tab = (n * (n + 1) * 8 + 255) // 256 * 256
    assert b2 + tab - 256 <= b <= b2 + tab + 256
