"""Host-side checks of the serving core (no GPU): class validation, pool
sizing and the budget check at creation."""
import ctypes as C

import pytest

from paper_1307_7867_amd import heatst as hs
from paper_1307_7867_amd import serving


def desc(classes, precision=hs.HS_MIXED):
    d = hs.ServerDesc()
    d.order, d.nnodes = 2, 5
    d.mg = hs.MgDesc(2, 1, 6.0 / 7.0, 3, 1e-10, 60, 0, precision, 2, 2, 1, 0)
    d.sweeps, d.sdc_tol, d.max_sweeps, d.forcing_c = 0, 1e-10, 40, 3.0
    d.nclasses = len(classes)
    for i, (n, s) in enumerate(classes):
        d.class_n[i], d.class_slots[i] = n, s
    return d


def sizes(d):
    sh, full = C.c_size_t(0), C.c_size_t(0)
    s = hs.lib().hs_server_pool_bytes(C.byref(d), C.byref(sh), C.byref(full))
    return s, sh.value, full.value


def request_bytes(d, n):
    out = C.c_size_t(0)
    s = hs.lib().hs_server_request_bytes(C.byref(d), n, C.byref(out))
    return s, out.value


@pytest.mark.parametrize("classes", [[], [(16, 2)], [(31, 0)], [(31, 2), (31, 1)], [(1023, 1)]])
def test_invalid_classes_rejected(classes):
    s, _, _ = sizes(desc(classes))
    assert s == hs.HS_EINVAL


def test_request_bytes_are_the_lane_fields_and_hierarchy():
    """A request of grid n holds its node data (U, F_I: 5 nodes; 4 quadrature
    fields; rhs, tmp) and the FP64 correction grids and FP32 grids of its
    hierarchy, nothing of the class's shared tables."""
    d = desc([(31, 3), (63, 2)])
    for n in (31, 63):
        s, b = request_bytes(d, n)
        assert s == hs.HS_OK
        N = n ** 3
        fields = (5 + 5 + 4 + 2) * N * 8
        grids, g = [], n
        while g >= 3:
            grids.append(g)
            g = (g - 1) // 2
        fp64 = sum(3 * k ** 3 * 8 for k in grids[1:])
        fp32 = sum(3 * k ** 3 * 4 for k in grids)
        assert fields + fp64 + fp32 <= b <= fields + fp64 + fp32 + 64 * 256
        assert b == serving.lane_bytes(n)
    assert request_bytes(d, 127)[0] == hs.HS_EINVAL


def test_pool_bytes_is_shared_plus_every_lane():
    d = desc([(31, 3), (63, 2)])
    s, sh, full = sizes(d)
    assert s == hs.HS_OK
    assert 0 < sh < 1 << 20            # lane states, tables and partials only
    assert full == sh + 3 * request_bytes(d, 31)[1] + 2 * request_bytes(d, 63)[1]


def test_create_rejects_pool_or_budget_below_one_request():
    d = desc([(31, 2), (63, 1)])
    _, sh, full = sizes(d)
    need = sh + request_bytes(d, 63)[1]
    h = C.c_void_p()
    # the checks happen before any device call; the pool pointer is never used
    st = hs.lib().hs_server_create(C.byref(d), C.c_void_p(256), full, need - 1, C.byref(h))
    assert st == hs.HS_ENOMEM
    st = hs.lib().hs_server_create(C.byref(d), C.c_void_p(256), need - 1, full, C.byref(h))
    assert st == hs.HS_ENOMEM


def test_capacities_follow_caps_and_budget():
    big = 10 ** 12
    caps = serving.capacities_for_budget(big, (31, 63, 127, 255, 511))
    assert caps == {n: serving.lane_cap(n) for n in (31, 63, 127, 255, 511)}
    small = 3 * serving.lane_bytes(255) + 1
    caps = serving.capacities_for_budget(small, (31, 255))
    assert caps[255] == 3 and caps[31] == serving.lane_cap(31)
