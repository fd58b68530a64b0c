"""Host-side checks of the serving core (no GPU): class validation, pool
sizing and admission by budget."""
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


def pool_bytes(d):
    out = C.c_size_t(0)
    s = hs.lib().hs_server_pool_bytes(C.byref(d), C.byref(out))
    return s, out.value


@pytest.mark.parametrize("classes", [[], [(16, 2)], [(31, 0)], [(31, 2), (31, 1)], [(1023, 1)]])
def test_invalid_classes_rejected(classes):
    s, _ = pool_bytes(desc(classes))
    assert s == hs.HS_EINVAL


def test_pool_bytes_is_sum_of_class_plans():
    s, total = pool_bytes(desc([(31, 3), (63, 2)]))
    assert s == hs.HS_OK
    per31 = serving.lane_bytes(31)
    per63 = serving.lane_bytes(63)
    assert total >= 2 * per63 + 3 * per31 * 0.9
    assert total <= 3 * per31 + 2 * per63 + (1 << 20)


def test_create_rejects_budget_below_need():
    d = desc([(31, 2)])
    s, need = pool_bytes(d)
    h = C.c_void_p()
    # the budget check happens before any device call; the pool pointer is never used
    st = hs.lib().hs_server_create(C.byref(d), C.c_void_p(256), need, need - 1, C.byref(h))
    assert st == hs.HS_ENOMEM
    st = hs.lib().hs_server_create(C.byref(d), C.c_void_p(256), need - 1, need, C.byref(h))
    assert st == hs.HS_ENOMEM


def test_slots_for_budget_respects_budget_and_weights():
    sizes, weights = (31, 63, 127), (8, 4, 2)
    budget = 2 * 10**9
    slots = serving.slots_for_budget(budget, sizes, weights)
    used = sum(slots[n] * serving.lane_bytes(n) for n in sizes)
    assert used <= budget
    assert all(slots[n] >= 1 for n in sizes)
    # every class is at its cap or the budget is exhausted for it
    for n in sizes:
        assert slots[n] == serving.slot_cap(n) or used + serving.lane_bytes(n) > budget
