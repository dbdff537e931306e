"""CPU checks of the work decomposition (pdd_plan_tickets, host only): the
tickets cover every (knot, path) pair exactly once in near-equal contiguous
ranges, the claim order is a permutation sorted as documented, and the XCD
split gives each XCD the cost share of its workgroups.  Expected costs and
Morton keys are recomputed here from the oracle's geometry."""
import ctypes as C

import numpy as np
import pytest

from paper_2301_05780_amd import pdd, workloads
from oracle.geometry import Geometry


def _morton(sx, sy):
    key = 0
    for b in range(16):
        key |= ((sx >> b) & 1) << (2 * b)
        key |= ((sy >> b) & 1) << (2 * b + 1)
    return key


def _workload(seed=0):
    w = dict(workloads.varcoef(), H=6, m=5, ext=2, domain=(-0.5, 1.0, 0.25, 1.75))
    g = Geometry(w["domain"], w["H"], w["m"], w["ext"])
    rng = np.random.default_rng(seed)
    w["n_paths_per_knot"] = rng.integers(1, 700, size=g.n).astype(np.int32)
    return w, g


@pytest.mark.parametrize("ppt", [1, 97, 256, 10 ** 6])
def test_tickets_cover_every_path_once(ppt):
    w, g = _workload()
    tickets, order, _ = pdd.plan_tickets(w, ppt)
    npk = w["n_paths_per_knot"]
    assert tickets.shape == (int(np.sum((npk + ppt - 1) // ppt)), 3)
    assert np.array_equal(np.sort(order), np.arange(tickets.shape[0]))
    # tickets are grouped by knot in canonical order, ranges contiguous from 0 to N_k
    assert np.all(np.diff(tickets[:, 0]) >= 0)
    for k in range(g.n):
        t = tickets[tickets[:, 0] == k]
        c = (npk[k] + ppt - 1) // ppt
        assert t.shape[0] == c
        assert t[0, 1] == 0 and t[-1, 2] == npk[k]
        assert np.array_equal(t[1:, 1], t[:-1, 2])
        sizes = t[:, 2] - t[:, 1]
        assert sizes.min() >= 1 and sizes.max() <= ppt and sizes.max() - sizes.min() <= 1


def test_longest_expected_first_order():
    w, g = _workload(1)
    tickets, order, xb = pdd.plan_tickets(w, 64)
    assert xb is None
    area = (g.box_i[:, 1] - g.box_i[:, 0]) * (g.box_i[:, 3] - g.box_i[:, 2])
    cost = area[tickets[:, 0]] * (tickets[:, 2] - tickets[:, 1])
    c = cost[order]
    assert np.all(np.diff(c) <= 0)
    # stable: equal costs keep the ticket order
    same = np.diff(c) == 0
    assert np.all(np.diff(order)[same] > 0)


def test_spatial_order_and_xcd_split():
    w, g = _workload(2)
    grid = 1000
    tickets, order, xb = pdd.plan_tickets(w, 50, spatial=True, grid=grid)
    key = np.array([_morton(int(g.ix[k]) // w["m"], int(g.iy[k]) // w["m"]) for k in tickets[:, 0]])
    ko = key[order]
    assert np.all(np.diff(ko) >= 0)
    same = np.diff(ko) == 0
    assert np.all(np.diff(order)[same] > 0)
    # the split: contiguous shares of the order, each XCD's expected cost in
    # proportion to its ceil((grid - x) / 8) workgroups
    T = tickets.shape[0]
    assert xb[0] == 0 and xb[8] == T and np.all(np.diff(xb) >= 0)
    area = (g.box_i[:, 1] - g.box_i[:, 0]) * (g.box_i[:, 3] - g.box_i[:, 2])
    cum = np.concatenate([[0.0], np.cumsum((area[tickets[:, 0]] * (tickets[:, 2] - tickets[:, 1]))[order])])
    before = 0
    for x in range(7):
        before += (grid - x + 7) // 8
        target = cum[-1] * before / grid
        b = xb[x + 1]
        assert cum[b] >= target and (b == 0 or cum[b - 1] < target or b == xb[x])


def test_every_ticket_of_the_large_table_workload():
    w = workloads.large_lut()
    tickets, order, xb = pdd.plan_tickets(w, 256, spatial=True, grid=768)
    assert tickets.shape[0] == 62465 * 40          # ceil(1e4 / 256) tickets per knot
    assert int((tickets[:, 2] - tickets[:, 1]).sum()) == 62465 * 10 ** 4
    assert xb[8] == tickets.shape[0]


def test_plan_rejects_bad_arguments():
    w, _ = _workload()
    with pytest.raises(pdd.PddError):
        pdd.plan_tickets(w, 0)
    with pytest.raises(pdd.PddError):
        pdd.plan_tickets(dict(w, n_paths_per_knot=np.zeros_like(w["n_paths_per_knot"])), 10)
    # the XCD split asks for the spatial order and at least one workgroup per XCD
    T = C.c_int64()
    xb = np.empty(9, dtype=np.int32)
    npk = np.ascontiguousarray(w["n_paths_per_knot"])
    for spatial, grid in ((0, 64), (1, 4)):
        st = pdd.lib().pdd_plan_tickets(C.byref(pdd.partition_of(w)), C.byref(pdd.knots_of(w)), npk.ctypes.data, 10,
                                        spatial, grid, C.byref(T), None, None, xb.ctypes.data)
        assert st == pdd.EINVAL
