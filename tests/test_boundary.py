"""C-ABI boundary tests that need no GPU: the library loads, exports every
function declared in include/mpdp.h, and rejects malformed input on the host
before any HIP call."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2202_13511_amd import mpdp, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for h in ("mpdp.h", "mpdp_scorer.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(mpdp_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_function():
    lib = mpdp.load()
    names = header_functions()
    assert set(names) == set(mpdp.EXPORTED)
    for name in names:
        assert hasattr(lib, name), name


def test_status_strings():
    for s in range(7):
        assert mpdp.mpdp_status_str(s) != "unknown status"
    assert mpdp.mpdp_status_str(99) == "unknown status"


def test_workspace_and_layout():
    assert mpdp.mpdp_workspace_bytes(0) == 0
    assert mpdp.mpdp_workspace_bytes(33) == 0
    for n in (2, 12, 25):
        ws = mpdp.mpdp_workspace_bytes(n)
        N = 1 << n
        assert ws >= 21 * N
        lay = mpdp.mpdp_memo_layout(n)
        assert all(v % 256 == 0 for v in lay.values())
        assert lay["cost"] + 8 * N <= lay["card"] and lay["card"] + 8 * N <= lay["left"]
        assert lay["left"] + 4 * N <= lay["op"] and lay["op"] + N <= ws
    with pytest.raises(mpdp.MpdpError):
        mpdp.mpdp_memo_layout(0)


def status_of(n, edges, card, sel, cm=0):
    try:
        mpdp.mpdp_optimize(W.Query(n, np.asarray(edges, np.uint32).reshape(-1, 2),
                                   np.asarray(card, np.float64), np.asarray(sel, np.float64)), cm)
    except mpdp.MpdpError as e:
        return e.status
    return mpdp.MPDP_OK


def test_validation_errors_without_gpu():
    good_e, good_c, good_s = [[0, 1], [1, 2]], [10.0, 20.0, 30.0], [0.5, 0.5]
    E = mpdp.MPDP_EINVAL
    assert status_of(0, [], [], []) == E
    assert status_of(33, [[i, i + 1] for i in range(32)], [2.0] * 33, [0.5] * 32) == mpdp.MPDP_ETOOLARGE
    assert status_of(3, [[0, 0], [1, 2]], good_c, good_s) == E             # self loop
    assert status_of(3, [[0, 1], [1, 0]], good_c, good_s) == E             # duplicate predicate
    assert status_of(3, [[0, 3], [1, 2]], good_c, good_s) == E             # endpoint out of range
    assert status_of(3, good_e, [0.5, 20.0, 30.0], good_s) == E            # card < 1
    assert status_of(3, good_e, [math.nan, 20.0, 30.0], good_s) == E
    assert status_of(3, good_e, [math.inf, 20.0, 30.0], good_s) == E
    assert status_of(3, good_e, good_c, [0.0, 0.5]) == E                   # sel outside (0, 1]
    assert status_of(3, good_e, good_c, [1.5, 0.5]) == E
    assert status_of(3, good_e, good_c, [math.nan, 0.5]) == E
    assert status_of(3, good_e, good_c, good_s, cm=7) == E                 # unknown cost model
    assert status_of(4, good_e, good_c + [5.0], good_s) == mpdp.MPDP_ENOTCONNECTED
    assert status_of(3, [], good_c, []) == E or status_of(3, [], good_c, []) == mpdp.MPDP_ENOTCONNECTED


def test_null_pointers_rejected():
    lib = mpdp.load()
    plan = (mpdp.mpdp_plan_node * 5)()
    cost = ctypes.c_double()
    card = (ctypes.c_double * 3)(1.0, 2.0, 3.0)
    # edges NULL with m > 0
    assert lib.mpdp_optimize(3, 2, None, card, None, 0, plan, ctypes.byref(cost), None) == mpdp.MPDP_EINVAL
    edges = (mpdp.mpdp_edge * 2)(mpdp.mpdp_edge(0, 1), mpdp.mpdp_edge(1, 2))
    sel = (ctypes.c_double * 2)(0.5, 0.5)
    assert lib.mpdp_optimize(3, 2, edges, None, sel, 0, plan, ctypes.byref(cost), None) == mpdp.MPDP_EINVAL
    assert lib.mpdp_optimize(3, 2, edges, card, sel, 0, None, ctypes.byref(cost), None) == mpdp.MPDP_EINVAL
    assert lib.mpdp_optimize(3, 2, edges, card, sel, 0, plan, None, None) == mpdp.MPDP_EINVAL
    # workspace variant: null workspace
    assert lib.mpdp_optimize_ws(3, 2, edges, card, sel, 0, None, 0, None, 0, plan, ctypes.byref(cost),
                                None) == mpdp.MPDP_EINVAL


def test_single_relation_needs_no_device():
    q = W.Query(1, np.zeros((0, 2), np.uint32), np.array([1234.0]), np.zeros(0))
    r = mpdp.mpdp_optimize(q, mpdp.MPDP_COST_PGLIKE)
    assert r.cost == 0.01 * 1234.0
    assert r.plan == [dict(left=-1, right=-1, relset=1, op=mpdp.MPDP_OP_SCAN, cost=0.01 * 1234.0, card=1234.0)]
    r = mpdp.mpdp_optimize(q, mpdp.MPDP_COST_COUT)
    assert r.cost == 0.0


def test_batch_validation_without_gpu():
    lib = mpdp.load()
    good = [W.chain(5, 0), W.star(6, 1)]
    assert mpdp.mpdp_batch_workspace_bytes(good) > 0
    assert mpdp.mpdp_batch_workspace_bytes(good + [W.chain(21, 2)]) == 0  # n > 20
    import torch  # noqa: F401  (tensor-free calls below never touch a device)

    def status(queries):
        qs, c, e, s = mpdp._batch_marshal(queries)
        plans = (mpdp.mpdp_plan_node * sum(2 * q.n - 1 for q in queries))()
        costs = np.zeros(len(queries))
        f64p = ctypes.POINTER(ctypes.c_double)
        return lib.mpdp_optimize_batch(len(queries), qs, e.ctypes.data_as(ctypes.POINTER(mpdp.mpdp_edge)),
                                       c.ctypes.data_as(f64p), s.ctypes.data_as(f64p), 0, None, 0, None, 0, plans,
                                       costs.ctypes.data_as(f64p), None, None, None)

    assert status(good + [W.chain(21, 2)]) == mpdp.MPDP_ETOOLARGE
    bad = W.chain(5, 3)
    bad.edges = bad.edges.copy()
    bad.edges[1] = [2, 2]
    assert status(good + [bad]) == mpdp.MPDP_EINVAL
    disc = W.Query(4, np.array([[0, 1], [2, 3]], np.uint32), np.full(4, 10.0), np.full(2, 0.5))
    assert status([disc]) == mpdp.MPDP_ENOTCONNECTED
    assert status(good) == mpdp.MPDP_EINVAL  # valid queries, but no workspace


def test_batch_schedule_tuner_and_graph_validation_without_gpu():
    """The scheduled batch call, the autotuner and the graph handle reject
    bad arguments on the host, before any HIP call."""
    lib = mpdp.load()
    import torch  # noqa: F401
    good = [W.chain(5, 0), W.star(6, 1), W.cycle_chords(4, n=7, chords=1)]
    qs, c, e, s = mpdp._batch_marshal(good)
    f64p = ctypes.POINTER(ctypes.c_double)
    ep = e.ctypes.data_as(ctypes.POINTER(mpdp.mpdp_edge))
    plans = (mpdp.mpdp_plan_node * sum(2 * q.n - 1 for q in good))()
    costs = np.zeros(len(good))

    def sched_status(pairs):
        sch = mpdp._schedules(good, pairs)
        return lib.mpdp_optimize_batch_sched(len(good), qs, ep, c.ctypes.data_as(f64p), s.ctypes.data_as(f64p), 0,
                                             None, 0, None, 0, sch, plans, costs.ctypes.data_as(f64p), None, None,
                                             None)

    for bad in ((3, 256), (0, 256), (8, 256), (4, 0), (4, 65536)):
        assert sched_status([bad] * 3) == mpdp.MPDP_EINVAL, bad
    # valid schedules pass validation and then stop at the missing workspace
    assert sched_status([(1, 1), (2, 65535), (4, 256)]) == mpdp.MPDP_EINVAL

    out = (mpdp.mpdp_batch_schedule * len(good))()
    st = mpdp.mpdp_batch_tune_stats()
    for reps, o in ((0, out), (17, out), (2, None)):
        assert lib.mpdp_batch_autotune(len(good), qs, ep, c.ctypes.data_as(f64p), s.ctypes.data_as(f64p), 0, None,
                                       0, None, reps, o, ctypes.byref(st)) == mpdp.MPDP_EINVAL

    h = ctypes.c_void_p(1)
    assert lib.mpdp_batch_graph_create(len(good), qs, 0, None, 0, None) == mpdp.MPDP_EINVAL
    assert lib.mpdp_batch_graph_create(len(good), qs, 0, None, 0, ctypes.byref(h)) == mpdp.MPDP_EINVAL
    assert h.value is None  # NULL on error
    assert lib.mpdp_batch_graph_create(len(good), qs, 7, None, 0, ctypes.byref(h)) == mpdp.MPDP_EINVAL
    big, _, _, _ = mpdp._batch_marshal([W.chain(21, 2)])
    assert lib.mpdp_batch_graph_create(1, big, 0, None, 0, ctypes.byref(h)) == mpdp.MPDP_ETOOLARGE
    short = (mpdp.mpdp_batch_query * 1)(mpdp.mpdp_batch_query(5, 3, 0, 0))  # m < n - 1
    assert lib.mpdp_batch_graph_create(1, short, 0, None, 0, ctypes.byref(h)) == mpdp.MPDP_EINVAL
    assert lib.mpdp_batch_graph_run(None, qs, ep, c.ctypes.data_as(f64p), s.ctypes.data_as(f64p), None, None,
                                    plans, costs.ctypes.data_as(f64p), None, None) == mpdp.MPDP_EINVAL
    lib.mpdp_batch_graph_destroy(None)


def test_batch_workspace_leaves_room_for_teams():
    """A cyclic query of 17 or more relations may be shared by a team of up
    to 8 workgroups, so the batch workspace holds 7 more queue entries of 64
    bytes and a team record for it; a tree of the same size, or a smaller
    cyclic query, needs none (their edge arrays differ by one edge only)."""
    base = [W.chain(10, s) for s in range(20)]
    size = lambda q: mpdp.mpdp_batch_workspace_bytes(base + [q])
    assert size(W.cycle(18, 1)) - size(W.chain(18, 1)) >= 7 * 64
    assert size(W.cycle(16, 1)) - size(W.chain(16, 1)) < 7 * 64
