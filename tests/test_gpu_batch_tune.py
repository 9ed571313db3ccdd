"""Batched kernel schedules, the schedule autotuner and the HIP-graph replay.

Schedules change only how a query's work is laid out (ranks per lane of a
tree query, which sets of a cyclic query go to the whole workgroup), so
every schedule must give the default schedule's plans and costs bit for
bit; the default batch is itself checked against the oracle in
test_gpu_batch.py.  Graph replays are checked against eager launches of the
same data, with eager work between the replays.
"""
import numpy as np
import pytest

from paper_2202_13511_amd import mpdp, workloads as W

pytestmark = pytest.mark.gpu


def same(a, b, names):
    for x, y, p, q, name in zip(a.costs, b.costs, a.plans, b.plans, names):
        assert np.float64(x).view(np.uint64) == np.float64(y).view(np.uint64), name
        assert p == q, name


@pytest.mark.parametrize("cm", [mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE])
def test_every_schedule_gives_the_default_result(cm):
    # the last four are cyclic with 19 or 20 relations: teams of workgroups
    big = [q for q in W.batch_mixed(40, 22, n_range=(19, 20)) if q.m != q.n - 1][:4]
    queries = W.batch_mixed(160, 21, n_range=(6, 16)) + [W.clique(11, 2), W.cycle_chords(5, n=16, chords=6)] + big
    names = [q.name for q in queries]
    ws = mpdp.batch_workspace(queries)
    ref = mpdp.mpdp_optimize_batch(queries, cm, ws)
    for tc, hc in ((1, 1), (2, 32), (4, 1024), (1, 65535), (2, 256)):
        print("schedule", tc, hc, flush=True)
        res = mpdp.mpdp_optimize_batch(queries, cm, ws, schedules=[(tc, hc)] * len(queries))
        same(res, ref, names)
        assert res.stats["connected_sets"] == ref.stats["connected_sets"]
        assert res.stats["ccp_pairs"] == ref.stats["ccp_pairs"]


def test_autotune_picks_valid_schedules_per_class():
    queries = W.batch_mixed(400, 5, n_range=(8, 18))
    names = [q.name for q in queries]
    ws = mpdp.batch_workspace(queries)
    sched, st = mpdp.mpdp_batch_autotune(queries, mpdp.MPDP_COST_COUT, ws, reps=1)
    print("tune", st, flush=True)
    assert st["launches"] == 5 and st["classes"] >= 10
    assert st["est_tuned_ms"] <= st["est_default_ms"] + 1e-9
    classes = {}
    for q, (tc, hc) in zip(queries, sched):
        assert tc in (1, 2, 4) and hc in (32, 64, 128, 256, 1024)
        tree = q.m == q.n - 1
        if tree:
            assert hc == 256
        else:
            assert tc == 4
        extra = q.m - (q.n - 1)
        key = (q.n, extra == 0, 0 if extra == 0 else 1 if extra <= 2 else 2 if extra <= 5 else 3)
        assert classes.setdefault(key, (tc, hc)) == (tc, hc), key  # one schedule per class
    ref = mpdp.mpdp_optimize_batch(queries, mpdp.MPDP_COST_COUT, ws)
    tuned = mpdp.mpdp_optimize_batch(queries, mpdp.MPDP_COST_COUT, ws, schedules=sched)
    same(tuned, ref, names)


def restat(queries, seed):
    """Same join graphs (same n and m), new statistics."""
    out = []
    for i, q in enumerate(queries):
        rng = np.random.Generator(np.random.PCG64([seed, i]))
        card = np.exp(rng.uniform(np.log(1e2), np.log(1e8), q.n))
        sel = rng.uniform(0.1, 1.0, q.m) / np.maximum(card[q.edges[:, 0]], card[q.edges[:, 1]]) if q.m else q.sel
        out.append(W.Query(q.n, q.edges.copy(), card, np.asarray(sel, np.float64), f"{q.name}/r{seed}"))
    return out


@pytest.mark.parametrize("cm", [mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE])
def test_graph_replays_match_eager_launches(cm):
    big = [q for q in W.batch_mixed(60, 8, n_range=(19, 20)) if q.m != q.n - 1][:12]  # teams of workgroups
    base = W.batch_mixed(300, 9, n_range=(6, 17)) + big
    # the same shape (n, m per query) with other topologies: a chain and a
    # star both have n - 1 edges
    swapped = [W.star(q.n, 77 + i) if (q.m == q.n - 1 and q.n >= 3 and i % 2) else q for i, q in enumerate(base)]
    # the large cyclic queries become rings with chords of the same n and m:
    # another predicted time, so other teams of workgroups in the same layout
    rings = [W.cycle_chords(90 + i, n=q.n, chords=q.m - q.n) if (q.n >= 19 and q.m > q.n) else q
             for i, q in enumerate(swapped)]
    assert [(q.n, q.m) for q in rings] == [(q.n, q.m) for q in base]
    data = [base, restat(base, 1), swapped, restat(swapped, 2), rings, base]
    ws = mpdp.batch_workspace(base)
    g = mpdp.BatchGraph(base, cm, ws)
    sched = [((1, 2, 4)[i % 3], 64 if i % 2 else 256) for i in range(len(base))]
    try:
        for rep, qs in enumerate(data):
            print("replay", rep, flush=True)
            names = [q.name for q in qs]
            got = g.run(qs, schedules=sched if rep % 2 else None)
            # eager work between replays, on the same workspace
            want = mpdp.mpdp_optimize_batch(qs, cm, ws)
            same(got, want, names)
            assert got.stats["ccp_pairs"] == want.stats["ccp_pairs"]
            assert np.all(got.latency_us > 0)
            one = mpdp.mpdp_optimize(qs[rep], cm)
            assert np.float64(got.costs[rep]).view(np.uint64) == np.float64(one.cost).view(np.uint64)
        with pytest.raises(mpdp.MpdpError):
            g.run(base[:-1] + [W.chain(base[-1].n, 1) if base[-1].m != base[-1].n - 1 else W.clique(5, 1)])
    finally:
        g.close()
