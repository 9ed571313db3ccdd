"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle, bit for
bit, on every memo entry of small queries that still span several levels,
both kernels (Alg. 2 tree kernel and Alg. 3 block kernel) and both cost
models, plus edge cases (two relations, ties, the largest bitmap width)."""
import numpy as np
import pytest

import oracle
from oracle.special import chain_interval_dp
from paper_2202_13511_amd import mpdp, workloads as W

pytestmark = pytest.mark.gpu

CMS = [mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE]


def run_ws(q, cm, flags=0):
    import torch
    ws = mpdp.workspace(q.n, cm, "cuda")
    res = mpdp.mpdp_optimize_ws(q, cm, ws, flags=flags)
    torch.cuda.synchronize()
    return res, mpdp.memo_arrays(ws, q.n)


def check_memo(q, gm, ref):
    mask = ref.has_plan()
    for name in ("cost", "card"):
        a = gm[name][mask].view(np.uint64)
        b = getattr(ref, name)[mask].view(np.uint64)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, (q.name, name, np.nonzero(mask)[0][bad[:5]])
    assert np.array_equal(gm["left"][mask], ref.left[mask]), q.name
    assert np.array_equal(gm["op"][mask], ref.op[mask]), q.name


def check_plan(q, res, ref):
    want = oracle.plan_from_memo(ref)
    assert len(res.plan) == len(want)
    for a, b in zip(res.plan, want):
        assert (a["relset"], a["left"], a["right"], a["op"]) == (b["relset"], b["left"], b["right"], b["op"])
        assert np.float64(a["cost"]).view(np.uint64) == np.float64(b["cost"]).view(np.uint64)
        assert np.float64(a["card"]).view(np.uint64) == np.float64(b["card"]).view(np.uint64)
    assert np.float64(res.cost).view(np.uint64) == np.float64(ref.root_cost).view(np.uint64)


def check_stats(q, res, ref, general):
    st = res.stats
    assert st["connected_sets"] == ref.connected_sets
    assert st["ccp_pairs"] == ref.ccp_ordered // 2
    assert st["candidates"] == (1 << q.n) - 1 - q.n
    if general:
        assert st["evaluated_pairs"] == oracle.mpdp(q, force_general=True).evaluated
    else:
        assert st["evaluated_pairs"] == ref.ccp_ordered


def families():
    qs = []
    for s in range(2):
        qs += [W.star(12, s), W.snowflake(14, s), W.random_tree(13, s), W.chain(12, s),
               W.cycle(11, s), W.clique(9, s), W.random_connected(12, s, 0.2),
               W.random_connected(11, 20 + s, 0.5), W.cycle_chords(s, n=13, chords=4)]
    qs += [W.all_equal_clique(9), W.from_edges(2, [[0, 1]], 3, "pair")]
    return qs


@pytest.mark.parametrize("cm", CMS)
def test_memo_parity_small(cm):
    for q in families():
        res, gm = run_ws(q, cm)
        ref = oracle.mpdp(q, cm)
        check_memo(q, gm, ref)
        check_plan(q, res, ref)
        tree = q.m == q.n - 1
        check_stats(q, res, ref, general=not tree)


@pytest.mark.parametrize("cm", CMS)
def test_block_kernel_on_trees(cm):
    """Alg. 3 kernel forced onto tree joins reaches the same memo."""
    for q in [W.star(11, 4), W.snowflake(15, 5), W.random_tree(12, 6)]:
        res, gm = run_ws(q, cm, flags=mpdp._FLAG_FORCE_GENERAL)
        ref = oracle.mpdp(q, cm)
        check_memo(q, gm, ref)
        check_plan(q, res, ref)
        check_stats(q, res, ref, general=True)


@pytest.mark.parametrize("cm", CMS)
def test_ablations_leave_results_unchanged(cm):
    """The measurement-only ablations (DPSUB's vertex-based candidates on the
    GPU; the tree kernel without LDS compaction; prune not fused into
    evaluate) reach the oracle's memo bit for bit; DPSUB evaluates 2^|S| - 2
    candidates per connected set (the oracle's DPSUB also counts the empty
    and the full subset)."""
    for q in [W.star(11, 4), W.snowflake(14, 5), W.cycle_chords(2, n=11, chords=3), W.clique(8, 1),
              W.random_connected(11, 3, 0.3)]:
        ref = oracle.mpdp(q, cm)
        res, gm = run_ws(q, cm, flags=mpdp.MPDP_FLAG_ABLATE_DPSUB)
        check_memo(q, gm, ref)
        check_plan(q, res, ref)
        d = oracle.dpsub(q, cm)
        assert res.stats["evaluated_pairs"] == d.evaluated - 2 * d.connected_sets, q.name
        assert 2 * res.stats["ccp_pairs"] == ref.ccp_ordered, q.name
        if q.m == q.n - 1:
            for flag in (mpdp.MPDP_FLAG_ABLATE_NO_COMPACTION, mpdp.MPDP_FLAG_ABLATE_UNFUSED_PRUNE):
                res, gm = run_ws(q, cm, flags=flag)
                check_memo(q, gm, ref)
                check_plan(q, res, ref)
                assert 2 * res.stats["ccp_pairs"] == ref.ccp_ordered, q.name


def test_self_allocating_entry_point():
    q = W.cycle_chords(7, n=12, chords=5)
    res = mpdp.mpdp_optimize(q, mpdp.MPDP_COST_PGLIKE)
    ref = oracle.mpdp(q, oracle.COST_PGLIKE)
    check_plan(q, res, ref)


def test_repeat_runs_identical():
    """Tie storm: every split costs the same; results must not depend on
    scheduling (three runs, same bits)."""
    q = W.all_equal_clique(12)
    outs = [run_ws(q, mpdp.MPDP_COST_COUT) for _ in range(3)]
    for res, gm in outs[1:]:
        for k in ("cost", "card", "left", "op"):
            assert np.array_equal(gm[k], outs[0][1][k])
    check_memo(q, outs[0][1], oracle.mpdp(q))


@pytest.mark.parametrize("cm", CMS)
def test_widest_bitmap_chain32(cm):
    """n = 32 fills the 32-bit relation bitmap (2^32 - 33 candidates);
    checked against the chain interval DP."""
    q = W.chain(32, 11)
    res = mpdp.mpdp_optimize(q, cm)
    ref = chain_interval_dp(q, cm)
    full = (1 << 32) - 1
    c, k, L, op = ref[full]
    assert res.cost == c
    assert res.plan[-1]["relset"] == full and res.plan[-1]["op"] == op
    assert res.plan[res.plan[-1]["left"]]["relset"] == L
    for nd in res.plan[32:]:
        S = nd["relset"]
        c, k, L, op = ref[S]
        assert nd["cost"] == c and nd["card"] == k and res.plan[nd["left"]]["relset"] == L
    assert res.stats["connected_sets"] == 32 * 33 // 2 - 32


def bits(x):
    return int(np.float64(x).view(np.uint64))


@pytest.mark.parametrize("cm", CMS)
def test_widest_star32(cm):
    """A 32-relation star fills the bitmap on the depth-one path (levels of
    up to C(31, 15) = 300 M connected sets).  Checked with what holds at any
    size: the counts of connected sets and csg-cmp pairs; the plan recosts
    to the root cost; every plan node of at most 16 relations equals the
    oracle's root of its induced sub-query; and under C_out the root cost is
    the closed form within rounding: every plan of a star joins one leaf at
    a time onto the hub, so C_out sums the cardinalities of the growing
    prefixes, and exchanging two neighbouring leaves shows that ascending
    card(v) * sel(0, v) is an optimal order (the clamp at 1 is monotone)."""
    q = W.star(32, 7)
    res = mpdp.mpdp_optimize(q, cm)
    assert res.stats["connected_sets"] == (1 << 31) - 1
    assert res.stats["ccp_pairs"] == 31 * (1 << 30)
    assert oracle.recost_plan(q, res.plan, cm) == res.cost
    checked = 0
    for nd in res.plan[32:]:
        S = nd["relset"]
        if bin(S).count("1") > 16:
            continue
        sub, rel = oracle.induced(q, S)
        m = oracle.mpdp(sub, cm)
        assert bits(nd["cost"]) == bits(m.root_cost) and bits(nd["card"]) == bits(m.card[m.full]), S
        assert res.plan[nd["left"]]["relset"] == oracle.expand(rel, int(m.left[m.full])), S
        assert nd["op"] == int(m.op[m.full]), S
        checked += 1
    assert checked == 15
    if cm == mpdp.MPDP_COST_COUT:
        f = sorted(float(q.card[v]) * float(q.sel[v - 1]) for v in range(1, 32))
        prefix, total = float(q.card[0]), 0.0
        for x in f:
            prefix *= x
            total += max(1.0, prefix)
        assert abs(res.cost - total) <= 1e-12 * total, (res.cost, total)


def test_recorded_sequence_replays():
    """Queries of up to 20 relations replay a launch sequence recorded once
    per workspace and shape: replays with new data, interleaved with other
    shapes, eager torch work and synchronizations, each match the oracle.
    A star and a chain of 12 relations share a workspace, model and size but
    not their level kernels (the star's tree has depth one from relation 0),
    so each must get its own recording."""
    import torch
    ws = {n: mpdp.workspace(n, 1, "cuda") for n in (12, 14)}
    refs = {}
    for rnd in range(4):
        for cm in (mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE):
            for q in (W.star(12, rnd), W.chain(12, rnd), W.snowflake(14, rnd), W.cycle_chords(rnd, n=12, chords=3),
                      W.random_connected(14, rnd, 0.3)):
                key = (q.name, cm)
                if key not in refs:
                    refs[key] = oracle.mpdp(q, cm)
                ref = refs[key]
                res = mpdp.mpdp_optimize_ws(q, cm, ws[q.n])
                check_plan(q, res, ref)
                assert res.stats["connected_sets"] == ref.connected_sets, q.name
                x = torch.arange(1000, device="cuda", dtype=torch.float32).sum()
                torch.cuda.synchronize()
                assert float(x) == 499500.0
