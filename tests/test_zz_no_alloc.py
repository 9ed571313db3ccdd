"""mpdp_optimize_noalloc (the entry point for callers that cannot allocate)
against mpdp_optimize_ws on the same queries: the same plan, root cost bits
and counters, on consecutive calls whose second query is smaller than the
first (the array keeps the first call's memo, which must not leak into the
second), and at the size limit."""
import numpy as np
import pytest

from paper_2202_13511_amd import mpdp, workloads as W

pytestmark = pytest.mark.gpu


def same(a, b, name):
    assert np.float64(a.cost).view(np.uint64) == np.float64(b.cost).view(np.uint64), name
    assert a.plan == b.plan, name
    for key in ("connected_sets", "ccp_pairs", "evaluated_pairs", "candidates"):
        assert a.stats[key] == b.stats[key], (name, key)


@pytest.mark.parametrize("cm", [mpdp.MPDP_COST_COUT, mpdp.MPDP_COST_PGLIKE])
def test_noalloc_matches_workspace_entry_point(cm):
    import torch
    # a large query, then a smaller one of another shape, then the largest
    # size the array takes, then a tree join
    queries = [W.cycle_chords(0, n=18, chords=6), W.star(12, 3), W.clique(14, 1),
               W.chain(20, 2), W.snowflake(20, 4)]
    for q in queries:
        print(f"noalloc {q.name} cm={cm}", flush=True)
        ws = mpdp.workspace(q.n, cm, "cuda")
        want = mpdp.mpdp_optimize_ws(q, cm, ws)
        del ws
        got = mpdp.mpdp_optimize_noalloc(q, cm)
        same(got, want, q.name)
        # again on torch's current stream
        got = mpdp.mpdp_optimize_noalloc(q, cm, stream=torch.cuda.current_stream())
        same(got, want, q.name)


def test_noalloc_limits():
    q = W.star(21, 0)
    with pytest.raises(mpdp.MpdpError) as e:
        mpdp.mpdp_optimize_noalloc(q, mpdp.MPDP_COST_COUT)
    assert e.value.status == mpdp.MPDP_ETOOLARGE
    q = W.star(8, 0)
    with pytest.raises(mpdp.MpdpError) as e:
        mpdp.mpdp_optimize_noalloc(q, mpdp.MPDP_COST_COUT, flags=mpdp.MPDP_FLAG_TIMING)
    assert e.value.status == mpdp.MPDP_EINVAL
    assert mpdp.mpdp_noalloc_scratch_bytes() >= mpdp.mpdp_workspace_bytes(mpdp.MPDP_NOALLOC_MAX_REL)
