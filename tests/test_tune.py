"""Schedule autotuner: the radix-order candidates (CPU) and one tuning pass of
each objective on a small lattice (GPU).  Schedules change speed and rounding
only; the parity of a radix order is in test_gpu_parity.py."""
import itertools

import pytest

from paper_2606_06247_amd import tune


def test_radix_order_candidates_index_the_lexicographic_orderings():
    """radix_order k >= 1 names the (k - 1)-th distinct ordering of the
    radices in lexicographic order from the ascending one; the candidates are
    the library order (0), ascending, descending, reversed and the two
    rotations, each once."""
    for L in (1120, 80, 100, 160, 200, 280, 392, 525, 256, 1029):
        rad = tune._factor(L)
        distinct = sorted(set(itertools.permutations(sorted(rad))))
        cands = tune.radix_order_candidates(L)
        assert cands[0] == 0
        orders = [tuple(rad)] + [distinct[k - 1] for k in cands[1:]]
        assert len(set(orders)) == len(orders)               # each ordering once
        assert all(1 <= k <= len(distinct) for k in cands[1:])
        want = {tuple(rad), distinct[0], distinct[-1], tuple(reversed(rad)),
                tuple(rad[1:] + rad[:1]), tuple(rad[-1:] + rad[:-1])}
        assert set(orders) == want
    assert tune.radix_order_candidates(1120) == [0, 1, 24, 15, 17]   # (8,4,5,7): asc, desc, rev, rot
    assert tune.radix_order_candidates(64) == [0]                       # one radix ordering only


def test_window_candidates_are_plannable_smooth_lengths():
    for n in (64, 96, 128, 1024):
        c = tune.window_candidates(n)
        assert c and all(L >= n + 4 and tune._factor(L) is not None for L in c)


@pytest.mark.gpu
@pytest.mark.parametrize("batch", [0, 2])
def test_tune_2d_returns_a_plannable_schedule(batch):
    from paper_2606_06247_amd import api
    ctx = api.Context(0)
    rec = tune.tune_2d(ctx, 64, "fp64", lines=(1,), batch=batch)
    assert set(rec) >= {"window_len", "lines_per_group", "radix_order", "ms", "default_ms", "trials"}
    assert rec["trials"] >= 1 and rec["ms"] > 0 and rec["radix_order"] >= 0
    prob = tune._problem_2d(64, "fp64", rec["window_len"], rec["lines_per_group"], rec["radix_order"])
    api.Plan(ctx, prob)
