"""Host-side scheduling of the serving loop (no GPU): which resident problems
an epoch advances under each policy."""
import types

import pytest

from paper_2409_16053_amd import serve


def _res(cells, rem):
    """Resident entries [request, handle, remaining steps] in arrival order."""
    return [[types.SimpleNamespace(pb=types.SimpleNamespace(cells=c)), None, k] for c, k in zip(cells, rem)]


def test_oldest_first_runs_the_oldest_and_fills_the_slack_in_arrival_order():
    srv = serve.Server(budget_bytes=1 << 30, epoch_steps=10, slack=0.25, min_epoch_work=1e6)
    big = 256 ** 3
    # oldest 256^3 (10 steps: 1.68e8), then two 32^3, a 256^3, a 64^3
    res = _res([big, 32 ** 3, 32 ** 3, big, 64 ** 3], [200, 10, 5, 100, 10])
    sel = srv._select(res)
    assert sel[0] == 0 and 3 not in sel       # the second large one waits
    assert sel == [0, 1, 2, 4]                # small ones ride in the 25% slack
    work = sum(res[i][0].pb.cells * min(res[i][2], 10) for i in sel)
    assert work <= 1.25 * big * 10


def test_oldest_first_floor_lets_small_problems_run_together():
    srv = serve.Server(budget_bytes=1 << 30, epoch_steps=10, slack=0.0, min_epoch_work=3 * 64 ** 3 * 10)
    res = _res([64 ** 3] * 5, [10] * 5)
    assert srv._select(res) == [0, 1, 2]


def test_all_policy_advances_everyone_and_bad_policy_is_refused():
    srv = serve.Server(budget_bytes=1 << 30, policy="all")
    assert srv._select(_res([8, 16, 32], [1, 2, 3])) == [0, 1, 2]
    with pytest.raises(ValueError):
        serve.Server(budget_bytes=1, policy="shortest")
