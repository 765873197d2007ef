"""Host logic of tail splitting (mq_plan_split): the plan's pieces cover each
split instance's steps in order, each piece waits for its predecessor queued
before it, and the reported makespans are those of a greedy list schedule of
the plan, recomputed here independently.  No GPU needed."""
import heapq
import os

import pytest

SETUP = 2  # steps charged per piece for its set-up


@pytest.fixture(scope="module")
def mq():
    import torch  # noqa: F401  (load the HIP runtime that torch ships first)
    from paper_2507_19246_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmq.so not built")
    import paper_2507_19246_amd as mq
    return mq


def list_schedule(durations, deps, slots):
    """Greedy list schedule: entries in order, each on the first free slot,
    not before its dependency has ended."""
    free = [0.0] * slots
    heapq.heapify(free)
    end = []
    for d, dep in zip(durations, deps):
        t = heapq.heappop(free)
        if dep >= 0:
            t = max(t, end[dep])
        end.append(t + d)
        heapq.heappush(free, t + d)
    return max(end) if end else 0.0


def three_level_mix():
    # 32 x 1024, 32 + 128 x 512, 128 + 512 x 256 steps (fine and coupled coarse runs)
    return [1024] * 32 + [512] * 160 + [256] * 640


def check_plan(steps, plan, slots):
    n = len(steps)
    seen = {}
    for e, (o, f, ln, d) in enumerate(zip(plan["orig"], plan["first"], plan["len"], plan["dep"])):
        assert 0 <= o < n and ln >= 1
        if f == 0:
            assert d == -1
        else:
            assert 0 <= d < e and plan["orig"][d] == o
            assert plan["first"][d] + plan["len"][d] == f
        seen.setdefault(o, []).append((f, ln))
    assert sorted(seen) == list(range(n))
    for o, parts in seen.items():
        pos = 0
        for f, ln in parts:
            assert f == pos
            pos += ln
        assert pos == steps[o]
    piece = [ln != steps[o] for o, ln in zip(plan["orig"], plan["len"])]
    dur = [ln + (SETUP if p else 0) for ln, p in zip(plan["len"], piece)]
    assert plan["makespan"][1] == pytest.approx(list_schedule(dur, plan["dep"], slots))
    assert plan["makespan"][0] == pytest.approx(list_schedule(steps, [-1] * n, slots))


def test_three_level_mix_is_split(mq):
    steps = three_level_mix()
    plan = mq.plan_split(steps, 256, 32)
    check_plan(steps, plan, 256)
    mk0, mk = plan["makespan"]
    assert mk0 == 1280.0  # every start and end is a multiple of 256 steps
    assert mk < 0.95 * mk0
    assert len(plan["orig"]) > len(steps)
    # the longest instances stay whole and come first
    assert plan["orig"][:32] == list(range(32)) and plan["len"][:32] == [1024] * 32
    # only instances of at most a quarter of the longest are split
    split = {o for o, ln in zip(plan["orig"], plan["len"]) if ln != steps[o]}
    assert split and all(steps[o] <= 256 for o in split)


@pytest.mark.parametrize("S", [16, 32, 64, 96])
def test_plan_invariants_for_piece_lengths(mq, S):
    steps = three_level_mix()
    plan = mq.plan_split(steps, 256, S)
    check_plan(steps, plan, 256)
    assert all(ln <= S for o, ln in zip(plan["orig"], plan["len"]) if ln != steps[o])


def test_no_split_when_it_does_not_pay(mq):
    # fewer instances than slots
    p = mq.plan_split([256] * 100, 256)
    assert p["orig"] == list(range(100)) and p["makespan"][0] == p["makespan"][1]
    # equal lengths: nothing to balance
    p = mq.plan_split([256] * 1000, 256)
    assert len(p["orig"]) == 1000
    # switched off
    p = mq.plan_split(three_level_mix(), 256, -1)
    assert len(p["orig"]) == len(three_level_mix())
    check_plan([7], mq.plan_split([7], 1), 1)


def test_plan_rejects_bad_input(mq):
    from paper_2507_19246_amd import _lib
    with pytest.raises(_lib.MQError):
        mq.plan_split([4, 0, 4], 2)
    with pytest.raises(_lib.MQError):
        mq.plan_split([4, 4], 0)
    with pytest.raises(_lib.MQError):
        mq.plan_split([4, 4], 2, -2)
