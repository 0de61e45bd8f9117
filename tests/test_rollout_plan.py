"""Host logic of the checkpointed rollout (no GPU): the backward plan visits
every step's adjoint exactly once in reverse order, recomputes each step at
most once and only from checkpoints the forward pass stored, keeps every
segment within the segment buffer, and never reads a kept slot after a
recomputation may have overwritten it (the segment buffer can alias the
first slots of the kept buffer)."""
import itertools

import pytest

from paper_1405_1253_amd.rollout import backward_plan, checkpoint_steps

CASES = [(n, k, c) for n, k, c in itertools.product((1, 7, 20, 100, 101), (0, 1, 5, 10, 20, 101),
                                                    (1, 3, 5, 10, 100)) if k <= n]


@pytest.mark.parametrize("n,keep,c", CASES)
def test_backward_plan(n, keep, c):
    plan = backward_plan(n, keep, c)
    saved = set(checkpoint_steps(n, keep, c))
    adj = [op[1] for op in plan if op[0] == "adjoint"]
    assert adj == list(range(n, 0, -1))                     # every step once, in reverse
    recomputes = [op for op in plan if op[0] == "recompute"]
    assert sum(b - a for _, a, b in recomputes) == n - keep  # each step at most once
    seen_recompute = False
    segment = None
    for op in plan:
        if op[0] == "recompute":
            _, a, b = op
            assert a in saved and 0 < b - a <= c
            seen_recompute, segment = True, (a, b)
        elif op[2] == "kept":
            _, t, _, i = op
            assert not seen_recompute                       # kept slots are read first
            assert 0 <= i < keep and t == n - keep + 1 + i
        else:
            _, t, _, i = op
            a, b = segment
            assert a < t <= b and i == t - a - 1


def test_checkpoints_with_the_kept_interval():
    """Interval = kept steps (ckpt_every = 0 in RolloutConfig): 5000 steps,
    1237 kept -> 3763 steps to recompute in 4 segments from the states after
    0, 1237, 2474 and 3711; the state after 4948 is stored as well (20
    states with an interval of 250)."""
    assert checkpoint_steps(5000, 1237, 1237) == [0, 1237, 2474, 3711, 4948]
    assert len(checkpoint_steps(5000, 1237, 250)) == 20
    plan = backward_plan(5000, 1237, 1237)
    assert [op[1:] for op in plan if op[0] == "recompute"] == [(3711, 3763), (2474, 3711), (1237, 2474),
                                                               (0, 1237)]


def test_checkpoints_every_interval_when_all_moments_are_kept():
    """A 2000-step rollout with a checkpoint every 100 steps stores the states
    after 0, 100, ..., 1900 even when every step's moments are kept (and the
    backward sweep then recomputes nothing)."""
    assert checkpoint_steps(2000, 2000, 100) == list(range(0, 2000, 100))
    assert [op for op in backward_plan(2000, 2000, 100) if op[0] == "recompute"] == []
