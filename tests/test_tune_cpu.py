"""The batch tuner's decisions with a scripted timer (host only: plans are
set and read through the library, no batch runs)."""
import pytest

from paper_1407_1465_amd import rsagpu, tune


def plan_of(width, kind):
    p = rsagpu.get_plan(width, kind)
    return (p.radix_bits, p.lanes_per_op, p.window_bits)


@pytest.fixture
def slot():
    width, kind = 32, 3
    yield width, kind
    rsagpu.set_plan(width, kind, 0, 0, 0)


def scripted(width, kind, script):
    """A timer whose n-th timing of plan P is script(P, n)."""
    calls = {}

    def timer():
        p = plan_of(width, kind)
        n = calls.get(p, 0)
        calls[p] = n + 1
        return script(p, n)
    return timer


def test_a_lucky_timing_does_not_move_the_descent(slot):
    width, kind = slot
    start = plan_of(width, kind)
    cands = [c for c in tune.candidate_plans(width, kind) if c != start]
    good, lucky = cands[0], cands[1]

    def script(p, n):
        if p == good:
            return 9.0                          # truly faster
        if p == lucky:
            return 5.0 if n == 0 else 11.0      # one lucky timing
        return 10.0
    chosen, ms = tune.tune_batch(None, [slot], timer=scripted(width, kind, script))
    assert chosen[slot] == good and plan_of(width, kind) == good
    assert ms == 9.0


def test_a_choice_that_loses_the_final_check_is_rolled_back(slot):
    width, kind = slot
    start = plan_of(width, kind)
    cands = [c for c in tune.candidate_plans(width, kind) if c != start]
    fickle = cands[0]

    def script(p, n):
        if p == fickle:
            return 9.0 if n < 2 else 10.5      # fast while tuned, slow when checked
        return 10.0
    chosen, ms = tune.tune_batch(None, [slot], timer=scripted(width, kind, script))
    assert chosen[slot] == start and plan_of(width, kind) == start
    assert ms == 10.0


def test_knobs_are_tuned_and_checked(slot):
    width, kind = slot
    state = {"forks": 3}

    def apply(v):
        state["forks"] = v

    def timer():
        return 8.0 if state["forks"] == 1 else 10.0
    chosen, ms = tune.tune_batch(None, [slot], timer=timer, knobs=[("forks", [3, 2, 1, 0], apply)])
    assert chosen["forks"] == 1 and state["forks"] == 1 and ms == 8.0
    assert chosen[slot] == plan_of(width, kind)
