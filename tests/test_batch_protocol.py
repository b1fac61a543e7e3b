"""A CPU model of the batched sweep's control words, graph by graph.

The batched sweep captures 16 sweeps per HIP graph, two launches each: the
global update of sweep k, whose first blocks test sweep k - 1 for every
scenario still running (the partial sums its local update left) and clear
the mask of each scenario that passed, then either stop the batch (no
scenario left, or the sweep limit) or set the sweep number to k; its other
blocks write x into the half k % 2 of a two-part buffer (the half is fixed
per graph node: node i computes sweep 16 g + i + 1), for the scenarios whose
mask they read as set. Those blocks run beside the test blocks, so they may
read a mask or the stop word before or after the test changes it: the model
runs both. The local update of sweep k follows the whole global launch and
skips every scenario whose mask is clear. The host replays the graph until
the stop word is set, and reads each scenario's x from the half of its last
tested sweep.

For stopping sweeps drawn per scenario, the model checks that every scenario
returns the state of its own stopping sweep (or the limit): x computed in
that sweep and not overwritten by a later global update, x_s and lambda of
that sweep, every sweep up to it tested once and in order, and that each
graph that does not stop advances the sweep number by 16. Planted mistakes
(a half chosen by the sweep number read at run time, the mask read by the
local update before the test, an off-by-one in the limit) are caught.
"""
import random

import pytest

GRAPH = 16


def run(stops, max_iter, check=True, late=False, bug=None):
    B = len(stops)
    ctrl = [0, 0]              # [sweep being computed, stopped]
    active = [True] * B
    iters = [0] * B
    xh = [[0, 0] for _ in range(B)]   # per scenario, the two halves: tag = sweep that wrote it
    xs = [0] * B               # sweep whose local update x_s / lambda hold
    tested = [[] for _ in range(B)]
    graphs = 0
    while True:
        before = ctrl[0]
        for i in range(GRAPH):
            if ctrl[1]:
                continue
            k = GRAPH * graphs + i + 1     # the sweep this node computes
            mask_before, stop_before = active[:], ctrl[1]
            t = ctrl[0]
            if t >= 1:
                for s in range(B):
                    if active[s]:
                        tested[s].append(t)
                        iters[s] = t
                        if check and t >= stops[s]:
                            active[s] = False
                limit = t >= max_iter if bug != "limit" else t > max_iter
                if not any(active) or limit:
                    ctrl[1] = 1
                else:
                    ctrl[0] = t + 1
            else:
                ctrl[0] = 1
            half = (i + 1) % 2 if bug != "half" else ctrl[0] % 2
            # update blocks: the mask and the stop word as read before or
            # after the test blocks changed them
            mask = active if late else mask_before
            stopped = ctrl[1] if late else stop_before
            for s in range(B):
                if mask[s] and not stopped:
                    xh[s][half] = k
            # local update after the whole launch
            local_mask = active if bug != "early-mask" else mask_before
            if not ctrl[1]:
                for s in range(B):
                    if local_mask[s]:
                        xs[s] = k
        graphs += 1
        if ctrl[1]:
            break
        assert ctrl[0] == before + GRAPH, "a graph that did not stop advanced the count wrongly"
        assert graphs < 10_000
    x = [xh[s][iters[s] % 2] if iters[s] >= 1 else 0 for s in range(B)]
    return ctrl[0], iters, x, xs, tested


def _check(stops, max_iter, check=True, late=False, bug=None):
    T, iters, x, xs, tested = run(stops, max_iter, check, late, bug)
    want = [min(s, max_iter) if check else max_iter for s in stops]
    assert iters == want
    assert T == max(want)
    assert x == want, "x of another sweep returned"
    assert xs == want, "x_s and lambda of another sweep returned"
    assert all(tested[s] == list(range(1, want[s] + 1)) for s in range(len(stops)))


@pytest.mark.parametrize("late", [False, True])
@pytest.mark.parametrize("stops,max_iter", [([1, 2, 3], 100), ([15, 16, 17], 100), ([16, 33, 32, 64], 100),
                                            ([5, 10**9], 40), ([10**9] * 3, 16), ([10**9] * 2, 17),
                                            ([7, 7, 7], 7)])
def test_each_scenario_returns_its_stopping_sweep(stops, max_iter, late):
    _check(stops, max_iter, late=late)


@pytest.mark.parametrize("late", [False, True])
def test_random_stopping_sweeps(late):
    rng = random.Random(2310)
    for _ in range(50):
        stops = [rng.randint(1, 120) for _ in range(rng.randint(1, 9))]
        _check(stops, rng.choice([50, 64, 97, 200]), late=late)


def test_fixed_sweep_count_without_the_test():
    _check([3, 9, 1], 37, check=False)


@pytest.mark.parametrize("bug", ["half", "early-mask", "limit"])
def test_planted_mistakes_are_caught(bug):
    caught = False
    for late in (False, True):
        for stops, max_iter in [([5, 9, 40], 100), ([16, 17], 100), ([10**9, 3], 40)]:
            try:
                _check(stops, max_iter, late=late, bug=bug)
            except AssertionError:
                caught = True
    assert caught, bug
