"""A CPU model of the streamed sweep's control words, graph by graph.

The streamed sweep captures 32 sweeps per HIP graph, two launches each: the
global update of sweep k, whose block 0 first tests sweep k - 1 (the partial
sums its local update left) and then either stops the solve or sets the
sweep number to k, writing x into the half k % 2 of a two-part buffer (the
half is fixed per graph node: node i computes sweep 32 g + i + 1), and the
local update of sweep k. Every launch returns at once after the stop. The
host replays the graph until the stop word is set and then copies the half
of the returned sweep into x.

The model runs that schedule for a stopping sweep T (the first sweep whose
test passes) or the sweep limit, and checks that the returned sweep is T (or
the limit), that its x is the x computed in sweep T and was not overwritten
by a later global update, that x_s and lambda are sweep T's, that every
sweep up to T was tested once and in order, and that each graph that does
not stop advances the sweep number by 32. A planted mistake (a half chosen
by k rather than by the node, an off-by-one in the limit, the stop word
read after the local update) is caught.
"""
import pytest

GRAPH = 32


def run(stop_at, max_iter, check=True, bug=None):
    ctrl = [0, 1 if max_iter == 0 else 0]  # [sweep being computed, stopped]
    xh = [None, None]   # the two halves of x: tag = sweep that wrote it
    xs = 0              # sweep whose local update x_s / lambda hold
    tested = []
    status_iters = 0
    graphs = 0
    while True:
        before = ctrl[0]
        for i in range(GRAPH):
            # global update of the node's sweep; block 0 tests first
            if ctrl[1]:
                continue
            t = ctrl[0]
            if t >= 1:
                tested.append(t)
                status_iters = t
                passed = check and t >= stop_at
                limit = t >= max_iter if bug != "limit" else t > max_iter
                if passed or limit:
                    ctrl[1] = 1
                else:
                    ctrl[0] = t + 1
            else:
                ctrl[0] = 1
            half = (i + 1) % 2 if bug != "half" else ctrl[0] % 2
            # the other blocks compute x for the node's sweep either way
            xh[half] = 32 * graphs + i + 1
            # local update of the node's sweep (returns after the stop)
            if bug == "late-stop" or not ctrl[1]:
                xs = 32 * graphs + i + 1
        graphs += 1
        if ctrl[1]:
            break
        assert ctrl[0] == before + GRAPH, "a graph that did not stop advanced the count wrongly"
        assert graphs < 10_000
    T = ctrl[0]
    x = xh[T % 2] if T >= 1 else None
    return T, x, xs, tested, status_iters


@pytest.mark.parametrize("stop_at,max_iter", [(1, 100), (2, 100), (31, 100), (32, 100), (33, 100), (64, 100),
                                              (65, 1000), (10**9, 1), (10**9, 32), (10**9, 33), (10**9, 97)])
def test_returned_state_is_the_stopping_sweep(stop_at, max_iter):
    T, x, xs, tested, iters = run(stop_at, max_iter)
    want = min(stop_at, max_iter)
    assert T == want and iters == want
    assert x == want, "x of another sweep returned"
    assert xs == want, "x_s and lambda of another sweep returned"
    assert tested == list(range(1, want + 1))


def test_no_sweep_for_a_zero_limit():
    T, x, xs, tested, iters = run(5, 0)
    assert T == 0 and x is None and xs == 0 and tested == [] and iters == 0


def test_fixed_sweep_count_without_the_test():
    T, x, xs, tested, iters = run(3, 70, check=False)
    assert T == 70 and x == 70 and xs == 70


@pytest.mark.parametrize("bug", ["half", "limit", "late-stop"])
def test_planted_mistakes_are_caught(bug):
    caught = False
    for stop_at, max_iter in [(5, 100), (32, 100), (10**9, 40)]:
        try:
            T, x, xs, tested, iters = run(stop_at, max_iter, bug=bug)
            want = min(stop_at, max_iter)
            assert T == want and x == want and xs == want
        except AssertionError:
            caught = True
    assert caught, bug
