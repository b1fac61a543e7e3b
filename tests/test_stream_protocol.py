"""A CPU model of the streamed sweep's control words, graph by graph.

The streamed sweep captures 32 sweeps per HIP graph, one launch each: the
launch of sweep k, whose block 0 tests sweep k - 1 (the block sums the
previous launch left) and then either stops the solve or sets the sweep
number to k, while its other blocks compute sweep k, writing x (and x_s,
lambda, the block sums) into the buffers of parity k % 2 (the parity is
fixed per graph node: node i computes sweep 32 g + i + 1). Those blocks may
see the stop word before or after block 0 sets it; every launch after the
stop returns at once. The host replays the graph until the stop word is
set and then copies the state of the returned sweep out of its buffers.

The model runs that schedule for a stopping sweep T (the first sweep whose
test passes) or the sweep limit, and checks that the returned sweep is T (or
the limit), that its x is the x computed in sweep T and was not overwritten
by a later launch, that x_s and lambda are sweep T's, that every sweep up
to T was tested once and in order, and that each graph that does not stop
advances the sweep number by 32. A planted mistake (a parity chosen by the
sweep number read at run time rather than by the node, an off-by-one in the
limit, x_s and lambda in one buffer) is caught.
"""
import pytest

GRAPH = 32


def run(stop_at, max_iter, check=True, late=False, bug=None):
    ctrl = [0, 1 if max_iter == 0 else 0]  # [sweep being computed, stopped]
    xh = [None, None]   # the two halves of x: tag = sweep that wrote it
    sh = [0, 0]         # the two buffers of x_s and lambda (buffer 0 starts with sweep 0)
    tested = []
    status_iters = 0
    graphs = 0
    while True:
        before = ctrl[0]
        for i in range(GRAPH):
            if ctrl[1]:
                continue  # every launch after the stop returns at once
            k = GRAPH * graphs + i + 1  # the sweep this node computes
            stop_before = ctrl[1]
            # block 0: the test of sweep k - 1
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
            par = (i + 1) % 2 if bug != "half" else ctrl[0] % 2
            # the other blocks compute sweep k unless they read the stop word
            # after block 0 set it
            if not (ctrl[1] if late else stop_before):
                xh[par] = k
                sh[par if bug != "one-buffer" else 0] = k
        graphs += 1
        if ctrl[1]:
            break
        assert ctrl[0] == before + GRAPH, "a graph that did not stop advanced the count wrongly"
        assert graphs < 10_000
    T = ctrl[0]
    x = xh[T % 2] if T >= 1 else None
    xs = sh[T % 2 if bug != "one-buffer" else 0]
    return T, x, xs, tested, status_iters


@pytest.mark.parametrize("late", [False, True])
@pytest.mark.parametrize("stop_at,max_iter", [(1, 100), (2, 100), (31, 100), (32, 100), (33, 100), (64, 100),
                                              (65, 1000), (10**9, 1), (10**9, 32), (10**9, 33), (10**9, 97)])
def test_returned_state_is_the_stopping_sweep(stop_at, max_iter, late):
    T, x, xs, tested, iters = run(stop_at, max_iter, late=late)
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


@pytest.mark.parametrize("bug", ["half", "limit", "one-buffer"])
def test_planted_mistakes_are_caught(bug):
    caught = False
    for late in (False, True):
        for stop_at, max_iter in [(5, 100), (32, 100), (10**9, 40)]:
            try:
                T, x, xs, tested, iters = run(stop_at, max_iter, late=late, bug=bug)
                want = min(stop_at, max_iter)
                assert T == want and x == want and xs == want
            except AssertionError:
                caught = True
    assert caught, bug
