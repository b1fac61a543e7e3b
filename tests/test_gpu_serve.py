"""GPU tests of the serving loop: results are the same alone and in the mix,
admission under a small HBM budget, rejection and cancellation."""
import numpy as np
import pytest

from conftest import feeder

pytestmark = pytest.mark.gpu


def _mix():
    from synth import make_feeder
    nets = [make_feeder("13", 50000 + i) for i in range(4)] + [make_feeder("123", 50010 + i) for i in range(3)]
    return nets


def test_result_same_alone_and_in_the_mix(gpu):
    P = gpu
    nets = _mix()
    opts = [P.ldopf_default_options(precision=i % 2) for i in range(len(nets))]
    alone = []
    srv = P.Server(max_slots=1)
    for net, o in zip(nets, opts):
        rid = srv.submit(net, o)
        state, st = srv.wait(rid, 120)
        assert state == P.ldopf.LDOPF_REQ_DONE and st.converged
        alone.append((srv.fetch(rid), st.iterations))
    srv.close()
    srv = P.Server(max_slots=8)
    ids = [srv.submit(net, o) for net, o in zip(nets, opts)]
    for rid, ((x, xs, lam), it) in zip(ids, alone):
        state, st = srv.wait(rid, 120)
        assert state == P.ldopf.LDOPF_REQ_DONE
        assert st.iterations == it
        x2, xs2, lam2 = srv.fetch(rid)
        np.testing.assert_array_equal(x, x2)
        np.testing.assert_array_equal(xs, xs2)
        np.testing.assert_array_equal(lam, lam2)
    s = srv.stats()
    assert s.completed == len(nets) and s.failed == 0
    assert s.peak_running >= 2  # requests were in flight together
    assert 0 < s.p50_ms <= s.p99_ms <= s.max_ms


def test_results_match_a_direct_solve(gpu):
    P = gpu
    net = feeder("123")
    direct = P.ldopf_create(net)
    st = direct.solve()
    srv = P.Server(max_slots=2)
    rid = srv.submit(net)
    state, st2 = srv.wait(rid, 120)
    assert state == P.ldopf.LDOPF_REQ_DONE and st2.iterations == st.iterations
    x, _, _ = srv.fetch(rid)
    np.testing.assert_array_equal(x, direct.get_global())


def test_admission_under_a_small_budget(gpu):
    """A budget that holds one 123-bus request at a time still serves them all."""
    P = gpu
    from synth import make_feeder
    nets = [make_feeder("123", 60000 + i) for i in range(3)]
    need = max(P.ldopf_request_estimate(n)[0] for n in nets)
    srv = P.Server(hbm_budget_bytes=int(1.5 * need), max_slots=4)
    ids = [srv.submit(n) for n in nets]
    for rid in ids:
        state, _ = srv.wait(rid, 120)
        assert state == P.ldopf.LDOPF_REQ_DONE
    s = srv.stats()
    assert s.peak_running == 1 and s.peak_bytes_in_use <= s.budget_bytes


def test_over_budget_and_cancel(gpu):
    P = gpu
    need = P.ldopf_request_estimate(feeder("123"))[0]
    srv = P.Server(hbm_budget_bytes=need // 2, max_slots=2)
    with pytest.raises(P.LdopfError) as e:
        srv.submit(feeder("123"))
    assert e.value.code == -5
    srv.close()
    srv = P.Server(max_slots=1)
    first = srv.submit(feeder("123"))
    later = [srv.submit(feeder("13")) for _ in range(3)]
    try:
        srv.cancel(later[-1])
        cancelled = True
    except P.LdopfError:
        cancelled = False  # it may already have run
    srv.wait(first, 120)
    for rid in later[:-1]:
        assert srv.wait(rid, 120)[0] == P.ldopf.LDOPF_REQ_DONE
    if cancelled:
        assert srv.poll(later[-1])[0] == P.ldopf.LDOPF_REQ_FAILED
