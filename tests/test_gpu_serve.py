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


def test_release_as_soon_as_done(gpu):
    """A client that polls in a tight loop and releases each request the
    moment it reads DONE: the server's bookkeeping stays whole (every request
    counted once, nothing in use afterwards) and a released request is gone."""
    P = gpu
    from synth import make_feeder
    srv = P.Server(max_slots=4)
    ids = [srv.submit(make_feeder("13", 51000 + i), P.ldopf_default_options(precision=i % 2)) for i in range(8)]
    pending = set(ids)
    while pending:
        for rid in list(pending):
            state, _ = srv.poll(rid)
            if state == P.ldopf.LDOPF_REQ_DONE:
                srv.release(rid)
                pending.discard(rid)
            else:
                assert state in (P.ldopf.LDOPF_REQ_QUEUED, P.ldopf.LDOPF_REQ_RUNNING)
    s = srv.stats()
    assert s.completed == 8 and s.failed == 0 and s.running == 0 and s.queued == 0
    assert s.bytes_in_use == 0
    with pytest.raises(P.LdopfError):
        srv.poll(ids[0])


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", f"converged_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} missing")
    return np.load(path)


def test_served_results_match_the_oracle_alone_and_in_the_mix(gpu):
    """Requests of every size of the serving workload, in both precisions:
    each result is bit for bit the same served alone (one slot) and in the
    mix (eight slots), and matches the oracle: the 2500- and 8500-bus feeders
    against their converged FP64 oracle solutions (same stopping sweep, x
    within 1e-6 in FP64; x and objective within 1e-4 and the stopping sweep
    within 2% in FP32-mixed), the small fresh feeders against the oracle run
    for the same number of sweeps (1e-6 FP64, 1e-4 FP32-mixed)."""
    from conftest import rel_err
    from oracle import admm, model
    from synth import make_feeder
    P = gpu
    reqs = [(feeder("8500"), 0, "8500"), (feeder("2500"), 1, "2500"), (feeder("2500"), 0, "2500")]
    reqs += [(make_feeder("13", 52000 + i), i % 2, None) for i in range(3)]
    reqs += [(make_feeder("123", 52100 + i), (i + 1) % 2, None) for i in range(2)]
    results = []
    for slots in (1, 8):
        srv = P.Server(max_slots=slots)
        ids = [srv.submit(net, P.ldopf_default_options(precision=prec)) for net, prec, _ in reqs]
        out = []
        for rid in ids:
            state, st = srv.wait(rid, 120)
            assert state == P.ldopf.LDOPF_REQ_DONE and st.converged
            out.append((st.iterations, srv.fetch(rid)))
        results.append(out)
        srv.close()
    for (it_a, (x_a, xs_a, l_a)), (it_b, (x_b, xs_b, l_b)) in zip(*results):
        assert it_a == it_b
        np.testing.assert_array_equal(x_a, x_b)
        np.testing.assert_array_equal(xs_a, xs_b)
        np.testing.assert_array_equal(l_a, l_b)
    for (net, prec, gold), (it, (x, xs, lam)) in zip(reqs, results[1]):
        if gold is not None:
            g = _golden(gold)
            T = int(g["t_stop"])
            if prec == 0:
                assert it == T
                assert rel_err(x, g["x"]) <= 1e-6 and rel_err(xs, g["xs"]) <= 1e-6 and rel_err(lam, g["lam"]) <= 1e-6
            else:
                assert abs(it - T) <= 0.02 * T
                assert rel_err(x, g["x"]) <= 1e-4
        else:
            tol = 1e-6 if prec == 0 else 1e-4
            ref = admm.solve(model.decompose(net), max_iter=it, check=False)
            assert rel_err(x, ref.x) <= tol and rel_err(xs, ref.xs) <= tol
            if prec == 0:
                assert rel_err(lam, ref.lam) <= tol
