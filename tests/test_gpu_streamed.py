"""GPU parity of the streamed sweep (operators and state in HBM, one launch
per sweep, graphs replayed by the host) against the FP64 oracle.

The streamed sweep is the path for problems whose operators and state do not
fit the LDS of one workgroup per CU. It computes the same steps as the
persistent sweep, so the bar is the same: 1e-6 relative (rel_err) on x, x_s
and lambda after the same number of sweeps, the history within 1e-6, and at
convergence the oracle's stopping sweep (one off only when the test sits on
its threshold). A 12,000-bus feeder (the 8500-bus recipe, more buses) does
not fit the persistent sweep in FP64, so the automatic choice takes the
streamed one; the oracle checks it at a fixed sweep count.
"""
import dataclasses

import numpy as np
import pytest

from conftest import feeder, oracle_prep, rel_err

pytestmark = pytest.mark.gpu


def _streamed(P, **kw):
    return P.ldopf_default_options(sweep_path=P.ldopf.LDOPF_PATH_STREAMED, **kw)


def _big_feeder():
    from synth import SPECS, make_feeder
    return make_feeder(dataclasses.replace(SPECS["8500"], n_bus=12000), 12000)


@pytest.mark.parametrize("name,T", [("13", 200), ("123", 100), ("123", 37), ("2500", 30)])
def test_streamed_fixed_sweeps(gpu, name, T):
    from oracle import admm
    P = gpu
    prob = P.ldopf_create(feeder(name), _streamed(P, max_iter=T, check_termination=0))
    assert prob.sizes().sweep_path == P.ldopf.LDOPF_PATH_STREAMED
    st = prob.solve()
    assert st.iterations == T
    ref = admm.solve(oracle_prep(name), max_iter=T, check=False)
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= 1e-6
    assert rel_err(xs, ref.xs) <= 1e-6
    assert rel_err(lam, ref.lam) <= 1e-6
    np.testing.assert_allclose(prob.get_history(), ref.history, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("name", ["13", "123"])
def test_streamed_converged(gpu, name):
    from oracle import admm
    P = gpu
    prob = P.ldopf_create(feeder(name), _streamed(P))
    st = prob.solve()
    ref = admm.solve(oracle_prep(name))
    assert st.converged == 1 and ref.converged
    assert st.pres <= st.eps_prim and st.dres <= st.eps_dual
    if st.iterations != ref.iters:
        assert abs(st.iterations - ref.iters) == 1
        t = min(st.iterations, ref.iters) - 1
        r = ref.history[t]
        assert min(abs(r[0] - r[2]) / r[2], abs(r[1] - r[3]) / r[3]) < 1e-9
    else:
        xs, lam = prob.get_local()
        assert rel_err(prob.get_global(), ref.x) <= 1e-6
        assert rel_err(xs, ref.xs) <= 1e-6
        assert rel_err(lam, ref.lam) <= 1e-6
    assert abs(prob.objective() - ref.objective) / max(1.0, abs(ref.objective)) <= 1e-6


def test_streamed_equals_persistent(gpu):
    """Both paths compute the same sweep: after 300 sweeps of the 8500-bus
    feeder they agree to summation order."""
    P = gpu
    net = feeder("8500")
    T = 300
    a = P.ldopf_create(net, P.ldopf_default_options(max_iter=T, check_termination=0))
    b = P.ldopf_create(net, _streamed(P, max_iter=T, check_termination=0))
    assert a.sizes().sweep_path == P.ldopf.LDOPF_PATH_PERSISTENT
    a.solve()
    b.solve()
    xa, la = a.get_local()
    xb, lb = b.get_local()
    assert rel_err(b.get_global(), a.get_global()) <= 1e-8
    assert rel_err(xb, xa) <= 1e-8
    assert rel_err(lb, la) <= 1e-8


def test_streamed_large_subsystem(gpu):
    """The 13-bus feeder as one subsystem of 261 variables (the kernel variant
    with up to sixteen rows per lane)."""
    from oracle import admm
    from test_gpu_large_subsystems import _create, single_subsystem_lp
    P = gpu
    lp1 = single_subsystem_lp(feeder("13"))
    T = 50
    prob = _create(P, lp1, _streamed(P, max_iter=T, check_termination=0))
    assert prob.sizes().sweep_path == P.ldopf.LDOPF_PATH_STREAMED
    prob.solve()
    ref = admm.solve(lp1, max_iter=T, check=False)
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= 1e-6
    assert rel_err(xs, ref.xs) <= 1e-6
    assert rel_err(lam, ref.lam) <= 1e-6


def test_streamed_mid_size_subsystems(gpu):
    """The 123-bus feeder merged into 79 subtrees of up to 111 variables
    (the kernel variant with up to four rows per lane), against the oracle on
    the same consensus LP."""
    from oracle import admm
    from test_gpu_large_subsystems import _create, subtree_lp
    P = gpu
    lp = subtree_lp(feeder("123"), 6)
    assert 64 < max(len(s.gidx) for s in lp.subs) <= 256
    T = 100
    prob = _create(P, lp, _streamed(P, max_iter=T, check_termination=0))
    assert prob.solve().iterations == T
    ref = admm.solve(lp, max_iter=T, check=False)
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= 1e-6
    assert rel_err(xs, ref.xs) <= 1e-6
    assert rel_err(lam, ref.lam) <= 1e-6
    np.testing.assert_allclose(prob.get_history(), ref.history, rtol=1e-6, atol=1e-12)


def test_warm_start_streamed(gpu):
    """150 sweeps == 60 sweeps, fetch, warm start, 90 sweeps. The streamed
    sweep keeps u = x_s - lambda / rho per copy and returns x_s = u + lambda /
    rho, so a warm start from the returned x_s forms u again up to one
    rounding: the two runs agree to 1e-13 (on this feeder bit for bit)."""
    P = gpu
    net = feeder("123")
    a = P.ldopf_create(net, _streamed(P, max_iter=150, check_termination=0))
    a.solve()
    xs_a, lam_a = a.get_local()
    b = P.ldopf_create(net, _streamed(P, max_iter=60, check_termination=0))
    b.solve()
    xs_m, lam_m = b.get_local()
    c = P.ldopf_create(net, _streamed(P, max_iter=90, check_termination=0))
    c.warm_start(xs_m, lam_m)
    c.solve()
    xs_c, lam_c = c.get_local()
    assert rel_err(xs_c, xs_a) <= 1e-13 and rel_err(lam_c, lam_a) <= 1e-13


def test_too_large_for_the_persistent_sweep(gpu):
    """12,000 buses in FP64: the persistent sweep refuses, the automatic
    choice streams, and 30 sweeps match the oracle."""
    from oracle import admm, model
    P = gpu
    net = _big_feeder()
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_create(net, P.ldopf_default_options(sweep_path=P.ldopf.LDOPF_PATH_PERSISTENT))
    assert e.value.code == P.ldopf.LDOPF_UNSUPPORTED
    T = 30
    prob = P.ldopf_create(net, P.ldopf_default_options(max_iter=T, check_termination=0))
    assert prob.sizes().sweep_path == P.ldopf.LDOPF_PATH_STREAMED
    st = prob.solve()
    assert st.iterations == T
    ref = admm.solve(admm.prepare(model.decompose(net)), max_iter=T, check=False)
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= 1e-6
    assert rel_err(xs, ref.xs) <= 1e-6
    assert rel_err(lam, ref.lam) <= 1e-6
    # in the FP32-mixed form the same feeder takes half the LDS and stays on
    # the persistent sweep
    p32 = P.ldopf_create(net, P.ldopf_default_options(max_iter=T, check_termination=0,
                                                      precision=P.ldopf.LDOPF_FP32_MIXED))
    assert p32.sizes().sweep_path == P.ldopf.LDOPF_PATH_PERSISTENT
    p32.solve()
    xs32, _ = p32.get_local()
    assert rel_err(p32.get_global(), ref.x) <= 1e-4
    assert rel_err(xs32, ref.xs) <= 1e-4


def test_streamed_refusals(gpu):
    P = gpu
    L = P.ldopf
    net = feeder("13")
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_create(net, _streamed(P, precision=L.LDOPF_FP32_MIXED))
    assert e.value.code == L.LDOPF_UNSUPPORTED
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_create(net, _streamed(P, residual_form=L.LDOPF_RESIDUAL_AGGREGATED))
    assert e.value.code == L.LDOPF_UNSUPPORTED
    prob = P.ldopf_create(net, _streamed(P, max_iter=10, check_termination=0))
    with pytest.raises(P.LdopfError) as e:
        prob.solve_noalloc()
    assert e.value.code == L.LDOPF_UNSUPPORTED
    other = P.ldopf_create(net, P.ldopf_default_options(max_iter=10, check_termination=0))
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_solve_many([other, prob])
    assert e.value.code == L.LDOPF_UNSUPPORTED
    with pytest.raises(P.LdopfError) as e:
        prob.set_options(P.ldopf_default_options(max_iter=10))  # the path is fixed at creation
    assert e.value.code == L.LDOPF_INVALID_ARGUMENT
    with pytest.raises(P.LdopfError) as e:
        prob.set_options(_streamed(P, max_iter=10, rho_update=L.LDOPF_RHO_BALANCE))
        prob.solve()
    assert e.value.code == L.LDOPF_UNSUPPORTED
    srv = P.Server()
    try:
        with pytest.raises(P.LdopfError) as e:
            srv.submit(net, _streamed(P))
        assert e.value.code == L.LDOPF_UNSUPPORTED
    finally:
        srv.close()
