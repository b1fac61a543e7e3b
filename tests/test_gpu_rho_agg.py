"""Residual balancing of rho and the aggregated residual form on the device,
against the FP64 oracle.

* Residual balancing (LDOPF_RHO_BALANCE; oracle admm.RhoBalance with lag 4):
  the same rho changes at the same sweeps (rho values are products of powers
  of tau, exact in binary), and x, x_s, lambda and the residual history
  within 1e-6 after a fixed number of sweeps; the same stopping sweep when
  run to the tolerance.
* The aggregated residual form (LDOPF_RESIDUAL_AGGREGATED; oracle
  form="aggregated"): the residual history within 1e-6 and the same stopping
  sweep; the iterate does not depend on the form.
"""
import numpy as np
import pytest

from conftest import feeder, oracle_prep, rel_err

pytestmark = pytest.mark.gpu


def _rule(**kw):
    from oracle import admm
    return admm.RhoBalance(mu=10.0, tau=2.0, period=kw.get("period", 20), lag=4, max_changes=kw.get("max_changes", 16))


def _opts(P, T=None, **kw):
    o = dict(kw)
    if T is not None:
        o.update(max_iter=T, check_termination=0)
    return P.ldopf_default_options(**o)


def _same_state(prob, ref, tol):
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= tol
    assert rel_err(xs, ref.xs) <= tol
    assert rel_err(lam, ref.lam) <= tol


@pytest.mark.parametrize("name,T", [("123", 1500), ("2500", 1300)])
def test_rho_balance_fixed_sweeps(gpu, name, T):
    from oracle import admm
    P = gpu
    prob = P.ldopf_create(feeder(name), _opts(P, T, rho_update=1, rho_period=20))
    st = prob.solve()
    ref = admm.solve(oracle_prep(name), max_iter=T, check=False, balance=_rule())
    assert ref.rho_log, "the rule should fire in this run"
    assert prob.get_rho_log() == ref.rho_log
    assert st.rho == ref.rho and st.rho_changes == len(ref.rho_log)
    _same_state(prob, ref, 1e-6)
    np.testing.assert_allclose(prob.get_history(), ref.history, rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("name", ["13", "123"])
def test_rho_balance_converged(gpu, name):
    from oracle import admm
    P = gpu
    prob = P.ldopf_create(feeder(name), _opts(P, rho_update=1, rho_period=20))
    st = prob.solve()
    ref = admm.solve(oracle_prep(name), balance=_rule())
    assert st.converged and ref.converged
    assert st.iterations == ref.iters
    assert prob.get_rho_log() == ref.rho_log
    _same_state(prob, ref, 1e-6)


def test_rho_balance_fp32_mixed(gpu):
    """FP32 bulk, FP64 test: the rule reads the same FP64 sums, so the
    changes are the oracle's as long as the FP32 residuals stay far from a
    tie; the iterate within 1e-4."""
    from oracle import admm
    P = gpu
    T = 1500
    prob = P.ldopf_create(feeder("123"), _opts(P, T, rho_update=1, rho_period=20, precision=1))
    prob.solve()
    ref = admm.solve(oracle_prep("123"), max_iter=T, check=False, balance=_rule())
    assert prob.get_rho_log() == ref.rho_log
    assert rel_err(prob.get_global(), ref.x) <= 1e-4


@pytest.mark.parametrize("name,T", [("13", 300), ("123", 200), ("2500", 30), ("8500", 100)])
def test_aggregated_residuals_fixed_sweeps(gpu, name, T):
    from oracle import admm
    P = gpu
    prob = P.ldopf_create(feeder(name), _opts(P, T, residual_form=1))
    st = prob.solve()
    assert st.iterations == T
    ref = admm.solve(oracle_prep(name), max_iter=T, check=False, form="aggregated")
    _same_state(prob, ref, 1e-6)
    np.testing.assert_allclose(prob.get_history(), ref.history, rtol=1e-6, atol=1e-12)
    # the form changes only the test's quantities, not the iterate
    paper = P.ldopf_create(feeder(name), _opts(P, T))
    paper.solve()
    np.testing.assert_array_equal(prob.get_global(), paper.get_global())


@pytest.mark.parametrize("name", ["13", "123"])
def test_aggregated_residuals_converged(gpu, name):
    from oracle import admm
    P = gpu
    prob = P.ldopf_create(feeder(name), _opts(P, residual_form=1))
    st = prob.solve()
    ref = admm.solve(oracle_prep(name), form="aggregated")
    assert st.converged and ref.converged
    if st.iterations != ref.iters:
        assert abs(st.iterations - ref.iters) == 1
        r = ref.history[min(st.iterations, ref.iters) - 1]
        assert min(abs(r[0] - r[2]) / r[2], abs(r[1] - r[3]) / r[3]) < 1e-9
    else:
        _same_state(prob, ref, 1e-6)


def test_aggregated_fp32_and_many_small_workgroups(gpu):
    """FP32 bulk with FP64 aggregated sums; and a plan of many small
    workgroups, where most variables are shared between workgroups and their
    aggregated sums cross the exchange."""
    from oracle import admm
    P = gpu
    T = 150
    ref = admm.solve(oracle_prep("123"), max_iter=T, check=False, form="aggregated")
    f32 = P.ldopf_create(feeder("123"), _opts(P, T, residual_form=1, precision=1))
    f32.solve()
    assert rel_err(f32.get_global(), ref.x) <= 1e-4
    np.testing.assert_allclose(f32.get_history()[:, [1, 3]], ref.history[:, [1, 3]], rtol=1e-3)
    small = P.ldopf_create(feeder("123"), _opts(P, T, residual_form=1, rows_per_part=64, block_threads=128))
    assert small.sizes().n_parts > 20
    small.solve()
    _same_state(small, ref, 1e-6)
    np.testing.assert_allclose(small.get_history(), ref.history, rtol=1e-6, atol=1e-12)


def test_both_together(gpu):
    from oracle import admm
    P = gpu
    T = 1500
    prob = P.ldopf_create(feeder("123"), _opts(P, T, residual_form=1, rho_update=1, rho_period=20))
    prob.solve()
    ref = admm.solve(oracle_prep("123"), max_iter=T, check=False, form="aggregated", balance=_rule())
    assert prob.get_rho_log() == ref.rho_log
    _same_state(prob, ref, 1e-6)
    np.testing.assert_allclose(prob.get_history(), ref.history, rtol=1e-6, atol=1e-12)
