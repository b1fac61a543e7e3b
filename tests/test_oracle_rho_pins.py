"""Pins of the oracle's residual balancing of rho (Section III-D names the
scheme; the rule is the classic one on relative residuals, see
oracle.admm.RhoBalance), and mutation tests that show the pins catch a
plausible mistake.

* A rule that never fires leaves the run bit for bit the fixed-rho run.
* The dual update ADMM-3 ties lambda to the primal residual in every sweep:
  lambda_t - lambda_{t-1} = rho_t (B x - x_s), so pres_t equals
  ||lambda_t - lambda_{t-1}|| / rho_t exactly (up to rounding) in every
  sweep, also in the sweeps where rho changes. Rescaling lambda on a change
  (right only for the scaled dual lambda / rho) breaks it there.
* The fixed point does not move: with rho changing, the run still reaches
  the LP optimum (HiGHS) on the 13-bus feeder at a tight tolerance.
* Changes happen only where the rule is evaluated (sweeps k * period),
  take effect lag sweeps later, and stop after max_changes.
"""
import numpy as np
import pytest

from conftest import feeder, oracle_prep
from oracle import admm, central


def _run(name, T, **kw):
    lams, xs, xg = [], [], []

    def keep(t, prep, st):
        lams.append(st.lam.copy())
        xs.append(st.xs.copy())
        xg.append(st.x.copy())

    res = admm.solve(oracle_prep(name), max_iter=T, check=False, on_iter=keep, **kw)
    return res, lams, xs, xg


def _rho_per_sweep(res, rho0, T):
    rho = np.full(T, rho0)
    for t, r in res.rho_log:
        rho[t - 1:] = r
    return rho


def test_a_rule_that_never_fires_is_the_fixed_rho_run():
    fixed = admm.solve(oracle_prep("123"), max_iter=400, check=False)
    quiet = admm.solve(oracle_prep("123"), max_iter=400, check=False,
                       balance=admm.RhoBalance(mu=1e300, period=10))
    assert quiet.rho_log == []
    np.testing.assert_array_equal(fixed.history, quiet.history)
    np.testing.assert_array_equal(fixed.xs, quiet.xs)
    np.testing.assert_array_equal(fixed.lam, quiet.lam)


def _dual_identity_worst(res, lams, xs, xg, rho0, T):
    prep = res.prep
    rho = _rho_per_sweep(res, rho0, T)
    lam_prev = np.zeros_like(lams[0])
    worst = 0.0
    for t in range(T):
        pres = np.linalg.norm(xg[t][prep.gidx] - xs[t])
        step = np.linalg.norm(lams[t] - lam_prev) / rho[t]
        worst = max(worst, abs(pres - step) / max(pres, 1e-300))
        lam_prev = lams[t]
    return worst


def test_dual_update_identity_holds_across_rho_changes():
    T = 1500
    res, lams, xs, xg = _run("123", T, balance=admm.RhoBalance(period=20))
    assert len(res.rho_log) >= 3  # the rule fired several times
    assert _dual_identity_worst(res, lams, xs, xg, 100.0, T) <= 1e-9


def test_changes_follow_the_schedule():
    rule = admm.RhoBalance(period=50, lag=4, max_changes=5)
    res = admm.solve(oracle_prep("123"), max_iter=2000, check=False, balance=rule)
    assert 0 < len(res.rho_log) <= 5
    prev = 100.0
    for t, r in res.rho_log:
        assert (t - rule.lag) % rule.period == 0
        assert r / prev in (pytest.approx(rule.tau), pytest.approx(1.0 / rule.tau))
        prev = r
    assert res.rho == prev


def test_fixed_point_unchanged_by_balancing():
    net = feeder("13")
    f_lp, _, _ = central.solve_central(net)
    res = admm.solve(oracle_prep("13"), eps_rel=1e-8, balance=admm.RhoBalance(period=20))
    assert res.converged and res.rho_log
    assert abs(res.objective - f_lp) <= 1e-5 * max(1.0, abs(f_lp))


def test_mutation_rescaled_dual_is_caught(monkeypatch):
    monkeypatch.setattr(admm, "rescale_dual", lambda lam, r0, r1: lam * (r0 / r1))
    T = 1500
    res, lams, xs, xg = _run("123", T, balance=admm.RhoBalance(period=20))
    assert res.rho_log
    assert _dual_identity_worst(res, lams, xs, xg, 100.0, T) > 1e-3
