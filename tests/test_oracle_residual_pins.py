"""Pins of the oracle's termination test (Section III-C) and initial point
(Section V-A), and mutation tests that show each pin catches a plausible
mistake.

* The residual norms are checked against the printed definitions evaluated
  with explicit 0-1 selection matrices B_s (a different route from the
  oracle's, which never forms B_s), on a real trajectory and on crafted
  states where each branch of the max in eps_prim is the active one.
* The dual residual is pinned by a fact of ADMM itself: when no bound is
  active, the global update's optimality condition makes the aggregated dual
  residual equal to the stationarity residual ||c + sum_s B_s' lambda_s|| of
  the iterate (and, when every variable has a single copy, the printed form
  equals it too).
* The test is invariant under scaling the cost and rho together: with a
  factor 4 (exact in binary floating point) the trajectory of x, x_s is bit
  for bit the same, lambda, dres and eps_dual scale by exactly 4, and the
  stopping sweep does not move.
* The initial point is pinned by the first sweep of the two-bus case,
  derived by hand (tests/golden/two_bus.json, "first_sweep").
"""
import json
import os

import numpy as np
import pytest

from conftest import oracle_prep
from oracle import admm, model
from synth import two_bus

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------- literal printed formulas
def _selection_matrices(prep):
    """B_s as dense 0-1 matrices: row j of B_s picks the global variable of copy j."""
    n = prep.lp.n
    out = []
    for s in range(len(prep.lp.subs)):
        g = prep.gidx[prep.offsets[s]:prep.offsets[s + 1]]
        B = np.zeros((g.size, n))
        B[np.arange(g.size), g] = 1.0
        out.append(B)
    return out


def _printed_residuals(Bs, offsets, x, xs, xs_prev, lam, rho, eps_rel):
    """pres, dres, eps_prim, eps_dual of Section III-C, each sum over s taken
    outside the norm as printed, with B_s applied as a matrix."""
    blk = lambda v, s: v[offsets[s]:offsets[s + 1]]  # noqa: E731
    S = len(Bs)
    pres = np.sqrt(sum(np.sum((Bs[s] @ x - blk(xs, s)) ** 2) for s in range(S)))
    dres = rho * np.sqrt(sum(np.sum((Bs[s].T @ (blk(xs, s) - blk(xs_prev, s))) ** 2) for s in range(S)))
    nz = np.sqrt(sum(np.sum((Bs[s] @ x) ** 2) for s in range(S)))
    nxs = np.sqrt(sum(np.sum(blk(xs, s) ** 2) for s in range(S)))
    nl = np.sqrt(sum(np.sum((Bs[s].T @ blk(lam, s)) ** 2) for s in range(S)))
    return np.array([pres, dres, eps_rel * max(nz, nxs), eps_rel * nl])


def test_history_equals_the_printed_residuals_on_a_trajectory():
    prep = oracle_prep("13")
    Bs = _selection_matrices(prep)
    states = [admm.initial_state(prep)]
    states[0] = admm.State(states[0].x, states[0].xs.copy(), states[0].lam.copy())
    res = admm.solve(prep, max_iter=40, check=False,
                     on_iter=lambda t, p, st: states.append(admm.State(st.x.copy(), st.xs.copy(), st.lam.copy())))
    for t in range(1, 41):
        want = _printed_residuals(Bs, prep.offsets, states[t].x, states[t].xs, states[t - 1].xs, states[t].lam,
                                  100.0, 1e-4)
        np.testing.assert_allclose(res.history[t - 1], want, rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("big", ["z", "xs"])
def test_residual_function_on_crafted_states(big):
    """Random states where ||B x|| (big = "z") or ||x_s|| (big = "xs") is the
    larger norm, so each branch of eps_prim's max is exercised."""
    prep = oracle_prep("13")
    Bs = _selection_matrices(prep)
    rng = np.random.default_rng(7 if big == "z" else 8)
    n, nl = prep.lp.n, prep.gidx.size
    x = rng.normal(size=n) * (10.0 if big == "z" else 0.1)
    xs = rng.normal(size=nl) * (0.1 if big == "z" else 10.0)
    xs_prev = rng.normal(size=nl)
    lam = rng.normal(size=nl) * 30.0
    got = admm.residuals(prep, x[prep.gidx], xs, xs_prev, lam, 37.0, 3e-3, 0.0, "paper")
    want = _printed_residuals(Bs, prep.offsets, x, xs, xs_prev, lam, 37.0, 3e-3)
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=0.0)


# ------------------------------------------- ADMM stationarity of the iterate
def _random_consensus_lp(seed, n=60, S=25, single_copy=False):
    """A consensus LP with no finite bounds (so the global update is never
    clipped) and feasible random rows."""
    rng = np.random.default_rng(seed)
    subs = []
    if single_copy:
        perm = rng.permutation(n)
        cuts = np.sort(rng.choice(np.arange(1, n), size=S - 1, replace=False))
        groups = np.split(perm, cuts)
    else:
        groups = []
        for s in range(S):
            k = int(rng.integers(3, 9))
            groups.append(rng.choice(n, size=k, replace=False))
        covered = np.zeros(n, bool)
        for g in groups:
            covered[g] = True
        groups.append(np.flatnonzero(~covered) if (~covered).any() else rng.choice(n, 2, replace=False))
    for g in groups:
        g = np.sort(np.asarray(g, dtype=np.int64))
        m = int(rng.integers(0, max(1, g.size - 1)))
        A = rng.normal(size=(m, g.size))
        b = A @ rng.normal(size=g.size)
        subs.append(model.Subsystem(g, A, b, ("random",)))
    c = rng.normal(size=n)
    lp = model.ConsensusLP(n, c, np.full(n, -np.inf), np.full(n, np.inf), subs, rng.normal(size=n))
    return lp


def _stationarity(prep, lam):
    """||c + sum_s B_s' lambda_s||: the gradient of the Lagrangian in x."""
    return np.linalg.norm(prep.lp.c + np.bincount(prep.gidx, weights=lam, minlength=prep.lp.n))


def test_aggregated_dual_residual_is_the_stationarity_residual():
    prep = admm.prepare(_random_consensus_lp(3))
    assert prep.N.max() >= 3  # several copies per variable
    lams = []
    res = admm.solve(prep, max_iter=30, check=False, form="aggregated",
                     on_iter=lambda t, p, st: lams.append(st.lam.copy()))
    for t in range(30):
        assert res.history[t, 1] == pytest.approx(_stationarity(prep, lams[t]), rel=1e-9)


def test_printed_dual_residual_is_the_stationarity_residual_with_single_copies():
    prep = admm.prepare(_random_consensus_lp(4, single_copy=True))
    assert prep.N.max() == 1
    lams = []
    res = admm.solve(prep, max_iter=30, check=False, form="paper",
                     on_iter=lambda t, p, st: lams.append(st.lam.copy()))
    for t in range(30):
        assert res.history[t, 1] == pytest.approx(_stationarity(prep, lams[t]), rel=1e-9)


# ------------------------------------------------------- scaling invariance
def _scaled(prep, f):
    lp = prep.lp
    lp2 = model.ConsensusLP(lp.n, lp.c * f, lp.lo, lp.hi, lp.subs, lp.x_init)
    return admm.Prepared(lp2, prep.gidx, prep.offsets, prep.Abar, prep.bbar, prep.Abar_blk, prep.N)


def test_termination_is_invariant_under_scaling_cost_and_rho():
    prep = oracle_prep("13")
    a = admm.solve(prep, rho=100.0)
    b = admm.solve(_scaled(prep, 4.0), rho=400.0)
    assert a.converged and b.converged and a.iters == b.iters
    np.testing.assert_array_equal(a.x, b.x)
    np.testing.assert_array_equal(a.xs, b.xs)
    np.testing.assert_array_equal(4.0 * a.lam, b.lam)
    np.testing.assert_array_equal(a.history * np.array([1.0, 4.0, 1.0, 4.0]), b.history)


# ------------------------------------------------------------ initial point
def _first_sweep_golden():
    return json.load(open(os.path.join(GOLDEN, "two_bus.json")))["first_sweep"]


def test_first_sweep_of_the_two_bus_case():
    g = _first_sweep_golden()
    lp = model.decompose(two_bus(alpha=0.0, fixed_source=True))
    res = admm.solve(lp, max_iter=1, check=False)
    np.testing.assert_array_equal(res.prep.N, g["copy_counts"])
    np.testing.assert_allclose(res.x, g["x"], rtol=0, atol=1e-15)
    np.testing.assert_allclose(res.xs, g["xs"], rtol=0, atol=1e-13)
    np.testing.assert_allclose(res.lam, g["lam"], rtol=0, atol=1e-11)
    np.testing.assert_allclose(res.history[0], [g["pres"], g["dres"], g["eps_prim"], g["eps_dual"]], rtol=1e-12)


def test_initial_value_rules():
    """Section V-A: no bounds -> 0, bounds -> their average, a voltage -> 1.
    A one-sided bound clips 0 into the box; lo = hi gives that value."""
    lo = np.array([-np.inf, -1.0, 0.5, -np.inf, 3.0, 0.9025, 1.0])
    hi = np.array([np.inf, 3.0, np.inf, -2.0, 3.0, 1.1025, 1.0])
    ix = model.Index(7, *({} for _ in range(11)), is_voltage=np.array([0, 0, 0, 0, 0, 1, 1], bool), kind=[])
    np.testing.assert_array_equal(model.init_values(ix, lo, hi), [0.0, 1.0, 0.5, -2.0, 3.0, 1.0, 1.0])


# ---------------------------------------------------------------- mutations
def test_mutation_voltage_at_its_midpoint_is_caught(monkeypatch):
    orig = model.init_values

    def midpoint_voltages(ix, lo, hi):
        out = orig(ix, lo, hi)
        both = np.isfinite(lo) & np.isfinite(hi) & ix.is_voltage
        out[both] = 0.5 * (lo[both] + hi[both])
        return out

    monkeypatch.setattr(model, "init_values", midpoint_voltages)
    with pytest.raises(AssertionError):
        test_first_sweep_of_the_two_bus_case()


def _mutant_residuals(kind):
    orig = admm.residuals

    def f(prep, z, xs, xs_prev, lam, rho, eps_rel, eps_abs, form):
        r = list(orig(prep, z, xs, xs_prev, lam, rho, eps_rel, eps_abs, form))
        if kind == "dres_without_rho":
            r[1] /= rho
        elif kind == "eps_prim_on_global_x":
            x = np.bincount(prep.gidx, weights=z, minlength=prep.lp.n) / prep.N
            r[2] = eps_rel * max(np.linalg.norm(x), np.linalg.norm(xs))
        elif kind == "dres_against_z":
            r[1] = rho * np.linalg.norm(xs - z) if form == "paper" else \
                rho * np.linalg.norm(np.bincount(prep.gidx, weights=xs - z, minlength=prep.lp.n))
        return tuple(r)

    return f


@pytest.mark.parametrize("kind,pin", [
    ("dres_without_rho", test_aggregated_dual_residual_is_the_stationarity_residual),
    ("dres_without_rho", test_termination_is_invariant_under_scaling_cost_and_rho),
    ("dres_against_z", test_aggregated_dual_residual_is_the_stationarity_residual),
    ("dres_against_z", test_history_equals_the_printed_residuals_on_a_trajectory),
    ("eps_prim_on_global_x", lambda: test_residual_function_on_crafted_states("z")),
])
def test_mutation_of_the_residuals_is_caught(monkeypatch, kind, pin):
    monkeypatch.setattr(admm, "residuals", _mutant_residuals(kind))
    with pytest.raises(AssertionError):
        pin()
