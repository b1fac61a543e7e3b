"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these checks re-types an oracle formula: each compares the oracle
with brute force, a closed form, a worked example, first-principles phasor
physics, an independent LP solver, or an invariant of the iteration. The
mutation tests at the end plant plausible mistakes in the oracle and show
that a pin catches each one.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.optimize

from conftest import feeder, oracle_lp, oracle_prep
from oracle import admm, central, model
from synth import FeederSpec, make_feeder, two_bus

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- global step
def _brute_global(c, lam_sum, copies, lo, hi, rho):
    """argmin over [lo, hi] of (c + sum lambda) x + rho/2 sum (x - x_k)^2 (ADMM-1, one variable)."""
    f = lambda x: (c + lam_sum) * x + 0.5 * rho * np.sum((x - copies) ** 2)  # noqa: E731
    if np.isfinite(lo) and np.isfinite(hi):
        r = scipy.optimize.minimize_scalar(f, bounds=(lo, hi), method="bounded", options={"xatol": 1e-12})
        return r.x
    r = scipy.optimize.minimize_scalar(f, bracket=(-10.0, 10.0), tol=1e-14)
    return float(np.clip(r.x, lo, hi))


def _global_case(seed, n=40, kmax=5, rho=100.0, unbounded=False):
    rng = np.random.default_rng(seed)
    N = rng.integers(1, kmax + 1, size=n)
    gidx = np.repeat(np.arange(n), N)
    xs = rng.normal(0, 1, gidx.size)
    lam = rng.normal(0, 30, gidx.size)
    c = rng.normal(0, 50, n)
    lo = rng.uniform(-1.5, 0, n)
    hi = lo + rng.uniform(0.1, 2.0, n)
    if unbounded:
        lo[:] = -np.inf
        hi[:] = np.inf
    lp = model.ConsensusLP(n, c, lo, hi, [])
    prep = admm.Prepared(lp, gidx, None, [], None, None, N.astype(float))
    return prep, xs, lam, rho


@pytest.mark.parametrize("unbounded", [False, True])
def test_global_update_is_the_minimizer_of_admm1(unbounded):
    prep, xs, lam, rho = _global_case(3, unbounded=unbounded)
    got = admm.global_update(prep, xs, lam, rho)
    for i in range(prep.lp.n):
        k = prep.gidx == i
        want = _brute_global(prep.lp.c[i], lam[k].sum(), xs[k], prep.lp.lo[i], prep.lp.hi[i], rho)
        assert abs(got[i] - want) <= 1e-7 * max(1.0, abs(want)), i


def test_global_update_special_cases():
    rho = 100.0
    lp = model.ConsensusLP(2, np.array([3.0, 1e9]), np.array([-np.inf, -1.0]), np.array([np.inf, 1.0]), [])
    prep = admm.Prepared(lp, np.array([0, 1]), None, [], None, None, np.array([1.0, 1.0]))
    x = admm.global_update(prep, np.array([0.7, 0.0]), np.array([2.0, 0.0]), rho)
    # a single copy with an inactive box: x = x_k - (c + lambda) / rho
    assert x[0] == pytest.approx(0.7 - 5.0 / rho, abs=1e-15)
    # a huge cost drives the variable to its lower bound
    assert x[1] == -1.0


# ----------------------------------------------------------------- local step
def _kkt_local(A, b, z, lam, rho):
    """Dense KKT solve of ADMM-2: min -lam'x + rho/2 ||z - x||^2 s.t. A x = b."""
    m, n = A.shape
    K = np.block([[rho * np.eye(n), A.T], [A, np.zeros((m, m))]])
    rhs = np.concatenate([rho * z + lam, b])
    return np.linalg.solve(K, rhs)[:n]


@pytest.mark.parametrize("m,n", [(3, 8), (6, 9), (1, 4), (9, 10)])
def test_local_update_solves_the_kkt_system(m, n):
    rng = np.random.default_rng(m * 100 + n)
    A = rng.normal(size=(m, n))
    b = rng.normal(size=m)
    Abar, bbar = admm.precompute(A, b)
    z = rng.normal(size=n)
    lam = rng.normal(size=n) * 10
    rho = 100.0
    x = (Abar @ (-rho * z - lam)) / rho + bbar
    np.testing.assert_allclose(x, _kkt_local(A, b, z, lam, rho), atol=1e-12)
    # projector identities of closed_2
    Pm = Abar + np.eye(n)
    np.testing.assert_allclose(Abar, Abar.T, atol=1e-14)
    np.testing.assert_allclose(Pm @ Pm, Pm, atol=1e-12)
    np.testing.assert_allclose(A @ Pm, A, atol=1e-12)
    np.testing.assert_allclose(A @ bbar, b, atol=1e-12)
    np.testing.assert_allclose(Abar @ bbar, 0.0, atol=1e-12)


def test_local_update_degenerate_shapes():
    rng = np.random.default_rng(0)
    n = 5
    Abar, bbar = admm.precompute(np.zeros((0, n)), np.zeros(0))
    v = rng.normal(size=n)
    np.testing.assert_array_equal(-Abar @ v + bbar, v)  # no rows: x_s = z + lambda / rho
    A = rng.normal(size=(n, n))
    b = rng.normal(size=n)
    Abar, bbar = admm.precompute(A, b)
    np.testing.assert_allclose(-Abar @ v + bbar, np.linalg.solve(A, b), atol=1e-10)  # square: x_s = A^-1 b


def test_rank_deficient_rows():
    rng = np.random.default_rng(5)
    A0 = rng.normal(size=(3, 7))
    b0 = rng.normal(size=3)
    A = np.vstack([A0, 2.0 * A0[1] - A0[2]])
    b = np.concatenate([b0, [2.0 * b0[1] - b0[2]]])
    Ab, bb = admm.precompute(A, b)
    Ab0, bb0 = admm.precompute(A0, b0)
    np.testing.assert_allclose(Ab, Ab0, atol=1e-12)
    np.testing.assert_allclose(bb, bb0, atol=1e-12)
    with pytest.raises(admm.InconsistentSubsystem):
        admm.precompute(A, b + np.array([0, 0, 0, 1.0]))


# ------------------------------------------------------------- worked example
@pytest.mark.parametrize("case", ["fixed_source_constant_power", "free_source_constant_impedance"])
def test_two_bus_worked_example(case):
    g = json.load(open(os.path.join(GOLDEN, "two_bus.json")))["cases"][case]
    net = two_bus(alpha=g["alpha"], fixed_source=g["w0_bounds"] == [1.0, 1.0])
    lp = model.decompose(net)
    assert lp.n == 12 and len(lp.subs) == 2
    assert sum(s.A.shape[0] for s in lp.subs) == 11
    res = admm.solve(lp, eps_rel=1e-10, max_iter=200000)
    assert res.converged
    x = res.x  # p^g, q^g, w0, w1, p^b, q^b, p^d, q^d, p01, q01, p10, q10
    for key, idx in (("pg", 0), ("qg", 1), ("w0", 2), ("w1", 3)):
        assert x[idx] == pytest.approx(g[key], abs=1e-6), key
    assert res.objective == pytest.approx(g["objective"], abs=1e-6)


# ---------------------------------------------------------- phasor physics pins
A_POS = np.exp(2j * math.pi / 3)
ALPHA = np.array([1.0, A_POS ** 2, A_POS])  # nominal phase a, b, c voltages


def _phasor_drop(R, X, p, q, ph):
    """w_i - w_j = 2 Re[conj(V_i) (Z I)] with V_i = nominal, I = conj(s / V_i), on phases ph."""
    Z = (R + 1j * X)[np.ix_(ph, ph)]
    V = ALPHA[ph]
    I = np.conj((p + 1j * q) / V)
    return 2.0 * np.real(np.conj(V) * (Z @ I))


def test_voltage_drop_rows_match_phasor_physics():
    rng = np.random.default_rng(11)
    for ph in ([0, 1, 2], [0, 1], [1, 2], [0, 2], [1]):
        R = rng.uniform(0.01, 0.05, (3, 3))
        R = (R + R.T) / 2
        X = rng.uniform(0.01, 0.05, (3, 3))
        X = (X + X.T) / 2
        Mp, Mq = model.m_matrices(R.ravel(), X.ravel())
        p = rng.normal(size=len(ph))
        q = rng.normal(size=len(ph))
        # voltage_mag_diff with tau = 1, no shunts: w_i - w_j = -(Mp p + Mq q)
        lhs = -(Mp[np.ix_(ph, ph)] @ p + Mq[np.ix_(ph, ph)] @ q)
        np.testing.assert_allclose(lhs, _phasor_drop(R, X, p, q, ph), atol=1e-12)


def _pi_line_state(eps, gi, bi, gj, bj, seed):
    """Exact single-phase AC state of a pi-model line i -> j with series
    impedance eps (r + jx), shunt admittances gi + j bi at i and gj + j bj at j,
    V_i = 1 and a unit series current: (w_i, w_j, p_ij, q_ij, p_ji, q_ji, |z|, |I|)."""
    rng = np.random.default_rng(seed)
    z = eps * complex(rng.uniform(0.2, 1.0), rng.uniform(0.2, 1.0))
    Is = np.exp(1j * rng.uniform(0.0, 2 * math.pi))  # unit series current, any direction
    Vi = 1.0 + 0.0j
    Vj = Vi - z * Is
    Sij = Vi * np.conj(Is + complex(gi, bi) * Vi)    # power entering the line at i
    Sji = Vj * np.conj(-Is + complex(gj, bj) * Vj)   # power entering the line at j
    return abs(Vi) ** 2, abs(Vj) ** 2, Sij.real, Sij.imag, Sji.real, Sji.imag, abs(z), abs(Is)


def _line_row_residuals(net, state):
    ix = model.build_index(net)
    wi, wj, pij, qij, pji, qji = state[:6]
    x = np.zeros(ix.n)
    x[ix.w[(0, 0)]], x[ix.w[(1, 0)]] = wi, wj
    x[ix.pij[(0, 0)]], x[ix.qij[(0, 0)]] = pij, qij
    x[ix.pji[(0, 0)]], x[ix.qji[(0, 0)]] = pji, qji
    return [sum(v * x[c] for c, v in row.items()) - rhs for row, rhs in model.line_rows(net, ix, 0)]


def test_line_shunt_terms_match_pi_model_physics():
    """Exact pi-model physics pins the shunt terms of powerloss-1, -2 and
    voltage_mag_diff: as the series impedance eps z -> 0, the loss rows err by
    the neglected series loss (O(eps)) and the drop row by |z I|^2 (O(eps^2));
    a wrong sign or a missing shunt term would leave an O(shunt) error."""
    gi, bi, gj, bj = 0.07, 0.11, 0.05, 0.09
    net = dict(two_bus(r=1.0, x=1.0))
    for key, val in (("line_gs_from", gi), ("line_bs_from", bi), ("line_gs_to", gj), ("line_bs_to", bj)):
        arr = np.zeros((1, 3))
        arr[0, 0] = val
        net[key] = arr
    for seed in range(5):
        for eps in (1e-3, 1e-4):
            st = _pi_line_state(eps, gi, bi, gj, bj, seed)
            zabs, iabs = st[6], st[7]
            # the oracle's rows use the line's r, x: give them this state's impedance
            rng = np.random.default_rng(seed)
            r, x = eps * rng.uniform(0.2, 1.0), eps * rng.uniform(0.2, 1.0)
            net["line_r"] = np.array([[r] + [0.0] * 8])
            net["line_x"] = np.array([[x] + [0.0] * 8])
            loss_p, loss_q, drop = _line_row_residuals(net, st)
            assert abs(loss_p) <= 1.01 * zabs * iabs ** 2
            assert abs(loss_q) <= 1.01 * zabs * iabs ** 2
            assert abs(drop) <= 1.01 * (zabs * iabs) ** 2
            # a wrong shunt term would cost g or b in the loss rows and about
            # 2 |z| g in the drop row, far above these bounds
            assert min(gi, bi, gj, bj) > 20 * zabs * iabs ** 2
            assert 2 * zabs * min(gi, bi) > 20 * (zabs * iabs) ** 2


def test_mutation_flipped_line_shunt_sign_is_caught(monkeypatch):
    """The physics pin fails for an oracle whose drop row adds g^s w_i."""
    orig = model.line_rows

    def flipped(net, ix, e):
        rows = orig(net, ix, e)
        gsi = net["line_gs_from"][e]
        out = []
        for k, (row, rhs) in enumerate(rows):
            row = dict(row)
            if k % 3 == 2:
                Mp, _ = model.m_matrices(net["line_r"][e], net["line_x"][e])
                row[ix.w[(int(net["line_from"][e]), 0)]] += 2 * Mp[0, 0] * gsi[0]
            out.append((row, rhs))
        return out

    monkeypatch.setattr(model, "line_rows", flipped)
    with pytest.raises(AssertionError):
        test_line_shunt_terms_match_pi_model_physics()


def test_delta_load_rows_match_balanced_delta_physics():
    """Bus injections of a delta load under nominal voltages satisfy VDLM-6..10."""
    net = make_feeder(FeederSpec(4, 1.0, 0.0, 2.4, "uniform100"), 1)
    net = dict(net)
    net["load_conn"] = np.array([1, 0, 0], dtype=np.uint8)
    net["load_phases"] = np.array([7, 7, 7], dtype=np.uint8)
    ix = model.build_index(net)
    rows = model.load_rows(net, ix, 0)[6:]  # the two sum rows and the four coupling rows
    rng = np.random.default_rng(2)
    sd = rng.uniform(0.1, 1, 3) + 1j * rng.uniform(0.1, 1, 3)  # branch powers ab, bc, ca
    Vd = np.array([ALPHA[0] - ALPHA[1], ALPHA[1] - ALPHA[2], ALPHA[2] - ALPHA[0]])
    Id = np.conj(sd / Vd)
    Il = np.array([Id[0] - Id[2], Id[1] - Id[0], Id[2] - Id[1]])
    sb = ALPHA * np.conj(Il)
    val = np.zeros(ix.n)
    for f in range(3):
        val[ix.pb[(0, f)]], val[ix.qb[(0, f)]] = sb[f].real, sb[f].imag
        val[ix.pd[(0, f)]], val[ix.qd[(0, f)]] = sd[f].real, sd[f].imag
    for coef, rhs in rows:
        assert abs(sum(v * val[g] for g, v in coef.items()) - rhs) <= 1e-12
    assert abs(Vd[0]) ** 2 == pytest.approx(3.0)  # w-hat = 3 w


def test_load_rows_linearize_the_zip_model():
    """p^d = a (1 + alpha/2 (w - 1)) is the tangent of a * |V|^alpha = a w^(alpha/2) at w = 1."""
    net = two_bus()
    ix = model.build_index(net)
    for alpha in (0.0, 1.0, 2.0):
        net["load_alpha"][0, 0] = alpha
        coef, rhs = model.load_rows(net, ix, 0)[0]
        a = net["load_a"][0, 0]
        slope = -coef[ix.w[(1, 0)]]
        assert slope == pytest.approx(a * alpha / 2.0)  # d/dw a w^(alpha/2) at w = 1
        assert rhs + slope == pytest.approx(a)  # value a at w = 1


# --------------------------------------------------------- fixed point at scale
def _sweep(net):
    """LinDistFlow by phasors: flows = downstream demand, w from the root down.

    Bus shunts draw (g^sh - j b^sh) w; with them the sweep is repeated until
    w stops changing.
    """
    nb = net["n_bus"]
    base = np.zeros((nb, 3), complex)
    for l in range(net["n_load"]):
        base[net["load_bus"][l]] += net["load_a"][l] + 1j * net["load_b"][l]
    shunt = net["bus_gsh"] - 1j * net["bus_bsh"]
    w = np.where(net["bus_whi"] > 0, 1.0, 0.0)
    for _ in range(200):
        flow = base + shunt * w
        for e in range(net["n_line"] - 1, -1, -1):
            flow[net["line_from"][e]] += flow[net["line_to"][e]]
        w_new = np.zeros((nb, 3))
        w_new[0] = 1.0
        for e in range(net["n_line"]):
            i, j = net["line_from"][e], net["line_to"][e]
            ph = model.phases(net["line_phases"][e])
            sj = flow[j][ph]
            d = _phasor_drop(net["line_r"][e].reshape(3, 3), net["line_x"][e].reshape(3, 3), sj.real, sj.imag, ph)
            w_new[j, ph] = w_new[i, ph] - d
        if np.abs(w_new - w).max() < 1e-15:
            break
        w = w_new
    return flow, w


@pytest.mark.parametrize("nbus,seed,shunts", [(13, 13, False), (60, 4, False), (13, 5, True)])
def test_fixed_point_is_the_lindistflow_sweep(nbus, seed, shunts):
    spec = FeederSpec(nbus, 0.6, 0.2, 2.4018, "uniform100", fixed_source=True, alpha_choices=(0,))
    net = dict(make_feeder(spec, seed))
    if shunts:
        on = net["bus_whi"] > 0
        rng = np.random.default_rng(seed)
        net["bus_gsh"] = np.where(on, rng.uniform(0, 0.02, on.shape), 0.0)
        net["bus_bsh"] = np.where(on, rng.uniform(0, 0.02, on.shape), 0.0)
    flow, w = _sweep(net)
    lp = model.decompose(net)
    assert lp.n - sum(s.A.shape[0] for s in lp.subs) == 3  # square up to the root voltages
    res = admm.solve(lp, eps_rel=1e-9, max_iter=400000)
    assert res.converged
    ix = model.build_index(net)
    for (i, f), g in ix.w.items():
        assert res.x[g] == pytest.approx(w[i, f], abs=2e-6)
    for (e, f), g in ix.pij.items():
        assert res.x[g] == pytest.approx(flow[net["line_to"][e], f].real, abs=2e-6)
    # the assembled central system with w_root = 1 has exactly this solution
    A, b, c, lo, hi, _ = central.central_lp(net)
    A = A.toarray()
    fix = np.zeros((3, lp.n))
    for f in range(3):
        fix[f, ix.w[(0, f)]] = 1.0
    xs = np.linalg.solve(np.vstack([A, fix]), np.concatenate([b, np.ones(3)]))
    for (i, f), g in ix.w.items():
        assert xs[g] == pytest.approx(w[i, f], abs=1e-12)


# ----------------------------------------------------------- LP optimum (HiGHS)
@pytest.mark.parametrize("name,eps,gap", [("13", 1e-7, 1e-6), ("123", 1e-4, 1e-3)])
def test_objective_matches_highs(name, eps, gap):
    f_lp, _, _ = central.solve_central(feeder(name))
    res = admm.solve(oracle_prep(name), eps_rel=eps)
    assert res.converged
    assert abs(res.objective - f_lp) / max(1.0, abs(f_lp)) <= gap


def test_kkt_certificate_from_admm_duals():
    res = admm.solve(oracle_prep("13"), eps_rel=1e-9)
    cert = central.kkt_certificate(res)
    assert cert["rowspace"] <= 1e-6
    assert cert["reduced_cost"] <= 1e-4 * cert["gscale"]


def test_single_subsystem_reaches_the_same_optimum():
    """S = 1 (the whole network one subsystem) and the decomposition agree."""
    net = feeder("13")
    A, b, c, lo, hi, ix = central.central_lp(net)
    lp1 = model.ConsensusLP(ix.n, c, lo, hi, [model.Subsystem(np.arange(ix.n), A.toarray(), b, ("all",))],
                            model.init_values(ix, lo, hi))
    r1 = admm.solve(lp1, eps_rel=1e-8)
    rS = admm.solve(oracle_prep("13"), eps_rel=1e-8)
    f_lp, _, _ = central.solve_central(net)
    assert r1.converged and rS.converged
    assert abs(r1.objective - f_lp) <= 1e-5 * max(1.0, abs(f_lp))
    assert abs(rS.objective - f_lp) <= 1e-5 * max(1.0, abs(f_lp))


# ------------------------------------------------------- trajectory invariants
def test_iteration_invariants():
    prep = oracle_prep("123")
    lp = prep.lp
    prev = {"lam": np.zeros(prep.gidx.size)}

    def check(t, prep, st):
        for s, sub in enumerate(lp.subs):
            xs = st.xs[prep.offsets[s]:prep.offsets[s + 1]]
            if sub.A.shape[0]:
                assert np.abs(sub.A @ xs - sub.b).max() <= 1e-10 * (1 + np.abs(sub.b).max())
        assert np.all(st.x >= lp.lo) and np.all(st.x <= lp.hi)
        z = st.x[prep.gidx]
        pres = np.linalg.norm(z - st.xs)
        assert pres == pytest.approx(np.linalg.norm(st.lam - prev["lam"]) / 100.0, rel=1e-9, abs=1e-14)
        prev["lam"] = st.lam.copy()

    admm.solve(prep, max_iter=60, check=False, on_iter=check)


# ------------------------------------------------------------------- structure
@pytest.mark.parametrize("name", ["13", "123", "2500"])
def test_decomposition_structure(name):
    net = feeder(name)
    lp = oracle_lp(name)
    n_leaf = int(model.leaves(net).sum())
    assert len(lp.subs) == net["n_bus"] + net["n_line"] - n_leaf  # Table 3 identity
    pv_phases = sum(bin(int(p)).count("1") for p in net["gen_phases"][1:])
    assert lp.n - sum(s.A.shape[0] for s in lp.subs) == 3 + 2 * pv_phases
    for s in lp.subs:
        assert np.all(np.diff(s.gidx) > 0)
    counts = np.bincount(np.concatenate([s.gidx for s in lp.subs]), minlength=lp.n)
    assert counts.min() >= 1


def test_residual_forms_agree_on_single_copy_variables():
    """With every variable in one subsystem the two residual forms coincide."""
    prep, xs, lam, rho = _global_case(1, kmax=1)
    z = xs + 0.1
    xs_prev = xs - 0.05
    a = admm.residuals(prep, z, xs, xs_prev, lam, rho, 1e-4, 0.0, "paper")
    b = admm.residuals(prep, z, xs, xs_prev, lam, rho, 1e-4, 0.0, "aggregated")
    np.testing.assert_allclose(a, b, rtol=1e-12)


# ------------------------------------------------------------------ mutations
def _printed_closed_1(prep, xs, lam, rho):
    """closed_1 exactly as printed: the rho on the sum of copies is missing."""
    lp = prep.lp
    sx = np.bincount(prep.gidx, weights=xs, minlength=lp.n)
    sl = np.bincount(prep.gidx, weights=lam, minlength=lp.n)
    xhat = -(lp.c + sl - sx) / (rho * prep.N)
    return np.minimum(np.maximum(xhat, lp.lo), lp.hi)


def test_mutation_printed_global_step_is_caught():
    prep, xs, lam, rho = _global_case(3)
    got = _printed_closed_1(prep, xs, lam, rho)
    bad = 0
    for i in range(prep.lp.n):
        k = prep.gidx == i
        want = _brute_global(prep.lp.c[i], lam[k].sum(), xs[k], prep.lp.lo[i], prep.lp.hi[i], rho)
        bad += abs(got[i] - want) > 1e-7 * max(1.0, abs(want))
    assert bad > 0


def test_mutation_transposed_m_matrix_is_caught():
    rng = np.random.default_rng(11)
    R = rng.uniform(0.01, 0.05, (3, 3))
    R = (R + R.T) / 2
    X = rng.uniform(0.01, 0.05, (3, 3))
    X = (X + X.T) / 2
    Mp, Mq = model.m_matrices(R.ravel(), X.ravel())
    p, q = rng.normal(size=3), rng.normal(size=3)
    lhs = -(Mp.T @ p + Mq.T @ q)
    assert np.abs(lhs - _phasor_drop(R, X, p, q, [0, 1, 2])).max() > 1e-3


def test_mutation_flipped_dual_sign_is_caught(monkeypatch):
    monkeypatch.setattr(admm, "dual_update", lambda lam, z, xs, rho: lam - rho * (z - xs))
    res = admm.solve(oracle_prep("13"), max_iter=5000)
    f_lp, _, _ = central.solve_central(feeder("13"))
    assert (not res.converged) or abs(res.objective - f_lp) > 1e-3 * abs(f_lp)
