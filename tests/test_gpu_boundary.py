"""The C ABI's other entry points and edge paths on the device, each against
the FP64 oracle or a stated error code:

* ldopf_create_lp (the consensus LP of Section III-A given directly) with a
  consistent dependent row (the "row reduction" of Section III-B): operators
  against the oracle's pseudo-inverse form, and the solve against the oracle;
  an inconsistent dependent row is refused (LDOPF_INCONSISTENT_SUBSYSTEM);
* degenerate subsystems: no rows (x_s = v) and square (x_s = A_s^-1 b_s),
  and S = 1, the whole network one subsystem;
* a feeder with delta loads, line and bus shunts and off-nominal taps
  (Section II-A: VDLM-4, VDLM-6..10, g^sh/b^sh, g^s/b^s, tau);
* non-finite state (LDOPF_NUMERICAL), and the device-pointer getters.
"""
import numpy as np
import pytest

from conftest import feeder, rel_err

pytestmark = pytest.mark.gpu


def _flat(lp):
    """The oracle's consensus LP as the arrays ldopf_create_lp takes."""
    n_s = np.array([len(s.gidx) for s in lp.subs], np.int32)
    m_s = np.array([s.A.shape[0] for s in lp.subs], np.int32)
    A = np.concatenate([s.A.ravel() for s in lp.subs])
    b = np.concatenate([s.b for s in lp.subs])
    gidx = np.concatenate([s.gidx for s in lp.subs]).astype(np.int64)
    return dict(n=lp.n, c=lp.c, lo=lp.lo, hi=lp.hi, x_init=lp.x_init, n_s=n_s, m_s=m_s, A=A, b=b, gidx=gidx)


def _create_lp(P, lp, opts=None):
    f = _flat(lp)
    return P.ldopf_create_lp(f["n"], f["c"], f["lo"], f["hi"], f["x_init"], f["n_s"], f["m_s"], f["A"], f["b"],
                             f["gidx"], opts)


def _with_dependent_row(lp, shift=0.0):
    """A copy of lp whose first subsystem with two or more rows gains the sum
    of its first two rows (right-hand side plus `shift`)."""
    import copy
    from oracle import model
    out = copy.deepcopy(lp)
    s = next(i for i, sub in enumerate(out.subs) if sub.A.shape[0] >= 2)
    sub = out.subs[s]
    row = sub.A[0] + sub.A[1]
    out.subs[s] = model.Subsystem(sub.gidx, np.vstack([sub.A, row]), np.append(sub.b, sub.b[0] + sub.b[1] + shift),
                                  sub.tag)
    return out, s


def _fixed(P, prob, lp, T, tol=1e-6):
    from oracle import admm
    prob.set_options(P.ldopf_default_options(max_iter=T, check_termination=0))
    st = prob.solve()
    assert st.iterations == T
    ref = admm.solve(lp, max_iter=T, check=False)
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= tol
    assert rel_err(xs, ref.xs) <= tol
    assert rel_err(lam, ref.lam) <= tol
    np.testing.assert_allclose(prob.get_history(), ref.history, rtol=1e-6, atol=1e-12)
    return ref


def test_create_lp_with_a_dependent_row_matches_oracle(gpu):
    from oracle import admm, model
    P = gpu
    lp, s = _with_dependent_row(model.decompose(feeder("13")))
    prob = _create_lp(P, lp)
    abar, bbar, rank = prob.get_operators()
    sub = lp.subs[s]
    assert rank[s] == np.linalg.matrix_rank(sub.A) == sub.A.shape[0] - 1
    Ab_ref, bb_ref = admm.precompute(sub.A, sub.b)
    n_s = [len(x.gidx) for x in lp.subs]
    off = sum(n * n for n in n_s[:s])
    n = n_s[s]
    np.testing.assert_allclose(abar[off:off + n * n].reshape(n, n), Ab_ref, rtol=0, atol=1e-12)
    prep = admm.prepare(lp)
    assert rel_err(bbar, prep.bbar) <= 1e-12
    _fixed(P, prob, prep, 200)


def test_create_lp_with_an_inconsistent_row_is_refused(gpu):
    from oracle import admm, model
    P = gpu
    lp, _ = _with_dependent_row(model.decompose(feeder("13")), shift=1.0)
    with pytest.raises(admm.InconsistentSubsystem):
        admm.prepare(lp)
    with pytest.raises(P.LdopfError) as e:
        _create_lp(P, lp)
    assert e.value.code == -4


def test_create_lp_degenerate_subsystems(gpu):
    """A subsystem without rows (its update is the plain average's copy) and
    a square one (its update is A_s^-1 b_s, whatever the consensus)."""
    from oracle import model
    P = gpu
    subs = [
        model.Subsystem(np.array([0, 1, 2]), np.array([[1.0, 1.0, 1.0]]), np.array([1.0]), ("a",)),
        model.Subsystem(np.array([1, 2, 3]), np.zeros((0, 3)), np.zeros(0), ("free",)),
        model.Subsystem(np.array([0, 3]), np.array([[2.0, 1.0], [1.0, 3.0]]), np.array([0.7, 0.4]), ("square",)),
    ]
    lp = model.ConsensusLP(4, np.array([1.0, -0.5, 0.25, 0.0]), np.array([-1.0, -1.0, 0.0, -np.inf]),
                           np.array([1.0, 1.0, 0.5, np.inf]), subs, np.array([0.0, 0.1, 0.2, 0.0]))
    prob = _create_lp(P, lp)
    _, _, rank = prob.get_operators()
    assert list(rank) == [1, 0, 2]
    ref = _fixed(P, prob, lp, 150)
    # the square subsystem's copies are its own solution after every sweep
    xs, _ = prob.get_local()
    np.testing.assert_allclose(xs[6:8], np.linalg.solve(subs[2].A, subs[2].b), rtol=0, atol=1e-14)
    assert ref.iters == 150


def test_single_subsystem_network(gpu):
    """S = 1: the two-bus network as one subsystem (all 12 variables, all 11
    rows) against the oracle, and its optimum (the hand-derived one)."""
    from oracle import admm, central, model
    from synth import two_bus
    P = gpu
    net = two_bus(fixed_source=True)
    A, b, c, lo, hi, ix = central.central_lp(net)
    lp = model.ConsensusLP(ix.n, c, lo, hi, [model.Subsystem(np.arange(ix.n), A.toarray(), b, ("all",))],
                           model.init_values(ix, lo, hi))
    prob = _create_lp(P, lp)
    assert prob.sizes().n_sub == 1
    _fixed(P, prob, lp, 100)
    prob.reset()
    prob.set_options(P.ldopf_default_options(eps_rel=1e-9))
    st = prob.solve()
    ref = admm.solve(lp, eps_rel=1e-9)
    assert st.converged and ref.converged and st.iterations == ref.iters
    np.testing.assert_allclose(prob.get_global()[[0, 1, 2, 3]], [0.5, 0.15, 1.0, 0.984], atol=1e-6)


@pytest.mark.parametrize("name", ["13", "123"])
@pytest.mark.parametrize("precision,tol", [(0, 1e-6), (1, 1e-4)])
def test_delta_loads_shunts_taps(gpu, name, precision, tol):
    from oracle import admm, model
    from synth import perturb_extras
    P = gpu
    net = perturb_extras(feeder(name), 7)
    assert (net["load_conn"] == 1).any() and np.any(net["line_tau"] != 1.0) and np.any(net["bus_gsh"] != 0.0)
    T = 200
    prob = P.ldopf_create(net, P.ldopf_default_options(max_iter=T, check_termination=0, precision=precision))
    prob.solve()
    ref = admm.solve(model.decompose(net), max_iter=T, check=False)
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= tol
    assert rel_err(xs, ref.xs) <= tol
    if precision == 0:
        assert rel_err(lam, ref.lam) <= tol


def test_delta_loads_shunts_taps_converged(gpu):
    """The 13-bus feeder with delta loads, shunts and off-nominal taps (a
    transformer or regulator is a line with per-phase tap ratios, as the
    paper models transformers) to eps_rel = 1e-4: the oracle's stopping sweep
    and state, and the objective against the LP optimum (HiGHS)."""
    from oracle import admm, central, model
    from synth import perturb_extras
    P = gpu
    net = perturb_extras(feeder("13"), 7)
    prob = P.ldopf_create(net)
    st = prob.solve()
    ref = admm.solve(model.decompose(net))
    assert st.converged and ref.converged and st.iterations == ref.iters
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= 1e-6
    assert rel_err(xs, ref.xs) <= 1e-6 and rel_err(lam, ref.lam) <= 1e-6
    f_lp, _, _ = central.solve_central(net)
    assert abs(prob.objective() - f_lp) <= 1e-3 * max(1.0, abs(f_lp))


def test_nonfinite_state(gpu):
    """A NaN warm start is refused; a finite state whose squares overflow
    stops the solve with LDOPF_NUMERICAL at the first sweep whose residual
    sums are not finite, and the handle stays usable."""
    P = gpu
    prob = P.ldopf_create(feeder("13"), P.ldopf_default_options(max_iter=50))
    nl = prob.sizes().n_local
    xs = np.zeros(nl)
    xs[3] = np.nan
    with pytest.raises(P.LdopfError) as e:
        prob.warm_start(xs, np.zeros(nl))
    assert e.value.code == -7
    prob.warm_start(np.full(nl, 1e300), np.zeros(nl))
    with pytest.raises(P.LdopfError) as e:
        prob.solve()
    assert e.value.code == -7
    prob.reset()
    st = prob.solve()
    assert st.iterations == 50 or st.converged


def test_device_getters_match_host(gpu):
    import torch
    P = gpu
    stream = torch.cuda.current_stream()
    prob = P.ldopf_create(feeder("123"), P.ldopf_default_options(max_iter=40, check_termination=0), stream=stream)
    prob.solve()
    s = prob.sizes()
    x = torch.full((s.n,), -1.0, dtype=torch.float64, device="cuda")
    xs = torch.full((s.n_local,), -1.0, dtype=torch.float64, device="cuda")
    lam = torch.full((s.n_local,), -1.0, dtype=torch.float64, device="cuda")
    prob.get_global_device(x.data_ptr(), s.n)
    prob.get_local_device(xs.data_ptr(), lam.data_ptr(), s.n_local)
    torch.cuda.synchronize()
    xs_h, lam_h = prob.get_local()
    np.testing.assert_array_equal(x.cpu().numpy(), prob.get_global())
    np.testing.assert_array_equal(xs.cpu().numpy(), xs_h)
    np.testing.assert_array_equal(lam.cpu().numpy(), lam_h)
    with pytest.raises(P.LdopfError) as e:
        prob.get_global_device(x.data_ptr(), s.n - 1)
    assert e.value.code == -8
