"""Large subsystems on the device: the whole network as one subsystem
(S = 1, which the consensus model of Section III-A allows) and a coarse
decomposition into subtrees, both given through ldopf_create_lp and both
against the FP64 oracle on the same consensus LP. The component-wise
decomposition of Section V-A gives subsystems of at most 39 variables; these
reach 261 (13-bus, S = 1) and 630 (123-bus, 11 subtrees)."""
import numpy as np
import pytest

from conftest import feeder, rel_err

pytestmark = pytest.mark.gpu


def _create(P, lp, opts=None):
    n_s = np.array([len(s.gidx) for s in lp.subs], np.int32)
    m_s = np.array([s.A.shape[0] for s in lp.subs], np.int32)
    A = np.concatenate([s.A.ravel() for s in lp.subs])
    b = np.concatenate([s.b for s in lp.subs])
    gidx = np.concatenate([s.gidx for s in lp.subs]).astype(np.int64)
    return P.ldopf_create_lp(lp.n, lp.c, lp.lo, lp.hi, lp.x_init, n_s, m_s, A, b, gidx, opts)


def single_subsystem_lp(net):
    from oracle import central, model
    A, b, c, lo, hi, ix = central.central_lp(net)
    return model.ConsensusLP(ix.n, c, lo, hi, [model.Subsystem(np.arange(ix.n), A.toarray(), b, ("all",))],
                             model.init_values(ix, lo, hi))


def subtree_lp(net, depth):
    """The component subsystems of Section V-A merged by subtree: every bus
    deeper than `depth` joins the subtree of its ancestor at that depth; a
    line goes with its child bus. Each row of LP_model stays in exactly one
    subsystem, so this is a consensus LP of the same problem."""
    from oracle import model
    lp = model.decompose(net)
    root = int(net["root"])
    children = {}
    for e in range(int(net["n_line"])):
        children.setdefault(int(net["line_from"][e]), []).append(int(net["line_to"][e]))
    region, depth_of, order = {root: root}, {root: 0}, [root]
    for u in order:
        for v in children.get(u, []):
            depth_of[v] = depth_of[u] + 1
            region[v] = v if depth_of[v] <= depth else region[u]
            order.append(v)
    groups = {}
    for s, sub in enumerate(lp.subs):
        bus = int(net["line_to"][sub.tag[1]]) if sub.tag[0] == "line" else int(sub.tag[1])
        groups.setdefault(region[bus], []).append(s)
    subs = []
    for g in groups.values():
        cols = np.unique(np.concatenate([lp.subs[s].gidx for s in g]))
        pos = {int(c): i for i, c in enumerate(cols)}
        A = np.zeros((sum(lp.subs[s].A.shape[0] for s in g), cols.size))
        r = 0
        for s in g:
            sub = lp.subs[s]
            A[r:r + sub.A.shape[0], [pos[int(c)] for c in sub.gidx]] = sub.A
            r += sub.A.shape[0]
        subs.append(model.Subsystem(cols, A, np.concatenate([lp.subs[s].b for s in g]), ("subtree",)))
    return model.ConsensusLP(lp.n, lp.c, lp.lo, lp.hi, subs, lp.x_init)


def _fixed(P, prob, lp, T):
    from oracle import admm
    prob.set_options(P.ldopf_default_options(max_iter=T, check_termination=0))
    assert prob.solve().iterations == T
    ref = admm.solve(lp, max_iter=T, check=False)
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), ref.x) <= 1e-6
    assert rel_err(xs, ref.xs) <= 1e-6
    assert rel_err(lam, ref.lam) <= 1e-6
    np.testing.assert_allclose(prob.get_history(), ref.history, rtol=1e-6, atol=1e-12)


def test_single_subsystem_13bus(gpu):
    from oracle import admm
    P = gpu
    lp = single_subsystem_lp(feeder("13"))
    prob = _create(P, lp)
    s = prob.sizes()
    assert s.n_sub == 1 and s.max_n == 261
    _, _, rank = prob.get_operators()
    assert rank[0] == np.linalg.matrix_rank(lp.subs[0].A)
    _fixed(P, prob, lp, 300)
    prob.reset()
    prob.set_options(P.ldopf_default_options())
    st = prob.solve()
    ref = admm.solve(lp)
    assert st.converged and ref.converged and st.iterations == ref.iters
    assert rel_err(prob.get_global(), ref.x) <= 1e-6


def test_subtree_decomposition_123bus(gpu):
    from oracle import admm, central
    P = gpu
    net = feeder("123")
    lp = subtree_lp(net, 3)
    assert max(len(s.gidx) for s in lp.subs) > 255
    prob = _create(P, lp)
    _fixed(P, prob, lp, 300)
    prob.reset()
    prob.set_options(P.ldopf_default_options())
    st = prob.solve()
    ref = admm.solve(lp)
    assert st.converged and st.iterations == ref.iters
    f_lp, _, _ = central.solve_central(net)
    assert abs(prob.objective() - f_lp) <= 1e-3 * abs(f_lp)


def test_subsystem_above_the_limit_is_refused(gpu):
    P = gpu
    lp = single_subsystem_lp(feeder("123"))  # 2,875 variables
    with pytest.raises(P.LdopfError) as e:
        _create(P, lp)
    assert e.value.code == -9
