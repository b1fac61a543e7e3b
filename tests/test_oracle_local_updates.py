"""Why several local updates per global update (one of the acceleration
schemes Section III-D names) are not built.

In this method the local update is an exact Euclidean projection (closed_2),
so repeating it with the same global x and lambda returns the same x_s. The
only way to make repeated local updates do something is to update the duals
(ADMM-3) after each of them, with x fixed; in the row space of A_s that
multiplies the dual step by the number of repetitions E. On the 13-bus
feeder that breaks the method: with E = 2 the test of Section III-C is not
met within 20,000 sweeps, and with E = 3 it is met at a point whose
objective is far from the LP optimum (HiGHS), where plain ADMM (E = 1)
converges to it.
"""
import numpy as np

from conftest import feeder, oracle_prep
from oracle import admm, central


def _run(E, max_iter):
    prep = oracle_prep("13")
    st = admm.initial_state(prep)
    xs, lam = st.xs.copy(), st.lam.copy()
    for t in range(1, max_iter + 1):
        x = admm.global_update(prep, xs, lam, 100.0)
        xs_prev = xs
        for _ in range(E):
            z, xs = admm.local_update(prep, x, lam, 100.0)
            lam = admm.dual_update(lam, z, xs, 100.0)
        r = admm.residuals(prep, z, xs, xs_prev, lam, 100.0, 1e-4, 0.0, "paper")
        if r[0] <= r[2] and r[1] <= r[3]:
            return t, float(prep.lp.c @ x)
    return None, float(prep.lp.c @ x)


def test_repeating_the_projection_alone_changes_nothing():
    prep = oracle_prep("13")
    res = admm.solve(prep, max_iter=50, check=False)
    x = admm.global_update(prep, res.xs, res.lam, 100.0)
    _, a = admm.local_update(prep, x, res.lam, 100.0)
    _, b = admm.local_update(prep, x, res.lam, 100.0)
    np.testing.assert_array_equal(a, b)


def test_repeated_local_and_dual_updates_do_not_reach_the_optimum():
    f_lp, _, _ = central.solve_central(feeder("13"))
    t1, f1 = _run(1, 20000)
    assert t1 is not None and abs(f1 - f_lp) <= 1e-3 * abs(f_lp)
    t2, _ = _run(2, 20000)
    assert t2 is None
    t3, f3 = _run(3, 20000)
    assert t3 is not None and abs(f3 - f_lp) > 0.5 * abs(f_lp)
