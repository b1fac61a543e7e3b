"""Centralized LP (LP_model) by HiGHS, and a KKT certificate from ADMM duals.

Used to pin the oracle's fixed point: ADMM on the consensus model must reach
the optimum of min c'x, A x = b, lo <= x <= hi.
"""
from __future__ import annotations

import numpy as np
import scipy.optimize
import scipy.sparse

from .model import central_rows


def central_lp(net: dict):
    ix, rows = central_rows(net)
    from .model import bounds_and_cost
    c, lo, hi = bounds_and_cost(net, ix)
    r, cidx, v = [], [], []
    b = np.zeros(len(rows))
    for k, (coef, rhs) in enumerate(rows):
        for g, val in coef.items():
            r.append(k)
            cidx.append(g)
            v.append(val)
        b[k] = rhs
    A = scipy.sparse.csr_matrix((v, (r, cidx)), shape=(len(rows), ix.n))
    return A, b, c, lo, hi, ix


def solve_central(net: dict):
    """HiGHS on the assembled LP; returns (objective, x, status message)."""
    A, b, c, lo, hi, _ = central_lp(net)
    bounds = list(zip([None if not np.isfinite(v) else v for v in lo],
                      [None if not np.isfinite(v) else v for v in hi]))
    res = scipy.optimize.linprog(c, A_eq=A, b_eq=b, bounds=bounds, method="highs")
    if res.status != 0:
        raise RuntimeError(f"HiGHS: {res.message}")
    return float(res.fun), res.x, res.message


def kkt_certificate(result):
    """Optimality measures of an ADMM result, built from its own duals.

    At a fixed point of the iteration, lambda_s lies in the row space of A_s
    (so lambda_s = A_s' mu_s), and the reduced cost g = c + sum_s B_s' lambda_s
    is zero at free variables, >= 0 at a variable on its lower bound and <= 0
    at one on its upper bound. Returns the largest violations.
    """
    prep = result.prep
    lp = prep.lp
    rowspace_err = 0.0
    for s, sub in enumerate(lp.subs):
        o0, o1 = prep.offsets[s], prep.offsets[s + 1]
        lam_s = result.lam[o0:o1]
        if sub.A.shape[0] == 0:
            rowspace_err = max(rowspace_err, float(np.abs(lam_s).max(initial=0.0)))
            continue
        mu, *_ = np.linalg.lstsq(sub.A.T, lam_s, rcond=None)
        rowspace_err = max(rowspace_err, float(np.abs(sub.A.T @ mu - lam_s).max(initial=0.0)))
    g = lp.c + np.bincount(prep.gidx, weights=result.lam, minlength=lp.n)
    x = result.x
    span = np.maximum(1.0, np.abs(x))
    tol = 1e-6 * span
    at_lo = np.abs(x - lp.lo) <= tol
    at_hi = np.abs(x - lp.hi) <= tol
    free = ~(at_lo | at_hi)
    viol = np.zeros(lp.n)
    viol[free] = np.abs(g[free])
    viol[at_lo & ~at_hi] = np.maximum(0.0, -g[at_lo & ~at_hi])
    viol[at_hi & ~at_lo] = np.maximum(0.0, g[at_hi & ~at_lo])
    return {"rowspace": rowspace_err, "reduced_cost": float(viol.max(initial=0.0)),
            "gscale": float(np.abs(lp.c).max(initial=1.0))}
