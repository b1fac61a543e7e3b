"""ADMM with closed-form updates on the consensus LP (oracle side, FP64).

Algorithm 1 of the paper, step by step:

* precompute, once per subsystem (Section III-B, closed_2):
  Abar_s = A_s' (A_s A_s')^-1 A_s - I and bbar_s = A_s' (A_s A_s')^-1 b_s;
  a rank-deficient A_s takes the pseudo-inverse form (the paper's "row
  reduction", which gives the same operators at full rank);
* initialization (Section V-A): lambda = 0; every copy starts at its global
  variable's starting value;
* each iteration: the global update (closed_1, in the form obtained by
  differentiating ADMM-1), the local update (closed_2), the dual update
  (ADMM-3) and the termination test (Section III-C) on the new iterate.

The global update: the printed closed_1 drops a factor rho on the sum of the
local copies; setting the derivative of the one-dimensional objective of
ADMM-1 to zero gives x_i = (sum_k x_k - (c_i + sum_k lambda_k) / rho) / N_i,
clipped into [lo_i, hi_i]. The tests pin this reading against brute-force
minimization of ADMM-1.

Residual forms: "paper" takes the norms of Section III-C literally (the sum
over subsystems is outside the B_s' product, so dres = rho * ||x_s - x_s_prev||
over all copies and eps_dual = eps_rel * ||lambda|| over all copies);
"aggregated" is the textbook form with B_s' summed first.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg
import scipy.sparse

from .model import ConsensusLP


class InconsistentSubsystem(ValueError):
    pass


def precompute(A: np.ndarray, b: np.ndarray):
    """Abar_s and bbar_s of closed_2 for one subsystem.

    Full row rank: Cholesky of A A' (the paper's formula). Otherwise the
    pseudo-inverse form Abar = A^+ A - I, bbar = A^+ b, after checking that
    b lies in the range of A.
    """
    m, n = A.shape
    eye = np.eye(n)
    if m == 0:
        return -eye, np.zeros(n)
    G = A @ A.T
    full_rank = False
    try:
        chol = scipy.linalg.cho_factor(G)
        full_rank = np.linalg.cond(G) < 1e12
    except np.linalg.LinAlgError:
        full_rank = False
    if full_rank:
        Abar = A.T @ scipy.linalg.cho_solve(chol, A) - eye
        bbar = A.T @ scipy.linalg.cho_solve(chol, b)
        return Abar, bbar
    Ap = np.linalg.pinv(A, rcond=1e-12)
    if np.linalg.norm(A @ (Ap @ b) - b) > 1e-10 * (1.0 + np.linalg.norm(b)):
        raise InconsistentSubsystem("A_s x = b_s has no solution")
    return Ap @ A - eye, Ap @ b


@dataclasses.dataclass
class Prepared:
    lp: ConsensusLP
    gidx: np.ndarray  # int64 [N_loc], every copy's global variable, subsystem by subsystem
    offsets: np.ndarray  # int64 [S+1], copy range of each subsystem
    Abar: list  # per subsystem
    bbar: np.ndarray  # [N_loc]
    Abar_blk: scipy.sparse.csr_matrix  # block diagonal of all Abar_s
    N: np.ndarray  # copies per global variable


def prepare(lp: ConsensusLP) -> Prepared:
    sizes = [len(s.gidx) for s in lp.subs]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    gidx = np.concatenate([s.gidx for s in lp.subs]).astype(np.int64) if lp.subs else np.zeros(0, np.int64)
    Abar, bbar = [], []
    for s in lp.subs:
        Ab, bb = precompute(s.A, s.b)
        Abar.append(Ab)
        bbar.append(bb)
    blk = block_diagonal(Abar, offsets)
    N = np.bincount(gidx, minlength=lp.n).astype(np.float64)
    if np.any(N == 0):
        raise ValueError("every global variable must have at least one local copy")
    bb = np.concatenate(bbar) if bbar else np.zeros(0)
    return Prepared(lp, gidx, offsets, Abar, bb, blk, N)


def block_diagonal(blocks: list, offsets: np.ndarray) -> scipy.sparse.csr_matrix:
    rows, cols, vals = [], [], []
    for s, B in enumerate(blocks):
        o = offsets[s]
        k = B.shape[0]
        r, c = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
        rows.append((r + o).ravel())
        cols.append((c + o).ravel())
        vals.append(B.ravel())
    n = int(offsets[-1])
    if not blocks:
        return scipy.sparse.csr_matrix((n, n))
    return scipy.sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                   shape=(n, n))


@dataclasses.dataclass
class State:
    x: np.ndarray  # global, [n]
    xs: np.ndarray  # local copies, [N_loc]
    lam: np.ndarray  # duals of B_s x = x_s, [N_loc]


def initial_state(prep: Prepared) -> State:
    """lambda = 0; every copy starts at its global variable's starting value."""
    lp = prep.lp
    if lp.x_init is not None:
        start = lp.x_init
    else:
        start = np.clip(np.zeros(lp.n), lp.lo, lp.hi)
        both = np.isfinite(lp.lo) & np.isfinite(lp.hi)
        start[both] = 0.5 * (lp.lo[both] + lp.hi[both])
    xs = start[prep.gidx].astype(np.float64)
    return State(np.full(lp.n, np.nan), xs, np.zeros_like(xs))


def global_update(prep: Prepared, xs: np.ndarray, lam: np.ndarray, rho: float) -> np.ndarray:
    """closed_1 (derived form): per global variable, the minimizer of ADMM-1
    restricted to [lo_i, hi_i]."""
    lp = prep.lp
    sum_x = np.bincount(prep.gidx, weights=xs, minlength=lp.n)
    sum_lam = np.bincount(prep.gidx, weights=lam, minlength=lp.n)
    xhat = (sum_x - (lp.c + sum_lam) / rho) / prep.N
    return np.minimum(np.maximum(xhat, lp.lo), lp.hi)


def local_update(prep: Prepared, x: np.ndarray, lam: np.ndarray, rho: float):
    """closed_2: x_s = (1/rho) Abar_s d_s + bbar_s with d_s = -rho B_s x - lambda_s."""
    z = x[prep.gidx]
    d = -rho * z - lam
    xs = (prep.Abar_blk @ d) / rho + prep.bbar
    return z, xs


def dual_update(lam: np.ndarray, z: np.ndarray, xs: np.ndarray, rho: float) -> np.ndarray:
    """ADMM-3: lambda_s += rho (B_s x - x_s)."""
    return lam + rho * (z - xs)


def residuals(prep: Prepared, z, xs, xs_prev, lam, rho, eps_rel, eps_abs, form):
    """pres, dres, eps_prim, eps_dual of Section III-C.

    Pinned (tests/test_oracle_residual_pins.py) against the printed norms
    evaluated with explicit 0-1 selection matrices B_s, against the ADMM
    identity "aggregated dual residual = stationarity residual of the
    iterate" when no bound is active, and by the invariance of the test
    under scaling the cost and rho together.
    """
    nloc = xs.shape[0]
    pres = np.linalg.norm(z - xs)
    if form == "paper":
        dres = rho * np.linalg.norm(xs - xs_prev)
        dual_norm = np.linalg.norm(lam)
        dim_d = nloc
    elif form == "aggregated":
        n = prep.lp.n
        dres = rho * np.linalg.norm(np.bincount(prep.gidx, weights=xs - xs_prev, minlength=n))
        dual_norm = np.linalg.norm(np.bincount(prep.gidx, weights=lam, minlength=n))
        dim_d = n
    else:
        raise ValueError(form)
    eps_p = np.sqrt(nloc) * eps_abs + eps_rel * max(np.linalg.norm(z), np.linalg.norm(xs))
    eps_d = np.sqrt(dim_d) * eps_abs + eps_rel * dual_norm
    return pres, dres, eps_p, eps_d


@dataclasses.dataclass
class RhoBalance:
    """Residual balancing of the penalty rho.

    Section III-D names residual balancing among the acceleration schemes
    that combine with the method, without fixing a rule. The rule here is
    the classic one (He, Yang and Wang 2000; Boyd et al. 2011, Section
    3.4.1) on relative residuals, as Wohlberg (2017) recommends: after sweep
    t, with r = pres / eps_prim and s = dres / eps_dual (the two ratios of
    the termination test of Section III-C),
      rho <- tau * rho  if r > mu * s,   rho <- rho / tau  if s > mu * r.
    The rule is evaluated after the sweeps that are multiples of `period`,
    the new rho is used from sweep t + lag on, and at most `max_changes`
    changes are made (after that rho stays fixed, so the usual convergence
    argument of ADMM applies to the rest of the run). lambda is the unscaled
    dual of B_s x = x_s and is kept as it is when rho changes (only a scaled
    dual lambda / rho would need rescaling); Abar_s and bbar_s do not depend
    on rho, so nothing is recomputed.
    """
    mu: float = 10.0
    tau: float = 2.0
    period: int = 100
    lag: int = 4
    max_changes: int = 16

    def __post_init__(self):
        if not (self.mu > 1.0 and self.tau > 1.0 and self.lag >= 1 and self.period >= self.lag
                and self.max_changes >= 0):
            raise ValueError("need mu > 1, tau > 1, lag >= 1, period >= lag, max_changes >= 0")


def rescale_dual(lam: np.ndarray, rho_old: float, rho_new: float) -> np.ndarray:
    """What a change of rho does to the dual: nothing. lambda_s is the
    unscaled multiplier of B_s x = x_s in ADMM-1..3; only the scaled form
    u = lambda / rho would be rescaled, by rho_old / rho_new."""
    return lam


def balance_factor(rule: RhoBalance, pres, dres, eps_p, eps_d) -> float:
    """The factor the residual-balancing rule applies to rho after a sweep
    (1 when neither relative residual dominates or a tolerance is zero)."""
    if eps_p <= 0.0 or eps_d <= 0.0:
        return 1.0
    r, s = pres / eps_p, dres / eps_d
    if r > rule.mu * s:
        return rule.tau
    if s > rule.mu * r:
        return 1.0 / rule.tau
    return 1.0


@dataclasses.dataclass
class Result:
    x: np.ndarray
    xs: np.ndarray
    lam: np.ndarray
    history: np.ndarray  # [iters, 4]: pres, dres, eps_prim, eps_dual
    iters: int
    converged: bool
    objective: float
    prep: Prepared
    rho: float = 0.0  # rho of the last sweep
    rho_log: list = dataclasses.field(default_factory=list)  # (first sweep, rho) of every change


class Float32Steps:
    """The global, local and dual updates with every operand and result in
    float32 (the FP32-mixed form: operators precomputed in FP64 and rounded
    to float32, the state in float32; the residual norms and the test stay
    FP64). Sums over copies accumulate in float32 in copy order."""

    def __init__(self, prep: Prepared):
        lp = prep.lp
        self.prep = prep
        self.Abar = prep.Abar_blk.astype(np.float32)
        self.bbar = prep.bbar.astype(np.float32)
        self.N = prep.N.astype(np.float32)
        self.c = lp.c.astype(np.float32)
        self.lo = lp.lo.astype(np.float32)
        self.hi = lp.hi.astype(np.float32)

    def global_update(self, xs, lam, rho):
        n = self.prep.lp.n
        sx = np.zeros(n, np.float32)
        sl = np.zeros(n, np.float32)
        np.add.at(sx, self.prep.gidx, xs)
        np.add.at(sl, self.prep.gidx, lam)
        r = np.float32(rho)
        return np.minimum(np.maximum((sx - (self.c + sl) / r) / self.N, self.lo), self.hi)

    def local_update(self, x, lam, rho):
        r = np.float32(rho)
        z = x[self.prep.gidx]
        d = -r * z - lam
        return z, (self.Abar @ d) / r + self.bbar

    @staticmethod
    def dual_update(lam, z, xs, rho):
        return lam + np.float32(rho) * (z - xs)


def solve(lp_or_prep, rho: float = 100.0, eps_rel: float = 1e-4, eps_abs: float = 0.0,
          max_iter: int = 1_000_000, check: bool = True, form: str = "paper",
          state: State | None = None, on_iter=None, balance: RhoBalance | None = None,
          precision: str = "fp64") -> Result:
    """Run Algorithm 1 until the termination test holds (or ``max_iter`` sweeps).

    ``check=False`` runs exactly ``max_iter`` sweeps. ``on_iter(t, prep, state)``
    is called after every sweep (tests use it to check invariants).
    ``balance``: residual balancing of rho (RhoBalance); None keeps rho fixed.
    ``precision="fp32"``: the three updates in float32 (Float32Steps); the
    residuals and the test in FP64.
    """
    prep = lp_or_prep if isinstance(lp_or_prep, Prepared) else prepare(lp_or_prep)
    st = state if state is not None else initial_state(prep)
    x, xs, lam = st.x, st.xs.copy(), st.lam.copy()
    if precision == "fp32":
        steps = Float32Steps(prep)
        g_up, l_up, d_up = steps.global_update, steps.local_update, steps.dual_update
        xs, lam = xs.astype(np.float32), lam.astype(np.float32)
    elif precision == "fp64":
        g_up = lambda xs_, lam_, r: global_update(prep, xs_, lam_, r)  # noqa: E731
        l_up = lambda x_, lam_, r: local_update(prep, x_, lam_, r)  # noqa: E731
        d_up = dual_update
    else:
        raise ValueError(precision)
    hist = []
    converged = False
    scheduled = {}  # sweep -> rho from that sweep on
    rho_log = []
    t = 0
    while t < max_iter:
        t += 1
        if t in scheduled:
            rho_new = scheduled.pop(t)
            lam = rescale_dual(lam, rho, rho_new)
            rho = rho_new
            rho_log.append((t, rho))
        x = g_up(xs, lam, rho)
        z, xs_new = l_up(x, lam, rho)
        lam = d_up(lam, z, xs_new, rho)
        if precision == "fp32":
            r = residuals(prep, z.astype(np.float64), xs_new.astype(np.float64), xs.astype(np.float64),
                          lam.astype(np.float64), rho, eps_rel, eps_abs, form)
        else:
            r = residuals(prep, z, xs_new, xs, lam, rho, eps_rel, eps_abs, form)
        xs = xs_new
        hist.append(r)
        if on_iter is not None:
            on_iter(t, prep, State(x, xs, lam))
        if check and r[0] <= r[2] and r[1] <= r[3]:
            converged = True
            break
        if balance is not None and t % balance.period == 0 and len(rho_log) + len(scheduled) < balance.max_changes:
            f = balance_factor(balance, *r)
            if f != 1.0:
                scheduled[t + balance.lag] = rho * f
    H = np.array(hist, dtype=np.float64).reshape(-1, 4)
    x, xs, lam = (np.asarray(v, dtype=np.float64) for v in (x, xs, lam))
    return Result(x, xs, lam, H, t, converged, float(prep.lp.c @ x), prep, rho, rho_log)
