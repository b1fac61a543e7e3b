"""Seeded synthetic radial multi-phase distribution feeders.

This module only draws inputs. It holds none of the solver's arithmetic: it
builds no LP rows, no operators and no ADMM step. Both the CPU oracle and the
GPU library consume the structure-of-arrays network it returns.

The network data follow the paper's nomenclature table (Section II): buses with
phase sets and squared-voltage bounds, lines with 3x3 series resistance and
reactance, shunts and taps, loads with reference powers a, b and load-type
exponents alpha, beta (the voltage-dependent load model), generators with
power boxes and a linear cost (the objective sums generator real power).

The paper measures on the IEEE 13/37/123/8500-bus feeders, whose data are not
available here. These feeders stand in for them with the same kind of
structure: a radial tree grown breadth-first, three-phase trunks with two- and
single-phase laterals, per-phase loads, one substation generator, optional
distributed PV units.

Layout of the returned dict (``n_*`` are Python ints, everything else numpy):

* ``bus_phases``  uint8 [n_bus]        phase bitmask, a=1, b=2, c=4
* ``bus_wlo``, ``bus_whi``  f64 [n_bus, 3]  squared-voltage bounds
* ``bus_gsh``, ``bus_bsh``  f64 [n_bus, 3]  bus shunt conductance/susceptance
* ``line_from``, ``line_to``  int32 [n_line]  parent bus -> child bus
* ``line_phases`` uint8 [n_line]
* ``line_r``, ``line_x``  f64 [n_line, 9]  row-major 3x3, per unit
* ``line_gs_from``, ``line_bs_from``, ``line_gs_to``, ``line_bs_to``  f64 [n_line, 3]
* ``line_tau``  f64 [n_line, 3]  tap ratio
* ``line_plo``, ``line_phi``, ``line_qlo``, ``line_qhi``  f64 [n_line, 3]
* ``load_bus`` int32, ``load_phases`` uint8, ``load_conn`` uint8 (0 wye, 1 delta)
* ``load_a``, ``load_b``, ``load_alpha``, ``load_beta``  f64 [n_load, 3]
* ``gen_bus`` int32, ``gen_phases`` uint8
* ``gen_plo``, ``gen_phi``, ``gen_qlo``, ``gen_qhi``, ``gen_cost_p``, ``gen_cost_q``  f64 [n_gen, 3]

Entries for phases a component does not carry are zero (bounds: +-inf).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

PHASE_BITS = (1, 2, 4)
INF = math.inf


@dataclasses.dataclass(frozen=True)
class FeederSpec:
    """Recipe for one synthetic feeder class."""

    n_bus: int
    frac3: float  # share of lines (by descending subtree size) with 3 phases
    frac2: float  # next share with 2 phases; the rest are single-phase
    v_ln_kv: float  # line-to-neutral base voltage of the feeder class
    load_dist: str  # "uniform100" (U[0,100] kW) or "lognormal5" (lognormal(ln 5 kW, 0.8))
    n_pv: int = 0
    fixed_source: bool = False  # root squared voltage fixed to [1, 1]
    alpha_choices: tuple = (0, 1, 2)  # load-type exponents drawn uniformly
    max_drop: float = 0.04  # repair target for the crude voltage-drop bound
    wlo: float = 0.9025
    whi: float = 1.1025


# The five workload classes: 13-bus, 123-bus + 4 PV, 8500-bus, 2500-bus (scenarios).
SPECS = {
    "13": FeederSpec(13, 0.6, 0.2, 2.4018, "uniform100"),
    "123": FeederSpec(123, 0.7, 0.2, 2.4018, "uniform100", n_pv=4),
    "2500": FeederSpec(2500, 0.2, 0.1, 7.2, "lognormal5"),
    "8500": FeederSpec(8500, 0.2, 0.1, 7.2, "lognormal5"),
}
DEFAULT_SEEDS = {"13": 13, "123": 123, "2500": 2500, "8500": 8500}


def _grow_tree(n_bus: int, rng: np.random.Generator):
    """Breadth-first growth: pop a bus, give it U{1,2,3} children, stop at n_bus."""
    parent = np.full(n_bus, -1, dtype=np.int64)
    queue = [0]
    count = 1
    head = 0
    while count < n_bus:
        b = queue[head]
        head += 1
        c = int(rng.integers(1, 4))
        for _ in range(min(c, n_bus - count)):
            parent[count] = b
            queue.append(count)
            count += 1
    return parent


def _subtree_sizes(parent: np.ndarray) -> np.ndarray:
    n = parent.shape[0]
    size = np.ones(n, dtype=np.int64)
    # children always carry larger ids than their parent (breadth-first growth)
    for v in range(n - 1, 0, -1):
        size[parent[v]] += size[v]
    return size


def _bits(mask: int):
    return [k for k in range(3) if mask & PHASE_BITS[k]]


def _mask(phases) -> int:
    m = 0
    for k in phases:
        m |= PHASE_BITS[k]
    return m


def make_feeder(spec: FeederSpec | str, seed: int) -> dict:
    """Draw one feeder. Same (spec, seed) gives the same arrays, bit for bit."""
    if isinstance(spec, str):
        spec = SPECS[spec]
    rng = np.random.Generator(np.random.PCG64(seed))
    nb = spec.n_bus
    if nb < 1:
        raise ValueError("n_bus must be >= 1")
    parent = _grow_tree(nb, rng)
    nl = nb - 1
    # line e connects parent[e+1] -> e+1 (children are created in id order)
    line_to = np.arange(1, nb, dtype=np.int32)
    line_from = parent[1:].astype(np.int32)

    # --- phases: rank lines by descending subtree size, ties by child id
    size = _subtree_sizes(parent)
    order = sorted(range(nl), key=lambda e: (-int(size[e + 1]), e + 1))
    n3 = int(round(spec.frac3 * nl))
    n2 = int(round(spec.frac2 * nl))
    want = np.ones(nl, dtype=np.int64)
    for rank, e in enumerate(order):
        want[e] = 3 if rank < n3 else (2 if rank < n3 + n2 else 1)
    bus_phases = np.zeros(nb, dtype=np.uint8)
    bus_phases[0] = 7
    line_phases = np.zeros(nl, dtype=np.uint8)
    for e in range(nl):  # parents are processed before children
        i, j = int(line_from[e]), int(line_to[e])
        par = _bits(int(bus_phases[i]))
        k = min(int(want[e]), len(par))
        if k == len(par):
            ph = par
        else:
            ph = sorted(rng.choice(par, size=k, replace=False).tolist())
        line_phases[e] = _mask(ph)
        bus_phases[j] = line_phases[e]

    # --- impedances: symmetric 3x3, upper entries U[0.1,0.5] ohm/km, times length
    zbase = spec.v_ln_kv ** 2 / 1.0  # ohm, S_base = 1 MVA per phase
    line_r = np.zeros((nl, 9))
    line_x = np.zeros((nl, 9))
    for e in range(nl):
        length = rng.uniform(0.1, 1.0)
        ru = rng.uniform(0.1, 0.5, size=6)
        xu = rng.uniform(0.1, 0.5, size=6)
        R = np.zeros((3, 3))
        X = np.zeros((3, 3))
        iu = np.triu_indices(3)
        R[iu] = ru
        X[iu] = xu
        R = R + np.triu(R, 1).T
        X = X + np.triu(X, 1).T
        ph = _bits(int(line_phases[e]))
        M = np.zeros((3, 3), dtype=bool)
        M[np.ix_(ph, ph)] = True
        line_r[e] = np.where(M, R * length / zbase, 0.0).ravel()
        line_x[e] = np.where(M, X * length / zbase, 0.0).ravel()

    # --- loads: one wye load per non-root bus on all its phases
    n_load = nb - 1
    load_bus = np.arange(1, nb, dtype=np.int32)
    load_phases = bus_phases[1:].copy()
    load_conn = np.zeros(n_load, dtype=np.uint8)
    load_a = np.zeros((n_load, 3))
    load_b = np.zeros((n_load, 3))
    load_alpha = np.zeros((n_load, 3))
    load_beta = np.zeros((n_load, 3))
    for l in range(n_load):
        ph = _bits(int(load_phases[l]))
        if spec.load_dist == "uniform100":
            pkw = rng.uniform(0.0, 100.0, size=len(ph))
        elif spec.load_dist == "lognormal5":
            pkw = rng.lognormal(mean=math.log(5.0), sigma=0.8, size=len(ph))
        else:
            raise ValueError(spec.load_dist)
        alpha = float(rng.choice(spec.alpha_choices))
        for t, k in enumerate(ph):
            load_a[l, k] = pkw[t] / 1000.0  # kW -> MW = pu on 1 MVA
            load_b[l, k] = 0.3 * pkw[t] / 1000.0
            load_alpha[l, k] = alpha
            load_beta[l, k] = alpha

    # --- crude voltage-drop bound and impedance repair (generator heuristic)
    kappa = _repair_scale(nb, line_from, line_to, line_phases, line_r, line_x,
                          load_bus, load_a, load_b, spec.max_drop)
    line_r *= kappa
    line_x *= kappa

    # --- generators: substation on abc, optional PV units
    ptot = load_a.sum(axis=0)
    gen_bus = [0]
    gen_phases = [7]
    plo = [[-2 * max(ptot[k], 0.005) for k in range(3)]]
    phi = [[2 * max(ptot[k], 0.005) for k in range(3)]]
    qlo = list(map(list, plo))
    qhi = list(map(list, phi))
    if spec.n_pv > 0:
        cand = np.arange(1, nb)
        pv_buses = sorted(rng.choice(cand, size=min(spec.n_pv, nb - 1), replace=False).tolist())
        for bsel in pv_buses:
            ph = _bits(int(bus_phases[bsel]))
            pmax = rng.uniform(0.0, 200.0, size=len(ph)) / 1000.0
            lo_p, hi_p, lo_q, hi_q = [0.0] * 3, [0.0] * 3, [0.0] * 3, [0.0] * 3
            for t, k in enumerate(ph):
                hi_p[k] = pmax[t]
                lo_q[k] = -0.3 * pmax[t]
                hi_q[k] = 0.3 * pmax[t]
            gen_bus.append(bsel)
            gen_phases.append(int(bus_phases[bsel]))
            plo.append(lo_p)
            phi.append(hi_p)
            qlo.append(lo_q)
            qhi.append(hi_q)
    n_gen = len(gen_bus)
    gph = np.array(gen_phases, dtype=np.uint8)
    gmask = np.array([[bool(g & PHASE_BITS[k]) for k in range(3)] for g in gph])
    gen_cost_p = np.where(gmask, 1.0, 0.0)
    gen_cost_q = np.zeros((n_gen, 3))

    bus_wlo = np.zeros((nb, 3))
    bus_whi = np.zeros((nb, 3))
    for i in range(nb):
        for k in _bits(int(bus_phases[i])):
            bus_wlo[i, k] = spec.wlo
            bus_whi[i, k] = spec.whi
    if spec.fixed_source:
        bus_wlo[0, :] = 1.0
        bus_whi[0, :] = 1.0

    lmask = np.array([[bool(p & PHASE_BITS[k]) for k in range(3)] for p in line_phases]).reshape(nl, 3)
    unb_lo = np.where(lmask, -INF, 0.0)
    unb_hi = np.where(lmask, INF, 0.0)
    return {
        "n_bus": nb, "n_line": nl, "n_load": n_load, "n_gen": n_gen, "root": 0,
        "bus_phases": bus_phases,
        "bus_wlo": bus_wlo, "bus_whi": bus_whi,
        "bus_gsh": np.zeros((nb, 3)), "bus_bsh": np.zeros((nb, 3)),
        "line_from": line_from, "line_to": line_to, "line_phases": line_phases,
        "line_r": line_r, "line_x": line_x,
        "line_gs_from": np.zeros((nl, 3)), "line_bs_from": np.zeros((nl, 3)),
        "line_gs_to": np.zeros((nl, 3)), "line_bs_to": np.zeros((nl, 3)),
        "line_tau": np.where(lmask, 1.0, 0.0),
        "line_plo": unb_lo.copy(), "line_phi": unb_hi.copy(),
        "line_qlo": unb_lo.copy(), "line_qhi": unb_hi.copy(),
        "load_bus": load_bus, "load_phases": load_phases, "load_conn": load_conn,
        "load_a": load_a, "load_b": load_b, "load_alpha": load_alpha, "load_beta": load_beta,
        "gen_bus": np.array(gen_bus, dtype=np.int32), "gen_phases": gph,
        "gen_plo": np.where(gmask, np.array(plo), 0.0), "gen_phi": np.where(gmask, np.array(phi), 0.0),
        "gen_qlo": np.where(gmask, np.array(qlo), 0.0), "gen_qhi": np.where(gmask, np.array(qhi), 0.0),
        "gen_cost_p": gen_cost_p, "gen_cost_q": gen_cost_q,
        "meta": {"kappa": kappa, "seed": seed, "spec": dataclasses.asdict(spec)},
    }


def _repair_scale(nb, line_from, line_to, line_phases, line_r, line_x,
                  load_bus, load_a, load_b, max_drop):
    """Scale factor for all impedances so a coarse voltage-drop estimate stays small.

    The estimate is independent of the LP: along every path from the root,
    phase phi of each line adds 2 * sum_psi (|R_phi,psi| + |X_phi,psi|) *
    (downstream real + reactive load on phase psi). If the largest estimate
    exceeds ``max_drop`` every R and X is multiplied by ``max_drop / estimate``.
    Lognormal loads on thousands of buses would otherwise push squared
    voltages outside [0.9025, 1.1025] and make the problem infeasible.
    """
    nl = line_from.shape[0]
    if nl == 0:
        return 1.0
    down = np.zeros((nb, 3))
    np.add.at(down, load_bus, load_a + load_b)
    for e in range(nl - 1, -1, -1):  # children have larger ids
        down[line_from[e]] += down[line_to[e]]
    drop = np.zeros((nb, 3))
    worst = 0.0
    for e in range(nl):
        Z = (np.abs(line_r[e]) + np.abs(line_x[e])).reshape(3, 3)
        drop[line_to[e]] = drop[line_from[e]] + 2.0 * (Z @ down[line_to[e]])
        worst = max(worst, float(drop[line_to[e]].max()))
    if worst > max_drop:
        return max_drop / worst
    return 1.0


def scale_loads(net: dict, factors: np.ndarray) -> dict:
    """Copy of ``net`` with each load's a and b multiplied by a per-load factor."""
    out = dict(net)
    out["load_a"] = net["load_a"] * factors[:, None]
    out["load_b"] = net["load_b"] * factors[:, None]
    return out


def scenario_factors(net: dict, n_scen: int, base_seed: int = 2500 * 1000,
                     lo: float = 0.7, hi: float = 1.3) -> np.ndarray:
    """Per-scenario, per-bus load multipliers U[lo, hi] (same on all phases).

    Scenario k draws from its own seed ``base_seed + k``. Returns [n_scen, n_load].
    """
    out = np.empty((n_scen, net["n_load"]))
    for k in range(n_scen):
        r = np.random.Generator(np.random.PCG64(base_seed + k))
        f_bus = r.uniform(lo, hi, size=net["n_bus"])
        out[k] = f_bus[net["load_bus"]]
    return out


def two_bus(r=0.01, x=0.02, a=0.5, b=0.15, alpha=0.0, fixed_source=True) -> dict:
    """Single-phase two-bus feeder: root generator, one line, one load at bus 1."""
    nb, nl = 2, 1
    w0lo, w0hi = (1.0, 1.0) if fixed_source else (0.9025, 1.1025)
    z = np.zeros(9)
    rr = z.copy(); rr[0] = r
    xx = z.copy(); xx[0] = x
    one = np.array([[1.0, 0.0, 0.0]])
    zero3 = np.zeros((1, 3))
    return {
        "n_bus": nb, "n_line": nl, "n_load": 1, "n_gen": 1, "root": 0,
        "bus_phases": np.array([1, 1], dtype=np.uint8),
        "bus_wlo": np.array([[w0lo, 0, 0], [0.9025, 0, 0]]),
        "bus_whi": np.array([[w0hi, 0, 0], [1.1025, 0, 0]]),
        "bus_gsh": np.zeros((2, 3)), "bus_bsh": np.zeros((2, 3)),
        "line_from": np.array([0], dtype=np.int32), "line_to": np.array([1], dtype=np.int32),
        "line_phases": np.array([1], dtype=np.uint8),
        "line_r": rr[None, :], "line_x": xx[None, :],
        "line_gs_from": zero3.copy(), "line_bs_from": zero3.copy(),
        "line_gs_to": zero3.copy(), "line_bs_to": zero3.copy(),
        "line_tau": one.copy(),
        "line_plo": np.array([[-INF, 0, 0]]), "line_phi": np.array([[INF, 0, 0]]),
        "line_qlo": np.array([[-INF, 0, 0]]), "line_qhi": np.array([[INF, 0, 0]]),
        "load_bus": np.array([1], dtype=np.int32), "load_phases": np.array([1], dtype=np.uint8),
        "load_conn": np.array([0], dtype=np.uint8),
        "load_a": np.array([[a, 0, 0]]), "load_b": np.array([[b, 0, 0]]),
        "load_alpha": np.array([[alpha, 0, 0]]), "load_beta": np.array([[alpha, 0, 0]]),
        "gen_bus": np.array([0], dtype=np.int32), "gen_phases": np.array([1], dtype=np.uint8),
        "gen_plo": np.array([[-10.0, 0, 0]]), "gen_phi": np.array([[10.0, 0, 0]]),
        "gen_qlo": np.array([[-10.0, 0, 0]]), "gen_qhi": np.array([[10.0, 0, 0]]),
        "gen_cost_p": one.copy(), "gen_cost_q": zero3.copy(),
        "meta": {"kappa": 1.0, "seed": None, "spec": "two_bus"},
    }


def perturb_extras(net: dict, seed: int, delta_frac: float = 0.3) -> dict:
    """Copy of ``net`` with nonzero shunts, off-nominal taps and some delta loads.

    Used by assembler tests only: exercises the shunt, tap and delta-load
    terms of the model that the workload feeders leave at zero / one / wye.
    Delta loads are placed only on three-phase buses.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in net.items()}
    bm = np.array([[bool(p & PHASE_BITS[k]) for k in range(3)] for p in net["bus_phases"]])
    lm = np.array([[bool(p & PHASE_BITS[k]) for k in range(3)] for p in net["line_phases"]]).reshape(-1, 3)
    out["bus_gsh"] = np.where(bm, rng.uniform(0, 1e-3, bm.shape), 0.0)
    out["bus_bsh"] = np.where(bm, rng.uniform(0, 1e-3, bm.shape), 0.0)
    for key in ("line_gs_from", "line_bs_from", "line_gs_to", "line_bs_to"):
        out[key] = np.where(lm, rng.uniform(0, 5e-4, lm.shape), 0.0)
    out["line_tau"] = np.where(lm, rng.uniform(0.97, 1.03, lm.shape), 0.0)
    conn = out["load_conn"]
    for l in range(net["n_load"]):
        if net["load_phases"][l] == 7 and rng.uniform() < delta_frac:
            conn[l] = 1
    out["load_conn"] = conn
    return out
