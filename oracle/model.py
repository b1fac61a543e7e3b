"""Network -> linearized OPF LP -> consensus decomposition (oracle side).

Follows Section II-A of the paper (operational bounds, power balance,
voltage-dependent load model, linearized power flow, objective), the abstract
LP form with its variable blocks (LP_model), the consensus model with bounds
kept only on the global vector (OurModel, Section III-A) and the decomposition
of Section V-A: one subsystem per line and per bus, each leaf bus merged into
its line, so S = buses + lines - leaves (Table 3).

Readings of the paper taken here (each one is listed with its reason in the
design notes of the repository):

* Each line is stored once, oriented i -> j. Its three rows per phase are
  written once; bus i's balance uses p_eij, bus j's uses p_eji.
* M^p and M^q are printed for three phases; a one- or two-phase line uses the
  principal submatrix on its phases.
* Delta loads exist only on three-phase buses; the sum constraint of the delta
  model means two rows (real and reactive).
* Subsystem membership is structural: a subsystem holds every variable its
  component's equations are written in, even where a coefficient is zero.
* The shunt terms inside the voltage-drop equation use the from side only, as
  printed.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SQ3 = math.sqrt(3.0)
PHASE_BITS = (1, 2, 4)


def phases(mask) -> list:
    return [k for k in range(3) if int(mask) & PHASE_BITS[k]]


def m_matrices(r: np.ndarray, x: np.ndarray):
    """M^p and M^q of a line from its 3x3 R and X, as printed in Section II-A."""
    r = r.reshape(3, 3)
    x = x.reshape(3, 3)
    Mp = np.array([
        [-2 * r[0, 0], r[0, 1] - SQ3 * x[0, 1], r[0, 2] + SQ3 * x[0, 2]],
        [r[1, 0] + SQ3 * x[1, 0], -2 * r[1, 1], r[1, 2] - SQ3 * x[1, 2]],
        [r[2, 0] - SQ3 * x[2, 0], r[2, 1] + SQ3 * x[2, 1], -2 * r[2, 2]],
    ])
    Mq = np.array([
        [-2 * x[0, 0], x[0, 1] + SQ3 * r[0, 1], x[0, 2] - SQ3 * r[0, 2]],
        [x[1, 0] - SQ3 * r[1, 0], -2 * x[1, 1], x[1, 2] + SQ3 * r[1, 2]],
        [x[2, 0] + SQ3 * r[2, 0], x[2, 1] - SQ3 * r[2, 1], -2 * x[2, 2]],
    ])
    return Mp, Mq


@dataclasses.dataclass
class Index:
    """Canonical positions of every variable in the global vector x.

    Block order of LP_model: generators (p^g, q^g per phase), squared voltages
    w per bus and phase, loads (p^b, q^b, p^d, q^d per phase), line flows
    (p_ij, q_ij, p_ji, q_ji per phase). Within a component, phases ascend.
    """

    n: int
    pg: dict  # (k, phi) -> index
    qg: dict
    w: dict  # (i, phi)
    pb: dict  # (l, phi)
    qb: dict
    pd: dict
    qd: dict
    pij: dict  # (e, phi)
    qij: dict
    pji: dict
    qji: dict
    is_voltage: np.ndarray  # bool [n]
    kind: list  # readable tag per index


def build_index(net: dict) -> Index:
    pg, qg, w, pb, qb, pd, qd, pij, qij, pji, qji = ({} for _ in range(11))
    kind = []
    pos = 0

    def take(d, key, tag):
        nonlocal pos
        d[key] = pos
        kind.append(tag + str(key))
        pos += 1

    for k in range(net["n_gen"]):
        for f in phases(net["gen_phases"][k]):
            take(pg, (k, f), "pg")
            take(qg, (k, f), "qg")
    for i in range(net["n_bus"]):
        for f in phases(net["bus_phases"][i]):
            take(w, (i, f), "w")
    for l in range(net["n_load"]):
        for f in phases(net["load_phases"][l]):
            take(pb, (l, f), "pb")
            take(qb, (l, f), "qb")
            take(pd, (l, f), "pd")
            take(qd, (l, f), "qd")
    for e in range(net["n_line"]):
        for f in phases(net["line_phases"][e]):
            take(pij, (e, f), "pij")
            take(qij, (e, f), "qij")
            take(pji, (e, f), "pji")
            take(qji, (e, f), "qji")
    is_v = np.zeros(pos, dtype=bool)
    for v in w.values():
        is_v[v] = True
    return Index(pos, pg, qg, w, pb, qb, pd, qd, pij, qij, pji, qji, is_v, kind)


def bounds_and_cost(net: dict, ix: Index):
    """x_lo, x_hi from the operational bounds; c from the objective (sum of p^g)."""
    lo = np.full(ix.n, -np.inf)
    hi = np.full(ix.n, np.inf)
    c = np.zeros(ix.n)
    for (k, f), v in ix.pg.items():
        lo[v], hi[v] = net["gen_plo"][k, f], net["gen_phi"][k, f]
        c[v] = net["gen_cost_p"][k, f]
    for (k, f), v in ix.qg.items():
        lo[v], hi[v] = net["gen_qlo"][k, f], net["gen_qhi"][k, f]
        c[v] = net["gen_cost_q"][k, f]
    for (i, f), v in ix.w.items():
        lo[v], hi[v] = net["bus_wlo"][i, f], net["bus_whi"][i, f]
    for (e, f), v in ix.pij.items():
        lo[v], hi[v] = net["line_plo"][e, f], net["line_phi"][e, f]
    for (e, f), v in ix.pji.items():
        lo[v], hi[v] = net["line_plo"][e, f], net["line_phi"][e, f]
    for (e, f), v in ix.qij.items():
        lo[v], hi[v] = net["line_qlo"][e, f], net["line_qhi"][e, f]
    for (e, f), v in ix.qji.items():
        lo[v], hi[v] = net["line_qlo"][e, f], net["line_qhi"][e, f]
    return c, lo, hi


def incidence(net: dict):
    """Per bus: incident lines, attached loads, attached generators."""
    nb = net["n_bus"]
    lines_at = [[] for _ in range(nb)]
    loads_at = [[] for _ in range(nb)]
    gens_at = [[] for _ in range(nb)]
    for e in range(net["n_line"]):
        lines_at[int(net["line_from"][e])].append(e)
        if int(net["line_to"][e]) != int(net["line_from"][e]):
            lines_at[int(net["line_to"][e])].append(e)
    for l in range(net["n_load"]):
        loads_at[int(net["load_bus"][l])].append(l)
    for k in range(net["n_gen"]):
        gens_at[int(net["gen_bus"][k])].append(k)
    return lines_at, loads_at, gens_at


# A row is (coefficients {global index: value}, right-hand side).

def _add(row, col, val):
    row[col] = row.get(col, 0.0) + val


def bus_rows(net: dict, ix: Index, i: int, inc) -> list:
    """Power balance at bus i, real then reactive, for each phase of the bus."""
    lines_at, loads_at, gens_at = inc
    rows = []
    for f in phases(net["bus_phases"][i]):
        rp, rq = {}, {}
        for e in lines_at[i]:
            if not (int(net["line_phases"][e]) & PHASE_BITS[f]):
                continue
            if net["line_from"][e] == i:
                _add(rp, ix.pij[(e, f)], 1.0)
                _add(rq, ix.qij[(e, f)], 1.0)
            if net["line_to"][e] == i:
                _add(rp, ix.pji[(e, f)], 1.0)
                _add(rq, ix.qji[(e, f)], 1.0)
        for l in loads_at[i]:
            if int(net["load_phases"][l]) & PHASE_BITS[f]:
                _add(rp, ix.pb[(l, f)], 1.0)
                _add(rq, ix.qb[(l, f)], 1.0)
        _add(rp, ix.w[(i, f)], net["bus_gsh"][i, f])
        _add(rq, ix.w[(i, f)], -net["bus_bsh"][i, f])
        for k in gens_at[i]:
            if int(net["gen_phases"][k]) & PHASE_BITS[f]:
                _add(rp, ix.pg[(k, f)], -1.0)
                _add(rq, ix.qg[(k, f)], -1.0)
        rows.append((rp, 0.0))
        rows.append((rq, 0.0))
    return rows


def load_rows(net: dict, ix: Index, l: int) -> list:
    """Voltage-dependent load model rows of load l.

    Wye: per phase p^d - (a alpha/2) w = a - a alpha/2, the reactive analogue,
    p^b = p^d and q^b = q^d. Delta (three-phase only): the same two model rows
    per phase with w-hat = 3w, the two sum rows and the four coupling rows.
    """
    i = int(net["load_bus"][l])
    ph = phases(net["load_phases"][l])
    a, b = net["load_a"][l], net["load_b"][l]
    al, be = net["load_alpha"][l], net["load_beta"][l]
    rows = []
    if int(net["load_conn"][l]) == 0:
        for f in ph:
            rows.append(({ix.pd[(l, f)]: 1.0, ix.w[(i, f)]: -a[f] * al[f] / 2.0}, a[f] - a[f] * al[f] / 2.0))
            rows.append(({ix.qd[(l, f)]: 1.0, ix.w[(i, f)]: -b[f] * be[f] / 2.0}, b[f] - b[f] * be[f] / 2.0))
            rows.append(({ix.pb[(l, f)]: 1.0, ix.pd[(l, f)]: -1.0}, 0.0))
            rows.append(({ix.qb[(l, f)]: 1.0, ix.qd[(l, f)]: -1.0}, 0.0))
        return rows
    if ph != [0, 1, 2]:
        raise ValueError(f"delta load {l} must be three-phase")
    for f in ph:
        rows.append(({ix.pd[(l, f)]: 1.0, ix.w[(i, f)]: -3.0 * a[f] * al[f] / 2.0}, a[f] - a[f] * al[f] / 2.0))
    for f in ph:
        rows.append(({ix.qd[(l, f)]: 1.0, ix.w[(i, f)]: -3.0 * b[f] * be[f] / 2.0}, b[f] - b[f] * be[f] / 2.0))
    P = lambda d, f: d[(l, f)]  # noqa: E731
    rp, rq = {}, {}
    for f in ph:
        _add(rp, P(ix.pb, f), 1.0)
        _add(rp, P(ix.pd, f), -1.0)
        _add(rq, P(ix.qb, f), 1.0)
        _add(rq, P(ix.qd, f), -1.0)
    rows.append((rp, 0.0))
    rows.append((rq, 0.0))
    # phases 1, 2, 3 of the coupling rows are a, b, c (indices 0, 1, 2)
    pb1, pb2, pb3 = (P(ix.pb, f) for f in ph)
    qb1, qb2, qb3 = (P(ix.qb, f) for f in ph)
    pd1, pd2, pd3 = (P(ix.pd, f) for f in ph)
    qd1, qd2, qd3 = (P(ix.qd, f) for f in ph)
    h = 0.5
    s = SQ3 / 2.0
    rows.append(({pb2: 1.5, qb2: -s, pd2: -1.0, pd1: -h, qd1: s}, 0.0))
    rows.append(({pb2: s, qb2: 1.5, pd1: -s, qd1: -h, qd2: -1.0}, 0.0))
    rows.append(({qb2: SQ3, pb3: 1.5, qb3: -s, pd1: -h, qd1: -s, pd3: -1.0}, 0.0))
    rows.append(({pb2: -SQ3, pb3: s, qb3: 1.5, pd1: s, qd1: -h, qd3: -1.0}, 0.0))
    return rows


def line_rows(net: dict, ix: Index, e: int) -> list:
    """Linearized power flow of line e = (i -> j): two loss rows and the
    voltage-drop row, per phase of the line."""
    i, j = int(net["line_from"][e]), int(net["line_to"][e])
    ph = phases(net["line_phases"][e])
    Mp, Mq = m_matrices(net["line_r"][e], net["line_x"][e])
    gsi, bsi = net["line_gs_from"][e], net["line_bs_from"][e]
    gsj, bsj = net["line_gs_to"][e], net["line_bs_to"][e]
    tau = net["line_tau"][e]
    rows = []
    for f in ph:
        r1 = {}
        _add(r1, ix.pij[(e, f)], 1.0)
        _add(r1, ix.pji[(e, f)], 1.0)
        _add(r1, ix.w[(i, f)], -gsi[f])
        _add(r1, ix.w[(j, f)], -gsj[f])
        r2 = {}
        _add(r2, ix.qij[(e, f)], 1.0)
        _add(r2, ix.qji[(e, f)], 1.0)
        _add(r2, ix.w[(i, f)], bsi[f])
        _add(r2, ix.w[(j, f)], bsj[f])
        # w_i - tau w_j + sum_psi Mp (p_ij - gs w_i) + sum_psi Mq (q_ij + bs w_i) = 0
        r3 = {}
        _add(r3, ix.w[(i, f)], 1.0)
        _add(r3, ix.w[(j, f)], -tau[f])
        for g in ph:
            _add(r3, ix.pij[(e, g)], Mp[f, g])
            _add(r3, ix.w[(i, g)], -Mp[f, g] * gsi[g])
            _add(r3, ix.qij[(e, g)], Mq[f, g])
            _add(r3, ix.w[(i, g)], Mq[f, g] * bsi[g])
        rows += [(r1, 0.0), (r2, 0.0), (r3, 0.0)]
    return rows


def bus_vars(net: dict, ix: Index, i: int, inc) -> set:
    """Variables of a bus component: its w, its generators, its loads and the
    flow at its end of every incident line."""
    lines_at, loads_at, gens_at = inc
    out = {ix.w[(i, f)] for f in phases(net["bus_phases"][i])}
    for k in gens_at[i]:
        for f in phases(net["gen_phases"][k]):
            out |= {ix.pg[(k, f)], ix.qg[(k, f)]}
    for l in loads_at[i]:
        for f in phases(net["load_phases"][l]):
            out |= {ix.pb[(l, f)], ix.qb[(l, f)], ix.pd[(l, f)], ix.qd[(l, f)]}
    for e in lines_at[i]:
        for f in phases(net["line_phases"][e]):
            if net["line_from"][e] == i:
                out |= {ix.pij[(e, f)], ix.qij[(e, f)]}
            if net["line_to"][e] == i:
                out |= {ix.pji[(e, f)], ix.qji[(e, f)]}
    return out


def line_vars(net: dict, ix: Index, e: int) -> set:
    i, j = int(net["line_from"][e]), int(net["line_to"][e])
    out = set()
    for f in phases(net["line_phases"][e]):
        out |= {ix.pij[(e, f)], ix.qij[(e, f)], ix.pji[(e, f)], ix.qji[(e, f)],
                ix.w[(i, f)], ix.w[(j, f)]}
    return out


@dataclasses.dataclass
class Subsystem:
    gidx: np.ndarray  # int64 [n_s], ascending global indices (the rows of B_s)
    A: np.ndarray  # [m_s, n_s]
    b: np.ndarray  # [m_s]
    tag: tuple  # ("line", e, merged_leaf_buses) or ("bus", i)


@dataclasses.dataclass
class ConsensusLP:
    """OurModel: min c'x, A_s x_s = b_s, B_s x = x_s, lo <= x <= hi."""

    n: int
    c: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    subs: list
    x_init: np.ndarray | None = None  # per global variable, copied into every x_s


def _dense(rows: list, cols: np.ndarray):
    pos = {int(g): t for t, g in enumerate(cols)}
    A = np.zeros((len(rows), len(cols)))
    b = np.zeros(len(rows))
    for r, (coef, rhs) in enumerate(rows):
        for g, v in coef.items():
            A[r, pos[g]] += v
        b[r] = rhs
    return A, b


def degrees(net: dict) -> np.ndarray:
    deg = np.zeros(net["n_bus"], dtype=np.int64)
    np.add.at(deg, net["line_from"], 1)
    np.add.at(deg, net["line_to"], 1)
    return deg


def leaves(net: dict) -> np.ndarray:
    """Leaf buses: non-root buses with exactly one incident line."""
    deg = degrees(net)
    is_leaf = deg == 1
    is_leaf[int(net["root"])] = False
    return is_leaf


def init_values(ix: Index, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Starting value of each global variable's copies (Section V-A): one for a
    squared voltage, the bound midpoint where both bounds are finite, zero
    (clipped into the box) otherwise.

    Pinned by the hand-derived first sweep of the two-bus case
    (tests/golden/two_bus.json, "first_sweep"), whose first global iterate
    is clip(x_init - c / (rho N))."""
    out = np.clip(np.zeros(ix.n), lo, hi)
    both = np.isfinite(lo) & np.isfinite(hi)
    out[both] = 0.5 * (lo[both] + hi[both])
    out[ix.is_voltage] = 1.0
    return out


def decompose(net: dict) -> ConsensusLP:
    """Component-wise decomposition with leaf merging (Section V-A).

    Subsystem order: one per line in line order (a leaf end bus merged into
    it), then one per non-leaf bus in bus order. Rows inside a subsystem: the
    line's rows, then for each merged leaf bus its balance rows and its loads'
    rows; a bus subsystem holds its balance rows then its loads' rows.
    Columns are the structural variable set, ascending.
    """
    ix = build_index(net)
    c, lo, hi = bounds_and_cost(net, ix)
    is_leaf = leaves(net)
    inc = incidence(net)

    def bus_block(i):
        rows = bus_rows(net, ix, i, inc)
        for l in inc[1][i]:
            rows += load_rows(net, ix, l)
        return rows, bus_vars(net, ix, i, inc)

    subs = []
    for e in range(net["n_line"]):
        rows = line_rows(net, ix, e)
        vars_ = line_vars(net, ix, e)
        merged = []
        for end in (int(net["line_from"][e]), int(net["line_to"][e])):
            if is_leaf[end]:
                brows, bvars = bus_block(end)
                rows += brows
                vars_ |= bvars
                merged.append(end)
        cols = np.array(sorted(vars_), dtype=np.int64)
        A, b = _dense(rows, cols)
        subs.append(Subsystem(cols, A, b, ("line", e, tuple(merged))))
    for i in range(net["n_bus"]):
        if is_leaf[i]:
            continue
        rows, vars_ = bus_block(i)
        cols = np.array(sorted(vars_), dtype=np.int64)
        A, b = _dense(rows, cols)
        subs.append(Subsystem(cols, A, b, ("bus", i)))
    return ConsensusLP(ix.n, c, lo, hi, subs, init_values(ix, lo, hi))


def central_rows(net: dict):
    """All rows of LP_model (A x = b) in one list: buses, loads, lines."""
    ix = build_index(net)
    inc = incidence(net)
    rows = []
    for i in range(net["n_bus"]):
        rows += bus_rows(net, ix, i, inc)
    for l in range(net["n_load"]):
        rows += load_rows(net, ix, l)
    for e in range(net["n_line"]):
        rows += line_rows(net, ix, e)
    return ix, rows
