"""The byte accounting of the measurement, pinned to the oracle's own
decomposition of the benchmark feeders (so that the algorithmic bytes the
bench divides by come from the problem, not from the device's report of it).

Per sweep of the plain form: w (sum_s n_s K_s + N_loc) for the rank-form
operators and bbar, N_loc (4 w + 4) for x_s and lambda read and written and
the int32 global index, 5 w n for x written and gathered with lo, hi, c;
K_s = min(r_s, n_s - r_s) with r_s the rank of A_s. The dense-operator
equivalent puts n_s^2 in place of n_s K_s. The batched form (FP32) counts
the operators once (shared ones for subsystems whose coefficients do not
scale with the load, one per scenario for the others) and per scenario
bbar, x_s and lambda read and written, the gather and the global x.
"""
import types

import numpy as np

import bench
from oracle import model
from synth import make_feeder, scenario_factors


def _shapes(net):
    lp = model.decompose(net)
    ns = np.array([len(s.gidx) for s in lp.subs])
    r = np.array([np.linalg.matrix_rank(s.A) for s in lp.subs])
    return lp, ns, np.minimum(r, ns - r)


def test_plain_sweep_bytes_of_the_8500_bus_feeder():
    lp, ns, K = _shapes(make_feeder("8500", 8500))
    sizes = types.SimpleNamespace(rank_words=int((ns * K).sum()), op_words=int((ns * ns).sum()),
                                  n_local=int(ns.sum()), n=lp.n)
    assert (sizes.rank_words, sizes.n_local, sizes.n) == (1_238_836, 178_428, 114_750)
    assert bench.algorithmic_bytes_per_sweep(sizes, 8) == 22_351_520
    assert bench.dense_equivalent_bytes_per_sweep(sizes, 8) == 38_385_680
    assert bench.algorithmic_bytes_per_sweep(sizes, 4) == 11_532_616  # the FP32-mixed form


def test_batched_sweep_bytes_of_the_2500_bus_feeder_with_256_scenarios():
    net = make_feeder("2500", 2500)
    lp, ns, K = _shapes(net)
    # a subsystem's operator differs per scenario when it holds a load whose
    # voltage coefficient (alpha or beta > 0) scales with the load factor
    vdep = {int(net["load_bus"][l]) for l in range(net["n_load"])
            if np.any(np.asarray(net["load_alpha"][l]) > 0) or np.any(np.asarray(net["load_beta"][l]) > 0)}
    per_scen = np.array([bool((set(s.tag[2]) if s.tag[0] == "line" else {s.tag[1]}) & vdep) for s in lp.subs])
    B = 256
    assert scenario_factors(net, B).shape[0] == B
    bs = types.SimpleNamespace(shared_operator_words=int((ns * K)[~per_scen].sum()),
                               scenario_operator_words=B * int((ns * K)[per_scen].sum()),
                               n_local=int(ns.sum()), n=lp.n, n_scen=B)
    assert int(per_scen.sum()) == 1670 and int((ns * K)[per_scen].sum()) == 176_710
    assert bench.batched_bytes_per_sweep(bs) == 538_763_084
