"""The seeded feeder generator: determinism and the shape rules of the workloads."""
import numpy as np
import pytest

from synth import SPECS, make_feeder, scenario_factors

PH = (1, 2, 4)


def test_same_seed_same_bytes():
    a = make_feeder("123", 123)
    b = make_feeder("123", 123)
    c = make_feeder("123", 124)
    for k, v in a.items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, b[k]), k
    assert not np.array_equal(a["load_a"], c["load_a"])


@pytest.mark.parametrize("name", ["13", "123", "2500", "8500"])
def test_radial_tree_and_phase_rules(name):
    spec = SPECS[name]
    net = make_feeder(name, 1000 + spec.n_bus)
    nb, nl = net["n_bus"], net["n_line"]
    assert nb == spec.n_bus and nl == nb - 1
    assert np.all(net["line_from"] < net["line_to"])  # parents come first: a tree rooted at 0
    assert np.array_equal(net["line_to"], np.arange(1, nb))
    for e in range(nl):
        i, j = net["line_from"][e], net["line_to"][e]
        assert net["line_phases"][e] & ~net["bus_phases"][i] == 0  # subset of the parent's phases
        assert net["bus_phases"][j] == net["line_phases"][e]
    counts = np.bincount([bin(int(p)).count("1") for p in net["line_phases"]], minlength=4)
    # the target mix before clamping to the parent's phase count
    assert counts[3] <= round(spec.frac3 * nl)
    assert counts[1] >= nl - round(spec.frac3 * nl) - round(spec.frac2 * nl)
    # per-phase loads on every non-root bus, Q = 0.3 P
    assert net["n_load"] == nb - 1
    np.testing.assert_allclose(net["load_b"], 0.3 * net["load_a"])
    assert np.all(net["bus_wlo"][net["bus_whi"] > 0] == 0.9025)
    assert net["n_gen"] == 1 + spec.n_pv


def test_scenarios_are_per_bus_factors():
    net = make_feeder("13", 13)
    f = scenario_factors(net, 4, base_seed=99)
    assert f.shape == (4, net["n_load"])
    assert f.min() >= 0.7 and f.max() <= 1.3
    assert np.array_equal(f, scenario_factors(net, 4, base_seed=99))
