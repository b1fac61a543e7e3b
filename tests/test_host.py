"""Host-side checks that need no GPU: the C ABI library loads and exports every
declared call, and its C++ assembly/decomposition equals the oracle's
independent Python assembly."""
import ctypes
import os
import re

import numpy as np
import pytest

from conftest import feeder
from synth import perturb_extras, two_bus

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ldopf.h")


def _declared():
    text = open(HEADER).read()
    return re.findall(r"LDOPF_API\s+[\w\s\*]+?\b(ldopf_\w+)\s*\(", text)


def test_header_declares_the_calls():
    names = _declared()
    assert "ldopf_create" in names and "ldopf_solve" in names
    assert len(names) == len(set(names))


def test_library_exports_every_declared_call():
    from paper_2310_09410_amd import _native
    lib = ctypes.CDLL(_native.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    # the binding declares exactly the header's calls
    assert set(_native.SIGNATURES) == set(_declared())


def _compare(net):
    from oracle import model
    import paper_2310_09410_amd as P
    d = P.ldopf_describe_network(net)
    lp = model.decompose(net)
    assert d["n"] == lp.n and d["S"] == len(lp.subs)
    np.testing.assert_array_equal(d["c"], lp.c)
    np.testing.assert_array_equal(d["lo"], lp.lo)
    np.testing.assert_array_equal(d["hi"], lp.hi)
    np.testing.assert_array_equal(d["x_init"], lp.x_init)
    ao = bo = go = 0
    for s, sub in enumerate(lp.subs):
        n, m = int(d["n_s"][s]), int(d["m_s"][s])
        assert (m, n) == sub.A.shape
        np.testing.assert_array_equal(d["gidx"][go:go + n], sub.gidx)
        np.testing.assert_allclose(d["A"][ao:ao + n * m].reshape(m, n), sub.A, rtol=0, atol=1e-15)
        np.testing.assert_allclose(d["b"][bo:bo + m], sub.b, rtol=0, atol=1e-15)
        ao += n * m
        bo += m
        go += n


@pytest.mark.parametrize("name", ["13", "123", "2500"])
def test_host_assembly_equals_oracle(name):
    _compare(feeder(name))


@pytest.mark.parametrize("name", ["13", "123"])
def test_host_assembly_equals_oracle_with_shunts_taps_delta(name):
    net = perturb_extras(feeder(name), 7)
    assert (net["load_conn"] == 1).any()
    _compare(net)


def test_host_assembly_two_bus():
    _compare(two_bus())


def _err(net):
    import paper_2310_09410_amd as P
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_describe_network(net)
    return e.value.code


def test_validation_errors():
    base = two_bus()
    bad = dict(base, line_to=np.array([5], np.int32))
    assert _err(bad) == -2  # index out of range
    bad = dict(base, line_phases=np.array([3], np.uint8))
    assert _err(bad) == -2  # line phase not carried by its buses
    bad = dict(base, load_conn=np.array([1], np.uint8))
    assert _err(bad) == -2  # delta load on one phase
    wlo = base["bus_wlo"].copy()
    wlo[1, 0] = 2.0
    assert _err(dict(base, bus_wlo=wlo)) == -3  # lo > hi
    a = base["load_a"].copy()
    a[0, 0] = np.nan
    assert _err(dict(base, load_a=a)) == -2  # NaN data
    assert _err(dict(base, n_bus=0)) == -1


def test_nullable_fields_take_defaults():
    import paper_2310_09410_amd as P
    net = dict(feeder("13"))
    full = P.ldopf_describe_network(net)
    for k in ("bus_gsh", "bus_bsh", "line_gs_from", "line_bs_from", "line_gs_to", "line_bs_to", "line_tau",
              "line_plo", "line_phi", "line_qlo", "line_qhi", "gen_cost_q"):
        net.pop(k)
    part = P.ldopf_describe_network(net)
    for k in ("c", "lo", "hi", "A", "b", "gidx"):
        np.testing.assert_array_equal(full[k], part[k])


def test_default_options():
    import paper_2310_09410_amd as P
    o = P.ldopf_default_options()
    assert o.rho == 100.0 and o.eps_rel == 1e-4 and o.max_iter == 1000000
    assert o.precision == 0 and o.residual_form == 0 and o.check_termination == 1
    assert o.sweep_path == P.ldopf.LDOPF_PATH_AUTO


@pytest.mark.parametrize("field,value", [
    ("block_threads", 64),     # one wave: no room for the test wave beside a row wave
    ("block_threads", 96),     # not a multiple of 64
    ("block_threads", 1088),   # above 1024
    ("rows_per_part", -1),
    ("rho", 0.0),
    ("eps_rel", -1.0),
    ("max_iter", -1),
    ("check_termination", 2),
    ("sweep_path", 3),
    ("reserved", 1),
])
def test_options_out_of_range_are_rejected_before_any_device_work(field, value):
    """Option bounds (include/ldopf.h, ldopf_options) are checked on the host
    before the device is touched, so they fail the same way with or without
    a GPU."""
    import paper_2310_09410_amd as P
    from paper_2310_09410_amd.ldopf import LdopfError
    o = P.ldopf_default_options()
    setattr(o, field, value)
    with pytest.raises(LdopfError) as e:
        P.ldopf_create(dict(feeder("13")), o)
    assert e.value.code == -1


def test_create_lp_validation_before_any_device_work():
    """ldopf_create_lp checks the B_s invariants of Section III-A (strictly
    ascending, hence distinct, global indices in a subsystem; every global
    variable with at least one copy, since closed_1 divides by N_i) and the
    bounds on the host, before touching the device."""
    import paper_2310_09410_amd as P
    n_s = np.array([2, 2], np.int32)
    m_s = np.array([1, 0], np.int32)
    A = np.array([1.0, 1.0])
    b = np.array([1.0])
    c, lo, hi = np.zeros(3), np.full(3, -1.0), np.ones(3)

    def code(**kw):
        args = dict(n=3, c=c, lo=lo, hi=hi, x_init=None, n_s=n_s, m_s=m_s, A=A, b=b,
                    gidx=np.array([0, 1, 1, 2], np.int64))
        args.update(kw)
        with pytest.raises(P.LdopfError) as e:
            P.ldopf_create_lp(args["n"], args["c"], args["lo"], args["hi"], args["x_init"], args["n_s"], args["m_s"],
                              args["A"], args["b"], args["gidx"])
        return e.value.code

    assert code(gidx=np.array([0, 0, 1, 2], np.int64)) == -1      # duplicate index inside a subsystem
    assert code(gidx=np.array([1, 0, 1, 2], np.int64)) == -1      # not ascending
    assert code(n=4, c=np.zeros(4), lo=np.full(4, -1.0), hi=np.ones(4)) == -1  # variable 3 has no copy (N_i = 0)
    assert code(gidx=np.array([0, 1, 1, 3], np.int64)) == -1      # index out of range
    assert code(lo=np.array([-1.0, 2.0, -1.0])) == -3             # lo > hi
    assert code(b=np.array([np.nan])) == -1                       # non-finite data
    assert code(x_init=np.array([0.0, np.inf, 0.0])) == -1


@pytest.mark.parametrize("field,value", [
    ("rho_update", 2), ("rho_period", 3), ("rho_max_changes", 1025), ("rho_mu", 1.0), ("rho_tau", 0.5),
    ("residual_form", 2),
])
def test_rho_and_residual_options_are_checked(field, value):
    import paper_2310_09410_amd as P
    o = P.ldopf_default_options(rho_update=1)
    setattr(o, field, value)
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_create(dict(feeder("13")), o)
    assert e.value.code == -1


@pytest.mark.parametrize("field", ["residual_form", "rho_update"])
def test_batch_refuses_what_it_does_not_run(field):
    import paper_2310_09410_amd as P
    net = feeder("13")
    o = P.ldopf_default_options(precision=1)
    setattr(o, field, 1)
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_batch_create(net, np.ones((2, int(net["n_load"]))), o)
    assert e.value.code == -9


def test_batch_argument_checks_before_any_device_work():
    """ldopf_batch_create checks the scenario count, the form and the load
    factors on the host before touching the device."""
    import paper_2310_09410_amd as P
    net = feeder("13")
    nl = int(net["n_load"])
    o32 = P.ldopf_default_options(precision=1)
    for n_scen in (0, 1025):
        with pytest.raises(P.LdopfError) as e:
            P.ldopf_batch_create(net, np.ones((n_scen, nl)), o32)
        assert e.value.code == -1
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_batch_create(net, np.ones((2, nl)), P.ldopf_default_options(precision=0))
    assert e.value.code == -9
    bad = np.ones((2, nl))
    bad[1, 0] = np.nan
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_batch_create(net, bad, o32)
    assert e.value.code == -1


@pytest.mark.parametrize("name", ["13", "123", "2500", "8500"])
def test_request_estimate_plans_on_the_host(name):
    """The serving admission's estimate assembles, decomposes and plans the
    sweep's workgroups on the host (full row rank assumed), with no GPU."""
    import paper_2310_09410_amd as P
    b, w = P.ldopf_request_estimate(feeder(name))
    assert b > 0 and 1 <= w <= 256
