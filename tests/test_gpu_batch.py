"""GPU parity of batched load scenarios: every scenario of a batch against an
oracle solve of the network with that scenario's loads, alone and in the mix.

Batched sweeps run in the FP32-mixed form, so the bar is 1e-4 relative
(rel_err) on x, x_s and the objective, always against the oracle after the
same number of sweeps. The stopping sweep itself is not held to the oracle's: near the
stop the dual test compares per-copy changes of about 1e-7 on values near 1,
which is FP32's resolution, so the sweep at which an FP32 run first passes
the test depends on rounding order (a float32 emulation of the same scenario
stops 12% later with one valid operator factorization and at the FP64 sweep
with another). It is held within 2% of the oracle's for all but at most one
scenario per feeder and within 25% for that one, and the returned state must
pass the test.
"""
import numpy as np
import pytest

from conftest import feeder, rel_err

pytestmark = pytest.mark.gpu


def _oracle(net, f, **kw):
    from oracle import admm, model
    from synth import scale_loads
    return admm.solve(model.decompose(scale_loads(net, f)), **kw)


def _factors(net, n, seed):
    from synth import scenario_factors
    return scenario_factors(net, n, base_seed=seed)


def test_batch_classes_and_sizes(gpu):
    P = gpu
    net = feeder("123")
    f = _factors(net, 8, 77)
    b = P.ldopf_batch_create(net, f)
    s = b.sizes()
    assert s.n_scen == 8 and s.n_scen_padded == 64
    assert s.n_mfma_subsystems > 0 and s.n_vector_subsystems > 0
    assert s.n_mfma_subsystems + s.n_vector_subsystems == s.n_sub


@pytest.mark.parametrize("name", ["13", "123"])
def test_batch_converged_matches_oracle(gpu, name):
    P = gpu
    net = feeder(name)
    f = _factors(net, 6, 1000 + len(name))
    b = P.ldopf_batch_create(net, f, P.ldopf_default_options(precision=1, max_iter=40000))
    st = b.solve()
    assert st.n_converged == 6 and st.code == 0
    gaps = []
    for k in range(6):
        ref = _oracle(net, f[k])
        sk = b.scenario(k)
        assert sk.converged
        assert sk.pres <= sk.eps_prim and sk.dres <= sk.eps_dual
        print(f"{name} scenario {k}: batched FP32 T_stop {sk.iterations}, FP64 oracle {ref.iters} "
              f"({(sk.iterations - ref.iters) / ref.iters:+.2%}); x vs converged oracle "
              f"{rel_err(b.get_global(k), ref.x):.2e}")
        gap = abs(sk.iterations - ref.iters) / ref.iters
        gaps.append(gap)
        assert gap <= 0.25, (k, sk.iterations, ref.iters)
        # the returned state against the oracle after the same number of sweeps
        same = _oracle(net, f[k], max_iter=sk.iterations, check=False)
        x = b.get_global(k)
        obj = float(ref.prep.lp.c @ x)
        assert abs(obj - same.objective) / max(1.0, abs(same.objective)) <= 1e-4
        assert rel_err(x, same.x) <= 1e-4
    # the FP64 stopping sweep within 2% (Section V-B, Table 5) for all but at
    # most one scenario per feeder (measured: 11 of these 12 at <= 0.01%,
    # 13-bus scenario 5 at +15%, the FP32-resolution case above)
    assert sum(g > 0.02 for g in gaps) <= 1, gaps


@pytest.mark.parametrize("T", [150, 37])
def test_batch_fixed_sweeps_match_oracle(gpu, T):
    """After T sweeps (an even and an odd count: x of sweep k is kept in the
    half k % 2 of a two-part buffer), every scenario against the oracle."""
    P = gpu
    net = feeder("123")
    f = _factors(net, 5, 31)
    b = P.ldopf_batch_create(net, f, P.ldopf_default_options(precision=1, max_iter=T, check_termination=0))
    st = b.solve()
    assert st.sweeps == T
    for k in range(5):
        ref = _oracle(net, f[k], max_iter=T, check=False)
        xs, lam = b.get_local(k)
        assert b.scenario(k).iterations == T
        assert rel_err(b.get_global(k), ref.x) <= 1e-4
        assert rel_err(xs, ref.xs) <= 1e-4


def test_batch_alone_equals_in_the_mix(gpu):
    P = gpu
    net = feeder("123")
    f = _factors(net, 9, 5)
    opts = P.ldopf_default_options(precision=1, rows_per_part=128)
    mix = P.ldopf_batch_create(net, f, opts)
    mix.solve()
    alone = P.ldopf_batch_create(net, f[4:5], opts)
    alone.solve()
    assert mix.scenario(4).iterations == alone.scenario(0).iterations
    np.testing.assert_array_equal(mix.get_global(4), alone.get_global(0))
    xa, la = alone.get_local(0)
    xm, lm = mix.get_local(4)
    np.testing.assert_array_equal(xa, xm)
    np.testing.assert_array_equal(la, lm)


def test_batch_ragged_tile_count(gpu):
    """130 scenarios: three 64-scenario tiles (a count that is not a
    multiple of the four tiles a global-update block takes) and a padded last
    tile; scenarios from every tile against the oracle after the same sweeps,
    and the last scenario equal bit for bit to a batch of its own."""
    P = gpu
    net = feeder("123")
    f = _factors(net, 130, 77)
    T = 60
    opts = P.ldopf_default_options(precision=1, max_iter=T, check_termination=0)
    b = P.ldopf_batch_create(net, f, opts)
    s = b.sizes()
    assert s.n_scen == 130 and s.n_scen_padded == 192
    assert b.solve().sweeps == T
    for k in (0, 63, 64, 127, 128, 129):
        ref = _oracle(net, f[k], max_iter=T, check=False)
        xs, lam = b.get_local(k)
        assert b.scenario(k).iterations == T
        assert rel_err(b.get_global(k), ref.x) <= 1e-4
        assert rel_err(xs, ref.xs) <= 1e-4
    alone = P.ldopf_batch_create(net, f[129:130], opts)
    alone.solve()
    np.testing.assert_array_equal(alone.get_global(0), b.get_global(129))


def test_batch_8500bus_feeder(gpu):
    """The largest feeder as a batch: 8500 buses x 128 scenarios (per-bus
    factors as in the benchmark), 20 fixed sweeps; the lightest and heaviest
    scenarios and one between against the oracle."""
    P = gpu
    net = feeder("8500")
    from synth import scenario_factors
    f = scenario_factors(net, 128, base_seed=8500 * 1000)
    T = 20
    b = P.ldopf_batch_create(net, f, P.ldopf_default_options(precision=1, max_iter=T, check_termination=0))
    assert b.solve().sweeps == T
    mean = f.mean(axis=1)
    for k in sorted({int(np.argmin(mean)), int(np.argmax(mean)), 77}):
        ref = _oracle(net, f[k], max_iter=T, check=False)
        xs, lam = b.get_local(k)
        assert rel_err(b.get_global(k), ref.x) <= 1e-4, k
        assert rel_err(xs, ref.xs) <= 1e-4, k


def test_batch_tuner_keeps_results(gpu, tmp_path):
    P = gpu
    net = feeder("123")
    f = _factors(net, 4, 9)
    opts = P.ldopf_default_options(precision=1, max_iter=100, check_termination=0)
    a = P.ldopf_batch_create(net, f, opts)
    a.solve()
    b = P.ldopf_batch_create(net, f, opts)
    cache = str(tmp_path / "tune.txt")
    r, w = b.tune(cache)
    assert r in (32, 64, 128, 256) and 1 <= w <= 512
    assert open(cache).read().strip()
    b.solve()
    for k in range(4):
        np.testing.assert_array_equal(a.get_global(k), b.get_global(k))


def test_batch_full_size_sampled_scenarios(gpu):
    """The batched workload bench.py times (2500-bus feeder x 256 scenarios,
    the bench's scenario factors, tiling chosen by the tuner) for 100 fixed
    sweeps; 32 scenarios against oracle solves of their scaled networks: the
    two with the lowest and highest mean load factor, and 30 spread evenly
    over the batch (the oracle takes about a second per scenario)."""
    P = gpu
    net = feeder("2500")
    from synth import scenario_factors
    f = scenario_factors(net, 256)
    T = 100
    b = P.ldopf_batch_create(net, f)
    b.tune(None)
    b.set_options(P.ldopf_default_options(precision=1, max_iter=T, check_termination=0))
    b.reset()
    st = b.solve()
    assert st.sweeps == T
    mean = f.mean(axis=1)
    picks = sorted({int(np.argmin(mean)), int(np.argmax(mean))} | {int(k) for k in np.linspace(0, 255, 30).round()})
    assert len(picks) >= 30
    for k in picks:
        ref = _oracle(net, f[k], max_iter=T, check=False)
        xs, lam = b.get_local(k)
        assert b.scenario(k).iterations == T
        assert rel_err(b.get_global(k), ref.x) <= 1e-4, k
        assert rel_err(xs, ref.xs) <= 1e-4, k
