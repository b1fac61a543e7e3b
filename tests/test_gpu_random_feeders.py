"""GPU parity on randomly drawn feeders: sizes, phase mixes, load kinds and
seeds other than the benchmark's, on both sweep paths and in both
precisions, against the FP64 oracle after the same number of sweeps (FP64
1e-6 on x, x_s and lambda; FP32-mixed 1e-4). Each feeder adds delta loads,
shunts and taps (the full feature set of Section II-A) to a random half of
the cases."""
import dataclasses

import numpy as np
import pytest

from conftest import rel_err

pytestmark = pytest.mark.gpu

CASES = list(range(8))


def _case(i):
    from synth import SPECS, make_feeder, perturb_extras
    rng = np.random.default_rng(7100 + i)
    base = SPECS["123"] if i % 2 else SPECS["2500"]
    spec = dataclasses.replace(base, n_bus=int(rng.integers(20, 400)), frac3=float(rng.uniform(0.1, 0.8)),
                               frac2=float(rng.uniform(0.0, 0.2)), n_pv=int(rng.integers(0, 3)))
    net = make_feeder(spec, 7100 + i)
    if i % 4 >= 2:
        net = perturb_extras(net, 7100 + i)
    return net


@pytest.mark.parametrize("i", CASES)
def test_random_feeder_both_paths(gpu, i):
    from oracle import admm, model
    P = gpu
    L = P.ldopf
    net = _case(i)
    T = 80
    ref = admm.solve(admm.prepare(model.decompose(net)), max_iter=T, check=False)
    for path in (L.LDOPF_PATH_PERSISTENT, L.LDOPF_PATH_STREAMED):
        prob = P.ldopf_create(net, P.ldopf_default_options(max_iter=T, check_termination=0, sweep_path=path))
        assert prob.solve().iterations == T
        xs, lam = prob.get_local()
        assert rel_err(prob.get_global(), ref.x) <= 1e-6, path
        assert rel_err(xs, ref.xs) <= 1e-6, path
        assert rel_err(lam, ref.lam) <= 1e-6, path
    p32 = P.ldopf_create(net, P.ldopf_default_options(max_iter=T, check_termination=0,
                                                      precision=L.LDOPF_FP32_MIXED))
    p32.solve()
    xs, _ = p32.get_local()
    assert rel_err(p32.get_global(), ref.x) <= 1e-4
    assert rel_err(xs, ref.xs) <= 1e-4
