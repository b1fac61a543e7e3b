"""Converged parity at the benchmarked sizes: the GPU solve to eps_rel = 1e-4
against the converged FP64 oracle stored by tests/golden/make_converged.py
(the oracle alone wrote those files; nothing in them came from the GPU).

FP64: the same stopping sweep (one off only when the test of the earlier
sweep sits on its threshold), and x, x_s, lambda and the objective within
1e-6 relative (rel_err). FP32-mixed: the objective and x within 1e-4 of the
converged oracle and the stopping sweep within 2% of the oracle's (the
precision claim of Section V-B, Table 5: the FP32 GPU run and the FP64 CPU
run take the same iteration count).
"""
import os

import numpy as np
import pytest

from conftest import feeder, rel_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    path = os.path.join(GOLDEN, f"converged_{name}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} missing: run tests/golden/make_converged.py {name}")
    return np.load(path)


def _tie(g, k):
    """The oracle's test of sweep k within 1e-9 of its threshold."""
    rows = list(g["hist_tail_sweeps"])
    if k not in rows:
        return False
    pres, dres, eps_p, eps_d = g["hist_tail"][rows.index(k)]
    return min(abs(pres - eps_p) / eps_p, abs(dres - eps_d) / eps_d) < 1e-9


@pytest.mark.parametrize("name", ["2500", "8500"])
def test_converged_fp64_matches_oracle(gpu, name):
    P = gpu
    g = _golden(name)
    prob = P.ldopf_create(feeder(name))
    st = prob.solve()
    assert st.converged == 1
    T = int(g["t_stop"])
    if st.iterations != T:
        assert abs(st.iterations - T) == 1 and _tie(g, min(st.iterations, T)), (st.iterations, T)
        return
    xs, lam = prob.get_local()
    assert rel_err(prob.get_global(), g["x"]) <= 1e-6
    assert rel_err(xs, g["xs"]) <= 1e-6
    assert rel_err(lam, g["lam"]) <= 1e-6
    f = float(g["objective"])
    assert abs(prob.objective() - f) / max(1.0, abs(f)) <= 1e-6
    H = prob.get_history()
    tail = g["hist_tail_sweeps"]
    np.testing.assert_allclose(H[tail - 1], g["hist_tail"], rtol=1e-6, atol=1e-12)
    thin = g["hist_thin_sweeps"]
    np.testing.assert_allclose(H[thin - 1], g["hist_thin"], rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("name", ["2500", "8500"])
def test_converged_fp32_mixed_against_oracle(gpu, name):
    P = gpu
    g = _golden(name)
    prob = P.ldopf_create(feeder(name), P.ldopf_default_options(precision=P.ldopf.LDOPF_FP32_MIXED))
    st = prob.solve()
    assert st.converged == 1
    T = int(g["t_stop"])
    gap = abs(st.iterations - T) / T
    f = float(g["objective"])
    ef = abs(prob.objective() - f) / max(1.0, abs(f))
    ex = rel_err(prob.get_global(), g["x"])
    print(f"{name} FP32-mixed: T_stop {st.iterations} vs oracle {T} (gap {gap:.2%}); "
          f"objective rel err {ef:.3e}; x rel err {ex:.3e}")
    assert gap <= 0.02
    assert ef <= 1e-4
    assert ex <= 1e-4
