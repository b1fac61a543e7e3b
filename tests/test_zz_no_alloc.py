"""The allocation-free solve (ldopf_solve_noalloc) against ldopf_solve.

Both run the same sweep kernel on the same handle state; only the device
memory of the sweep's synchronisation words differs (the library's static
array instead of the handle's buffers), so results must agree bit for bit.
Two calls in a row, the second on a smaller feeder, so that the second reuses
the array the first left behind.
"""
import numpy as np
import pytest

from conftest import feeder

pytestmark = pytest.mark.gpu


def _same(a, sa, b, sb):
    assert sa.code == sb.code and sa.iterations == sb.iterations and sa.converged == sb.converged
    assert sa.sweeps_computed == sb.sweeps_computed
    for f in ("pres", "dres", "eps_prim", "eps_dual"):
        assert getattr(sa, f) == getattr(sb, f), f
    np.testing.assert_array_equal(a.get_global(), b.get_global())
    xa, la = a.get_local()
    xb, lb = b.get_local()
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(la, lb)


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_solve_twice_second_smaller(gpu, precision):
    P = gpu
    for name in ("123", "13"):
        opts = P.ldopf_default_options(precision=precision)
        ref = P.ldopf_create(feeder(name), opts)
        sr = ref.solve()
        assert sr.converged
        na = P.ldopf_create(feeder(name), opts)
        assert 0 < na.sizes().sync_bytes <= 4 << 20
        sn = na.solve_noalloc()
        _same(na, sn, ref, sr)
        # no history buffer on a handle that never ran ldopf_solve
        assert na.get_history().shape == (0, 4)


def test_noalloc_fixed_sweeps_and_history(gpu):
    """After one ldopf_solve (which allocates the history buffer) the
    allocation-free solve records the same history."""
    P = gpu
    T = 120
    opts = P.ldopf_default_options(max_iter=T, check_termination=0)
    ref = P.ldopf_create(feeder("123"), opts)
    sr = ref.solve()
    na = P.ldopf_create(feeder("123"), opts)
    na.solve()
    na.reset()
    sn = na.solve_noalloc()
    _same(na, sn, ref, sr)
    np.testing.assert_array_equal(na.get_history(), ref.get_history())
    # a smaller one right after, on the same array
    small = P.ldopf_create(feeder("13"), opts)
    ref_small = P.ldopf_create(feeder("13"), opts)
    _same(small, small.solve_noalloc(), ref_small, ref_small.solve())


def test_noalloc_rejects_more_than_the_static_array(gpu):
    """A consensus LP whose few global variables are shared by every one of
    256 workgroups needs 256^2 exchange words per variable; beyond the
    array's 4 MiB the call fails before running anything."""
    P = gpu
    nv, S = 6, 256
    gidx = np.tile(np.arange(nv, dtype=np.int64), S)
    n_s = np.full(S, nv, np.int32)
    m_s = np.ones(S, np.int32)
    A = np.tile(np.ones(nv), S)          # one row per subsystem: sum of its copies = 1
    b = np.ones(S)
    opts = P.ldopf_default_options(max_iter=10, check_termination=0, rows_per_part=1)
    prob = P.ldopf_create_lp(nv, np.zeros(nv), np.full(nv, -1.0), np.full(nv, 1.0), None, n_s, m_s, A, b, gidx, opts)
    s = prob.sizes()
    if s.sync_bytes <= 4 << 20:
        pytest.skip(f"plan has {s.n_parts} workgroups, {s.sync_bytes} bytes: fits the array")
    with pytest.raises(P.LdopfError) as e:
        prob.solve_noalloc()
    assert e.value.code == -5
    # the ordinary solve still runs it
    assert prob.solve().iterations == 10
