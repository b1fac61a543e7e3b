"""Several feeders in one persistent launch (ldopf_solve_many): every problem
runs Algorithm 1 on its own inside the shared launch, so each result must
equal the problem's own ldopf_solve bit for bit (the same kernels on the same
plan); ldopf_solve itself is held to the oracle by the parity tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _nets():
    from synth import make_feeder
    return ([make_feeder("13", 53000 + i) for i in range(5)] + [make_feeder("123", 53100 + i) for i in range(3)]
            + [make_feeder("2500", 2500)])


def _same(a, sa, b, sb):
    assert sa.code == sb.code and sa.iterations == sb.iterations and sa.converged == sb.converged
    for f in ("pres", "dres", "eps_prim", "eps_dual"):
        assert getattr(sa, f) == getattr(sb, f), f
    np.testing.assert_array_equal(a.get_global(), b.get_global())
    xa, la = a.get_local()
    xb, lb = b.get_local()
    np.testing.assert_array_equal(xa, xb)
    np.testing.assert_array_equal(la, lb)
    np.testing.assert_array_equal(a.get_history(), b.get_history())


@pytest.mark.parametrize("kw", [dict(), dict(precision=1), dict(residual_form=1),
                                dict(max_iter=700, check_termination=0)])
def test_many_equals_each_alone(gpu, kw):
    P = gpu
    nets = _nets()
    together = [P.ldopf_create(n, P.ldopf_default_options(**kw)) for n in nets]
    sts = P.ldopf_solve_many(together)
    assert len(sts) == len(nets)
    for net, h, st in zip(nets, together, sts):
        alone = P.ldopf_create(net, P.ldopf_default_options(**kw))
        _same(h, st, alone, alone.solve())
    # and again from where they stopped (a second shared launch on the same handles)
    if "max_iter" in kw:
        sts2 = P.ldopf_solve_many(together[::-1])
        assert all(s.iterations == 700 for s in sts2)


def test_many_refuses_what_it_cannot_run(gpu):
    P = gpu
    from conftest import feeder
    a = P.ldopf_create(feeder("13"))
    b = P.ldopf_create(feeder("13"), P.ldopf_default_options(precision=1))
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_solve_many([a, b])
    assert e.value.code == -1
    with pytest.raises(P.LdopfError) as e:
        P.ldopf_solve_many([a, a])
    assert e.value.code == -1
    big = P.ldopf_create(feeder("8500"))
    mid = P.ldopf_create(feeder("2500"))
    if big.sizes().n_parts + mid.sizes().n_parts > 256:
        with pytest.raises(P.LdopfError) as e:
            P.ldopf_solve_many([big, mid])
        assert e.value.code == -9
