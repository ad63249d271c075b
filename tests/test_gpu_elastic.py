"""GPU parity of the elastic path against the FP64 checker (forward, adjoint, dot test)."""
import numpy as np
import pytest

from helpers import dev, el_case, host, make_el, oracle_el, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prop():
    from paper_2004_10519_amd import prop as P
    P.lib()
    return P


@pytest.mark.parametrize("so,shape", [(8, (70, 37, 29)), (4, (66, 20, 40)), (12, (40, 22, 30))])
def test_elastic_forward_parity(prop, orc, so, shape):
    case = el_case(shape, so, 5, 80)
    p, shot = make_el(case, prop)
    d = host(p.forward(shot))
    fields = [host(p.read_state(i)) for i in range(9)]
    g, mod = oracle_el(case, orc)
    do, fo = orc.elastic_forward(g, mod, case["src"], case["wav"], case["rec"], case["kind"])
    assert rel_l2(d, do) <= 1e-4, rel_l2(d, do)
    for a, b in zip(fields, fo):
        assert rel_l2(a, b) <= 1e-4


@pytest.mark.parametrize("so,shape", [(8, (70, 37, 29)), (4, (66, 20, 40))])
def test_elastic_adjoint_parity(prop, orc, so, shape):
    case = el_case(shape, so, 5, 60)
    p, shot = make_el(case, prop)
    rec = np.random.default_rng(2).standard_normal((case["nt"], len(case["rec"]))).astype(np.float32)
    s = host(p.adjoint(shot, dev(rec)))
    fields = [host(p.read_state(i)) for i in range(9)]
    g, mod = oracle_el(case, orc)
    so_, fo = orc.elastic_adjoint(g, mod, case["src"], case["rec"], rec, case["kind"])
    assert rel_l2(s, so_) <= 1e-4, rel_l2(s, so_)
    for a, b in zip(fields, fo):
        assert rel_l2(a, b) <= 1e-4


def test_elastic_gpu_dot_test(prop):
    case = el_case((70, 37, 29), 8, 5, 100)
    p, shot = make_el(case, prop)
    rng = np.random.default_rng(12)
    x = dev(rng.standard_normal(case["wav"].shape))
    shot.wavelet = x
    Fx = p.forward(shot)
    # y = a component along Fx plus independent noise of the same norm: white-noise y alone makes
    # <Fx, y> a near-cancelling sum that amplifies FP32 rounding
    xi = dev(rng.standard_normal((case["nt"], len(case["rec"]))))
    y = (Fx * (xi.norm() / Fx.norm()) + xi).contiguous()
    FTy = p.adjoint(shot, y)
    a, b = prop.dot_f64(Fx, y), prop.dot_f64(x, FTy)
    assert abs(a - b) / abs(a) < 1e-5, (a, b)
