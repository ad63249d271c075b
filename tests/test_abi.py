"""The C-ABI library loads and exports every symbol that include/prop.h declares (no GPU calls),
and host-side validation that needs no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "prop.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(prop_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("prop_create", "prop_forward", "prop_adjoint", "prop_gradient", "prop_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2004_10519_amd import prop
    if not os.path.exists(prop.LIB_PATH):
        pytest.skip("libprop.so not built")
    L = ctypes.CDLL(prop.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert sorted(prop.EXPORTS) == _declared()


def test_cfl_bound_matches_the_checker(orc):
    """prop_cfl_dt is host arithmetic: compare with the checker's bound (no device needed)."""
    from paper_2004_10519_amd import prop
    if not os.path.exists(prop.LIB_PATH):
        pytest.skip("libprop.so not built")
    for so in (4, 8, 12, 16):
        g = prop.Grid((50, 40, 30), (12.5, 10.0, 8.0), space_order=so, dt=1e-3, nt=10)
        og = orc.Grid((50, 40, 30), (12.5, 10.0, 8.0), space_order=so)
        a = prop.cfl_dt(prop.TTI, g, 4725.0, 0.3)
        b = orc.tti_dt_max(og, 4725.0, 0.3)
        assert abs(a - b) / b < 1e-6
        a = prop.cfl_dt(prop.ELASTIC, g, 4725.0)
        b = orc.elastic_dt_max(og, 4725.0)
        assert abs(a - b) / b < 1e-12
    g2 = prop.Grid((101, 1, 101), (10.0, 1.0, 10.0), space_order=4, dt=1e-3, nt=10)
    assert abs(prop.cfl_dt(prop.TTI, g2, 1500.0, 0.1) - 6.272038915e-3) < 1e-11
    bad = prop.Grid((101, 1, 101), (10.0, 1.0, 10.0), space_order=5, dt=1e-3, nt=10)
    assert prop.cfl_dt(prop.TTI, bad, 1500.0, 0.1) < 0


def test_workload_time_steps_are_stable(orc):
    """Every workload's fixed dt is below the checker's stability bound for its model's largest velocity."""
    from paper_2004_10519_amd import configs
    w = configs.tti2d_101()
    og = orc.Grid(w.shape, w.spacing, space_order=w.space_order)
    assert w.dt <= orc.tti_dt_max(og, 1500.0, 0.1) * 0.81
    for w, vmax in ((configs.tti3d_512(), 4725.0), (configs.ttigrad(), 4725.0)):
        og = orc.Grid(w.shape, w.spacing, space_order=w.space_order)
        assert w.dt <= orc.tti_dt_max(og, vmax, 0.3) * 0.81
    w = configs.el3d_400()
    og = orc.Grid(w.shape, w.spacing, space_order=w.space_order)
    assert w.dt <= orc.elastic_dt_max(og, 4725.0) * 0.81
    w = configs.el2d_marine()   # layers up to 4.5 km/s with a +5 % perturbation
    og = orc.Grid(w.shape, w.spacing, space_order=w.space_order)
    assert w.dt <= orc.elastic_dt_max(og, 4725.0) * 0.81
