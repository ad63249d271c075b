"""Batched shots (shot groups on uneven windows of one model) against plain per-shot calls and against
the FP64 checker's per-window results summed in FP64, and the 64^3 gradient against the FP64
checker's stored gradient (full 2000 steps)."""
import os

import numpy as np
import pytest
import torch

from helpers import dev, host, rel_l2

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def prop():
    from paper_2004_10519_amd import prop as P
    P.lib()
    return P


def _setup(prop, nt=120, scheme=None):
    """Three shots on uneven windows of a 100 x 80 x 60 model, space order 8 (default scheme: the
    fused pass), or the given step scheme."""
    from paper_2004_10519_amd import inputs
    shape, h, so, nbl = (100, 80, 60), (10.0, 10.0, 10.0), 8, 6
    mdl = inputs.tti_model(shape, nbl, 31)
    arrs = [inputs.slowness_squared(mdl["vp"]), mdl["eps"], mdl["delta"], mdl["theta"], mdl["phi"]]
    dt = 8e-4
    g = prop.Grid(shape, h, space_order=so, nbl=nbl, dt=dt, nt=nt, v_ref=1500.0)
    mt = [dev(a) for a in arrs]
    p = prop.Propagator(prop.TTI, g, mt)
    p._keep_model = mt
    p._host_model = [np.asarray(a, np.float64) for a in arrs]
    if scheme is not None:
        p.set_option("scheme", scheme)
    wins = [((3, 5, 0), (70, 41, 50)), ((20, 0, 4), (80, 77, 56)), ((0, 30, 0), (37, 50, 60))]
    shots = []
    for k, (o, n) in enumerate(wins):
        cx, cy = h[0] * (o[0] + n[0] / 2 + 0.3), h[1] * (o[1] + n[1] / 2 - 0.2)
        src = np.array([[cx, cy, h[2] * (o[2] + nbl + 3.3)]], np.float32)
        xs = h[0] * (o[0] + np.linspace(nbl, n[0] - 1 - nbl, 9))
        ys = h[1] * (o[1] + np.linspace(nbl, n[1] - 1 - nbl, 7))
        X, Y = np.meshgrid(xs, ys)
        rec = np.stack([X.ravel(), Y.ravel(), np.full(X.size, h[2] * (o[2] + nbl + 2.0))], axis=1).astype(np.float32)
        wav = dev(inputs.ricker(20.0 + 3 * k, dt, nt)[:, None])
        shots.append(prop.Shot(src, wav, rec, win_origin=o, win_shape=n))
    return p, shots


@pytest.mark.parametrize("scheme", [None, 3])
def test_batched_forward_equals_plain(prop, scheme):
    p, shots = _setup(prop, scheme=scheme)
    plain = [host(p.forward(s)).copy() for s in shots]
    outs = p.forward_batched(shots)
    for a, b in zip(outs, plain):
        assert np.array_equal(host(a), b)


@pytest.mark.parametrize("dtype,n_ckpt", [("f16", 5), ("f32", 5), ("f16", 1)])
def test_batched_gradient_equals_plain_sum(prop, dtype, n_ckpt):
    p, shots = _setup(prop, nt=100)
    rng = np.random.default_rng(7)
    res = [dev(rng.standard_normal((100, s.nrec))) for s in shots]
    total = np.zeros(p.grid.arr_shape)
    for s, r in zip(shots, res):
        g = host(p.gradient(s, r, n_ckpt=n_ckpt, ckpt_dtype=dtype)).astype(np.float64)
        (ox, oy, oz), (nx, ny, nz) = s.win_origin, s.win_shape
        total[oz:oz + nz, oy:oy + ny, ox:ox + nx] += g
    gg = torch.zeros(p.grid.arr_shape, dtype=torch.float64, device="cuda")
    p.gradient_batched(shots, res, gg, n_ckpt=n_ckpt, ckpt_dtype=dtype)
    assert np.array_equal(host(gg), total)


def test_batched_groups_split_by_memory_budget(prop):
    """A tiny budget forces one shot per group; results do not change."""
    p, shots = _setup(prop, nt=60)
    rng = np.random.default_rng(8)
    res = [dev(rng.standard_normal((60, s.nrec))) for s in shots]
    g1 = torch.zeros(p.grid.arr_shape, dtype=torch.float64, device="cuda")
    p.gradient_batched(shots, res, g1, n_ckpt=4, ckpt_dtype="f16")
    assert p.get_option("info_groups") == 1
    p.set_option("batch_mb", 1)
    g2 = torch.zeros(p.grid.arr_shape, dtype=torch.float64, device="cuda")
    p.gradient_batched(shots, res, g2, n_ckpt=4, ckpt_dtype="f16")
    assert p.get_option("info_groups") == len(shots)
    assert np.array_equal(host(g1), host(g2))


@pytest.mark.parametrize("scheme", [None, 3])
def test_graphs_and_autotuned_tiles_change_no_bit(prop, scheme):
    """HIP-graph launches and autotuned tiles give the same bits as per-step launches with the fixed
    tiles, for forward, adjoint, gradient and both batched calls; every call is made twice (graphs
    are recorded again per call) with eager work and host synchronisation in between.  For the
    default (fused) scheme and the four-field two-pass scheme (its pass 2 keeps a delay ring in LDS)."""
    p, shots = _setup(prop, nt=100, scheme=scheme)
    rng = np.random.default_rng(9)
    res = [dev(rng.standard_normal((100, s.nrec))) for s in shots]

    def run_all():
        out = [host(p.forward(shots[0])).copy(), host(p.adjoint(shots[1], res[1])).copy(),
               host(p.gradient(shots[2], res[2], n_ckpt=6, ckpt_dtype="f16")).copy()]
        out += [host(a).copy() for a in p.forward_batched(shots)]
        gg = torch.zeros(p.grid.arr_shape, dtype=torch.float64, device="cuda")
        p.gradient_batched(shots, res, gg, n_ckpt=6, ckpt_dtype="bf16")
        out.append(host(gg).copy())
        return out

    ref = run_all()
    assert p.get_option("info_graphs") == 0
    p.set_option("graph", 1)
    p.set_option("autotune", 1)
    for rep in range(2):
        g0 = p.get_option("info_graphs")
        got = run_all()
        assert p.get_option("info_graphs") > g0
        assert p.get_option("info_tile1") in (0, 1) and p.get_option("info_tile2") in (0, 1)
        assert p.get_option("info_zc1") > 0 and p.get_option("info_zc2") > 0
        torch.ones(1000, device="cuda").sum().item()       # eager work between the runs
        for a, b in zip(got, ref):
            assert np.array_equal(a, b), f"repeat {rep}"


def test_graph_runs_span_watchdog_checks(prop):
    """A forward of 1100 steps is recorded as three graphs (watchdog every 500 steps); same bits."""
    from paper_2004_10519_amd import inputs
    shape, h = (48, 40, 36), (10.0, 10.0, 10.0)
    mdl = inputs.tti_model(shape, 4, 33)
    mt = [dev(a) for a in (inputs.slowness_squared(mdl["vp"]), mdl["eps"], mdl["delta"], mdl["theta"], mdl["phi"])]
    g = prop.Grid(shape, h, space_order=4, nbl=4, dt=8e-4, nt=1100, v_ref=1500.0)
    p = prop.Propagator(prop.TTI, g, mt)
    src = np.array([[240.0, 200.0, 80.0]], np.float32)
    rec = np.array([[100.0, 120.0, 30.0], [333.0, 250.0, 60.0]], np.float32)
    shot = prop.Shot(src, dev(inputs.ricker(25.0, 8e-4, 1100)[:, None]), rec)
    a = host(p.forward(shot)).copy()
    p.set_option("graph", 1)
    b = host(p.forward(shot)).copy()
    assert p.get_option("info_graphs") == 3
    assert np.array_equal(a, b)
    with pytest.raises(prop.PropError):
        p.set_option("tile1", 2)
    with pytest.raises(prop.PropError):
        p.set_option("info_groups", 1)


@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f16", 1e-3),
                                       pytest.param("bf16", 1e-3, marks=pytest.mark.xfail(
                                           strict=True, reason="BF16 keeps 8 mantissa bits (relative rounding "
                                                               "2^-9 per checkpoint value): measured 2.0e-3")),
                                       ("bf16", 2.5e-3)], ids=["f32", "f16", "bf16-bar", "bf16-regression"])
def test_gradient_64cubed_vs_checker(prop, dtype, tol):
    """64^3, so 8, 2000 steps, 48 checkpoints: GPU gradient vs the FP64 checker's stored gradient."""
    import importlib.util
    spec = importlib.util.spec_from_file_location("mk", os.path.join(HERE, "golden", "make_ttigrad64.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    gold = np.load(os.path.join(HERE, "golden", "ttigrad64.npz"))["grad"].astype(np.float64)
    w, m0, res = mk.case()
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, v_ref=w.v_ref)
    mt = [dev(m0[k]) for k in ("m", "eps", "delta", "theta", "phi")]
    p = prop.Propagator(prop.TTI, g, mt)
    shot = prop.Shot(w.src_xyz, dev(w.wavelet()), w.rec_xyz)
    gg = host(p.gradient(shot, dev(res), n_ckpt=48, ckpt_dtype=dtype)).astype(np.float64)
    err = rel_l2(gg, gold)
    # also without the singular neighbourhoods of the source and the receiver plane
    mask = np.ones_like(gold, bool)
    mask[w.nbl + 4 - 5:w.nbl + 4 + 6] = False
    err_masked = rel_l2(gg[mask], gold[mask])
    print(f"64^3 gradient rel-L2 vs FP64 ({dtype} checkpoints): {err:.3e} (masked {err_masked:.3e})")
    assert err <= tol


def test_batched_image_equals_plain_sum(prop):
    p, shots = _setup(prop, nt=90)
    rng = np.random.default_rng(17)
    data = [dev(rng.standard_normal((90, s.nrec))) for s in shots]
    total = np.zeros(p.grid.arr_shape)
    for s, r in zip(shots, data):
        im = host(p.image(s, r, n_ckpt=4, ckpt_dtype="f16")).astype(np.float64)
        (ox, oy, oz), (nx, ny, nz) = s.win_origin, s.win_shape
        total[oz:oz + nz, oy:oy + ny, ox:ox + nx] += im
    gi = torch.zeros(p.grid.arr_shape, dtype=torch.float64, device="cuda")
    p.image_batched(shots, data, gi, n_ckpt=4, ckpt_dtype="f16")
    assert np.array_equal(host(gi), total)
    assert np.abs(total).max() > 0


def _oracle_window(orc, p, s, arrs, nbl=6):
    """The checker's grid and model on a shot's window (absolute coordinates: origin at the window's
    first node)."""
    (ox, oy, oz), (nx, ny, nz) = s.win_origin, s.win_shape
    h = p.grid.spacing
    g = orc.Grid((nx, ny, nz), h, origin=(ox * h[0], oy * h[1], oz * h[2]), space_order=p.grid.space_order,
                 nbl=nbl, dt=p.grid.dt, nt=p.grid.nt, vref=p.grid.v_ref)
    sl = (slice(oz, oz + nz), slice(oy, oy + ny), slice(ox, ox + nx))
    return g, orc.TTIModel.from_arrays(g, *(a[sl] for a in arrs)), sl


@pytest.fixture(scope="module")
def batched_checker(prop, orc):
    """The FP64 checker's gradient and image of the three windowed shots (100 steps), each shot on its
    own window, summed over the shots in FP64; with the residuals that drive them."""
    p, shots = _setup(prop, nt=100)
    arrs = p._host_model
    rng = np.random.default_rng(71)
    res = [rng.standard_normal((100, s.nrec)).astype(np.float32) for s in shots]
    go = np.zeros(p.grid.arr_shape)
    io = np.zeros(p.grid.arr_shape)
    for s, r in zip(shots, res):
        g, mod, sl = _oracle_window(orc, p, s, arrs)
        wav = host(s.wavelet).astype(np.float64)
        # the checker takes observed data: d_obs = d - r gives the residual d - d_obs = r
        d, _, _ = orc.tti_forward(g, mod, s.src_xyz, wav, s.rec_xyz)
        _, gw, _ = orc.tti_gradient(g, mod, s.src_xyz, wav, s.rec_xyz, d - r)
        go[sl] += gw
        io[sl] += orc.tti_image(g, mod, s.src_xyz, wav, s.rec_xyz, r)
    p.close()
    return res, go, io


@pytest.mark.parametrize("dtype,n_ckpt,tol", [("f32", 5, 1e-4), ("f16", 5, 1e-3), ("f16", 1, 1e-3)])
def test_batched_gradient_and_image_vs_checker(prop, batched_checker, dtype, n_ckpt, tol):
    """Batched FP64 gradient and image of the three windowed shots against the FP64 checker's per-window
    gradients and images summed in FP64."""
    res, go, io = batched_checker
    p, shots = _setup(prop, nt=100)
    gg = torch.zeros(p.grid.arr_shape, dtype=torch.float64, device="cuda")
    p.gradient_batched(shots, [dev(r) for r in res], gg, n_ckpt=n_ckpt, ckpt_dtype=dtype)
    gi = torch.zeros(p.grid.arr_shape, dtype=torch.float64, device="cuda")
    p.image_batched(shots, [dev(r) for r in res], gi, n_ckpt=n_ckpt, ckpt_dtype=dtype)
    eg, ei = rel_l2(host(gg), go), rel_l2(host(gi), io)
    print(f"batched vs FP64 checker ({dtype}, n_ckpt {n_ckpt}): gradient {eg:.2e}, image {ei:.2e}")
    assert eg <= tol and ei <= tol, (eg, ei)
