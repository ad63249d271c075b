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


def _to_2d(case):
    case["src"] = np.ascontiguousarray(case["src"][:, [0, 2]])
    case["rec"] = np.ascontiguousarray(case["rec"][:, [0, 2]])
    return case


@pytest.mark.parametrize("so", [4, 8])
def test_elastic_forward_parity_2d(prop, orc, so):
    """2D (x, z): ny = 1; vy, txy and tyz stay exactly zero, tyy follows the normal strains."""
    case = _to_2d(el_case((90, 1, 61), so, 5, 80))
    p, shot = make_el(case, prop)
    d = host(p.forward(shot))
    fields = [host(p.read_state(i)) for i in range(9)]
    g, mod = oracle_el(case, orc)
    do, fo = orc.elastic_forward(g, mod, case["src"], case["wav"], case["rec"], case["kind"])
    assert rel_l2(d, do) <= 1e-4, rel_l2(d, do)
    for i, (a, b) in enumerate(zip(fields, fo)):
        if np.abs(b).max() > 0:
            assert rel_l2(a, b) <= 1e-4, (i, rel_l2(a, b))
        else:
            assert not a.any(), i


@pytest.mark.parametrize("so", [4, 8])
def test_elastic_adjoint_parity_2d(prop, orc, so):
    """2D adjoint: source traces and the final adjoint fields against the checker; v~_y, tau~_xy,
    tau~_yz and tau~_yy (no receiver drives it in 2D, where the stress tensor is 2 x 2) stay exactly
    zero, as the 2D passes never store them."""
    case = _to_2d(el_case((90, 1, 61), so, 5, 60))
    p, shot = make_el(case, prop)
    rec = np.random.default_rng(4).standard_normal((case["nt"], len(case["rec"]))).astype(np.float32)
    s = host(p.adjoint(shot, dev(rec)))
    fields = [host(p.read_state(i)) for i in range(9)]
    g, mod = oracle_el(case, orc)
    so_, fo = orc.elastic_adjoint(g, mod, case["src"], case["rec"], rec, case["kind"])
    assert rel_l2(s, so_) <= 1e-4, rel_l2(s, so_)
    for i, (a, b) in enumerate(zip(fields, fo)):
        if np.abs(b).max() > 0:
            assert rel_l2(a, b) <= 1e-4, (i, rel_l2(a, b))
        else:
            assert not a.any(), i
    assert not any(fields[i].any() for i in (1, 4, 6, 8))


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


@pytest.mark.parametrize("so,shape", [(8, (70, 37, 29)), (4, (66, 1, 40))])
def test_elastic_gradient_parity(prop, orc, so, shape):
    """Gradient with respect to (vp, vs, rho) against the checker's adjoint-state gradient (residual
    from a perturbed model), with FP32 checkpoints every 12 steps."""
    from paper_2004_10519_amd import inputs
    case = el_case(shape, so, 5, 60)
    if shape[1] == 1:
        case = _to_2d(case)
    p, shot = make_el(case, prop)
    g, mod = oracle_el(case, orc)
    m = case["model"]
    pert = 1 + 0.03 * inputs.random_unit_field(g.arr_shape, 5, 2.0)
    dobs, _ = orc.elastic_forward(g, orc.ElasticModel.from_velocities(g, m["vp"] * pert, m["vs"] * pert, m["rho"]),
                                  case["src"], case["wav"], case["rec"], case["kind"])
    d = host(p.forward(shot)).astype(np.float64)
    res = (d - dobs).astype(np.float32)
    gg = host(p.gradient(shot, dev(res), n_ckpt=5, ckpt_dtype="f32"))
    _, go, _ = orc.elastic_gradient(g, m["vp"], m["vs"], m["rho"], case["src"], case["wav"], case["rec"],
                                    d - res.astype(np.float64), case["kind"])
    for name, a, b in zip(("vp", "vs", "rho"), gg, go):
        err = rel_l2(a, b)
        print(f"elastic gradient {name}: rel-L2 {err:.3e}")
        assert err <= 1e-3, (name, err)
    # checkpoints are exact FP32 copies: any segmentation gives the same bits
    g1 = host(p.gradient(shot, dev(res), n_ckpt=1, ckpt_dtype="f32"))
    assert np.array_equal(g1, gg)


# ---- free surface on the top face (vacuum rows above row nbl, no absorbing layer on that face)
FS_CASES = [((70, 37, 29), 8), ((90, 1, 61), 8), ((66, 20, 40), 4)]


def _fluid_top(case):
    """A fluid on the surface row and the R rows below it, which an image free surface needs."""
    case["model"]["vs"][:case["nbl"] + case["so"] // 2 + 1] = 0.0
    return case


def _fs_case(shape, so, nt, mode=True):
    case = el_case(shape, so, 5 if mode is True else max(5, so - 2), nt, free_surface=mode)
    if mode == "image":
        case = _fluid_top(case)
    if shape[1] == 1:
        case = _to_2d(case)
    # source below the surface, near it (the ghost and the surface waves matter)
    case["src"][0, -1] = case["h"][2] * (case["nbl"] + 3.4)
    return case


@pytest.mark.parametrize("mode", [True, "image"])
@pytest.mark.parametrize("shape,so", FS_CASES)
def test_free_surface_forward_parity(prop, orc, shape, so, mode):
    case = _fs_case(shape, so, 80, mode)
    p, shot = make_el(case, prop)
    d = host(p.forward(shot))
    fields = [host(p.read_state(i)) for i in range(9)]
    g, mod = oracle_el(case, orc)
    do, fo = orc.elastic_forward(g, mod, case["src"], case["wav"], case["rec"], case["kind"])
    assert rel_l2(d, do) <= 1e-4, rel_l2(d, do)
    for i, (a, b) in enumerate(zip(fields, fo)):
        if np.abs(b).max() > 0:
            assert rel_l2(a, b) <= 1e-4, (i, rel_l2(a, b))
        else:
            assert not a.any(), i
    nb = case["nbl"]
    if mode is True:
        for c in (3, 4, 5):   # normal stresses vanish in the vacuum rows
            assert not fields[c][:nb].any()
    else:                     # odd images of the tractions above the surface row, tau_zz = 0 on it
        assert not fields[3][:nb + 1].any() and not fields[4][:nb + 1].any() and not fields[5][nb].any()
        for k in range(1, nb + 1):
            assert np.array_equal(fields[5][nb - k], -fields[5][nb + k])
            assert np.array_equal(fields[7][nb - k], -fields[7][nb + k - 1])
            assert np.array_equal(fields[8][nb - k], -fields[8][nb + k - 1])


@pytest.mark.parametrize("mode", [True, "image"])
@pytest.mark.parametrize("shape,so", FS_CASES[:2])
def test_free_surface_adjoint_parity_and_dot(prop, orc, shape, so, mode):
    case = _fs_case(shape, so, 60, mode)
    p, shot = make_el(case, prop)
    rng = np.random.default_rng(3)
    rec = rng.standard_normal((case["nt"], len(case["rec"]))).astype(np.float32)
    s = host(p.adjoint(shot, dev(rec)))
    g, mod = oracle_el(case, orc)
    so_, _ = orc.elastic_adjoint(g, mod, case["src"], case["rec"], rec, case["kind"])
    assert rel_l2(s, so_) <= 1e-4, rel_l2(s, so_)
    x = dev(rng.standard_normal(case["wav"].shape))
    shot.wavelet = x
    Fx = p.forward(shot)
    xi = dev(rng.standard_normal((case["nt"], len(case["rec"]))))
    y = (Fx * (xi.norm() / Fx.norm()) + xi).contiguous()
    FTy = p.adjoint(shot, y)
    a, b = prop.dot_f64(Fx, y), prop.dot_f64(x, FTy)
    assert abs(a - b) / abs(a) < 1e-5, (a, b)


@pytest.mark.parametrize("mode", [True, "image"])
@pytest.mark.parametrize("shape,so", FS_CASES[:2])
def test_free_surface_gradient_parity(prop, orc, shape, so, mode):
    from paper_2004_10519_amd import inputs
    case = _fs_case(shape, so, 60, mode)
    p, shot = make_el(case, prop)
    g, mod = oracle_el(case, orc)
    m = case["model"]
    pert = 1 + 0.03 * inputs.random_unit_field(g.arr_shape, 5, 2.0)
    dobs, _ = orc.elastic_forward(g, orc.ElasticModel.from_velocities(g, m["vp"] * pert, m["vs"] * pert, m["rho"]),
                                  case["src"], case["wav"], case["rec"], case["kind"])
    d = host(p.forward(shot)).astype(np.float64)
    res = (d - dobs).astype(np.float32)
    gg = host(p.gradient(shot, dev(res), n_ckpt=5, ckpt_dtype="f32"))
    _, go, _ = orc.elastic_gradient(g, m["vp"], m["vs"], m["rho"], case["src"], case["wav"], case["rec"],
                                    d - res.astype(np.float64), case["kind"])
    for name, a, b in zip(("vp", "vs", "rho"), gg, go):
        err = rel_l2(a, b)
        print(f"free-surface elastic gradient {name}: rel-L2 {err:.3e}")
        assert err <= 1e-3, (name, err)
    nb = case["nbl"]
    assert not gg[0][:nb].any() and not gg[1][:nb].any()
    if mode == "image":
        assert not gg[2][:nb].any()


def test_free_surface_rejections(prop):
    from helpers import tti_case
    case = el_case((40, 20, 30), 8, 3, 10, free_surface=True)
    with pytest.raises(prop.PropError, match="nbl >= space_order"):
        make_el(case, prop)
    case = el_case((40, 20, 30), 8, 5, 10, free_surface="image")
    with pytest.raises(prop.PropError, match="nbl >= space_order - 2"):
        make_el(case, prop)
    case = el_case((40, 20, 30), 8, 6, 10, free_surface="image")
    case["model"]["vs"][:] = 1000.0
    with pytest.raises(prop.PropError, match="fluid"):
        make_el(case, prop)
    tcase = tti_case((40, 20, 30), 8, 5, 10)
    g = prop.Grid(tcase["shape"], tcase["h"], space_order=8, nbl=5, dt=tcase["dt"], nt=10, free_surface=True)
    mt = [dev(tcase["model"][k]) for k in ("m", "eps", "delta", "theta", "phi")]
    with pytest.raises(prop.PropError, match="elastic only"):
        prop.Propagator(prop.TTI, g, mt)
    case = el_case((40, 20, 30), 8, 5, 10, free_surface=True)
    p, shot = make_el(case, prop)
    off = prop.Shot(case["src"], dev(case["wav"]), case["rec"], case["kind"], win_origin=(0, 0, 1),
                    win_shape=(40, 20, 29))
    with pytest.raises(prop.PropError, match="starts at z index 0"):
        p.forward(off)


# ---- the fused velocity-stress step (3D forward up to space order 8) against the two passes
@pytest.mark.parametrize("so,shape,nt,zc,fs", [(8, (70, 37, 29), 61, 0, False), (8, (70, 37, 29), 60, 5, False),
                                              (6, (45, 19, 33), 41, 7, False), (4, (66, 20, 40), 50, 0, False),
                                              (2, (33, 17, 24), 37, 3, False), (8, (70, 37, 29), 47, 9, True),
                                              (4, (66, 20, 40), 40, 0, True), (4, (66, 20, 40), 41, 7, "image")])
def test_fused_elastic_step_bitwise_equals_two_passes(prop, so, shape, nt, zc, fs):
    """The fused step forms v+ and tau+ with the two passes' expressions, term for term, so traces
    and every final field are equal bit for bit: ragged tiles in x and y, one and several z chunks
    (short ones: many chunk seams, each recomputing v+ on 2R planes beyond it), an odd step count
    (the final state is copied back to the first buffer set), the free surface."""
    case = el_case(shape, so, 5, nt, free_surface=fs)
    if fs:
        case["src"][0, -1] = case["h"][2] * (case["nbl"] + 3.4)
    if fs == "image":
        case = _fluid_top(case)
    out = []
    for fused in (0, 1):
        p, shot = make_el(case, prop)
        p.set_option("el_fused", fused)
        if zc:
            p.set_option("zc", zc)
        p.set_timing(True)
        d = host(p.forward(shot)).copy()
        f = [host(p.read_state(i)).copy() for i in range(9)]
        launches = {k: p.kernel_time(k)[1] for k in (2, 3, 4)}
        out.append((d, f, launches))
        p.close()
    (d0, f0, l0), (d1, f1, l1) = out
    assert l0 == {2: nt, 3: nt, 4: 0} and l1 == {2: 0, 3: 0, 4: nt}, (l0, l1)
    assert np.abs(d0).max() > 0
    assert np.array_equal(d0, d1), rel_l2(d1, d0)
    for i in range(9):
        assert np.array_equal(f0[i], f1[i]), (i, rel_l2(f1[i], f0[i]))


def test_fused_elastic_checkpoints_feed_the_gradient(prop):
    """A saving forward on the fused step keeps the checkpoints of the buffer set that holds each
    state; the gradient that reuses them equals the one that runs its own (two-pass) forward sweep."""
    case = el_case((70, 37, 29), 8, 5, 61)
    p, shot = make_el(case, prop)
    p.set_option("el_fused", 1)
    rec = dev(np.random.default_rng(4).standard_normal((case["nt"], len(case["rec"]))))
    g_fresh = host(p.gradient(shot, rec, n_ckpt=6, ckpt_dtype="f32")).copy()
    p.forward(shot, save_ckpt=6, ckpt_dtype="f32")
    g_reuse = host(p.gradient(shot, rec, n_ckpt=0, ckpt_dtype="f32"))
    assert np.array_equal(g_reuse, g_fresh), rel_l2(g_reuse, g_fresh)


# ---- tile heights of the elastic passes (TILE1: velocity pass, TILE2: stress pass and imaging
# condition; 0: 64 x 8, 1: 64 x 16; default 0 and 1)
@pytest.mark.parametrize("so,shape,zc", [(8, (70, 37, 29), 0), (4, (66, 20, 40), 7), (12, (40, 22, 30), 0),
                                         (8, (130, 45, 33), 5)])
def test_elastic_tile_rows_change_no_bit(prop, so, shape, zc):
    """Forward traces and final fields and adjoint source traces are equal bit for bit with 64 x 8
    and 64 x 16 tiles in either pass: each point is formed by the same expressions, whichever tile
    computes it (ragged tiles in x and y, one and several z chunks).  So is the (vp, vs, rho)
    gradient while the imaging condition keeps its tile height; with the other height it runs
    another instantiation of that kernel, whose products and sums the compiler may contract into
    fused multiply-adds differently: rounding level."""
    case = el_case(shape, so, 5, 41)
    rec = dev(np.random.default_rng(6).standard_normal((case["nt"], len(case["rec"]))))
    out = []
    for t1, t2 in ((None, None), (1, 1), (0, 0)):
        p, shot = make_el(case, prop)
        if t1 is None:
            assert (p.get_option("tile1"), p.get_option("tile2")) == (0, 1)
        else:
            p.set_option("tile1", t1)
            p.set_option("tile2", t2)
        if zc:
            p.set_option("zc", zc)
        d = host(p.forward(shot)).copy()
        f = [host(p.read_state(i)).copy() for i in range(9)]
        a = host(p.adjoint(shot, rec)).copy()
        g = host(p.gradient(shot, rec, n_ckpt=4, ckpt_dtype="f32")).copy()
        out.append((d, f, a, g))
        p.close()
    d0, f0, a0, g0 = out[0]
    assert np.abs(d0).max() > 0 and np.abs(g0).max() > 0
    for k, (d1, f1, a1, g1) in enumerate(out[1:]):
        assert np.array_equal(d0, d1), (k, rel_l2(d1, d0))
        for i in range(9):
            assert np.array_equal(f0[i], f1[i]), (k, i, rel_l2(f1[i], f0[i]))
        assert np.array_equal(a0, a1), (k, rel_l2(a1, a0))
        if k == 0:
            assert np.array_equal(g0, g1), rel_l2(g1, g0)
        else:
            assert rel_l2(g1, g0) <= 1e-6, rel_l2(g1, g0)
