"""GPU parity of the TTI path (HIP library through the C ABI) against the FP64 checker.

Bar: FP32 traces and wavefields within relative L2 1e-4 of the FP64 checker; adjoint dot test
(FP32 arithmetic, FP64 inner products) within 1e-5; gradient within 1e-3 (per checkpoint type);
codec bit-exact; determinism bitwise.
"""
import numpy as np
import pytest
import torch

from helpers import dev, host, make_tti, oracle_tti, rel_l2, tti_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prop():
    from paper_2004_10519_amd import prop as P
    P.lib()
    return P


BF16_REASON = ("BF16 keeps 8 mantissa bits: a checkpoint level carries a relative rounding error of up to "
               "2^-9, above the 1e-3 gradient bar (measured 4.7e-3 here, 2.0e-3 on the 64^3 case); FP16 meets it")


# two passes (six-field / four-field temporaries), one fused pass, two fused single-field passes
SCHEMES = [0, 2, 3, 4]


@pytest.mark.parametrize("scheme", SCHEMES)
def test_tti2d_101_full_parity(prop, orc, scheme):
    """The 2D constant-medium case at full length: 101 x 101, so 4, 500 steps, 101 surface receivers."""
    from paper_2004_10519_amd import configs
    w = configs.tti2d_101()
    mdl = w.make_model()
    case = dict(shape=w.shape, h=w.spacing, so=w.space_order, nbl=w.nbl, nt=w.nt, dt=w.dt, model=mdl,
                src=w.src_xyz, rec=w.rec_xyz, wav=w.wavelet())
    p, shot = make_tti(case, prop, scheme)
    d = host(p.forward(shot))
    fields = [host(p.read_state(i)) for i in range(4)]
    g, mod = oracle_tti(case, orc)
    do, (po, qo, pmo, qmo), _ = orc.tti_forward(g, mod, case["src"], case["wav"], case["rec"])
    assert rel_l2(d, do) <= 1e-4
    for a, b in zip(fields, (po, qo, pmo, qmo)):
        assert rel_l2(a, b) <= 1e-4


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("so,shape", [(8, (70, 37, 29)), (12, (67, 20, 40)), (4, (130, 18, 21)), (8, (90, 1, 77)),
                                      (16, (75, 33, 45))])
def test_tti_forward_parity(prop, orc, so, shape, scheme):
    """Several tiles and ragged tails in x, y and z, absorbing layers, two off-grid sources."""
    case = tti_case(shape, so, 5, 90)
    p, shot = make_tti(case, prop, scheme)
    d = host(p.forward(shot))
    pf, qf = host(p.read_state(0)), host(p.read_state(1))
    g, mod = oracle_tti(case, orc)
    do, (po, qo, _, _), _ = orc.tti_forward(g, mod, case["src"], case["wav"], case["rec"])
    assert rel_l2(d, do) <= 1e-4, rel_l2(d, do)
    assert rel_l2(pf, po) <= 1e-4 and rel_l2(qf, qo) <= 1e-4


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("so,shape", [(8, (70, 37, 29)), (12, (67, 20, 40)), (8, (90, 1, 77))])
def test_tti_adjoint_parity(prop, orc, so, shape, scheme):
    case = tti_case(shape, so, 5, 80)
    p, shot = make_tti(case, prop, scheme)
    rng = np.random.default_rng(3)
    rec = rng.standard_normal((case["nt"], len(case["rec"]))).astype(np.float32)
    s = host(p.adjoint(shot, dev(rec)))
    yp = host(p.read_state(0))
    g, mod = oracle_tti(case, orc)
    so_, (ypo, _) = orc.tti_adjoint(g, mod, case["src"], case["rec"], rec)
    assert rel_l2(s, so_) <= 1e-4, rel_l2(s, so_)
    assert rel_l2(yp, ypo) <= 1e-4


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("shape", [(70, 37, 29), (90, 1, 77)])
def test_tti_gpu_dot_test(prop, shape, scheme):
    case = tti_case(shape, 8, 5, 100)
    p, shot = make_tti(case, prop, scheme)
    rng = np.random.default_rng(11)
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


def _bandlimited_residual(case, seed):
    """Data-like residual: white noise filtered by the source's Ricker spectrum (band-limited)."""
    from paper_2004_10519_amd import inputs
    rng = np.random.default_rng(seed)
    wn = rng.standard_normal((case["nt"], len(case["rec"])))
    k = inputs.ricker(25.0, case["dt"], 81, t0=40 * case["dt"]).astype(np.float64)
    out = np.stack([np.convolve(wn[:, i], k, mode="same") for i in range(wn.shape[1])], axis=1)
    return out.astype(np.float32)


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f16", 1e-3),
                                       pytest.param("bf16", 1e-3, marks=pytest.mark.xfail(strict=True,
                                                                                          reason=BF16_REASON)),
                                       ("bf16", 6e-3)], ids=["f32", "f16", "bf16-bar", "bf16-regression"])
def test_tti_gradient_parity(prop, orc, dtype, tol, scheme):
    case = tti_case((40, 36, 32), 8, 5, 150, nrec=30)
    p, shot = make_tti(case, prop, scheme)
    res = _bandlimited_residual(case, 4)
    gg = host(p.gradient(shot, dev(res), n_ckpt=7, ckpt_dtype=dtype))
    g, mod = oracle_tti(case, orc)
    # the checker takes observed data: d_obs = d - res gives the residual d - d_obs = res
    d, _, _ = orc.tti_forward(g, mod, case["src"], case["wav"], case["rec"])
    _, go, _ = orc.tti_gradient(g, mod, case["src"], case["wav"], case["rec"], d - res)
    err = rel_l2(gg, go)
    print(f"gradient rel-L2 vs FP64 ({dtype} checkpoints): {err:.3e}")
    assert err <= tol, err


@pytest.mark.parametrize("dtype,tol", [("f16", 1e-3),
                                       pytest.param("bf16", 1e-3, marks=pytest.mark.xfail(strict=True,
                                                                                          reason=BF16_REASON)),
                                       ("bf16", 1.5e-3)], ids=["f16", "bf16-bar", "bf16-regression"])
def test_tti_gradient_whole_run_16bit_storage(prop, orc, dtype, tol):
    """n_ckpt = 1 with a 16-bit type stores every forward level in FP16/BF16 (per-row scales) and
    runs two sweeps."""
    case = tti_case((40, 36, 32), 8, 5, 150, nrec=30)
    p, shot = make_tti(case, prop)
    res = _bandlimited_residual(case, 4)
    gg = host(p.gradient(shot, dev(res), n_ckpt=1, ckpt_dtype=dtype))
    g, mod = oracle_tti(case, orc)
    d, _, _ = orc.tti_forward(g, mod, case["src"], case["wav"], case["rec"])
    _, go, _ = orc.tti_gradient(g, mod, case["src"], case["wav"], case["rec"], d - res)
    err = rel_l2(gg, go)
    print(f"gradient rel-L2 vs FP64 (whole run stored in {dtype}): {err:.3e}")
    assert err <= tol, err
    im = host(p.image(shot, dev(res), n_ckpt=1, ckpt_dtype=dtype))
    io = orc.tti_image(g, mod, case["src"], case["wav"], case["rec"], res)
    assert rel_l2(im, io) <= tol, rel_l2(im, io)


def test_tti_gradient_single_segment_equals_full_storage(prop, orc):
    """n_ckpt = 1 keeps the whole forward wavefield (no checkpoint rounding): FP32-level agreement."""
    case = tti_case((40, 36, 32), 8, 5, 120, nrec=30)
    p, shot = make_tti(case, prop)
    res = _bandlimited_residual(case, 5)
    gg = host(p.gradient(shot, dev(res), n_ckpt=1, ckpt_dtype="f32"))
    g, mod = oracle_tti(case, orc)
    d, _, _ = orc.tti_forward(g, mod, case["src"], case["wav"], case["rec"])
    _, go, _ = orc.tti_gradient(g, mod, case["src"], case["wav"], case["rec"], d - res)
    assert rel_l2(gg, go) <= 1e-4


@pytest.mark.parametrize("so,shape", [(4, (83, 29, 41)), (8, (70, 37, 29)), (12, (67, 20, 40)), (16, (75, 33, 45)),
                                      (8, (90, 1, 77))])
def test_four_field_scheme_bitwise_equals_six(prop, so, shape):
    """Four-field scheme: pass 1 stores t and the scalar n . grad q, pass 2 forms n (n . grad q) from
    it and the axis. Those products are the floats the six-field pass 1 stores, so forward traces,
    adjoint traces and the gradient (FP32 checkpoints) are equal bit for bit, for every tile variant
    and short z-chunks."""
    case = tti_case(shape, so, 5, 60)
    p0, shot = make_tti(case, prop, 0)
    d0 = host(p0.forward(shot)).copy()
    rec = np.random.default_rng(3).standard_normal(d0.shape).astype(np.float32)
    a0 = host(p0.adjoint(shot, dev(rec))).copy()
    g0 = host(p0.gradient(shot, dev(rec), n_ckpt=4, ckpt_dtype="f32")).copy()
    for t1, t2, zc in ((1, 1, 0), (0, 0, 5), (1, 0, 3)):
        p3, shot3 = make_tti(case, prop, 3, tile1=t1, tile2=t2, zc=zc)
        assert np.array_equal(host(p3.forward(shot3)), d0), (t1, t2, zc)
        assert np.array_equal(host(p3.adjoint(shot3, dev(rec))), a0), (t1, t2, zc)
        assert np.array_equal(host(p3.gradient(shot3, dev(rec), n_ckpt=4, ckpt_dtype="f32")), g0), (t1, t2, zc)


@pytest.mark.parametrize("so", [4, 8, 12, 16])
def test_six_field_scheme_tiles_and_chunks(prop, so):
    """Six-field scheme: both tile variants of each pass and short z-chunks (more chunk seams and
    queue refills) give the traces of its default launch bit for bit (every point is computed by the
    same expressions); pass 2 takes pass 1's z-chunk unless its own is set."""
    case = tti_case((83, 29, 41), so, 5, 60)
    p0, shot = make_tti(case, prop, 0)
    ref = host(p0.forward(shot)).copy()
    for t1 in (0, 1):
        for t2 in (0, 1):
            for zc in (0, 5):
                p, shot = make_tti(case, prop, 0, tile1=t1, tile2=t2, zc=zc)
                assert np.array_equal(host(p.forward(shot)), ref), (t1, t2, zc)
                assert p.get_option("info_zc2") == p.get_option("info_zc1")
                if zc:
                    assert p.get_option("info_zc1") == zc
    p, shot = make_tti(case, prop, 0, zc=7, zc2=4)
    assert np.array_equal(host(p.forward(shot)), ref)
    assert (p.get_option("info_zc1"), p.get_option("info_zc2")) == (7, 4)


@pytest.mark.parametrize("so", [2, 4, 8, 12])
def test_fused_scheme_tiles_and_chunks(prop, so):
    """Fused scheme: both tile variants and short z-chunks (chunk seams, warm-up of the queues and
    accumulators at every chunk start) give the traces of its default launch to 1e-6 and the
    six-field scheme's to 1e-5 (the z divergence is summed in another order)."""
    case = tti_case((83, 29, 41), so, 5, 60)
    p0, shot = make_tti(case, prop, 0)
    six = host(p0.forward(shot)).copy()
    p2, shot = make_tti(case, prop, 2)
    ref = host(p2.forward(shot)).copy()
    assert rel_l2(ref, six) <= 1e-5, rel_l2(ref, six)
    for t2 in (0, 1):
        for zc in (0, 3, 17):
            p, shot = make_tti(case, prop, 2, tile2=t2, zc=zc, zc2=zc)
            d = host(p.forward(shot))
            assert rel_l2(d, ref) <= 1e-6, (t2, zc, rel_l2(d, ref))


def test_fused_scheme_rejects_wide_stencils(prop):
    case = tti_case((40, 20, 30), 16, 5, 10)
    p, _ = make_tti(case, prop, 0)
    with pytest.raises(prop.PropError, match="space orders up to 12"):
        p.set_option("scheme", 2)
    with pytest.raises(prop.PropError, match="space orders up to 12"):
        p.set_option("scheme", 4)
    for bad in (1, 5, -1):
        with pytest.raises(prop.PropError, match="scheme must be"):
            p.set_option("scheme", bad)


def test_codec_bit_exact(prop, orc):
    rng = np.random.default_rng(9)
    f = (rng.standard_normal(100003) * 10.0 ** rng.uniform(-4, 3, 100003)).astype(np.float32)
    f[:4] = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.5 + 2 ** -9], np.float32) * 512
    for dt in ("f16", "bf16"):
        codes, scale = prop.ckpt_encode(dev(f), dt)
        s_o, c_o = orc.ckpt_encode(f, dt)
        assert float(host(scale)[0]) == s_o
        assert np.array_equal(host(codes).view(np.uint16), c_o)
        dec = host(prop.ckpt_decode(codes, scale, dt))
        assert np.array_equal(dec, orc.ckpt_decode(s_o, c_o, dt))
    codes, scale = prop.ckpt_encode(dev(np.zeros(10, np.float32)), "bf16")
    assert float(host(scale)[0]) == 1.0 and not host(codes).any()
    sub = np.array([3e-41, -1e-40, 0.0, 2e-45], np.float32)       # subnormal maximum
    for dt in ("f16", "bf16"):
        codes, scale = prop.ckpt_encode(dev(sub), dt)
        s_o, c_o = orc.ckpt_encode(sub, dt)
        assert float(host(scale)[0]) == s_o == 2.0 ** -126
        assert np.array_equal(host(codes).view(np.uint16), c_o)


def test_dot_f64(prop):
    rng = np.random.default_rng(1)
    a = rng.standard_normal(1_000_003).astype(np.float32)
    b = rng.standard_normal(1_000_003).astype(np.float32)
    r = prop.dot_f64(dev(a), dev(b))
    ref = float(np.dot(a.astype(np.float64), b.astype(np.float64)))
    assert abs(r - ref) <= 1e-12 * np.abs(a.astype(np.float64) * b).sum()
    assert prop.dot_f64(dev(a), dev(b)) == r


def test_determinism(prop):
    case = tti_case((70, 37, 29), 8, 5, 60)
    p, shot = make_tti(case, prop)
    d1 = host(p.forward(shot)).copy()
    d2 = host(p.forward(shot))
    assert np.array_equal(d1, d2)


def test_error_paths(prop):
    case = tti_case((40, 36, 32), 8, 5, 10)
    g = prop.Grid(case["shape"], case["h"], space_order=7, nbl=5, dt=case["dt"], nt=10)
    mt = [dev(case["model"][k]) for k in ("m", "eps", "delta", "theta", "phi")]
    with pytest.raises(prop.PropError) as e:
        prop.Propagator(prop.TTI, g, mt)
    assert e.value.code == prop.PROP_EINVAL
    g = prop.Grid(case["shape"], case["h"], space_order=8, nbl=5, dt=case["dt"] * 2, nt=10)
    with pytest.raises(prop.PropError) as e:
        prop.Propagator(prop.TTI, g, mt)
    assert e.value.code == prop.PROP_EUNSTABLE
    bad = [mt[0], mt[2], mt[1], mt[3], mt[4]]   # epsilon < delta
    g = prop.Grid(case["shape"], case["h"], space_order=8, nbl=5, dt=case["dt"], nt=10)
    with pytest.raises(prop.PropError) as e:
        prop.Propagator(prop.TTI, g, bad)
    assert e.value.code == prop.PROP_EUNSTABLE
    p = prop.Propagator(prop.TTI, g, mt)
    shot = prop.Shot(case["src"], dev(case["wav"][:10]), case["rec"] + 1e4)
    with pytest.raises(prop.PropError) as e:
        p.forward(shot)
    assert e.value.code == prop.PROP_EINVAL
    with pytest.raises(prop.PropError) as e:
        p.read_state(0)
    assert e.value.code == prop.PROP_ESTATE


@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("dtype,tol", [("f32", 1e-4), ("f16", 1e-3)])
def test_tti_image_parity(prop, orc, dtype, tol, scheme):
    """Zero-lag cross-correlation image of one shot against the checker's image."""
    case = tti_case((40, 36, 32), 8, 5, 150, nrec=30)
    p, shot = make_tti(case, prop, scheme)
    data = _bandlimited_residual(case, 6)
    im = host(p.image(shot, dev(data), n_ckpt=7, ckpt_dtype=dtype))
    g, mod = oracle_tti(case, orc)
    io = orc.tti_image(g, mod, case["src"], case["wav"], case["rec"], data)
    err = rel_l2(im, io)
    print(f"image rel-L2 vs FP64 ({dtype} checkpoints): {err:.3e}")
    assert err <= tol, err


def test_isotropic_reduction_vs_acoustic_stepper(prop, orc):
    """eps = delta = 0 and a vertical axis: p = q and the TTI scheme is the acoustic leapfrog with the
    composed Laplacian -sum_a D_a^T D_a; compare with the checker's independent acoustic stepper."""
    from paper_2004_10519_amd import inputs
    shape, h, so, nt = (60, 44, 52), (10.0, 11.0, 9.0), 8, 120
    mdl = inputs.tti_model(shape, 0, 12)
    m = inputs.slowness_squared(mdl["vp"])
    z = np.zeros_like(m)
    case = tti_case(shape, so, 0, nt)
    case["model"] = {"m": m, "eps": z, "delta": z, "theta": z, "phi": z}
    p, shot = make_tti(case, prop)
    d = host(p.forward(shot))
    pf, qf = host(p.read_state(0)), host(p.read_state(1))
    g = orc.Grid(shape, h, space_order=so, nbl=0, dt=case["dt"], nt=nt)
    da, ua = orc.acoustic_wide_forward(g, m, case["src"], case["wav"], case["rec"])
    assert rel_l2(d, da) <= 1e-4, rel_l2(d, da)
    assert rel_l2(pf, ua) <= 1e-4 and np.array_equal(pf, qf)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_degenerate_shots(prop, orc, scheme):
    """No source: all-zero traces; no receivers: the state still evolves; one time step; a window of
    the smallest allowed size (2 nbl + 2 points per axis) inside a larger grid; a grid thinner than
    the stencil (5 x 3 x 2 points at space order 12, no absorbing layer)."""
    case = tti_case((70, 37, 29), 8, 5, 40)
    p, shot = make_tti(case, prop, scheme)
    silent = prop.Shot(np.zeros((0, 3), np.float32), None, case["rec"])
    assert not host(p.forward(silent)).any()
    blind = prop.Shot(case["src"], dev(case["wav"]), np.zeros((0, 3), np.float32))
    p.forward(blind)
    pf = host(p.read_state(0))
    g, mod = oracle_tti(case, orc)
    _, (po, _, _, _), _ = orc.tti_forward(g, mod, case["src"], case["wav"], None)
    assert rel_l2(pf, po) <= 1e-4
    one = tti_case((70, 37, 29), 8, 5, 1)
    p1, s1 = make_tti(one, prop, scheme)
    d1 = host(p1.forward(s1))
    g1, mod1 = oracle_tti(one, orc)
    do1, _, _ = orc.tti_forward(g1, mod1, one["src"], one["wav"], one["rec"])
    assert rel_l2(d1, do1) <= 1e-6
    # smallest window: 12 x 12 x 12 with nbl 5, at an offset inside the 70 x 37 x 29 grid
    o, n = (30, 11, 9), (12, 12, 12)
    hh = case["h"]
    src = np.array([[hh[0] * (o[0] + 5.5), hh[1] * (o[1] + 6.2), hh[2] * (o[2] + 5.7)]], np.float32)
    rec = np.array([[hh[0] * (o[0] + 2.0), hh[1] * (o[1] + 9.0), hh[2] * (o[2] + 3.3)],
                    [hh[0] * (o[0] + 11.0), hh[1] * (o[1] + 11.0), hh[2] * (o[2] + 11.0)]], np.float32)
    wav = dev(case["wav"][:, :1])
    dw = host(p.forward(prop.Shot(src, wav, rec, win_origin=o, win_shape=n)))
    sub = (slice(o[2], o[2] + n[2]), slice(o[1], o[1] + n[1]), slice(o[0], o[0] + n[0]))
    gw = orc.Grid(n, hh, origin=tuple(o[a] * hh[a] for a in range(3)), space_order=8, nbl=5, dt=case["dt"],
                  nt=case["nt"], vref=1500.0)
    mw = orc.TTIModel.from_arrays(gw, *(case["model"][k][sub] for k in ("m", "eps", "delta", "theta", "phi")))
    dow, _, _ = orc.tti_forward(gw, mw, src, case["wav"][:, :1], rec)
    assert rel_l2(dw, dow) <= 1e-4, rel_l2(dw, dow)
    with pytest.raises(prop.PropError):       # one point short of 2 nbl + 2
        p.forward(prop.Shot(src, wav, rec, win_origin=o, win_shape=(11, 12, 12)))
    thin = tti_case((5, 3, 2), 12, 0, 12, nsrc=1, nrec=3)
    pt, st = make_tti(thin, prop, scheme)
    dt_ = host(pt.forward(st))
    gt, mt = oracle_tti(thin, orc)
    dot_, _, _ = orc.tti_forward(gt, mt, thin["src"], thin["wav"], thin["rec"])
    assert np.abs(dot_).max() > 0 and rel_l2(dt_, dot_) <= 1e-4, rel_l2(dt_, dot_)


@pytest.mark.parametrize("so,shape", [(8, (70, 37, 29)), (12, (67, 20, 40)), (4, (90, 1, 77))])
def test_split_scheme_bitwise_equals_fused(prop, so, shape):
    """The split scheme forms H0 u and Hz v with the fused pass's expressions in the same order (h goes
    through memory as the same float): forward traces and final state, adjoint and gradient are
    bitwise those of the fused scheme."""
    case = tti_case(shape, so, 5, 60, nrec=19)
    res = dev(np.random.default_rng(3).standard_normal((case["nt"], len(case["rec"]))))
    out = []
    for scheme in (2, 4):
        p, shot = make_tti(case, prop, scheme)
        d = host(p.forward(shot)).copy()
        st = [host(p.read_state(i)).copy() for i in range(4)]
        a = host(p.adjoint(shot, res)).copy()
        g = host(p.gradient(shot, res, n_ckpt=4, ckpt_dtype="f16")).copy()
        out.append([d, a, g] + st)
        p.close()
    for x, y in zip(*out):
        assert np.array_equal(x, y)
