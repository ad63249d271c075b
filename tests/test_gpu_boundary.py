"""The C ABI's contract beyond the propagators' numbers (GPU):

* the gradient's row codecs bit for bit against the checker's twin (oracle.encode_rows,
  oracle.ckpt_pair_encode_rows / ckpt_pair_decode_rows);
* checkpoints saved by prop_forward and reused by prop_gradient / prop_image (bitwise equal to a
  fresh gradient), PROP_ESTATE once they are invalidated;
* the autograd Function TTIModelling against Propagator.gradient and the FP64 checker's gradient,
  for a whole-grid shot and a windowed shot;
* failures forced from the host: a NaN wavelet sample trips the non-finite watchdog
  (PROP_EUNSTABLE), an absurd grid fails its allocation (PROP_ENOMEM).
"""
import numpy as np
import pytest
import torch

from codec_cases import rows_fixture
from helpers import dev, host, make_el, make_tti, el_case, oracle_tti, rel_l2, tti_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prop():
    from paper_2004_10519_amd import prop as P
    P.lib()
    return P


def _u16(t):
    return host(t).view(np.uint16)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
@pytest.mark.parametrize("nx", [700, 37])
def test_row_codecs_bit_exact_against_twin(prop, orc, dtype, nx):
    f = rows_fixture()[:, :, :nx].copy()
    rng = np.random.default_rng(31)
    prev = (f * (1 + 0.05 * rng.standard_normal(f.shape))).astype(np.float32)
    # checkpoint pair: level and level difference
    ca, cb, sa, sb = prop.ckpt_encode_rows(dev(f), dev(prev), True, dtype)
    ra, rb, rsa, rsb = orc.ckpt_pair_encode_rows(f, prev, dtype)
    assert np.array_equal(_u16(ca), ra) and np.array_equal(_u16(cb), rb)
    assert np.array_equal(host(sa), rsa) and np.array_equal(host(sb), rsb)
    cur, prv = prop.ckpt_decode_rows(ca, cb, sa, sb, dtype)
    rc, rp = orc.ckpt_pair_decode_rows(ra, rb, rsa, rsb, dtype)
    assert np.array_equal(host(cur), rc) and np.array_equal(host(prv), rp)
    # per-step store of two independent fields
    ca, cb, sa, sb = prop.ckpt_encode_rows(dev(f), dev(prev), False, dtype)
    ra, rsa = orc.encode_rows(f, dtype)
    rb, rsb = orc.encode_rows(prev, dtype)
    assert np.array_equal(_u16(ca), ra) and np.array_equal(_u16(cb), rb)
    assert np.array_equal(host(sa), rsa) and np.array_equal(host(sb), rsb)


def test_row_codec_rejects_bad_shapes(prop):
    a = dev(np.zeros((1, 1, 4), np.float32))
    with pytest.raises(prop.PropError):
        prop.ckpt_encode_rows(a, a, True, "f32")
    bad = torch.zeros((70000, 1, 1), device="cuda")
    with pytest.raises(prop.PropError):
        prop.ckpt_encode_rows(bad, bad, True, "f16")


def _res(case, seed):
    rng = np.random.default_rng(seed)
    return dev(rng.standard_normal((case["nt"], len(case["rec"]))))


@pytest.mark.parametrize("n_ckpt,dtype", [(7, "f16"), (7, "f32"), (1, "f16"), (1, "f32")])
def test_tti_saved_checkpoints_reused_bitwise(prop, n_ckpt, dtype):
    case = tti_case((38, 30, 28), 8, 4, 90, nrec=17)
    p, shot = make_tti(case, prop, 2)
    res = _res(case, 41)
    d0 = host(p.forward(shot)).copy()
    g_fresh = host(p.gradient(shot, res, n_ckpt, dtype)).copy()
    i_fresh = host(p.image(shot, res, n_ckpt, dtype)).copy()
    with pytest.raises(prop.PropError) as e:      # nothing saved yet
        p.gradient(shot, res, 0)
    assert e.value.code == prop.PROP_ESTATE
    d1 = host(p.forward(shot, save_ckpt=n_ckpt, ckpt_dtype=dtype)).copy()
    assert np.array_equal(d0, d1)
    assert np.array_equal(host(p.gradient(shot, res, 0)), g_fresh)
    p.adjoint(shot, res)                          # adjoint and plain forward keep the checkpoints
    p.forward(shot)
    assert np.array_equal(host(p.gradient(shot, res, n_ckpt, dtype)), g_fresh)
    assert np.array_equal(host(p.image(shot, res, 0)), i_fresh)
    # another wavelet array is another shot
    other = type(shot)(shot.src_xyz, shot.wavelet.clone(), shot.rec_xyz)
    with pytest.raises(prop.PropError) as e:
        p.gradient(other, res, 0)
    assert e.value.code == prop.PROP_ESTATE
    # a model change invalidates them
    p.set_model(p._model)
    with pytest.raises(prop.PropError) as e:
        p.gradient(shot, res, 0)
    assert e.value.code == prop.PROP_ESTATE
    # so does a gradient that stores checkpoints of its own
    p.forward(shot, save_ckpt=n_ckpt, ckpt_dtype=dtype)
    p.gradient(shot, res, n_ckpt + 2, dtype)
    with pytest.raises(prop.PropError) as e:
        p.gradient(shot, res, 0)
    assert e.value.code == prop.PROP_ESTATE


def test_elastic_saved_checkpoints_reused_bitwise(prop):
    case = el_case((30, 26, 28), 8, 4, 70)
    p, shot = make_el(case, prop)
    res = _res(case, 42)
    d0 = host(p.forward(shot)).copy()
    g_fresh = host(p.gradient(shot, res, 6, "f32")).copy()
    d1 = host(p.forward(shot, save_ckpt=6, ckpt_dtype="f32")).copy()
    assert np.array_equal(d0, d1)
    assert np.array_equal(host(p.gradient(shot, res, 0)), g_fresh)
    assert np.array_equal(host(p.gradient(shot, res, 6, "f32")), g_fresh)
    with pytest.raises(prop.PropError) as e:      # elastic checkpoints are FP32
        p.forward(shot, save_ckpt=6, ckpt_dtype="f16")
    assert e.value.code == prop.PROP_EINVAL
    p.set_model(p._model)
    with pytest.raises(prop.PropError) as e:
        p.gradient(shot, res, 0)
    assert e.value.code == prop.PROP_ESTATE


@pytest.mark.parametrize("windowed", [False, True])
def test_ttimodelling_autograd(prop, orc, windowed):
    """torch.autograd.grad of 1/2 ||F(m) - d_obs||^2 through TTIModelling equals Propagator.gradient
    (bitwise: the backward reuses the forward's checkpoints) and the FP64 checker's gradient (FP32
    checkpoints, 1e-4); a windowed shot's gradient is the window's, zero elsewhere."""
    case = tti_case((44, 34, 30), 8, 4, 100, nrec=21)
    if windowed:
        o, n = (4, 3, 0), (36, 28, 30)
        lo = np.array([o[0] * case["h"][0], o[1] * case["h"][1], 0.0])
        hi = lo + np.array([(n[0] - 1) * case["h"][0], (n[1] - 1) * case["h"][1], (n[2] - 1) * case["h"][2]])
        case["rec"] = np.clip(case["rec"], lo, hi).astype(np.float32)
        case["src"] = np.clip(case["src"], lo + 50.0, hi - 50.0).astype(np.float32)
    p, shot = make_tti(case, prop, 2)
    if windowed:
        shot = prop.Shot(case["src"], shot.wavelet, case["rec"], win_origin=o, win_shape=n)
    rng = np.random.default_rng(5)
    dobs = dev(rng.standard_normal((case["nt"], len(case["rec"]))) * 1e-3)
    m = dev(case["model"]["m"]).requires_grad_(True)
    aniso = [dev(case["model"][k]) for k in ("eps", "delta", "theta", "phi")]
    d = prop.TTIModelling.apply(m, p, aniso, shot, 5, "f32")
    J = 0.5 * ((d - dobs) ** 2).sum()
    (gm,) = torch.autograd.grad(J, m)
    gm = host(gm).astype(np.float64)
    assert gm.shape == p.grid.arr_shape
    res = (d.detach() - dobs).contiguous()
    gref = host(p.gradient(shot, res, 5, "f32")).astype(np.float64)
    if windowed:
        (ox, oy, oz), (nx, ny, nz) = o, n
        inner = gm[oz:oz + nz, oy:oy + ny, ox:ox + nx]
        assert np.array_equal(inner, gref)
        out = gm.copy()
        out[oz:oz + nz, oy:oy + ny, ox:ox + nx] = 0
        assert not out.any()
        return
    assert np.array_equal(gm, gref)
    g, mod = oracle_tti(case, orc)
    r = host(res).astype(np.float64)
    dd, _, _ = orc.tti_forward(g, mod, case["src"], case["wav"], case["rec"])
    _, go, _ = orc.tti_gradient(g, mod, case["src"], case["wav"], case["rec"], dd - r)
    err = rel_l2(gm, go)
    print(f"TTIModelling gradient vs FP64: {err:.2e}")
    assert err <= 1e-4, err


def test_nan_wavelet_trips_the_watchdog(prop):
    """A NaN in the wavelet (NaN arithmetic does not fault) reaches the wavefield; the non-finite check
    at the end of the run returns PROP_EUNSTABLE instead of traces."""
    case = tti_case((30, 28, 26), 8, 4, 40, nrec=5)
    p, shot = make_tti(case, prop, 2)
    w = case["wav"].copy()
    w[7, 0] = np.nan
    shot.wavelet = dev(w)
    with pytest.raises(prop.PropError) as e:
        p.forward(shot)
    assert e.value.code == prop.PROP_EUNSTABLE
    shot.wavelet = dev(case["wav"])               # the handle stays usable
    assert np.isfinite(host(p.forward(shot))).all()


@pytest.mark.parametrize("kind", ["tti", "elastic"])
def test_absurd_grid_fails_allocation(prop, kind):
    """A 10^13-point grid: creating the handle needs its derived coefficients (160 TB and more), so
    the device allocation fails before any kernel touches the (small) model arrays: PROP_ENOMEM."""
    n = 21544
    g = prop.Grid((n, n, n), (10.0, 10.0, 10.0), space_order=8, nbl=0, dt=1e-4, nt=1)
    small = [torch.ones(16, device="cuda") for _ in range(5)]
    with pytest.raises(prop.PropError) as e:
        prop.Propagator(prop.TTI if kind == "tti" else prop.ELASTIC, g, small)
    assert e.value.code == prop.PROP_ENOMEM
