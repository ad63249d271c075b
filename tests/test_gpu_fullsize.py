"""Parity at the benchmark workloads' full sizes, in the launch configuration bench.py times
(autotuned tiles), on outputs the FP64 checker can compute, and properties that hold at any size.

* 512^3 so12 TTI and 400^3 so8 elastic: a few time steps from the workload's own source.  After n
  steps the wavefield is exactly zero beyond n * (stencil reach per step) points from the source, so
  the checker runs on a sub-grid that contains that support plus a full absorbing layer of its own
  (where the field is zero, so its damping acts on zeros).  The sub-grid keeps the full grid's top
  face, so the absorbing layer the source sits next to is the same on both sides.  The GPU fields
  and traces must match the checker there and be exactly zero everywhere else.
* 512^3 so12 TTI dot test over 20 steps and 65536 receivers.
* 256^3 so8 gradient (2000 steps; 48 FP16 checkpoints, or the whole run stored in FP16): central
  finite differences of the FP64 misfit and the Taylor remainder's slope along five seeded smooth
  model perturbations.
* 2D marine elastic workload (1701 x 391, free surface over the water layer): the first 800 steps,
  all 3242 traces, against the checker on the whole grid.
"""
import math

import numpy as np
import pytest
import torch

from helpers import dev, host, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prop():
    from paper_2004_10519_amd import prop as P
    P.lib()
    return P


@pytest.fixture(scope="module")
def tti512_model():
    """The 512^3 workload's seeded model (generated once for the module)."""
    from paper_2004_10519_amd import configs
    return configs.tti3d_512(nt=1).make_model()


def _tti512(nt, model):
    from paper_2004_10519_amd import configs
    w = configs.tti3d_512(nt=nt)
    w.model = model
    return w


def _subgrid(w, reach):
    """Index ranges [lo, hi) per axis (x, y, z) of a sub-grid holding the support after the steps
    plus an absorbing layer; z starts at the top face."""
    s = np.asarray(w.src_xyz[0], np.float64) / np.asarray(w.spacing)
    lo, hi = [], []
    for a in range(3):
        l_ = int(math.floor(s[a] - reach)) - w.nbl - 2
        h_ = int(math.ceil(s[a] + reach)) + w.nbl + 3
        lo.append(max(l_, 0) if a < 2 else 0)
        hi.append(min(h_, w.shape[a]))
    assert lo[0] > w.nbl and lo[1] > w.nbl and hi[0] < w.shape[0] - w.nbl and hi[1] < w.shape[1] - w.nbl
    return lo, hi


def _inside(xyz, lo, hi, h):
    u = np.asarray(xyz, np.float64) / np.asarray(h)
    return np.all((u >= np.asarray(lo)) & (u <= np.asarray(hi) - 1), axis=1)


def _compare_fields(gpu_full, ref_sub, lo, hi, tol):
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    assert rel_l2(gpu_full[sl], ref_sub) <= tol, rel_l2(gpu_full[sl], ref_sub)
    rest = gpu_full.copy()
    rest[sl] = 0
    assert not rest.any()


def test_tti512_so12_first_steps_vs_checker(prop, orc, tti512_model):
    nt = 6
    w = _tti512(nt, tti512_model)
    mdl = w.make_model()
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=nt, v_ref=w.v_ref)
    mt = [dev(mdl[k]) for k in ("m", "eps", "delta", "theta", "phi")]
    p = prop.Propagator(prop.TTI, g, mt)
    p.set_option("autotune", 1)
    shot = prop.Shot(w.src_xyz, dev(w.wavelet()), w.rec_xyz)
    d = host(p.forward(shot))
    pf, qf = host(p.read_state(0)), host(p.read_state(1))
    lo, hi = _subgrid(w, 2 * (w.space_order // 2) * nt + 2)
    shp = tuple(hi[a] - lo[a] for a in range(3))
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    gs = orc.Grid(shp, w.spacing, origin=tuple(lo[a] * w.spacing[a] for a in range(3)), space_order=w.space_order,
                  nbl=w.nbl, dt=w.dt, nt=nt, vref=w.v_ref)
    mod = orc.TTIModel.from_arrays(gs, *(mdl[k][sl] for k in ("m", "eps", "delta", "theta", "phi")))
    ins = _inside(w.rec_xyz, lo, hi, w.spacing)
    do, (po, qo, _, _), _ = orc.tti_forward(gs, mod, w.src_xyz, w.wavelet(), w.rec_xyz[ins])
    assert np.abs(po).max() > 0
    _compare_fields(pf, po, lo, hi, 1e-4)
    _compare_fields(qf, qo, lo, hi, 1e-4)
    assert rel_l2(d[:, ins], do) <= 1e-4
    assert not d[:, ~ins].any()


def test_el400_so8_first_steps_vs_checker(prop, orc):
    from paper_2004_10519_amd import configs
    nt = 8
    w = configs.el3d_400(nt=nt)
    mdl = w.make_model()
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=nt, v_ref=w.v_ref)
    mt = [dev(mdl[k]) for k in ("vp", "vs", "rho")]
    p = prop.Propagator(prop.ELASTIC, g, mt)
    shot = prop.Shot(w.src_xyz, dev(w.wavelet()), w.rec_xyz, w.rec_kind)
    d = host(p.forward(shot))
    fields = [host(p.read_state(i)) for i in range(9)]
    lo, hi = _subgrid(w, 2 * (w.space_order // 2) * nt + 2)
    shp = tuple(hi[a] - lo[a] for a in range(3))
    sl = (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))
    gs = orc.Grid(shp, w.spacing, origin=tuple(lo[a] * w.spacing[a] for a in range(3)), space_order=w.space_order,
                  nbl=w.nbl, dt=w.dt, nt=nt, vref=w.v_ref)
    mod = orc.ElasticModel.from_velocities(gs, *(mdl[k][sl] for k in ("vp", "vs", "rho")))
    ins = _inside(w.rec_xyz, lo, hi, w.spacing)
    do, fo = orc.elastic_forward(gs, mod, w.src_xyz, w.wavelet(), w.rec_xyz[ins], w.rec_kind[ins])
    for a, b in zip(fields, fo):
        if np.abs(b).max() > 1e-30:
            _compare_fields(a, b, lo, hi, 1e-4)
        else:
            # the shear stresses: the source sits in the water layer (mu = 0) and after 8 steps the
            # wave has only just reached the solid below, where the checker's values are ~1e-47,
            # beneath FP32's range (smallest normal 1.2e-38)
            assert np.abs(a).max() < 1e-30
    assert rel_l2(d[:, ins], do) <= 1e-4
    assert not d[:, ~ins].any()


def test_tti512_so12_dot_test(prop, tti512_model):
    nt = 20
    w = _tti512(nt, tti512_model)
    mdl = w.make_model()
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=nt, v_ref=w.v_ref)
    mt = [dev(mdl[k]) for k in ("m", "eps", "delta", "theta", "phi")]
    p = prop.Propagator(prop.TTI, g, mt)
    p.set_option("autotune", 1)
    rng = np.random.default_rng(21)
    x = dev(rng.standard_normal((nt, 1)))
    shot = prop.Shot(w.src_xyz, x, w.rec_xyz)
    Fx = p.forward(shot)
    xi = dev(rng.standard_normal((nt, len(w.rec_xyz))))
    y = (Fx * (xi.norm() / Fx.norm()) + xi).contiguous()
    FTy = p.adjoint(shot, y)
    a, b = prop.dot_f64(Fx, y), prop.dot_f64(x, FTy)
    assert abs(a - b) / abs(a) < 1e-5, (a, b)


def test_ttigrad256_finite_differences_five_directions(prop):
    """The 256^3 gradient workload (so 8, 2000 steps) against finite differences of the FP64 misfit
    J = 1/2 ||F(m) s - d_obs||^2 along five seeded smooth directions (seeds 100-104: N(0,1) smoothed
    with sigma 6, zero in the absorbing layers and above the receivers, max |dm| = 1e-2 max |m|), with
    steps h in {1, 1/2, 1/4}; FP16 storage: 48 checkpoints, and the whole run (n_ckpt = 1, 134 GB).
    Central differences: (J(m + h dm) - J(m - h dm)) / 2h -> <g, dm> with an O(h^2) error.  Taylor
    remainder R(h) = |J(m + h dm) - J(m) - h <g, dm>| = O(h^2): slope log2(R(h) / R(h/2)) near 2."""
    from paper_2004_10519_amd import configs, inputs
    w = configs.ttigrad()
    true = w.model_list()
    m0 = configs.ttigrad_starting_model(w)
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, v_ref=w.v_ref)
    tt = [dev(a) for a in true]
    p = prop.Propagator(prop.TTI, g, tt)
    p.set_option("autotune", 1)
    shot = prop.Shot(w.src_xyz, dev(w.wavelet()), w.rec_xyz)
    dobs = p.forward(shot).clone()
    base = [m0[k] for k in ("m", "eps", "delta", "theta", "phi")]
    aniso = [dev(a) for a in base[1:]]

    def J(mm):
        arrs = [dev(mm)] + aniso
        p.set_model(arrs)
        r = (p.forward(shot) - dobs).contiguous()
        return 0.5 * prop.dot_f64(r, r), r, arrs

    j0, res, keep = J(base[0])
    grads = {n: host(p.gradient(shot, res, n_ckpt=n, ckpt_dtype="f16")).astype(np.float64) for n in (48, 1)}
    rows = []
    for seed in range(100, 105):
        dm = inputs.random_unit_field(w.arr_shape, seed, 6.0).astype(np.float64)
        dm[: w.nbl + 4] = 0.0                   # zero above the receivers and in the top layer
        dm[-w.nbl:] = 0.0
        dm[:, :w.nbl] = 0.0
        dm[:, -w.nbl:] = 0.0
        dm[:, :, :w.nbl] = 0.0
        dm[:, :, -w.nbl:] = 0.0
        dm *= 1e-2 * np.abs(base[0]).max() / np.abs(dm).max()
        jp, jm = {}, {}
        for hh in (1.0, 0.5, 0.25):
            jp[hh] = J((base[0] + hh * dm).astype(np.float32))[0]
            jm[hh] = J((base[0] - hh * dm).astype(np.float32))[0]
        for n, gr in grads.items():
            gd = float(np.vdot(gr, dm))
            fd = {hh: (jp[hh] - jm[hh]) / (2 * hh) for hh in jp}
            rem = {hh: abs(jp[hh] - j0 - hh * gd) for hh in jp}
            slopes = [math.log2(rem[a] / rem[a / 2]) for a in (1.0, 0.5)]
            rows.append((seed, n, gd, fd, slopes))
    # a direction nearly orthogonal to the gradient has a directional derivative below the FP32
    # noise of the misfit differences, so every error is taken against the scale of the directional
    # derivatives (the largest |<g, dm>| of the five directions)
    scale = max(abs(r[2]) for r in rows)
    for seed, n, gd, fd, slopes in rows:
        err = {hh: abs(v - gd) / scale for hh, v in fd.items()}
        print(f"256^3 seed {seed} n_ckpt {n}: <g,dm> {gd:.6e}; central FD error / max|<g,dm>| "
              + ", ".join(f"h={hh}: {e:.2e}" for hh, e in err.items())
              + f"; Taylor slopes {slopes[0]:.2f}, {slopes[1]:.2f}")
    for seed, n, gd, fd, slopes in rows:
        err = {hh: abs(v - gd) / scale for hh, v in fd.items()}
        assert min(err.values()) < 1e-3, (seed, n, err)
        assert 1.8 < slopes[0] < 2.2 and 1.8 < slopes[1] < 2.2, (seed, n, slopes)


def test_el2d_marine_free_surface_vs_checker(prop, orc):
    """Full shape of the 2D marine workload, first 800 steps (0.72 s: the direct wave and its surface
    ghost, the sea-bed reflection back near the surface, the transmitted waves at the sea bed):
    traces of both receiver lines and the final fields against the checker, for the workload's image
    free surface and for the vacuum form; the image rows hold odd copies of tau_zz, the surface row
    none, the vacuum rows no normal stress."""
    import dataclasses
    from paper_2004_10519_amd import configs
    w0 = configs.el2d_marine(nt=800)
    assert w0.free_surface == "image"
    for mode in ("image", True):
        _marine_vs_checker(prop, orc, dataclasses.replace(w0, free_surface=mode))


def _marine_vs_checker(prop, orc, w):
    m = w.make_model()
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, v_ref=w.v_ref,
                  free_surface=w.free_surface)
    mt = [dev(m[k]) for k in ("vp", "vs", "rho")]
    p = prop.Propagator(prop.ELASTIC, g, mt)
    shot = prop.Shot(w.src_xyz, dev(w.wavelet()), w.rec_xyz, w.rec_kind)
    d = host(p.forward(shot))
    fields = [host(p.read_state(i)) for i in range(9)]
    og = orc.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, vref=w.v_ref,
                  free_surface=w.free_surface)
    mod = orc.ElasticModel.from_velocities(og, m["vp"], m["vs"], m["rho"])
    do, fo = orc.elastic_forward(og, mod, w.src_xyz, w.wavelet(), w.rec_xyz, w.rec_kind)
    npr = int((w.rec_kind == 0).sum())
    for name, sl in (("pressure", slice(0, npr)), ("vz", slice(npr, None))):
        err = rel_l2(d[:, sl], do[:, sl])
        print(f"el2d_marine ({w.free_surface}) {name} traces rel-L2 {err:.2e}")
        assert np.abs(do[:, sl]).max() > 0 and err <= 1e-4, (name, err)
    for i in (0, 2, 3, 5, 7):   # vx, vz, txx, tzz, txz (2D)
        assert rel_l2(fields[i], fo[i]) <= 1e-4, i
    nb = w.nbl
    if w.free_surface == "image":
        assert not fields[3][:nb + 1].any() and not fields[5][nb].any()
        assert np.array_equal(fields[5][nb - 3], -fields[5][nb + 3])
    else:
        for c in (3, 5):
            assert not fields[c][:nb].any()


def _golden_module():
    import importlib.util
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    spec = importlib.util.spec_from_file_location("mk128", os.path.join(here, "golden", "make_parity128.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    return mk, os.path.join(here, "golden")


@pytest.mark.parametrize("kind", ["tti", "elastic"])
def test_parity128_full_length_vs_checker(prop, kind):
    """The benchmark recipes at 128^3 over their full lengths (TTI so12, 3000 steps; elastic so8, 2000
    steps), in the benchmark's launch configuration (library default scheme, autotuned tiles), against
    the FP64 checker's stored results (tests/golden/make_parity128.py): every 4th sample of every
    trace (rel-L2 1e-4), and the wavefields on the three central planes after MID steps (the wave
    still in the grid) and at the end (by then the absorbing layers have taken most of the energy, so
    each plane's error is measured against its norm after MID steps).
    Bar per plane: 1e-4 of that norm, or, for TTI, 4 times the departure that storing the levels in
    FP32 alone causes in the checker, if larger: q's equation has near-zero-frequency modes (fields
    nearly constant along the symmetry axis, where Hz vanishes) that integrate rounding noise instead
    of propagating it away, so after 400 steps FP32 storage alone moves q by 1.7-3.8e-4 (p by 3e-5)."""
    import dataclasses
    import os
    mk, gdir = _golden_module()
    w = mk.tti_case() if kind == "tti" else mk.elastic_case()
    gold = np.load(os.path.join(gdir, "tti128_so12.npz" if kind == "tti" else "el128_so8.npz"))
    m = w.make_model()
    keys = ("m", "eps", "delta", "theta", "phi") if kind == "tti" else ("vp", "vs", "rho")
    mt = [dev(m[k]) for k in keys]
    names = ("p", "q") if kind == "tti" else mk.EL_FIELDS

    def run(nt):
        g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=nt, v_ref=w.v_ref)
        p = prop.Propagator(prop.TTI if kind == "tti" else prop.ELASTIC, g, mt)
        if kind == "tti":
            p.set_option("autotune", 1)
        ws = dataclasses.replace(w, nt=nt)
        shot = prop.Shot(w.src_xyz, dev(ws.wavelet()), w.rec_xyz, w.rec_kind)
        d = host(p.forward(shot)).copy()
        nz, ny, nx = g.arr_shape
        pl = {}
        for i, name in enumerate(names):
            f = host(p.read_state(i))
            pl.update({f"{name}_xz": f[:, ny // 2, :], f"{name}_yz": f[:, :, nx // 2], f"{name}_xy": f[nz // 2, :, :]})
        p.close()
        return d, pl

    d, final = run(w.nt)
    _, mid = run(int(gold["mid"]))
    err = rel_l2(d[::int(gold["tsub"])], gold["traces"])
    print(f"{kind} 128^3: traces rel-L2 {err:.2e}")
    assert err <= 1e-4, err
    bad = []
    for when, got in (("mid_", mid), ("", final)):
        for k, v in got.items():
            scale = np.linalg.norm(gold[f"mid_{k}"].astype(np.float64))
            if scale == 0:
                continue
            ref = gold[f"{when}{k}"].astype(np.float64)
            e = np.linalg.norm(v - ref)
            bound = 1e-4 * scale
            fp32 = f"fp32store_{when}{k}"
            if fp32 in gold.files:
                bound = max(bound, 4 * np.linalg.norm(gold[fp32].astype(np.float64) - ref))
            print(f"  {when or 'end_'}{k}: error {e / scale:.2e} of the plane's norm (bound {bound / scale:.2e})")
            if e > bound:
                bad.append((when or "end", k, e / scale, bound / scale))
    assert not bad, bad
