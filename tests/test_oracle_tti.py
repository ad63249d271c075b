"""Pins of the oracle's TTI operators and time stepping (no GPU).

* rotation algebra: H0 + Hz = -sum_a D_a^T D_a for any tilt/azimuth fields (the rotation is
  orthonormal pointwise), H0 and Hz symmetric negative semidefinite;
* the literal -D_i^T D_i form equals the projector form div((I - n n^T) grad) computed
  independently from D alone;
* plane-wave symbol: the step's operator equals -C diag(A~, B~) on cos(k.x) in the interior,
  with A~, B~ from the discrete Fourier symbol of the stencils (pins the placement of
  1+2eps and sqrt(1+2delta) and the mix-first order of the adjoint);
* spatial order of H0, Hz on a Gaussian bump against analytic second derivatives;
* TTI(eps = delta = 0, any angles) reduces to an independent acoustic stepper;
* symmetries (tilt 90 deg = x/z swap; tilt -> -tilt = x mirror); kinematics (horizontal
  speed vp sqrt(1+2 eps)); time-step bound versus power iteration.
"""
import math

import numpy as np
import pytest

from paper_2004_10519_amd import inputs


def _angles(g, seed):
    rng = np.random.default_rng(seed)
    th = rng.uniform(-1.2, 1.2, g.arr_shape)
    ph = rng.uniform(-3, 3, g.arr_shape) if g.ndim == 3 else np.zeros(g.arr_shape)
    return th, ph


@pytest.mark.parametrize("shape", [(9, 8, 7), (13, 1, 11)])
@pytest.mark.parametrize("so", [4, 8])
def test_rotation_invariance_and_symmetry(orc, shape, so):
    g = orc.Grid(shape, (10.0, 12.0, 8.0), space_order=so)
    th, ph = _angles(g, 1)
    rng = np.random.default_rng(2)
    u = rng.standard_normal(g.arr_shape)
    v = rng.standard_normal(g.arr_shape)
    H0u, Hzu = orc.tti_H(g, th, ph, u, 0), orc.tti_H(g, th, ph, u, 1)
    lap = sum(-orc.dcen(g, ax, orc.dcen(g, ax, u), transpose=True) for ax in g.axes())
    assert np.abs(H0u + Hzu - lap).max() <= 1e-13 * np.abs(lap).max()
    for grp, Hu in ((0, H0u), (1, Hzu)):
        Hv = orc.tti_H(g, th, ph, v, grp)
        assert abs(np.vdot(Hu, v) - np.vdot(u, Hv)) <= 1e-13 * np.abs(Hu).sum() * np.abs(v).max()
        assert np.vdot(Hu, u) <= 1e-12 * abs(np.vdot(lap, u))


@pytest.mark.parametrize("shape", [(9, 8, 7), (13, 1, 11)])
def test_literal_form_equals_projector_form(orc, shape):
    g = orc.Grid(shape, (10.0, 12.0, 8.0), space_order=8)
    th, ph = _angles(g, 3)
    f = np.random.default_rng(4).standard_normal(g.arr_shape)
    if g.ndim == 3:
        n = [np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)]
    else:
        n = [np.sin(th), None, np.cos(th)]
    grad = {ax: orc.dcen(g, ax, f) for ax in g.axes()}
    w = sum(n[ax] * grad[ax] for ax in g.axes())
    H0 = sum(orc.dcen(g, ax, grad[ax] - n[ax] * w) for ax in g.axes())
    Hz = sum(orc.dcen(g, ax, n[ax] * w) for ax in g.axes())
    s = np.abs(H0).max()
    assert np.abs(orc.tti_H(g, th, ph, f, 0) - H0).max() <= 1e-13 * s
    assert np.abs(orc.tti_H(g, th, ph, f, 1) - Hz).max() <= 1e-13 * s


def _symbol(orc, so, k, h):
    a = [float(x) for x in orc.fd_centered(so)]
    return 2.0 / h * sum(a[j] * math.sin((j + 1) * k * h) for j in range(len(a)))


@pytest.mark.parametrize("adjoint", [False, True])
@pytest.mark.parametrize("ndim", [2, 3])
def test_step_operator_plane_wave_symbol(orc, adjoint, ndim):
    so = 8
    shape = (40, 1, 36) if ndim == 2 else (28, 26, 24)
    h = (10.0, 9.0, 8.0)
    g = orc.Grid(shape, h, space_order=so, dt=1e-3)
    eps, delta, th, ph = 0.22, 0.09, 0.5, (0.7 if ndim == 3 else 0.0)
    k = np.array([0.021, 0.017 if ndim == 3 else 0.0, 0.029])
    nz, ny, nx = g.arr_shape
    Z, Y, X = np.meshgrid(np.arange(nz) * h[2], np.arange(ny) * h[1], np.arange(nx) * h[0], indexing="ij")
    phase = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    P, Q = 0.8, -1.3
    m = np.full(g.arr_shape, 1 / 2000.0 ** 2)
    mod = orc.TTIModel.from_arrays(g, m, np.full(g.arr_shape, eps), np.full(g.arr_shape, delta),
                                   np.full(g.arr_shape, th), np.full(g.arr_shape, ph))
    p, q = P * phase, Q * phase
    pn, qn = orc._tti_step(g, mod, np.zeros(g.arr_shape), adjoint, p, q, 2 * p, 2 * q)
    Lp, Lq = pn * m / g.dt ** 2, qn * m / g.dt ** 2
    kt = np.array([_symbol(orc, so, k[0], h[0]), _symbol(orc, so, k[1], h[1]) if ndim == 3 else 0.0,
                   _symbol(orc, so, k[2], h[2])])
    n = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
    Bt = float(n @ kt) ** 2
    At = float(kt @ kt) - Bt
    A, B = 1 + 2 * eps, math.sqrt(1 + 2 * delta)
    if not adjoint:
        ep, eq = -(A * At * P + B * Bt * Q), -(B * At * P + Bt * Q)
    else:
        ep, eq = -At * (A * P + B * Q), -Bt * (B * P + Q)
    r2 = so  # interior = at least 2r from every face
    sl = tuple(slice(r2, s - r2) if s > 1 else slice(None) for s in g.arr_shape)
    scale = abs(ep) + abs(eq)
    assert np.abs(Lp[sl] - ep * phase[sl]).max() <= 1e-10 * scale
    assert np.abs(Lq[sl] - eq * phase[sl]).max() <= 1e-10 * scale


@pytest.mark.parametrize("so", [4, 8])
def test_spatial_order_gaussian_bump(orc, so):
    """2D: H0 f and Hz f versus Delta f - n^T (grad grad f) n and n^T (grad grad f) n."""
    th = 0.6
    n = np.array([math.sin(th), math.cos(th)])
    errs = []
    for N in (41, 81):
        L = 400.0
        h = L / (N - 1)
        g = orc.Grid((N, 1, N), (h, 1.0, h), space_order=so)
        x = np.arange(N) * h
        Z, X = np.meshgrid(x, x, indexing="ij")
        c, s = L / 2, 30.0
        rx, rz = X - c, Z - c
        f = np.exp(-(rx ** 2 + rz ** 2) / (2 * s * s))
        fxx = f * (rx * rx / s ** 4 - 1 / s ** 2)
        fzz = f * (rz * rz / s ** 4 - 1 / s ** 2)
        fxz = f * (rx * rz / s ** 4)
        nHn = n[0] ** 2 * fxx + 2 * n[0] * n[1] * fxz + n[1] ** 2 * fzz
        thf = np.full(g.arr_shape, th)
        H0 = orc.tti_H(g, thf, np.zeros(g.arr_shape), f.reshape(g.arr_shape), 0).reshape(N, N)
        Hz = orc.tti_H(g, thf, np.zeros(g.arr_shape), f.reshape(g.arr_shape), 1).reshape(N, N)
        b = 2 * so  # stay clear of the truncated faces
        inner = (slice(b, N - b), slice(b, N - b))
        errs.append(max(np.abs(H0 - (fxx + fzz - nHn))[inner].max(), np.abs(Hz - nHn)[inner].max()))
    rate = math.log(errs[0] / errs[1]) / math.log(80 / 40)
    assert abs(rate - so) < 0.6, (errs, rate)


def _tti_setup(orc, shape, so, nbl, dt, nt, seed, iso=False):
    h = (10.0, 10.0, 10.0)
    g = orc.Grid(shape, h, space_order=so, nbl=nbl, dt=dt, nt=nt, vref=1500.0)
    mdl = inputs.tti_model(shape, nbl, seed)
    m = inputs.slowness_squared(mdl["vp"])
    if iso:
        mdl["eps"][:] = 0.0
        mdl["delta"][:] = 0.0
    mod = orc.TTIModel.from_arrays(g, m, mdl["eps"], mdl["delta"], mdl["theta"], mdl["phi"])
    nx, ny, nz = shape
    if g.ndim == 3:
        src = np.array([[h[0] * (nx // 2 + 0.3), h[1] * (ny // 2 - 0.2), h[2] * (nz // 2 + 0.4)]])
        rec = np.array([[h[0] * (2.5 + i), h[1] * (ny / 2 + 0.7 * i - 3), h[2] * 2.3] for i in range(nx - 5)])
    else:
        src = np.array([[h[0] * (nx // 2 + 0.3), h[2] * (nz // 2 + 0.4)]])
        rec = np.array([[h[0] * (1.5 + i), h[2] * 2.3] for i in range(nx - 3)])
    wav = inputs.ricker(25.0, dt, nt).astype(np.float64).reshape(nt, 1)
    return g, mod, src, wav, rec


@pytest.mark.parametrize("shape", [(30, 1, 28), (16, 15, 14)])
def test_isotropic_reduction_to_acoustic(orc, shape):
    g, mod, src, wav, rec = _tti_setup(orc, shape, 8, 0, 1e-3, 60, 11, iso=True)
    d, (p, q, _, _), _ = orc.tti_forward(g, mod, src, wav, rec)
    da, ua = orc.acoustic_wide_forward(g, mod.m, src, wav, rec)
    assert np.abs(p - q).max() <= 1e-13 * np.abs(p).max()
    assert np.abs(d - da).max() <= 1e-12 * np.abs(da).max()
    assert np.abs(p - ua).max() <= 1e-12 * np.abs(ua).max()


def test_tilt_symmetries(orc):
    N = 41
    g = orc.Grid((N, 1, N), (10.0, 1.0, 10.0), space_order=8, nbl=6, dt=1e-3, nt=120, vref=2000.0)
    c = 10.0 * (N // 2)
    src = np.array([[c, c]])
    wav = inputs.ricker(20.0, g.dt, g.nt).astype(np.float64).reshape(-1, 1)
    m = np.full(g.arr_shape, 1 / 2000.0 ** 2)
    e, dl = np.full(g.arr_shape, 0.2), np.full(g.arr_shape, 0.1)

    def run(theta):
        mod = orc.TTIModel.from_arrays(g, m, e, dl, np.full(g.arr_shape, theta), np.zeros(g.arr_shape))
        _, (p, q, _, _), _ = orc.tti_forward(g, mod, src, wav, None)
        return p.reshape(N, N), q.reshape(N, N)

    p0, q0 = run(0.0)
    p90, q90 = run(math.pi / 2)
    s = np.abs(p0).max()
    assert np.abs(p90 - p0.T).max() <= 1e-11 * s
    assert np.abs(q90 - q0.T).max() <= 1e-11 * s
    pa, _ = run(0.4)
    pb, _ = run(-0.4)
    assert np.abs(pb - pa[:, ::-1]).max() <= 1e-11 * np.abs(pa).max()
    assert np.abs(pa - pa[:, ::-1]).max() > 1e-3 * np.abs(pa).max()  # the tilt does matter


@pytest.mark.slow
def test_kinematics_horizontal_speed(orc):
    """Constant medium, vertical symmetry axis: the qP front moves at vp along z and vp sqrt(1+2 eps)
    along x.  First-break lags between two receivers on each axis, within 3 dt."""
    N, h, vp, eps = 201, 5.0, 2000.0, 0.25
    g = orc.Grid((N, 1, N), (h, 1.0, h), space_order=8, nbl=0, dt=5e-4, nt=440, vref=vp)
    c = h * (N // 2)
    R1, R2 = 150.0, 350.0
    rec = np.array([[c + R1, c], [c + R2, c], [c, c + R1], [c, c + R2]])
    wav = inputs.ricker(25.0, g.dt, g.nt).astype(np.float64)
    # smooth source density (a point source also excites the fast checkerboard mode of the
    # composed centred stencil, which would pollute first breaks)
    ax = np.arange(N) * h - c
    Zg, Xg = np.meshgrid(ax, ax, indexing="ij")
    rho = np.exp(-(Xg ** 2 + Zg ** 2) / (2 * (2 * h) ** 2)).reshape(g.arr_shape)
    m = np.full(g.arr_shape, 1 / vp ** 2)
    mod = orc.TTIModel.from_arrays(g, m, np.full(g.arr_shape, eps), np.full(g.arr_shape, 0.1),
                                   np.zeros(g.arr_shape), np.zeros(g.arr_shape))
    d, _, _ = orc.tti_forward(g, mod, None, None, rec, force=lambda n: (rho * wav[n], rho * wav[n]))

    def first_break(a):
        # the qP wave arrives first; later energy includes the slow pseudo-acoustic shear artefact
        return np.argmax(np.abs(a) > 0.02 * np.abs(a).max()) * g.dt

    def lag(a, b):
        return first_break(b) - first_break(a)

    lx, lz = lag(d[:, 0], d[:, 1]), lag(d[:, 2], d[:, 3])
    assert abs(lz - (R2 - R1) / vp) <= 3 * g.dt
    assert abs(lx - (R2 - R1) / (vp * math.sqrt(1 + 2 * eps))) <= 3 * g.dt
    assert abs(lx - (R2 - R1) / vp) > 10 * g.dt  # an isotropic speed would fail


@pytest.mark.parametrize("ndim", [2, 3])
def test_time_step_bound_vs_power_iteration(orc, ndim):
    shape = (24, 1, 22) if ndim == 2 else (12, 11, 10)
    g = orc.Grid(shape, (10.0, 10.0, 10.0), space_order=8, dt=1e-3)
    mdl = inputs.tti_model(shape, 0, 21)
    m = inputs.slowness_squared(mdl["vp"]).astype(np.float64)
    mod = orc.TTIModel.from_arrays(g, m, mdl["eps"], mdl["delta"], mdl["theta"], mdl["phi"])
    rng = np.random.default_rng(5)
    p, q = rng.standard_normal(g.arr_shape), rng.standard_normal(g.arr_shape)
    lam = 0.0
    for _ in range(150):
        pn, qn = orc._tti_step(g, mod, np.zeros(g.arr_shape), False, p, q, 2 * p, 2 * q)
        Lp, Lq = pn * m / g.dt ** 2, qn * m / g.dt ** 2  # L(p, q)
        Ap, Aq = Lp / m, Lq / m                              # m^-1 L
        lam = math.sqrt(np.vdot(Ap, Ap) + np.vdot(Aq, Aq)) / math.sqrt(np.vdot(p, p) + np.vdot(q, q))
        p, q = Ap / lam, Aq / lam
    vmax = float(np.max(1 / np.sqrt(m)))
    dtmax = orc.tti_dt_max(g, vmax, float(mdl["eps"].max()))
    assert lam * dtmax ** 2 / 4 <= 1.0 + 1e-9, (lam * dtmax ** 2 / 4)
    assert lam * dtmax ** 2 / 4 > 0.3  # the bound is not vacuous
