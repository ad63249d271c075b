"""Adjoint and gradient pins of the oracle (no GPU).

* dot tests |<Fx, y> - <x, F^T y>| / |<Fx, y>| < 1e-12 in FP64 for the user map
  (wavelet -> traces) and for a dense space-time map (forcing at every point and step ->
  every state), with absorbing layers, so boundaries and damping are probed;
* negative control: the forward operator used as its own adjoint fails, because the TTI
  operator is not self-adjoint;
* gradient with respect to m: Taylor test (second-order remainder) and central finite
  differences along random directions.
"""
import numpy as np
import pytest

from paper_2004_10519_amd import inputs


def _tti_case(orc, shape, nbl=3, nt=40, seed=7, so=8):
    h = (10.0, 11.0, 9.0)
    g = orc.Grid(shape, h, space_order=so, nbl=nbl, dt=1e-3, nt=nt, vref=1800.0)
    mdl = inputs.tti_model(shape, nbl, seed)
    mod = orc.TTIModel.from_arrays(g, inputs.slowness_squared(mdl["vp"]), mdl["eps"], mdl["delta"],
                                   mdl["theta"], mdl["phi"])
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    if g.ndim == 3:
        src = np.array([[h[0] * (nx / 2 + 0.3), h[1] * (ny / 2 - 0.4), h[2] * (nz / 2 + 0.2)],
                        [h[0] * 2.6, h[1] * 3.1, h[2] * (nz - 1.5)]])
        rec = np.stack([rng.uniform(0, (nx - 1) * h[0], 9), rng.uniform(0, (ny - 1) * h[1], 9),
                        rng.uniform(0, (nz - 1) * h[2], 9)], axis=1)
    else:
        src = np.array([[h[0] * (nx / 2 + 0.3), h[2] * (nz / 2 + 0.2)], [h[0] * 1.4, h[2] * 2.6]])
        rec = np.stack([rng.uniform(0, (nx - 1) * h[0], 7), rng.uniform(0, (nz - 1) * h[2], 7)], axis=1)
        rec[0] = [(nx - 1) * h[0], (nz - 1) * h[2]]  # last-node clamp
    return g, mod, src, rec


@pytest.mark.parametrize("shape", [(20, 1, 18), (11, 10, 9)])
def test_tti_dot_user_map(orc, shape):
    g, mod, src, rec = _tti_case(orc, shape)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((g.nt, len(src)))
    y = rng.standard_normal((g.nt, len(rec)))
    Fx, _, _ = orc.tti_forward(g, mod, src, x, rec)
    FTy, _ = orc.tti_adjoint(g, mod, src, rec, y)
    lhs, rhs = np.vdot(Fx, y), np.vdot(x, FTy)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


@pytest.mark.parametrize("shape", [(16, 1, 14), (9, 8, 7)])
def test_tti_dot_dense_map_and_negative_control(orc, shape, monkeypatch):
    g, mod, _, _ = _tti_case(orc, shape, nt=12)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((g.nt, 2) + g.arr_shape)
    Y = rng.standard_normal((g.nt, 2) + g.arr_shape)
    out = np.zeros_like(X)
    orc.tti_forward(g, mod, None, None, None, force=lambda n: (X[n, 0], X[n, 1]),
                    callback=lambda n, p, q: out.__setitem__(n, np.stack([p, q])))
    adj = np.zeros_like(Y)
    orc.tti_adjoint(g, mod, None, None, None, force=lambda n: (Y[n, 0], Y[n, 1]),
                    callback=lambda k, p, q: adj.__setitem__(k - 1, np.stack([p, q])))
    lhs, rhs = np.vdot(out, Y), np.vdot(X, adj)
    assert abs(lhs - rhs) / abs(lhs) < 1e-12
    # negative control: use the forward operator in the backward recursion
    step = orc._tti_step
    monkeypatch.setattr(orc, "_tti_step", lambda g_, m_, e_, adjoint, *a: step(g_, m_, e_, False, *a))
    adj2 = np.zeros_like(Y)
    orc.tti_adjoint(g, mod, None, None, None, force=lambda n: (Y[n, 0], Y[n, 1]),
                    callback=lambda k, p, q: adj2.__setitem__(k - 1, np.stack([p, q])))
    assert abs(lhs - np.vdot(X, adj2)) / abs(lhs) > 1e-6


def _J(orc, g, mod, src, wav, rec, dobs):
    d, _, _ = orc.tti_forward(g, mod, src, wav, rec)
    r = d - dobs
    return 0.5 * float(np.sum(r * r))


@pytest.mark.parametrize("shape", [(24, 1, 22), (10, 9, 12)])
def test_tti_gradient_taylor_and_fd(orc, shape):
    g, mod, src, rec = _tti_case(orc, shape, nbl=4, nt=60, seed=9)
    wav = inputs.ricker(30.0, g.dt, g.nt).astype(np.float64)[:, None].repeat(len(src), axis=1)
    # observed data from a perturbed "true" model
    true = orc.TTIModel(mod.m * (1 + 0.05 * inputs.random_unit_field(g.arr_shape, 3, 2.0)), mod.eps,
                        mod.delta, mod.theta, mod.phi)
    dobs, _, _ = orc.tti_forward(g, true, src, wav, rec)
    J0, grad, _ = orc.tti_gradient(g, mod, src, wav, rec, dobs)
    for seed in (100, 101):
        dm = inputs.random_unit_field(g.arr_shape, seed, 1.5).astype(np.float64)
        dm *= 1e-2 * np.abs(mod.m).max() / np.abs(dm).max()
        gd = float(np.vdot(grad, dm))
        res = []
        for hh in (1.0, 0.5, 0.25):
            mp = orc.TTIModel(mod.m + hh * dm, mod.eps, mod.delta, mod.theta, mod.phi)
            res.append(abs(_J(orc, g, mp, src, wav, rec, dobs) - J0 - hh * gd))
        assert res[0] / res[1] > 3.5 and res[1] / res[2] > 3.5, res  # O(h^2) remainder
        hh = 0.01
        jp = _J(orc, g, orc.TTIModel(mod.m + hh * dm, mod.eps, mod.delta, mod.theta, mod.phi), src, wav, rec, dobs)
        jm = _J(orc, g, orc.TTIModel(mod.m - hh * dm, mod.eps, mod.delta, mod.theta, mod.phi), src, wav, rec, dobs)
        fd = (jp - jm) / (2 * hh)
        assert abs(fd - gd) / abs(gd) < 1e-5, (fd, gd)


@pytest.mark.parametrize("shape", [(22, 1, 20), (10, 9, 11)])
def test_tti_image_of_second_difference_is_the_gradient(orc, shape):
    """The adjoint recursion is time-invariant, so driving it with the second difference of the data,
    d[n] - 2 d[n+1] + d[n+2], gives the second difference of the adjoint state.  Hence the zero-lag
    image of that data equals -dt^2 times the gradient for residual d (summation by parts; f^0 = 0 and
    y^{N+1} = y^{N+2} = 0).  A shifted pairing of f^k with y^{k+-1} breaks this."""
    g, mod, src, rec = _tti_case(orc, shape, nbl=3, nt=45, seed=4)
    wav = inputs.ricker(30.0, g.dt, g.nt).astype(np.float64)[:, None].repeat(len(src), axis=1)
    rng = np.random.default_rng(12)
    d = rng.standard_normal((g.nt, len(rec)))
    d2 = d.copy()
    d2[:-1] -= 2 * d[1:]
    d2[:-2] += d[2:]
    img = orc.tti_image(g, mod, src, wav, rec, d2)
    traces, _, _ = orc.tti_forward(g, mod, src, wav, rec)
    _, grad, _ = orc.tti_gradient(g, mod, src, wav, rec, traces - d)
    assert np.linalg.norm(img + g.dt ** 2 * grad) <= 1e-11 * np.linalg.norm(img)


def test_tti_image_one_step_closed_form(orc):
    """N = 1: f^1 = P_s^T s^0 / a in p and q, y^1 = P_r^T d^0 / a in p only, so I = f_p^1 y_p^1 with
    a = m/dt^2 + eta/(2 dt)."""
    g, mod, src, rec = _tti_case(orc, (12, 10, 9), nbl=2, nt=1, seed=6)
    rec = np.concatenate([src + np.array([[3.0, -2.0, 1.5]]), rec])   # receivers beside the sources
    wav = np.array([[1.7, -0.6]])
    d = np.array([np.linspace(-1.0, 2.0, len(rec))])
    img = orc.tti_image(g, mod, src, wav, rec, d)
    a = mod.m / g.dt ** 2 + orc.tti_eta(g) / (2 * g.dt)
    fs, fr = np.zeros(g.arr_shape), np.zeros(g.arr_shape)
    orc.inject(orc.sparse_setup(g, src), fs, wav[0])
    orc.inject(orc.sparse_setup(g, rec), fr, d[0])
    expect = (fs / a) * (fr / a)
    assert np.abs(expect).max() > 0
    assert np.allclose(img, expect, rtol=1e-13, atol=1e-13 * np.abs(expect).max())
