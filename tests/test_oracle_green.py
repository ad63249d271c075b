"""Oracle against the textbook 3D and 2D acoustic Green's functions (no GPU).

TTI with eps = delta = theta = phi = 0 is the isotropic wave equation m u_tt - Delta u = f.
A Gaussian source density rho(x) s(t) (spatially smooth, so the checkerboard mode of the
composed centred stencil is not excited) gives the retarded-potential solution
    u(r, t) = c/(2r) int_0^inf rho(r') r' [S(t - |r - r'|/c) - S(t - (r + r')/c)] dr',
with S the antiderivative of the Ricker wavelet, S(t) = (t - t0) exp(-(pi f0 (t - t0))^2).
Trace sample n belongs to time (n+1) dt.  This pins amplitude, speed and the timing convention.
"""
import math

import numpy as np
import pytest


@pytest.mark.slow
def test_green_3d_gaussian_source(orc):
    N, h, vp, f0, dt, nt = 61, 10.0, 2000.0, 12.0, 1e-3, 260
    g = orc.Grid((N, N, N), (h, h, h), space_order=8, nbl=0, dt=dt, nt=nt, vref=vp)
    c = h * (N // 2)
    sig = 2.0 * h
    ax = np.arange(N) * h - c
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    rho = np.exp(-(X ** 2 + Y ** 2 + Z ** 2) / (2 * sig ** 2)) / ((2 * math.pi) ** 1.5 * sig ** 3)
    t0 = 1.0 / f0
    wav = (1 - 2 * (math.pi * f0 * (np.arange(nt) * dt - t0)) ** 2) * np.exp(-(math.pi * f0 * (np.arange(nt) * dt - t0)) ** 2)
    S = lambda t: (t - t0) * np.exp(-(math.pi * f0 * (t - t0)) ** 2)
    m = np.full(g.arr_shape, 1 / vp ** 2)
    zero = np.zeros(g.arr_shape)
    mod = orc.TTIModel.from_arrays(g, m, zero, zero, zero, zero)
    recs = np.array([[c + 150.0, c, c], [c, c + 120.0, c], [c, c, c + 170.0], [c + 100, c + 100, c]])
    d, _, _ = orc.tti_forward(g, mod, None, None, recs, force=lambda n: (rho * wav[n], rho * wav[n]))
    rp = np.linspace(0, 8 * sig, 3000)
    rhor = np.exp(-rp ** 2 / (2 * sig ** 2)) / ((2 * math.pi) ** 1.5 * sig ** 3)
    win = (np.arange(nt) + 1) * dt < 0.2  # before the first reflection from the truncated faces
    for k, rv in enumerate(np.linalg.norm(recs - c, axis=1)):
        errs = []
        for shift in (-1, 0, 1):
            t = (np.arange(nt) + 1 + shift) * dt
            ana = np.array([vp / (2 * rv) * np.trapezoid(rhor * rp * (S(tt - np.abs(rv - rp) / vp) - S(tt - (rv + rp) / vp)), rp)
                            for tt in t])
            errs.append(np.linalg.norm((d[:, k] - ana)[win]) / np.linalg.norm(ana[win]))
        assert errs[1] < 0.015, errs
        assert errs[0] > 4 * errs[1] and errs[2] > 4 * errs[1], errs


@pytest.mark.slow
def test_green_2d_gaussian_source(orc):
    """2D: the Green's function of m u_tt - Delta u = delta(x) delta(t) is
    G(R, tau) = H(tau - R/c) / (2 pi sqrt(tau^2 - R^2/c^2)).  For the Gaussian density
    rho(x) = exp(-|x|^2 / (2 sig^2)) / (2 pi sig^2), the angular integral over the source disc gives
    the kernel K(r, R) = exp(-(r - R)^2 / (2 sig^2)) I0e(r R / sig^2) / sig^2, and with R = c tau sin(a)
        g(r, tau) = int R K(r, R) G(R, tau) dR = c^2 tau / (2 pi) int_0^{pi/2} sin(a) K(r, c tau sin a) da,
    a smooth integrand.  The trace is then u(r, t) = int_0^t s(t - tau) g(r, tau) dtau with the
    wavelet starting at t = 0, and trace sample n belongs to time (n + 1) dt."""
    from scipy.special import i0e
    N, h, vp, f0, dt, nt = 241, 10.0, 2000.0, 12.0, 1e-3, 320
    g = orc.Grid((N, 1, N), (h, 1.0, h), space_order=8, nbl=0, dt=dt, nt=nt, vref=vp)
    c = h * (N // 2)
    sig = 2.0 * h
    ax = np.arange(N) * h - c
    Z, X = np.meshgrid(ax, ax, indexing="ij")
    rho = (np.exp(-(X ** 2 + Z ** 2) / (2 * sig ** 2)) / (2 * math.pi * sig ** 2))[:, None, :]
    t0 = 1.0 / f0
    s = lambda t: np.where(t >= 0, (1 - 2 * (math.pi * f0 * (t - t0)) ** 2) * np.exp(-(math.pi * f0 * (t - t0)) ** 2), 0.0)
    wav = s(np.arange(nt) * dt)
    m = np.full(g.arr_shape, 1 / vp ** 2)
    zero = np.zeros(g.arr_shape)
    mod = orc.TTIModel.from_arrays(g, m, zero, zero, zero, zero)
    recs = np.array([[c + 150.0, c], [c, c + 230.0], [c - 120.0, c + 120.0]])
    d, _, _ = orc.tti_forward(g, mod, None, None, recs, force=lambda n: (rho * wav[n], rho * wav[n]))
    dtau = dt / 16
    tau = np.arange(1, int((nt + 2) * dt / dtau) + 1) * dtau
    al = np.linspace(0.0, math.pi / 2, 801)
    win = (np.arange(nt) + 1) * dt < 0.3   # before the first reflection from the truncated faces
    for k, rv in enumerate(np.linalg.norm(recs - c, axis=1)):
        R = vp * tau[:, None] * np.sin(al)[None, :]
        K = np.exp(-(rv - R) ** 2 / (2 * sig ** 2)) * i0e(rv * R / sig ** 2) / sig ** 2
        gk = vp ** 2 * tau / (2 * math.pi) * np.trapezoid(np.sin(al)[None, :] * K, al, axis=1)
        errs = []
        for shift in (-1, 0, 1):
            t = (np.arange(nt) + 1 + shift) * dt
            ana = np.array([np.trapezoid(s(tt - tau) * gk, tau) for tt in t])
            errs.append(np.linalg.norm((d[:, k] - ana)[win]) / np.linalg.norm(ana[win]))
        assert errs[1] < 0.006, errs   # measured 0.16-0.24 %
        assert errs[0] > 10 * errs[1] and errs[2] > 10 * errs[1], errs
