"""Oracle against the textbook 3D acoustic Green's function (no GPU).

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
