"""Write tests/golden/ttigrad64.npz: the FP64 checker's TTI gradient at 64^3 (C3 recipe scaled down).

Calls only oracle/ and the seeded input generators.  Case: 64^3 grid, 12.5 m, space order 8,
10-point absorbing layers, 2000 steps of 1.116 ms, smoothed starting model of the seed-3 layered
TTI model, source at the centre 4 points below the layer, 32 x 32 receivers 2 points below it,
15 Hz Ricker; the adjoint is driven by a seeded band-limited residual (the gradient is linear in
the residual, so a data-like residual exercises the same arithmetic as d - d_obs).
Run: python tests/golden/make_ttigrad64.py   (a few minutes, ~9 GB of host memory)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2004_10519_amd import configs, inputs  # noqa: E402


def case():
    w = configs.ttigrad(n=64, nt=2000, nbl=10, nrec=32, seed=3)
    m0 = configs.ttigrad_starting_model(w)
    rng = np.random.default_rng(2024)
    wn = rng.standard_normal((w.nt, len(w.rec_xyz)))
    k = inputs.ricker(15.0, w.dt, 121, t0=60 * w.dt).astype(np.float64)
    res = np.stack([np.convolve(wn[:, i], k, mode="same") for i in range(wn.shape[1])], axis=1).astype(np.float32)
    return w, m0, res


def main():
    w, m0, res = case()
    g = oracle.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, vref=w.v_ref)
    mod = oracle.TTIModel.from_arrays(g, m0["m"], m0["eps"], m0["delta"], m0["theta"], m0["phi"])
    d, _, _ = oracle.tti_forward(g, mod, w.src_xyz, w.wavelet(), w.rec_xyz)
    _, grad, _ = oracle.tti_gradient(g, mod, w.src_xyz, w.wavelet(), w.rec_xyz, d - res)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ttigrad64.npz")
    np.savez_compressed(out, grad=grad.astype(np.float32), nt=w.nt, seed=3,
                        note="FP64 checker gradient, see make_ttigrad64.py")
    print(out, float(np.abs(grad).max()))


if __name__ == "__main__":
    main()
