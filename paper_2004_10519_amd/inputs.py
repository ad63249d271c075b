"""Seeded synthetic inputs shared by the propagator library's tests and benchmarks.

This module only *makes inputs*: earth models, source wavelets and acquisition
geometry.  It holds none of the propagators' arithmetic (no finite
differences, no damping, no time stepping), so both the HIP library and the
FP64 checker can consume exactly the same FP32 arrays.

Recipe (the paper's workloads use an SEG/EAGE-derived TTI model, Marmousi-ii
and a SEAM-like model, none of which is available; these seeded stand-ins have
the same kind of structure and value ranges):

* layered P velocity, 10 flat layers, 1.5 km/s at the top to 4.5 km/s at the
  bottom, interface depths drawn uniformly in the physical part of the model,
  times (1 + 5 % x smooth noise);
* Thomsen epsilon in [0, 0.3] (smooth noise), delta = epsilon / 2 so that
  epsilon >= delta everywhere (the pseudo-acoustic system is only stable
  when epsilon >= delta);
* tilt and azimuth in [-45, 45] degrees (smooth noise), in radians;
* elastic: vs = vp / 1.8 except vs = 0 in the water (top) layer, density from
  Gardner's relation rho = 310 vp^0.25 (kg/m^3, vp in m/s);
* Ricker wavelet with peak at t0 = 1/f0.

Arrays follow the library's layout: shape (nz, ny, nx), x fastest, FP32.
Generation happens in FP64 and is rounded to FP32 once at the end (the fast
recipe for very large TTI models, ``tti_model(parallel=k)``, draws and smooths
its noise in FP32 on k threads).
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.ndimage as ndi

__all__ = [
    "ricker", "tti_model", "elastic_model", "smooth", "slowness_squared",
    "surface_receivers", "random_unit_field",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def ricker(f0: float, dt: float, nt: int, t0: float | None = None) -> np.ndarray:
    """Ricker wavelet sampled at t = n*dt, n = 0..nt-1, peak 1 at t0 (default 1/f0)."""
    if t0 is None:
        t0 = 1.0 / f0
    t = np.arange(nt, dtype=np.float64) * dt - t0
    a = (math.pi * f0 * t) ** 2
    return ((1.0 - 2.0 * a) * np.exp(-a)).astype(np.float32)


def smooth(field: np.ndarray, sigma: float, threads: int = 8, dtype=np.float64) -> np.ndarray:
    """Gaussian smoothing (sigma in grid points, kernel truncated at 3 sigma, reflecting edges).

    ``dtype`` in (FP64 by default), the same out.  The filter is separable: one 1D pass per axis, in
    axis order, exactly as ``scipy.ndimage.gaussian_filter`` does it; each pass is split into slabs
    along another axis and run on ``threads`` threads, which gives the same bits as the
    single-threaded filter.
    """
    a = np.asarray(field, dtype=dtype)
    if sigma <= 0:
        return a
    for ax in range(a.ndim):
        if a.shape[ax] == 1:
            a = ndi.gaussian_filter1d(a, sigma, axis=ax, truncate=3.0, mode="reflect")
            continue
        split = max((d for d in range(a.ndim) if d != ax), key=lambda d: a.shape[d], default=None)
        n = a.shape[split] if split is not None else 1
        nth = max(1, min(threads, n, a.size // (1 << 20)))
        if nth == 1:
            a = ndi.gaussian_filter1d(a, sigma, axis=ax, truncate=3.0, mode="reflect")
            continue
        out = np.empty_like(a)

        def run(c, a=a, ax=ax, split=split, n=n, nth=nth, out=out):
            sl = [slice(None)] * a.ndim
            sl[split] = slice(c * n // nth, (c + 1) * n // nth)
            sl = tuple(sl)
            out[sl] = ndi.gaussian_filter1d(a[sl], sigma, axis=ax, truncate=3.0, mode="reflect")

        with ThreadPoolExecutor(nth) as ex:
            list(ex.map(run, range(nth)))
        a = out
    return a


def _minmax(a: np.ndarray, lo: float, hi: float) -> np.ndarray:
    amin, amax = float(a.min()), float(a.max())
    if amax <= amin:
        return np.full_like(a, 0.5 * (lo + hi))
    return lo + (hi - lo) * (a - amin) / (amax - amin)


def _smooth_noise(shape, sigma, rng) -> np.ndarray:
    """N(0,1) noise drawn in a fixed order, returned unsmoothed (smoothing is done in parallel later)."""
    return rng.standard_normal(shape)


def _parallel_noise(shape, seq: np.random.SeedSequence, threads: int) -> np.ndarray:
    """FP32 N(0,1) noise, one independent PCG64 stream per z-slab (children of ``seq``), drawn on
    ``threads`` threads: the same bits for any thread count."""
    out = np.empty(shape, dtype=np.float32)
    nz = shape[0]
    nslab = min(nz, 64)
    kids = seq.spawn(nslab)

    def run(c):
        sl = slice(c * nz // nslab, (c + 1) * nz // nslab)
        np.random.Generator(np.random.PCG64(kids[c])).standard_normal(out=out[sl], dtype=np.float32)

    with ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(nslab)))
    return out


def _layer_index(nz: int, nbl: int, seed_rng: np.random.Generator, nlayers: int) -> np.ndarray:
    """Layer number (0..nlayers-1) of every depth index 0..nz-1."""
    nz_phys = max(nz - 2 * nbl, 1)
    depths = np.sort(seed_rng.uniform(0.1, 0.95, nlayers - 1)) * nz_phys + nbl
    k = np.arange(nz, dtype=np.float64)
    return np.searchsorted(depths, k, side="right")


def tti_model(shape_xyz, nbl: int, seed: int, nlayers: int = 10, vmin: float = 1500.0,
              vmax: float = 4500.0, pert: float = 0.05, eps_max: float = 0.3,
              angle_max_deg: float = 45.0, progress=None, parallel: int = 0) -> dict:
    """Seeded TTI model: dict of FP32 arrays vp (m/s), eps, delta, theta, phi (rad), shape (nz, ny, nx).

    For 2D grids pass ny = 1; phi is then zero.  ``progress``, if given, is called with a short
    message after each generation stage (large models take minutes).

    ``parallel`` > 0 selects the fast recipe for very large models, run on that many threads: the
    same distributions, but the noise comes from independent streams spawned from the seed (one per
    z-slab) and is drawn and smoothed in FP32, so its values differ from the default recipe's.
    """
    say = progress if progress is not None else (lambda msg: None)
    nx, ny, nz = (int(s) for s in shape_xyz)
    shp = (nz, ny, nx)
    sigmas = (4.0, 8.0, 8.0, 8.0)
    if parallel > 0:
        seq_layers, *seq_noise = np.random.SeedSequence(seed).spawn(1 + len(sigmas))
        layer = _layer_index(nz, nbl, np.random.Generator(np.random.PCG64(seq_layers)), nlayers)
        noises = [_parallel_noise(shp, q, parallel) for q in seq_noise]
    else:
        rng = _rng(seed)
        layer = _layer_index(nz, nbl, rng, nlayers)
        noises = [_smooth_noise(shp, s, rng) for s in sigmas]
    v_layer = vmin + (vmax - vmin) * layer / (nlayers - 1)
    say("noise drawn")
    sm = []
    for i, sig in enumerate(sigmas):
        if parallel > 0:
            sm.append(smooth(noises[i], sig, threads=parallel, dtype=np.float32))
        else:
            sm.append(smooth(noises[i], sig))
        noises[i] = None
        say(f"field {i + 1}/4 smoothed")
    amax = math.radians(angle_max_deg)
    if parallel > 0:
        return _tti_finish_parallel(sm, v_layer, pert, eps_max, amax, ny == 1, parallel)
    xi_v = _minmax(sm[0], -1.0, 1.0)
    vp = v_layer[:, None, None] * (1.0 + pert * xi_v)
    eps = eps_max * _minmax(sm[1], 0.0, 1.0)
    delta = 0.5 * eps
    theta = amax * _minmax(sm[2], -1.0, 1.0)
    phi = amax * _minmax(sm[3], -1.0, 1.0)
    if ny == 1:
        phi[:] = 0.0
    return {k: np.ascontiguousarray(v, dtype=np.float32)
            for k, v in (("vp", vp), ("eps", eps), ("delta", delta), ("theta", theta), ("phi", phi))}


def _slabs(n: int, threads: int, fn) -> None:
    """Run fn(slice) over ``threads`` contiguous slabs of range(n) on as many threads."""
    k = max(1, min(threads, n))
    with ThreadPoolExecutor(k) as ex:
        list(ex.map(lambda c: fn(slice(c * n // k, (c + 1) * n // k)), range(k)))


def _tti_finish_parallel(sm, v_layer, pert, eps_max, amax, flat, threads) -> dict:
    """The default recipe's mapping of the smoothed fields to parameters, slab by slab on threads
    (FP64 arithmetic per slab, FP32 results)."""
    nz = sm[0].shape[0]
    ext = []
    for a in sm:
        lo = np.empty(nz)
        hi = np.empty(nz)

        def red(sl, a=a, lo=lo, hi=hi):
            lo[sl] = a[sl].min(axis=(1, 2))
            hi[sl] = a[sl].max(axis=(1, 2))

        _slabs(nz, threads, red)
        ext.append((float(lo.min()), float(hi.max())))
    out = {k: np.empty(sm[0].shape, np.float32) for k in ("vp", "eps", "delta", "theta", "phi")}

    def unit(i, sl, lo, hi):
        amin, amax_ = ext[i]
        if amax_ <= amin:
            return np.full(sm[i][sl].shape, 0.5 * (lo + hi))
        return lo + (hi - lo) * (sm[i][sl].astype(np.float64) - amin) / (amax_ - amin)

    def run(sl):
        out["vp"][sl] = v_layer[sl, None, None] * (1.0 + pert * unit(0, sl, -1.0, 1.0))
        eps = eps_max * unit(1, sl, 0.0, 1.0)
        out["eps"][sl] = eps
        out["delta"][sl] = 0.5 * eps
        out["theta"][sl] = amax * unit(2, sl, -1.0, 1.0)
        out["phi"][sl] = 0.0 if flat else amax * unit(3, sl, -1.0, 1.0)

    _slabs(nz, threads, run)
    return out


def elastic_model(shape_xyz, nbl: int, seed: int, nlayers: int = 10, vmin: float = 1500.0,
                  vmax: float = 4500.0, pert: float = 0.05, vp_vs: float = 1.8) -> dict:
    """Seeded isotropic elastic model: FP32 vp, vs (m/s), rho (kg/m^3); layer 0 is water (vs = 0)."""
    nx, ny, nz = (int(s) for s in shape_xyz)
    shp = (nz, ny, nx)
    rng = _rng(seed)
    layer = _layer_index(nz, nbl, rng, nlayers)
    v_layer = vmin + (vmax - vmin) * layer / (nlayers - 1)
    xi = _minmax(smooth(rng.standard_normal(shp), 4.0), -1.0, 1.0)
    water = (layer == 0)[:, None, None]
    vp = v_layer[:, None, None] * np.where(water, 1.0, 1.0 + pert * xi)
    vs = np.where(water, 0.0, vp / vp_vs)
    rho = 310.0 * vp ** 0.25
    return {k: np.ascontiguousarray(v, dtype=np.float32) for k, v in (("vp", vp), ("vs", vs), ("rho", rho))}


def marine_elastic_model(shape_xyz, surface_row: int, water_rows: int, seed: int, nlayers: int = 9,
                         vmin: float = 1600.0, vmax: float = 4500.0, pert: float = 0.05,
                         vp_vs: float = 1.8) -> dict:
    """Seeded marine elastic model: FP32 vp, vs (m/s), rho (kg/m^3), shape (nz, ny, nx).  Water
    (vp 1500 m/s, vs 0) from the top down to surface_row + water_rows (the rows above surface_row
    become vacuum under a free surface), then nlayers elastic layers between vmin and vmax with a
    smoothed +-pert perturbation, vs = vp / vp_vs, Gardner density 310 vp^0.25."""
    nx, ny, nz = (int(s) for s in shape_xyz)
    shp = (nz, ny, nx)
    rng = _rng(seed)
    bed = surface_row + water_rows
    depths = np.sort(rng.uniform(0.0, 0.9, nlayers - 1)) * (nz - bed) + bed
    k = np.arange(nz, dtype=np.float64)
    layer = np.searchsorted(depths, k, side="right")
    v_layer = vmin + (vmax - vmin) * layer / max(nlayers - 1, 1)
    xi = _minmax(smooth(rng.standard_normal(shp), 4.0), -1.0, 1.0)
    water = (k < bed)[:, None, None]
    vp = np.where(water, 1500.0, v_layer[:, None, None] * (1.0 + pert * xi))
    vs = np.where(water, 0.0, vp / vp_vs)
    rho = 310.0 * vp ** 0.25
    return {k_: np.ascontiguousarray(v, dtype=np.float32) for k_, v in (("vp", vp), ("vs", vs), ("rho", rho))}


def slowness_squared(vp: np.ndarray, threads: int = 1) -> np.ndarray:
    """The model parameter m = 1/vp^2 (s^2/m^2) as FP32, computed in FP64 from the FP32 velocities
    (over slabs of the first axis on ``threads`` threads: the same bits)."""
    if threads <= 1 or np.ndim(vp) == 0:
        v = np.asarray(vp, dtype=np.float64)
        return (1.0 / (v * v)).astype(np.float32)
    out = np.empty(np.shape(vp), np.float32)

    def run(sl):
        v = np.asarray(vp[sl], dtype=np.float64)
        out[sl] = 1.0 / (v * v)

    _slabs(out.shape[0], threads, run)
    return out


def random_unit_field(shape, seed: int, sigma: float = 0.0) -> np.ndarray:
    """Seeded N(0,1) field (optionally smoothed), FP32; used for perturbations and dot tests."""
    a = _rng(seed).standard_normal(shape)
    if sigma > 0:
        a = smooth(a, sigma)
    return a.astype(np.float32)


def surface_receivers(shape_xyz, spacing, origin, nbl: int, depth_index: float, nrx: int, nry: int,
                      inset: float = 0.25) -> np.ndarray:
    """Receiver coordinates (metres, FP32, nrec x ndim) on an even lattice over the physical x-y interior.

    The lattice spans [nbl + inset, n - 1 - nbl - inset] in index units so that it is generally off-grid.
    For 2D grids (ny = 1) pass nry = 1; the result is then nrec x 2 (x, z).
    """
    nx, ny, nz = shape_xyz
    hx, hy, hz = spacing
    ox, oy, oz = origin
    xs = ox + hx * np.linspace(nbl + inset, nx - 1 - nbl - inset, nrx)
    z = oz + hz * depth_index
    if ny == 1:
        return np.stack([xs, np.full_like(xs, z)], axis=1).astype(np.float32)
    ys = oy + hy * np.linspace(nbl + inset, ny - 1 - nbl - inset, nry)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], axis=1).astype(np.float32)
