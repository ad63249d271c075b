"""Workload definitions (sizes, geometry and seeds of the benchmark and parity cases).

Only input recipes live here (they call ``inputs``); the time steps are fixed numbers chosen at
about 0.8 of the stability bound of each workload, so that neither the checker nor the library
has to supply them to the other.

  tti2d_101    2D TTI, 101 x 101, h 10 m, space order 4, 500 steps, constant medium (parity case)
  tti3d_512    3D TTI, 512^3, h 12.5 m, space order 12, 3000 steps, 40-point layers (benchmark)
  el3d_400     3D elastic, 400^3, h 10 m, space order 8, 2000 steps, 40-point layers
  ttigrad_256  3D TTI gradient, 256^3, h 12.5 m, space order 8, 2000 steps (and a 64^3 check)
  batch_64     64 TTI shots on windows of a 1024 x 1024 x 512 model, space order 8, 1500 steps
  el2d_marine  2D elastic, 1701 x 391, h 10 m, space order 8, 5 s, free surface (method of images)
               over a 450 m water layer; pressure 5 m below the surface and vz on the sea bed (the
               paper's 2D example's geometry on a seeded layered model)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import inputs


@dataclass
class Workload:
    name: str
    kind: str                     # "tti" or "elastic"
    shape: tuple                  # (nx, ny, nz)
    spacing: tuple
    space_order: int
    nt: int
    nbl: int
    dt: float
    seed: int
    f0: float
    src_xyz: np.ndarray
    rec_xyz: np.ndarray
    rec_kind: np.ndarray = None
    v_ref: float = 1500.0
    free_surface: object = False  # True: vacuum rows above the surface; "image": method of images
    model_threads: int = 0        # > 0: the fast FP32 model recipe on that many threads
    model: dict = field(default_factory=dict, repr=False)

    @property
    def ndim(self):
        return 2 if self.shape[1] == 1 else 3

    @property
    def arr_shape(self):
        return (self.shape[2], self.shape[1], self.shape[0])

    @property
    def npts(self):
        return int(np.prod(self.shape))

    def wavelet(self, nt=None) -> np.ndarray:
        nt = self.nt if nt is None else nt
        w = inputs.ricker(self.f0, self.dt, nt)
        return np.repeat(w[:, None], len(self.src_xyz), axis=1).astype(np.float32)

    def make_model(self, progress=None) -> dict:
        """FP32 model arrays keyed by parameter name (``progress`` reports generation stages)."""
        if self.model:
            return self.model
        if self.name == "tti2d_101":
            shp = self.arr_shape
            vp = np.full(shp, 1500.0, np.float32)
            self.model = {"m": inputs.slowness_squared(vp), "eps": np.full(shp, 0.1, np.float32),
                          "delta": np.full(shp, 0.05, np.float32), "theta": np.full(shp, math.radians(30), np.float32),
                          "phi": np.zeros(shp, np.float32)}
        elif self.kind == "tti":
            mdl = inputs.tti_model(self.shape, self.nbl, self.seed, progress=progress, parallel=self.model_threads)
            self.model = {"m": inputs.slowness_squared(mdl["vp"], threads=max(1, self.model_threads)),
                          "eps": mdl["eps"], "delta": mdl["delta"], "theta": mdl["theta"], "phi": mdl["phi"]}
        elif self.name == "el2d_marine":
            self.model = inputs.marine_elastic_model(self.shape, self.nbl, MARINE_WATER_ROWS, self.seed)
        else:
            self.model = inputs.elastic_model(self.shape, self.nbl, self.seed)
        return self.model

    def model_list(self, progress=None):
        """FP32 model arrays in the library's parameter order."""
        m = self.make_model(progress)
        keys = ("m", "eps", "delta", "theta", "phi") if self.kind == "tti" else ("vp", "vs", "rho")
        return [m[k] for k in keys]


def _centre_src(shape, h, nbl, zidx, dx=0.0, dy=0.0):
    nx, ny, nz = shape
    cx = h[0] * (nbl + (nx - 1 - 2 * nbl) / 2.0 + dx)
    cy = h[1] * (nbl + (ny - 1 - 2 * nbl) / 2.0 + dy)
    return np.array([[cx, cy, h[2] * zidx]], dtype=np.float32)


def tti2d_101() -> Workload:
    shape, h = (101, 1, 101), (10.0, 1.0, 10.0)
    src = np.array([[500.0, 500.0]], dtype=np.float32)
    rec = np.stack([np.arange(101) * 10.0, np.zeros(101)], axis=1).astype(np.float32)
    return Workload("tti2d_101", "tti", shape, h, 4, 500, 0, 5.018e-3, 0, 10.0, src, rec, v_ref=1500.0)


def tti3d_512(nt: int = 3000, n: int = 512) -> Workload:
    shape, h, nbl = (n, n, n), (12.5, 12.5, 12.5), 40
    src = _centre_src(shape, h, nbl, nbl + 4.5, 0.3, 0.3)
    rec = inputs.surface_receivers(shape, h, (0, 0, 0), nbl, nbl + 2, 256, 256)
    return Workload(f"tti3d_{n}", "tti", shape, h, 12, nt, nbl, 1.0e-3, 1, 15.0, src, rec, v_ref=1500.0)


def el3d_400(nt: int = 2000, n: int = 400) -> Workload:
    shape, h, nbl = (n, n, n), (10.0, 10.0, 10.0), 40
    src = _centre_src(shape, h, nbl, nbl + 10)
    r = inputs.surface_receivers(shape, h, (0, 0, 0), nbl, nbl + 2, 200, 200)
    rec = np.concatenate([r, r], axis=0)
    kind = np.concatenate([np.zeros(len(r), np.int32), np.ones(len(r), np.int32)])
    return Workload(f"el3d_{n}", "elastic", shape, h, 8, nt, nbl, 0.760e-3, 2, 12.0, src, rec, kind, v_ref=1500.0)


def ttigrad(n: int = 256, nt: int = 2000, nbl: int = 40, nrec: int = 128, seed: int = 3) -> Workload:
    shape, h = (n, n, n), (12.5, 12.5, 12.5)
    src = _centre_src(shape, h, nbl, nbl + 4)
    rec = inputs.surface_receivers(shape, h, (0, 0, 0), nbl, nbl + 2, nrec, nrec)
    return Workload(f"ttigrad_{n}", "tti", shape, h, 8, nt, nbl, 1.116e-3, seed, 15.0, src, rec, v_ref=1500.0)


def ttigrad_starting_model(w: Workload) -> dict:
    """Smoothed starting model of the gradient workload (vp smoothed with sigma = 10 points)."""
    mdl = inputs.tti_model(w.shape, w.nbl, w.seed)
    vp0 = inputs.smooth(mdl["vp"], 10.0).astype(np.float32)
    return {"m": inputs.slowness_squared(vp0), "eps": mdl["eps"], "delta": mdl["delta"], "theta": mdl["theta"],
            "phi": mdl["phi"]}


def batch_64(nshot: int = 64, nt: int = 1500, shape=(1024, 1024, 512), seed_model: int = 4, seed_win: int = 5):
    """64 TTI shots on uneven windows of one seeded model.

    Windows: edges uniform in [128, 320] per axis (seed 5), x-y origin uniform within the model, z
    origin 0; 32-point absorbing layers inside each window.  Per shot: source at the window centre,
    4 points below the layer; receivers on every 4th node of the window interior, 2 points below
    the layer.  The 0.5 G-point model uses the fast FP32 recipe of ``inputs.tti_model`` on 16
    threads.  Returns (model Workload, list of (origin, shape, src_xyz, rec_xyz)).
    """
    h, nbl = (12.5, 12.5, 12.5), 32
    w = Workload("batch_64", "tti", tuple(shape), h, 8, nt, nbl, 1.116e-3, seed_model, 15.0,
                 np.zeros((1, 3), np.float32), np.zeros((0, 3), np.float32), v_ref=1500.0, model_threads=16)
    rng = np.random.Generator(np.random.PCG64(seed_win))
    shots = []
    for _ in range(nshot):
        n = [int(rng.integers(128, 321)) for _ in range(3)]
        n = [min(n[a], shape[a]) for a in range(3)]
        o = [int(rng.integers(0, shape[0] - n[0] + 1)), int(rng.integers(0, shape[1] - n[1] + 1)), 0]
        src = np.array([[h[0] * (o[0] + (n[0] - 1) / 2 + 0.3), h[1] * (o[1] + (n[1] - 1) / 2 + 0.3),
                         h[2] * (nbl + 4)]], np.float32)
        xs = h[0] * (o[0] + np.arange(nbl, n[0] - nbl, 4))
        ys = h[1] * (o[1] + np.arange(nbl, n[1] - nbl, 4))
        X, Y = np.meshgrid(xs, ys)
        rec = np.stack([X.ravel(), Y.ravel(), np.full(X.size, h[2] * (nbl + 2))], axis=1).astype(np.float32)
        shots.append((tuple(o), tuple(n), src, rec))
    return w, shots


MARINE_WATER_ROWS = 45   # 450 m of water at 10 m


def el2d_marine(nt: int = 5556) -> Workload:
    """Free surface on the top face at row nbl (the rows above it are vacuum), explosive source 10 m
    below it at x = 5 km of the physical frame, pressure receivers 5 m below the surface and vz
    receivers on the sea bed, every 10 m across the physical width; dt 0.9 ms (5 s in 5556 steps)."""
    shape, h, nbl = (1701, 1, 391), (10.0, 1.0, 10.0), 40
    z0 = nbl * h[2]
    src = np.array([[nbl * h[0] + 5000.0, z0 + 10.0]], dtype=np.float32)
    xs = nbl * h[0] + np.arange(0, shape[0] - 2 * nbl) * h[0]
    rp = np.stack([xs, np.full(xs.size, z0 + 5.0)], axis=1)
    rv = np.stack([xs, np.full(xs.size, z0 + MARINE_WATER_ROWS * h[2])], axis=1)
    rec = np.concatenate([rp, rv], axis=0).astype(np.float32)
    kind = np.concatenate([np.zeros(xs.size, np.int32), np.ones(xs.size, np.int32)])
    return Workload("el2d_marine", "elastic", shape, h, 8, nt, nbl, 0.9e-3, 9, 12.0, src, rec, kind,
                    v_ref=1500.0, free_surface="image")
