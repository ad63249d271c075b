"""Shared helpers of the GPU parity tests: run the HIP path and the checker on the same inputs."""
import numpy as np
import torch

from paper_2004_10519_amd import inputs


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def tti_case(shape, so, nbl, nt, seed=5, h=(10.0, 11.0, 9.0), nsrc=2, nrec=23, dt=None):
    """A small seeded TTI case with off-grid sources/receivers spread over the whole window
    (including the absorbing layer and the last-node clamp)."""
    nx, ny, nz = shape
    ndim = 2 if ny == 1 else 3
    mdl = inputs.tti_model(shape, nbl, seed)
    model = {"m": inputs.slowness_squared(mdl["vp"]), "eps": mdl["eps"], "delta": mdl["delta"],
             "theta": mdl["theta"], "phi": mdl["phi"]}
    rng = np.random.default_rng(seed + 100)
    ext = [(nx - 1) * h[0], (ny - 1) * h[1], (nz - 1) * h[2]]
    axes = (0, 2) if ndim == 2 else (0, 1, 2)
    src = np.stack([rng.uniform(0.3, 0.7, nsrc) * ext[a] for a in axes], axis=1)
    rec = np.stack([rng.uniform(0.0, 1.0, nrec) * ext[a] for a in axes], axis=1)
    rec[0] = [ext[a] for a in axes]
    rec[1] = [0.0 for a in axes]
    if dt is None:
        dt = 0.8 * 2.0 / (4725.0 * np.sqrt(1.6 * _sd(so) * sum(1 / h[a] ** 2 for a in axes)))
    wav = np.stack([inputs.ricker(25.0, dt, nt), 0.5 * inputs.ricker(18.0, dt, nt, t0=0.07)], axis=1)[:, :nsrc]
    return dict(shape=shape, h=h, so=so, nbl=nbl, nt=nt, dt=float(dt), model=model, src=src.astype(np.float32),
                rec=rec.astype(np.float32), wav=np.ascontiguousarray(wav, dtype=np.float32), ndim=ndim)


def _sd(so):
    import oracle
    return oracle.symbol_max_sq(so)


def el_case(shape, so, nbl, nt, seed=6, h=(10.0, 9.0, 8.0), nrec=20, free_surface=False):
    nx, ny, nz = shape
    model = inputs.elastic_model(shape, nbl, seed)
    rng = np.random.default_rng(seed + 7)
    ext = [(nx - 1) * h[0], (ny - 1) * h[1], (nz - 1) * h[2]]
    src = np.array([[0.47 * ext[0], 0.52 * ext[1], 0.55 * ext[2]]])
    rec = np.stack([rng.uniform(0, 1, nrec) * ext[0], rng.uniform(0, 1, nrec) * ext[1],
                    rng.uniform(0.05, 0.95, nrec) * ext[2]], axis=1)
    kind = (np.arange(nrec) % 2).astype(np.int32)
    dt = 0.8 * min(h) / (4725.0 * np.sqrt(3) * {2: 1.0, 4: 1.16667, 6: 1.24167, 8: 1.28631, 12: 1.33906}[so])
    wav = inputs.ricker(30.0, dt, nt)[:, None]
    return dict(shape=shape, h=h, so=so, nbl=nbl, nt=nt, dt=float(dt), model=model, src=src.astype(np.float32),
                rec=rec.astype(np.float32), kind=kind, wav=np.ascontiguousarray(wav, dtype=np.float32),
                free_surface=free_surface)


def make_tti(case, prop, scheme=0, **options):
    """TTI propagator for a test case; scheme 0 = six-field pass-1 temporaries, 2 = one fused pass,
    3 = four-field temporaries (t and n . grad q), 4 = two fused single-field passes (schemes 2 and 4
    support space orders up to 12: the test is skipped beyond)."""
    if scheme in (2, 4) and case["so"] > 12:
        import pytest
        pytest.skip("the fused and split schemes support space orders up to 12")
    g = prop.Grid(case["shape"], case["h"], space_order=case["so"], nbl=case["nbl"], dt=case["dt"], nt=case["nt"],
                  v_ref=1500.0)
    mt = [dev(case["model"][k]) for k in ("m", "eps", "delta", "theta", "phi")]
    p = prop.Propagator(prop.TTI, g, mt)
    p._keep_model = mt
    p.set_option("scheme", scheme)
    for k, v in options.items():
        p.set_option(k, v)
    shot = prop.Shot(case["src"], dev(case["wav"]), case["rec"])
    return p, shot


def make_el(case, prop):
    g = prop.Grid(case["shape"], case["h"], space_order=case["so"], nbl=case["nbl"], dt=case["dt"], nt=case["nt"],
                  v_ref=1500.0, free_surface=case.get("free_surface", False))
    mt = [dev(case["model"][k]) for k in ("vp", "vs", "rho")]
    p = prop.Propagator(prop.ELASTIC, g, mt)
    p._keep_model = mt
    shot = prop.Shot(case["src"], dev(case["wav"]), case["rec"], case["kind"])
    return p, shot


def oracle_tti(case, orc):
    g = orc.Grid(case["shape"], case["h"], space_order=case["so"], nbl=case["nbl"], dt=case["dt"], nt=case["nt"],
                 vref=1500.0)
    m = case["model"]
    mod = orc.TTIModel.from_arrays(g, m["m"], m["eps"], m["delta"], m["theta"], m["phi"])
    return g, mod


def oracle_el(case, orc):
    g = orc.Grid(case["shape"], case["h"], space_order=case["so"], nbl=case["nbl"], dt=case["dt"], nt=case["nt"],
                 vref=1500.0, free_surface=case.get("free_surface", False))
    m = case["model"]
    return g, orc.ElasticModel.from_velocities(g, m["vp"], m["vs"], m["rho"])
