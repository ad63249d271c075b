#!/usr/bin/env python3
"""Benchmark of the propagator library on one MI355X.

One "step" is one whole modelling run of the 3D TTI workload tti3d_512 (512^3 grid, 12.5 m,
space order 12, 3000 time steps, 40-point absorbing layers, 15 Hz source, 256 x 256 receivers),
with all inputs resident in HBM: every time step's stencil launches, source injection and
receiver interpolation.  Metric: grid points updated per second (GPts/s = 512^3 * 3000 / time);
ms_per_step is one whole run, ms_per_time_step one of its 3000 time steps.

The JSON line also carries
  roofline      the method's algorithmic bytes of one time step (44 B/pt) times the points of one
                launch of the dominant kernel, over that kernel's mean launch time (HIP events on the
                library's stream during the timed steps), against the 8 TB/s HBM peak; step_frac is
                the same bytes over the whole time step;
  cpu_baseline  the FP64 checker timed on this host on bounded samples of the TTI and elastic workloads;
  paths         the other measured paths (TTI adjoint, elastic forward / adjoint / gradient, 2D marine
                elastic, TTI gradient, 64 batched shots against 64 plain calls); --only-main skips them.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per grid point of one launch of each stencil kernel (FP32).  TTI, per scheme
# (0: six-field temporaries, 2: one fused pass, 3: four-field temporaries, 4: split) and direction:
#   scheme 0 pass 1: read u, v, n_x, n_y; write t (3), s (3)                              -> 10 x 4
#   scheme 0 pass 2: read t, s (6), f, f- for p and q (4), m, 1+2eps, sqrt(1+2delta) (3);
#                    write p+, q+ (2); adjoint also writes w = C y+ (2)                  -> 15 / 17 x 4
#   scheme 2 (one fused pass, class 1): read u, v, f- for p and q (4), n_x, n_y, m, 1+2eps,
#                    sqrt(1+2delta) (5); write p+, q+ (2); adjoint reads y too and writes
#                    w = C y+ (2)                                                         -> 11 / 15 x 4
#   scheme 4 pass A: read u, n_x, n_y; write h = H0 u                                    ->  4 x 4
#   scheme 4 pass B: read v, n_x, n_y, h, f and f- of p (2), f- of q, m, 1+2eps, sqrt(1+2delta);
#                    write p+, q+ (2); adjoint reads f of q too and writes w = C y+ (2)  -> 12 / 15 x 4
# Elastic:
#   el_vel:    read 9 fields + buoyancy; write 3                                  -> 13 x 4
#   el_stress: read 9 fields + lambda, mu; write 6                                -> 17 x 4
#   el_fused:  read 9 fields + lambda, mu, buoyancy; write 9 (one step)           -> 21 x 4
TTI_KERNEL_BYTES = {(0, 0, False): 40, (0, 1, False): 60, (0, 0, True): 40, (0, 1, True): 68,
                    (2, 1, False): 44, (2, 1, True): 60,
                    (3, 0, False): 32, (3, 1, False): 60, (3, 0, True): 32, (3, 1, True): 68,
                    (4, 0, False): 16, (4, 1, False): 48, (4, 0, True): 16, (4, 1, True): 60}
KERNEL_BYTES_PER_PT = {2: 52, 3: 68, 4: 84}
TTI_SCHEME = None   # step scheme of every TTI handle (--scheme); None = the library default
FIXED_TILES = None  # (tile1, zc1, tile2, zc2) of the main run instead of the autotuner (--tiles)


def kernel_bytes(kclass: int, scheme: int = 0, adjoint: bool = False) -> int:
    return TTI_KERNEL_BYTES[(scheme, kclass, adjoint)] if kclass in (0, 1) else KERNEL_BYTES_PER_PT[kclass]


# minimum bytes per point per time step of the whole method (fused reading, FP32)
METHOD_BYTES_PER_PT = {"tti": 44, "elastic": 84}
# TTI FLOPs per point after the paper's symbolic optimisation (Table ttiFLOPs), used only to quote a
# FLOP-rate equivalent beside the paper's own figures
TTI_PAPER_FLOPS_PER_PT = {4: 95, 8: 102, 12: 160, 16: 276}


_T_START = time.perf_counter()


def log(*a):
    """Progress line on stderr, stamped with the seconds since the benchmark started."""
    print(f"{time.perf_counter() - _T_START:7.1f}s", *a, file=sys.stderr, flush=True)


# sources of each TTI scheme's stencil kernels (the counters in profiles/pmc_traffic.json hold only
# while these are unchanged)
SCHEME_SOURCES = {0: "tti.hip", 2: "tti_fused.hip", 3: "tti.hip", 4: "tti_split.hip"}


def kernel_source_hash(scheme: int) -> str:
    h = hashlib.sha256()
    for f in ("common.h", "jobs.h", SCHEME_SOURCES[scheme]):
        with open(os.path.join(ROOT, "paper_2004_10519_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(kclass: int, npts: int, scheme: int = 0, tile=None, space_order: int = 12):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/pmc_traffic.json), if they were
    taken on the current kernel source with the same tile variant and z-chunk; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    ent = rec.get(f"{kclass}/{scheme}/so{space_order}")
    if not ent or ent.get("source_hash") != kernel_source_hash(scheme) or ent.get("npts") != npts:
        return None
    if tile is not None and ent.get("tile") != list(tile):
        return None
    return ent.get("bytes_per_launch")


def setup_tti(w, torch, prop):
    arrs = w.model_list()
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, v_ref=w.v_ref,
                  free_surface=w.free_surface)
    p = prop.Propagator(prop.TTI if w.kind == "tti" else prop.ELASTIC, g, dev)
    p._keep = dev
    if w.kind == "tti":
        if TTI_SCHEME is not None:
            p.set_option("scheme", TTI_SCHEME)
        if FIXED_TILES:
            for k, v in zip(("tile1", "zc", "tile2", "zc2"), FIXED_TILES):
                p.set_option(k, v)
        else:
            p.set_option("autotune", 1)
    shot = prop.Shot(w.src_xyz, torch.from_numpy(w.wavelet()).cuda(), w.rec_xyz, w.rec_kind)
    return p, shot


def timed(torch, fn, steps, warmup, label=None):
    """Mean wall time of `steps` calls after `warmup` untimed ones; with a label, one progress line per
    call on stderr (long legs would otherwise stay silent for minutes)."""
    for i in range(warmup):
        fn()
        if label:
            torch.cuda.synchronize()
            log(f"[bench] {label}: warm-up {i + 1}/{warmup}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn()
        if label:
            log(f"[bench] {label}: step {i + 1}/{steps} issued ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, budget_s: float = 8.0, el_budget_s: float = 5.0):
    """The FP64 checker on sub-volumes of the benchmark model (the TTI step of the headline) and of the
    elastic 400^3 model (a bounded sample of each workload)."""
    import oracle
    from paper_2004_10519_amd import configs
    n = min(192, w.shape[0])
    mdl = w.make_model()
    sl = tuple(slice(s // 2 - n // 2, s // 2 - n // 2 + n) if s > 1 else slice(None) for s in w.arr_shape)
    arrs = [np.ascontiguousarray(mdl[k][sl]) for k in ("m", "eps", "delta", "theta", "phi")]
    shape = (arrs[0].shape[2], arrs[0].shape[1], arrs[0].shape[0])
    g = oracle.Grid(shape, w.spacing, space_order=w.space_order, nbl=w.nbl // 4, dt=w.dt, nt=1, vref=w.v_ref)
    mod = oracle.TTIModel.from_arrays(g, *arrs)
    eta = oracle.tti_eta(g)
    zeros = [np.zeros(g.arr_shape) for _ in range(4)]
    rng = np.random.default_rng(0)
    zeros[0][...] = rng.standard_normal(g.arr_shape)
    oracle._tti_step(g, mod, eta, False, *zeros)   # warm-up (page faults)
    steps, t0 = 0, time.perf_counter()
    while True:
        oracle._tti_step(g, mod, eta, False, *zeros)
        steps += 1
        el = time.perf_counter() - t0
        if el > budget_s or steps >= 50:
            break
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    out = {"value": round(int(np.prod(shape)) * steps / el / 1e9, 5), "unit": "GPts/s", "cores": cores,
           "kind": "oracle", "cpu_model": cpu_model(),
           "sample": f"{shape[0]}x{shape[1]}x{shape[2]} centre sub-volume of the {w.name} model, "
                     f"space order {w.space_order}, {steps} FP64 time steps in {el:.1f} s"}
    # elastic: the velocity-stress step of the el3d_400 workload on a centre sub-volume
    we = configs.el3d_400(nt=1)
    ne = 160
    me = we.make_model()
    sle = tuple(slice(s // 2 - ne // 2, s // 2 - ne // 2 + ne) for s in we.arr_shape)
    ge = oracle.Grid((ne, ne, ne), we.spacing, space_order=we.space_order, nbl=we.nbl // 4, dt=we.dt, nt=1,
                     vref=we.v_ref)
    emod = oracle.ElasticModel.from_velocities(ge, *(np.ascontiguousarray(me[k][sle]) for k in ("vp", "vs", "rho")))
    damp = np.ascontiguousarray(oracle.elastic_damp(ge))
    v = [rng.standard_normal(ge.arr_shape) for _ in range(3)]
    t = [np.zeros(ge.arr_shape) for _ in range(6)]
    oracle._el_call(oracle.lib().orc_el_step, ge, emod, damp, v, t)
    steps, t0 = 0, time.perf_counter()
    while True:
        oracle._el_call(oracle.lib().orc_el_step, ge, emod, damp, v, t)
        steps += 1
        el = time.perf_counter() - t0
        if el > el_budget_s or steps >= 50:
            break
    out["elastic"] = {"value": round(ne ** 3 * steps / el / 1e9, 5), "unit": "GPts/s",
                      "sample": f"{ne}^3 centre sub-volume of the {we.name} model, space order {we.space_order}, "
                                f"{steps} FP64 velocity-stress steps in {el:.1f} s"}
    return out


def kernel_roof(p, classes, npts, scheme=0, adjoint=False):
    kt = {k: p.kernel_time(k) for k in classes}
    out = {}
    for k, (ms, n, name) in kt.items():
        if n == 0:
            continue
        avg = ms / 1e3 / n
        b = kernel_bytes(k, scheme, adjoint)
        out[name] = {"mean_launch_ms": round(avg * 1e3, 4), "launches": n, "bytes_per_point": b,
                     "GBps_algorithmic": round(b * npts / avg / 1e9, 1),
                     "frac_of_8TBs": round(b * npts / avg / 1e9 / HBM_PEAK_GBS, 4)}
    return out


def measure_tti_adjoint(torch, prop, w, p, shot):
    rec = torch.randn((w.nt, len(w.rec_xyz)), device="cuda")
    torch.cuda.synchronize()
    p.set_timing(True)
    t = timed(torch, lambda: p.adjoint(shot, rec), 1, 0)
    roof = kernel_roof(p, (0, 1), w.npts, p.get_option("scheme"), adjoint=True)
    p.set_timing(False)
    g = w.npts * w.nt / t / 1e9
    return {"workload": w.name, "GPts/s": round(g, 3), "ms": round(t * 1e3, 1),
            "method_hbm_frac": round(g * METHOD_BYTES_PER_PT["tti"] / HBM_PEAK_GBS, 4), "kernels": roof}


def measure_elastic(torch, prop, nt):
    from paper_2004_10519_amd import configs
    w = configs.el3d_400(nt=nt)
    log(f"[bench] generating {w.name} model ...")
    p, shot = setup_tti(w, torch, prop)
    p.forward(shot)
    torch.cuda.synchronize()
    p.set_timing(True)
    t = timed(torch, lambda: p.forward(shot), 1, 0)
    roof = kernel_roof(p, (2, 3, 4), w.npts)
    p.set_timing(False)
    rec = torch.randn((w.nt, len(w.rec_xyz)), device="cuda")
    torch.cuda.synchronize()
    ta = timed(torch, lambda: p.adjoint(shot, rec), 1, 0)
    g, ga = w.npts * w.nt / t / 1e9, w.npts * w.nt / ta / 1e9
    # the fused velocity-stress step (opt-in; bitwise the same traces)
    p.set_option("el_fused", 1)
    p.set_timing(True)
    tf = timed(torch, lambda: p.forward(shot), 1, 0)
    roof_f = kernel_roof(p, (4,), w.npts)
    p.set_timing(False)
    p.set_option("el_fused", 0)
    # gradient with respect to (vp, vs, rho), 48 FP32 checkpoints (a residual-shaped random input:
    # the cost does not depend on the values)
    log("[bench] elastic gradient ...")
    tg = timed(torch, lambda: p.gradient(shot, rec, n_ckpt=48, ckpt_dtype="f32"), 1, 0)
    gg = w.npts * w.nt / tg / 1e9
    p.close()
    return {"workload": w.name, "grid": list(w.shape), "space_order": w.space_order, "time_steps": w.nt,
            "forward_GPts/s": round(g, 3), "adjoint_GPts/s": round(ga, 3),
            "gradient_vp_vs_rho_GPts/s": round(gg, 3), "gradient_checkpoints": 48,
            "forward_method_hbm_frac": round(g * METHOD_BYTES_PER_PT["elastic"] / HBM_PEAK_GBS, 4),
            "forward_kernels": roof,
            "forward_fused_step_GPts/s": round(w.npts * w.nt / tf / 1e9, 3), "forward_fused_kernel": roof_f}


def measure_marine(torch, prop):
    """The 2D marine elastic workload (free surface over a water layer), 5 s of modelling."""
    from paper_2004_10519_amd import configs
    w = configs.el2d_marine()
    p, shot = setup_tti(w, torch, prop)
    p.forward(shot)
    torch.cuda.synchronize()
    t = timed(torch, lambda: p.forward(shot), 1, 0)
    d = p.forward(shot)
    npr = int((w.rec_kind == 0).sum())
    peak = [float(d[:, :npr].abs().max()), float(d[:, npr:].abs().max())]
    # gradient with respect to (vp, vs, rho), 48 FP32 checkpoints, for a residual-shaped input
    res = torch.randn_like(d)
    p.gradient(shot, res, n_ckpt=48, ckpt_dtype="f32")
    torch.cuda.synchronize()
    tg = timed(torch, lambda: p.gradient(shot, res, n_ckpt=48, ckpt_dtype="f32"), 1, 0)
    p.close()
    return {"workload": w.name, "grid": list(w.shape), "space_order": w.space_order, "time_steps": w.nt,
            "free_surface": w.free_surface, "s": round(t, 4), "GPts/s": round(w.npts * w.nt / t / 1e9, 3),
            "gradient_vp_vs_rho_s": round(tg, 4), "gradient_checkpoints": 48,
            "receivers": {"pressure_5m": npr, "vz_seabed": len(w.rec_xyz) - npr},
            "peak_pressure": peak[0], "peak_vz": peak[1]}


def measure_gradient(torch, prop, nt, dtypes=("bf16", "f16")):
    from paper_2004_10519_amd import configs
    w = configs.ttigrad(n=256, nt=nt)
    log(f"[bench] generating {w.name} models ...")
    true = [np.ascontiguousarray(a) for a in w.model_list()]
    m0 = configs.ttigrad_starting_model(w)
    start = [m0[k] for k in ("m", "eps", "delta", "theta", "phi")]
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, v_ref=w.v_ref)
    dt_ = [torch.from_numpy(a).cuda() for a in true]
    p = prop.Propagator(prop.TTI, g, dt_)
    if TTI_SCHEME is not None:
        p.set_option("scheme", TTI_SCHEME)
    p.set_option("autotune", 1)
    shot = prop.Shot(w.src_xyz, torch.from_numpy(w.wavelet()).cuda(), w.rec_xyz)
    dobs = p.forward(shot).clone()
    ds_ = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in start]
    p.set_model(ds_)
    res = (p.forward(shot) - dobs).contiguous()
    p.adjoint(shot, res)   # the autotuner's choice for the adjoint direction, outside the timed calls
    torch.cuda.synchronize()
    out = {"workload": w.name, "grid": list(w.shape), "space_order": w.space_order, "time_steps": w.nt,
           "checkpoints": 48}
    ref = None
    for dt in ("f32",) + tuple(dtypes):
        holder = []
        t = timed(torch, lambda: holder.append(p.gradient(shot, res, 48, dt)), 1, 0)
        gr = holder[0]
        gp = w.npts * w.nt / t / 1e9
        ent = {"GPts/s": round(gp, 3), "ms": round(t * 1e3, 1),
               "method_hbm_frac_156B": round(gp * 156 / HBM_PEAK_GBS, 4)}
        if ref is None:
            ref = gr.double()
        else:
            ent["rel_l2_vs_f32_checkpoints"] = float(((gr.double() - ref).norm() / ref.norm()).item())
        out[dt] = ent
    # whole run stored in FP16 (n_ckpt = 1): two sweeps instead of three; method bytes per point and
    # step: forward 44 + store 4 + adjoint 44 + read 4 + gradient read-modify-write 8 = 104
    holder = []
    t = timed(torch, lambda: holder.append(p.gradient(shot, res, 1, "f16")), 1, 0)
    gr = holder[0]
    gp = w.npts * w.nt / t / 1e9
    out["f16_whole_run"] = {"GPts/s": round(gp, 3), "ms": round(t * 1e3, 1), "checkpoints": 0,
                            "store_GB": round(w.nt * 2 * w.npts * 2 / 1e9, 1),
                            "method_hbm_frac_104B": round(gp * 104 / HBM_PEAK_GBS, 4),
                            "rel_l2_vs_f32_checkpoints": float(((gr.double() - ref).norm() / ref.norm()).item())}
    # one FWI iteration: modelling (for the residual), then the gradient.  A saving forward keeps the
    # checkpoints (or, with n_ckpt = 1, the whole run in FP16) and the gradient reuses them: one
    # forward sweep less (48 checkpoints: 3 sweeps instead of 4; whole run: 2 instead of 3)
    fwi = {}
    for label, n in (("48_f16_checkpoints", 48), ("whole_run_f16", 1)):
        def plain(n=n):
            p.forward(shot)
            p.gradient(shot, res, n, "f16")

        def saved(n=n):
            p.forward(shot, save_ckpt=n, ckpt_dtype="f16")
            p.gradient(shot, res, 0)

        t_plain = timed(torch, plain, 1, 0)
        t_saved = timed(torch, saved, 1, 0)
        fwi[label] = {"forward_then_gradient_s": round(t_plain, 4), "saving_forward_then_reuse_s": round(t_saved, 4),
                      "speedup": round(t_plain / t_saved, 3)}
    out["fwi_iteration"] = fwi
    out["scheme"] = p.get_option("scheme")
    p.close()
    return out


def copy_bandwidth(torch, nbytes=1 << 31, reps=10):
    """Device-to-device copy rate (bytes read + written per second) of torch's copy kernel on 2 GiB,
    and the read-only rate of torch's sum over the same 2 GiB."""
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2 * nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    # read-only rate of the same buffer (torch's sum reduction)
    a.sum()
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        a.sum()
    e1.record()
    torch.cuda.synchronize()
    rgbs = nbytes * reps / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs, rgbs


def measure_batched(torch, prop, nt, nshot):
    """Batched checkpointed gradient of many shots vs the plain per-shot baseline (FP32 checkpoints,
    one call per shot, per-shot host FP64 sum)."""
    from paper_2004_10519_amd import configs
    w, geo = configs.batch_64(nshot=nshot, nt=nt)
    log(f"[bench] generating {w.name} model {w.shape} ({nshot} shots) ...")
    arrs = w.model_list(progress=lambda msg: log(f"[bench]   model: {msg}"))
    g = prop.Grid(w.shape, w.spacing, space_order=w.space_order, nbl=w.nbl, dt=w.dt, nt=w.nt, v_ref=w.v_ref)
    dev_ = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]
    del arrs
    p = prop.Propagator(prop.TTI, g, dev_)
    if TTI_SCHEME is not None:
        p.set_option("scheme", TTI_SCHEME)
    wav = torch.from_numpy(np.ascontiguousarray(w.wavelet()[:, :1])).cuda()
    shots = [prop.Shot(src, wav, rec, win_origin=o, win_shape=n) for (o, n, src, rec) in geo]
    gen = torch.Generator(device="cuda").manual_seed(0)
    res = [torch.randn((w.nt, s.nrec), device="cuda", generator=gen) for s in shots]
    pts = sum(int(np.prod(n)) for (_, n, _, _) in geo)
    log(f"[bench] {nshot} shots, {pts / 1e6:.1f} M window points, {w.nt} steps")
    # batched (FP16 checkpoints, device FP64 sum); issued in calls of up to 16 shots so that
    # progress is reported; each call adds its shots into gb in shot order
    chunk = 16
    p.set_option("graph", 1)
    p.set_option("autotune", 1)
    gb = torch.zeros(w.arr_shape, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(0, nshot, chunk):
        p.gradient_batched(shots[c:c + chunk], res[c:c + chunk], gb, n_ckpt=48, ckpt_dtype="f16")
        torch.cuda.synchronize()
        log(f"[bench]   batched: {min(c + chunk, nshot)}/{nshot} shots, {time.perf_counter() - t0:.1f} s")
    tb = time.perf_counter() - t0
    tiles_b = {k: p.get_option("info_" + k) for k in ("tile1", "zc1", "tile2", "zc2")}
    graphs_b = p.get_option("info_graphs")
    groups_b = p.get_option("info_groups")
    # plain: sequential per-shot calls, per-step launches, fixed tiles, FP32 checkpoints, host FP64 sum
    p.set_option("graph", 0)
    p.set_option("autotune", 0)
    gp = np.zeros(w.arr_shape, dtype=np.float64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (s, r) in enumerate(zip(shots, res)):
        gw = p.gradient(s, r, n_ckpt=48, ckpt_dtype="f32").cpu().numpy()
        (ox, oy, oz), (nx, ny, nz) = s.win_origin, s.win_shape
        gp[oz:oz + nz, oy:oy + ny, ox:ox + nx] += gw
        if (i + 1) % 8 == 0:
            log(f"[bench]   plain: {i + 1}/{nshot} shots, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    gbh = gb.cpu().numpy()
    err = float(np.linalg.norm(gbh - gp) / np.linalg.norm(gp))
    del gb
    torch.cuda.empty_cache()
    scheme = p.get_option("scheme")
    p.close()
    return {"workload": w.name, "model": list(w.shape), "shots": nshot, "window_points": pts, "time_steps": w.nt,
            "space_order": w.space_order, "checkpoints": 48, "scheme": scheme,
            "batched": {"s": round(tb, 2), "GPts/s": round(pts * w.nt / tb / 1e9, 3), "checkpoint_dtype": "f16",
                        "graphs": graphs_b, "last_group_tiles": tiles_b, "groups_last_call": groups_b,
                        "method_hbm_frac_156B": round(pts * w.nt / tb / 1e9 * 156 / HBM_PEAK_GBS, 4)},
            "plain": {"s": round(tp, 2), "GPts/s": round(pts * w.nt / tp / 1e9, 3), "checkpoint_dtype": "f32"},
            "speedup": round(tp / tb, 3), "rel_l2_batched_vs_plain": err}


def main():
    global TTI_SCHEME, FIXED_TILES
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nt", type=int, default=None, help="override the number of time steps (short runs)")
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--space-order", type=int, default=None,
                    help="space order of the main TTI run instead of 12 (profiles of other stencil widths)")
    ap.add_argument("--only-main", action="store_true", help="skip the adjoint, elastic and gradient paths")
    ap.add_argument("--batched", type=int, default=64, metavar="NSHOT",
                    help="shots of the batched-vs-plain gradient comparison (default 64, the full workload; "
                         "0 skips it)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--budget", type=float, default=500.0,
                    help="wall-time budget in seconds: a measured leg that would end past it is skipped")
    ap.add_argument("--tiles", default=None, metavar="T1,Z1,T2,Z2",
                    help="fixed tile variants and z-chunks of the two TTI passes instead of the autotuner "
                         "(counter runs: the profiler serialises launches, which would mislead the autotuner)")
    ap.add_argument("--scheme", type=int, default=TTI_SCHEME, choices=(0, 2, 3, 4),
                    help="TTI step scheme: 0 two passes with six-field temporaries, "
                         "2 one fused pass, 3 two passes with four-field temporaries, "
                         "4 two fused single-field passes (default: the library's choice per space "
                         "order, fused up to 8)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one device copy of 512 MiB (calibrates rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    TTI_SCHEME = args.scheme
    if args.tiles:
        FIXED_TILES = [int(v) for v in args.tiles.split(",")]
        if len(FIXED_TILES) != 4:
            ap.error("--tiles takes four integers")
    if args.gpus != 1:
        print(f"bench.py: measures one GPU only; --gpus {args.gpus} is not supported "
              "(several GPUs would each take a shot group and sum the gradient with one all-reduce)",
              file=sys.stderr)
        sys.exit(2)

    T0 = time.perf_counter()
    import torch
    from paper_2004_10519_amd import configs, prop
    prop.lib()
    torch.cuda.set_device(0)

    if args.copy_probe:
        a = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("[bench] copy probe: 536870912 bytes read, 536870912 bytes written")
        del a, b

    w = configs.tti3d_512(nt=args.nt or 3000, n=args.size)
    if args.space_order:
        w = dataclasses.replace(w, space_order=args.space_order)
    log(f"[bench] generating {w.name} model {w.shape} ...")
    t0 = time.perf_counter()
    p, shot = setup_tti(w, torch, prop)
    log(f"[bench] setup {time.perf_counter() - t0:.1f} s; timing {args.steps} step(s) after {args.warmup} warm-up")
    npts = w.npts

    def run():
        p.forward(shot)

    for i in range(args.warmup):
        run()
        torch.cuda.synchronize()
        log(f"[bench] {w.name}: warm-up {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    p.set_timing(True)
    t_step = timed(torch, run, args.steps, 0, label=w.name)
    kt = {k: p.kernel_time(k) for k in (0, 1)}
    kt = {k: v for k, v in kt.items() if v[1] > 0}   # the fused scheme launches class 1 only
    p.set_timing(False)
    gpts = npts * w.nt / t_step / 1e9
    log(f"[bench] {w.name}: {t_step * 1e3:.1f} ms/step, {gpts:.2f} GPts/s")

    dom = max(kt, key=lambda k: kt[k][0])
    ms_tot, nl, name = kt[dom]
    avg_s = ms_tot / 1e3 / max(nl, 1)
    scheme = p.get_option("scheme")
    tiles = [p.get_option(k) for k in ("info_tile1", "info_zc1", "info_tile2", "info_zc2")]
    # achieved: the method's algorithmic bytes of one time step (44 B per point, FP32) times the points
    # one launch of the dominant kernel updates, over its mean launch time
    method_b = METHOD_BYTES_PER_PT["tti"]
    achieved = method_b * npts / avg_s / 1e9
    traffic = traffic_from_profiles(dom, npts, scheme, tiles[2 * dom:2 * dom + 2], w.space_order)
    t_ts = t_step / w.nt
    roof = {"bound": "hbm", "kernel": name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "basis": f"{method_b} B/pt (one TTI time step: read p, q at two levels and m, eps, delta, theta, "
                     f"phi; write p+, q+) x {npts} points per launch",
            "algorithmic_bytes_per_launch": method_b * npts, "scheme": scheme,
            "mean_launch_ms": round(avg_s * 1e3, 4), "launches": nl,
            "step_frac": round(method_b * npts / t_ts / 1e9 / HBM_PEAK_GBS, 4),
            "kernels": {kt[k][2]: {"mean_launch_ms": round(kt[k][0] / max(kt[k][1], 1), 4),
                                   "own_bytes_per_point": kernel_bytes(k, scheme),
                                   "GBps_own_bytes": round(kernel_bytes(k, scheme) * npts /
                                                           (kt[k][0] / 1e3 / max(kt[k][1], 1)) / 1e9, 1)}
                        for k in kt}}
    roof["tiles"] = {"pass1": {"variant": tiles[0], "zc": tiles[1]}, "pass2": {"variant": tiles[2], "zc": tiles[3]},
                     "autotuned": not FIXED_TILES}
    if not args.copy_probe:   # (counter runs calibrate on the probe copy alone)
        copy_gbs, read_gbs = copy_bandwidth(torch)
        roof["copy_GBps"] = round(copy_gbs, 1)
        roof["read_GBps"] = round(read_gbs, 1)
        roof["frac_of_copy"] = round(achieved / copy_gbs, 4)
        log(f"[bench] device copy {copy_gbs:.0f} GB/s; dominant kernel {achieved:.0f} GB/s algorithmic")

    paths = {}
    if not args.only_main:
        log("[bench] TTI adjoint ...")
        paths["tti_adjoint"] = measure_tti_adjoint(torch, prop, w, p, shot)
    out = {"metric": f"GPts/s (TTI forward, {w.shape[0]}^3, so{w.space_order})", "value": round(gpts, 3), "unit": "GPts/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 2),
           "time_steps_per_step": w.nt, "ms_per_time_step": round(t_ts * 1e3, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded layered TTI model, Ricker source)",
           "config": {"workload": w.name, "grid": list(w.shape), "spacing_m": w.spacing[0],
                      "space_order": w.space_order, "time_steps": w.nt, "nbl": w.nbl, "receivers": len(w.rec_xyz),
                      "parallelism": "single GPU"},
           "roofline": roof}
    if w.space_order in TTI_PAPER_FLOPS_PER_PT:
        fpp = TTI_PAPER_FLOPS_PER_PT[w.space_order]
        out["flop_equivalent"] = {"TFLOP/s": round(gpts * fpp / 1e3, 2), "flop_per_point": fpp,
                                  "basis": "the paper's optimised TTI FLOP count per point (Table ttiFLOPs)"}
    p.close()
    del p
    torch.cuda.empty_cache()
    # the remaining legs, each started only while the whole run stays inside the time budget (the
    # estimates are generous wall times on one MI355X; a skipped leg is recorded as such)
    def leg(name, est_s, fn, where):
        left = args.budget - (time.perf_counter() - T0)
        if left < est_s:
            where[name] = {"skipped": f"time budget: {left:.0f} s left, the leg takes about {est_s:.0f} s"}
            log(f"[bench] {name}: skipped ({left:.0f} s left)")
            return
        where[name] = fn()
        torch.cuda.empty_cache()

    if not args.only_main:
        nt_el = 2000 if args.nt is None else min(args.nt, 2000)
        nt_gr = 2000 if args.nt is None else min(args.nt, 2000)
        leg("elastic", 60, lambda: measure_elastic(torch, prop, nt_el), paths)
        leg("tti_gradient", 60, lambda: measure_gradient(torch, prop, nt_gr), paths)
        out["paths"] = paths
    if not args.no_cpu:
        log("[bench] CPU baseline (FP64 checker) ...")
        out["cpu_baseline"] = cpu_baseline(w)
    if not args.only_main:
        if args.batched:
            leg("batched_vs_plain", 200, lambda: measure_batched(torch, prop, args.nt or 1500, args.batched), paths)
        log("[bench] 2D marine elastic (free surface) ...")
        leg("elastic_2d_marine", 15, lambda: measure_marine(torch, prop), paths)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
