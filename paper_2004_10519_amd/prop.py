"""Thin Python binding of the C ABI in ``include/prop.h`` (argument marshalling only).

Every numerical step runs in the HIP library ``libprop.so``; PyTorch provides device memory
and the stream.  If the library is missing this module raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libprop.so")

PROP_OK, PROP_EINVAL, PROP_ENOMEM, PROP_EHIP, PROP_EUNSTABLE, PROP_ESTATE = 0, -1, -2, -3, -4, -5
TTI, ELASTIC = 1, 2
CKPT = {"f32": 0, "f16": 1, "bf16": 2}

EXPORTS = ["prop_create", "prop_cfl_dt", "prop_set_model", "prop_forward", "prop_adjoint", "prop_gradient",
           "prop_image", "prop_forward_batched", "prop_gradient_batched", "prop_image_batched", "prop_read_state", "prop_set_timing",
           "prop_kernel_time", "prop_set_option", "prop_get_option", "prop_ckpt_encode", "prop_ckpt_decode",
           "prop_ckpt_encode_rows", "prop_ckpt_decode_rows", "prop_dot_f64", "prop_dot_f64_noalloc", "prop_destroy",
           "prop_last_error"]

# option / info codes of prop_set_option and prop_get_option
OPTIONS = {"graph": 1, "autotune": 2, "tile1": 3, "tile2": 4, "zc": 5, "xcd": 6, "batch_mb": 7, "scheme": 8, "zc2": 9,
           "el_fused": 10,
           "info_tile1": 101, "info_tile2": 102, "info_zc1": 103, "info_zc2": 104, "info_graphs": 105,
           "info_groups": 106}


class PropError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"prop error {code}: {msg}")
        self.code = code


class CGrid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int32), ("shape", ctypes.c_int64 * 3), ("spacing", ctypes.c_double * 3),
                ("origin", ctypes.c_double * 3), ("space_order", ctypes.c_int32), ("time_order", ctypes.c_int32),
                ("nbl", ctypes.c_int32), ("dt", ctypes.c_double), ("nt", ctypes.c_int32), ("v_ref", ctypes.c_double),
                ("free_surface", ctypes.c_int32)]


class CModel(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p * 5)]


class CShot(ctypes.Structure):
    _fields_ = [("win_origin", ctypes.c_int64 * 3), ("win_shape", ctypes.c_int64 * 3),
                ("nsrc", ctypes.c_int32), ("src_xyz", ctypes.c_void_p), ("src_wavelet", ctypes.c_void_p),
                ("nrec", ctypes.c_int32), ("rec_xyz", ctypes.c_void_p), ("rec_kind", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libprop.so (built by ``paper_2004_10519_amd.build_lib``); raise if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.prop_create.argtypes = [ctypes.POINTER(vp), i32, ctypes.POINTER(CGrid), ctypes.POINTER(CModel), vp]
        L.prop_cfl_dt.argtypes = [i32, ctypes.POINTER(CGrid), dbl, dbl]
        L.prop_cfl_dt.restype = dbl
        L.prop_set_model.argtypes = [vp, ctypes.POINTER(CModel)]
        L.prop_forward.argtypes = [vp, ctypes.POINTER(CShot), vp, i32, i32]
        L.prop_adjoint.argtypes = [vp, ctypes.POINTER(CShot), vp, vp]
        L.prop_gradient.argtypes = [vp, ctypes.POINTER(CShot), vp, vp, i32, i32]
        L.prop_image.argtypes = [vp, ctypes.POINTER(CShot), vp, vp, i32, i32]
        L.prop_image_batched.argtypes = [vp, i32, ctypes.POINTER(CShot), ctypes.POINTER(vp), vp, i32, i32]
        L.prop_forward_batched.argtypes = [vp, i32, ctypes.POINTER(CShot), ctypes.POINTER(vp)]
        L.prop_gradient_batched.argtypes = [vp, i32, ctypes.POINTER(CShot), ctypes.POINTER(vp), vp, i32, i32]
        L.prop_read_state.argtypes = [vp, i32, vp]
        L.prop_set_timing.argtypes = [vp, i32]
        L.prop_kernel_time.argtypes = [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                       ctypes.POINTER(ctypes.c_char_p)]
        L.prop_set_option.argtypes = [vp, i32, i64]
        L.prop_get_option.argtypes = [vp, i32, ctypes.POINTER(i64)]
        L.prop_ckpt_encode.argtypes = [vp, i64, i32, vp, vp, vp]
        L.prop_ckpt_decode.argtypes = [vp, vp, i64, i32, vp, vp]
        L.prop_ckpt_encode_rows.argtypes = [vp, vp, i64, i64, i64, i32, i32, vp, vp, vp, vp, vp]
        L.prop_ckpt_decode_rows.argtypes = [vp, vp, vp, vp, i64, i64, i64, i32, vp, vp, vp]
        L.prop_dot_f64.argtypes = [vp, vp, i64, ctypes.POINTER(dbl), vp]
        L.prop_dot_f64_noalloc.argtypes = [vp, vp, i64, ctypes.POINTER(dbl), vp]
        L.prop_destroy.argtypes = [vp]
        L.prop_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("prop_cfl_dt", "prop_last_error"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int):
    if rc != PROP_OK:
        raise PropError(rc, lib().prop_last_error().decode())


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _dev(t: Optional[torch.Tensor], dtype=torch.float32):
    if t is None:
        return None
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous CUDA {dtype} tensor")
    return t.data_ptr()


@dataclass
class Grid:
    shape: tuple                 # (nx, ny, nz); ny = 1 in 2D
    spacing: tuple
    origin: tuple = (0.0, 0.0, 0.0)
    space_order: int = 8
    nbl: int = 0
    dt: float = 1e-3
    nt: int = 1
    v_ref: float = 1500.0
    free_surface: object = False   # elastic: free surface on the top face (vacuum rows above row nbl);
                                   # "image": the same with the method of images for the tractions

    @property
    def ndim(self) -> int:
        return 2 if self.shape[1] == 1 else 3

    @property
    def arr_shape(self):
        return (self.shape[2], self.shape[1], self.shape[0])

    def c(self, kind: int) -> CGrid:
        g = CGrid()
        g.ndim = self.ndim
        for i in range(3):
            g.shape[i] = int(self.shape[i])
            g.spacing[i] = float(self.spacing[i])
            g.origin[i] = float(self.origin[i])
        g.space_order = int(self.space_order)
        g.time_order = 2 if kind == TTI else 1
        g.nbl = int(self.nbl)
        g.dt = float(self.dt)
        g.nt = int(self.nt)
        g.v_ref = float(self.v_ref)
        g.free_surface = 2 if self.free_surface == "image" else int(bool(self.free_surface))
        return g


@dataclass
class Shot:
    """One source experiment: host coordinates, device wavelet (nt x nsrc), optional window."""
    src_xyz: np.ndarray
    wavelet: Optional[torch.Tensor]
    rec_xyz: np.ndarray
    rec_kind: Optional[np.ndarray] = None
    win_origin: tuple = (0, 0, 0)
    win_shape: tuple = (0, 0, 0)
    _keep: list = field(default_factory=list, repr=False)

    @property
    def nsrc(self) -> int:
        return 0 if self.src_xyz is None else int(np.asarray(self.src_xyz).reshape(len(self.src_xyz), -1).shape[0])

    @property
    def nrec(self) -> int:
        return 0 if self.rec_xyz is None else int(np.asarray(self.rec_xyz).shape[0])

    def c(self) -> CShot:
        s = CShot()
        for i in range(3):
            s.win_origin[i] = int(self.win_origin[i])
            s.win_shape[i] = int(self.win_shape[i])
        src = None if self.src_xyz is None else np.ascontiguousarray(self.src_xyz, dtype=np.float32)
        rec = None if self.rec_xyz is None else np.ascontiguousarray(self.rec_xyz, dtype=np.float32)
        kind = None if self.rec_kind is None else np.ascontiguousarray(self.rec_kind, dtype=np.int32)
        self._keep = [src, rec, kind]
        s.nsrc = 0 if src is None else src.shape[0]
        s.src_xyz = None if src is None else src.ctypes.data
        s.src_wavelet = _dev(self.wavelet)
        s.nrec = 0 if rec is None else rec.shape[0]
        s.rec_xyz = None if rec is None else rec.ctypes.data
        s.rec_kind = None if kind is None else kind.ctypes.data
        return s


def cfl_dt(kind: int, grid: Grid, vmax: float, eps_max: float = 0.0) -> float:
    return float(lib().prop_cfl_dt(kind, ctypes.byref(grid.c(kind)), vmax, eps_max))


class Propagator:
    """A propagator handle for one grid and model (TTI: m, eps, delta, theta, phi; elastic: vp, vs, rho)."""

    def __init__(self, kind: int, grid: Grid, model: Sequence[torch.Tensor], stream=None):
        self.kind, self.grid = kind, grid
        self._h = ctypes.c_void_p()
        self._model = list(model)
        self._stream = _stream(stream)
        cg = grid.c(kind)
        cm = self._cmodel(self._model)
        _check(lib().prop_create(ctypes.byref(self._h), kind, ctypes.byref(cg), ctypes.byref(cm), self._stream))

    def _cmodel(self, model) -> CModel:
        cm = CModel()
        for i, t in enumerate(model):
            cm.p[i] = _dev(t)
        return cm

    def set_model(self, model: Sequence[torch.Tensor]):
        self._model = list(model)
        _check(lib().prop_set_model(self._h, ctypes.byref(self._cmodel(self._model))))

    def _win_shape(self, shot: Shot):
        if any(shot.win_shape):
            nx, ny, nz = shot.win_shape
            return (nz, ny, nx)
        return self.grid.arr_shape

    def forward(self, shot: Shot, out: Optional[torch.Tensor] = None, save_ckpt: int = 0,
                ckpt_dtype: str = "f16") -> torch.Tensor:
        """Traces of one shot.  save_ckpt = n >= 1 also keeps the checkpoints that gradient / image with
        n_ckpt = n and this ckpt_dtype use, so that they skip their forward sweep (n_ckpt = 0 there
        asks for that reuse)."""
        nt = self.grid.nt
        if out is None:
            out = torch.empty((nt, shot.nrec), dtype=torch.float32, device="cuda")
        cs = shot.c()
        _check(lib().prop_forward(self._h, ctypes.byref(cs), _dev(out) if shot.nrec else None, int(save_ckpt),
                                  CKPT[ckpt_dtype]))
        return out

    def adjoint(self, shot: Shot, rec: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:
            out = torch.empty((self.grid.nt, shot.nsrc), dtype=torch.float32, device="cuda")
        cs = shot.c()
        _check(lib().prop_adjoint(self._h, ctypes.byref(cs), _dev(rec) if shot.nrec else None,
                                  _dev(out) if shot.nsrc else None))
        return out

    def gradient(self, shot: Shot, residual: torch.Tensor, n_ckpt: int = 48, ckpt_dtype: str = "f16",
                 out: Optional[torch.Tensor] = None) -> torch.Tensor:
        if out is None:   # elastic: the gradients with respect to vp, vs and rho, stacked
            shp = self._win_shape(shot)
            out = torch.empty(((3,) + shp) if self.kind == ELASTIC else shp, dtype=torch.float32, device="cuda")
        cs = shot.c()
        _check(lib().prop_gradient(self._h, ctypes.byref(cs), _dev(residual) if shot.nrec else None, _dev(out),
                                   int(n_ckpt), CKPT[ckpt_dtype]))
        return out

    def image(self, shot: Shot, rec_in: torch.Tensor, n_ckpt: int = 48, ckpt_dtype: str = "f16",
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Zero-lag cross-correlation image sum_k sum_f f^k y_f^k of one shot (y driven by rec_in)."""
        if out is None:
            out = torch.empty(self._win_shape(shot), dtype=torch.float32, device="cuda")
        cs = shot.c()
        _check(lib().prop_image(self._h, ctypes.byref(cs), _dev(rec_in) if shot.nrec else None, _dev(out),
                                int(n_ckpt), CKPT[ckpt_dtype]))
        return out

    def image_batched(self, shots: Sequence[Shot], rec_in: Sequence[torch.Tensor], image: torch.Tensor,
                      n_ckpt: int = 48, ckpt_dtype: str = "f16") -> torch.Tensor:
        """Sum of the shots' zero-lag images, accumulated in FP64 into ``image`` (whole grid)."""
        arr = (CShot * len(shots))(*[s.c() for s in shots])
        ptrs = (ctypes.c_void_p * len(shots))(*[_dev(r) for r in rec_in])
        _check(lib().prop_image_batched(self._h, len(shots), arr, ptrs, _dev(image, torch.float64), int(n_ckpt),
                                        CKPT[ckpt_dtype]))
        return image

    def forward_batched(self, shots: Sequence[Shot], outs: Optional[list] = None) -> list:
        if outs is None:
            outs = [torch.empty((self.grid.nt, s.nrec), dtype=torch.float32, device="cuda") for s in shots]
        arr = (CShot * len(shots))(*[s.c() for s in shots])
        ptrs = (ctypes.c_void_p * len(shots))(*[_dev(o) for o in outs])
        _check(lib().prop_forward_batched(self._h, len(shots), arr, ptrs))
        return outs

    def gradient_batched(self, shots: Sequence[Shot], residuals: Sequence[torch.Tensor], grad: torch.Tensor,
                         n_ckpt: int = 48, ckpt_dtype: str = "f16") -> torch.Tensor:
        arr = (CShot * len(shots))(*[s.c() for s in shots])
        ptrs = (ctypes.c_void_p * len(shots))(*[_dev(r) for r in residuals])
        _check(lib().prop_gradient_batched(self._h, len(shots), arr, ptrs, _dev(grad, torch.float64), int(n_ckpt),
                                           CKPT[ckpt_dtype]))
        return grad

    def read_state(self, field_id: int, shape=None) -> torch.Tensor:
        out = torch.empty(shape if shape is not None else self.grid.arr_shape, dtype=torch.float32, device="cuda")
        _check(lib().prop_read_state(self._h, int(field_id), _dev(out)))
        return out

    def set_timing(self, enable: bool):
        _check(lib().prop_set_timing(self._h, int(bool(enable))))

    def set_option(self, name: str, value: int):
        """Set a run-time option: graph, autotune, tile1, tile2, zc, zc2, xcd, batch_mb, scheme, el_fused."""
        _check(lib().prop_set_option(self._h, OPTIONS[name], int(value)))

    def get_option(self, name: str) -> int:
        """Read an option, or info_tile1/2, info_zc1/2 (last TTI launch shape), info_graphs, info_groups."""
        v = ctypes.c_int64()
        _check(lib().prop_get_option(self._h, OPTIONS[name], ctypes.byref(v)))
        return v.value

    def kernel_time(self, kclass: int):
        ms, n, name = ctypes.c_double(), ctypes.c_int64(), ctypes.c_char_p()
        _check(lib().prop_kernel_time(self._h, int(kclass), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(name)))
        return ms.value, n.value, name.value.decode()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().prop_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dot_f64(a: torch.Tensor, b: torch.Tensor, stream=None) -> float:
    res = ctypes.c_double()
    _check(lib().prop_dot_f64(_dev(a), _dev(b), a.numel(), ctypes.byref(res), _stream(stream)))
    return res.value


def dot_f64_noalloc(a: torch.Tensor, b: torch.Tensor, stream=None) -> float:
    """dot_f64 through the allocation-free entry point (static device scratch)."""
    res = ctypes.c_double()
    _check(lib().prop_dot_f64_noalloc(_dev(a), _dev(b), a.numel(), ctypes.byref(res), _stream(stream)))
    return res.value


def ckpt_encode(f: torch.Tensor, dtype: str, stream=None):
    """Returns (codes, scale) with codes int16 (f16/bf16 bit patterns) or float32 (f32)."""
    n = f.numel()
    codes = torch.empty(n, dtype=torch.float32 if dtype == "f32" else torch.int16, device="cuda")
    scale = torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib().prop_ckpt_encode(_dev(f), n, CKPT[dtype], codes.data_ptr(), scale.data_ptr(), _stream(stream)))
    return codes, scale


def ckpt_decode(codes: torch.Tensor, scale: torch.Tensor, dtype: str, stream=None) -> torch.Tensor:
    n = codes.numel()
    f = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().prop_ckpt_decode(codes.data_ptr(), scale.data_ptr(), n, CKPT[dtype], f.data_ptr(), _stream(stream)))
    return f


def ckpt_encode_rows(a: torch.Tensor, b: torch.Tensor, pair: bool, dtype: str, stream=None):
    """Row codec of the gradient's stores on dense (nz, ny, nx) fields: pair = True codes a and a - b
    (a checkpoint pair), pair = False codes a and b independently.  Returns (codes_a, codes_b, scales_a,
    scales_b): int16 bit patterns (nz, ny, nx) and FP32 scales (nz, ny), one per x-row."""
    nz, ny, nx = a.shape
    ca = torch.empty(a.shape, dtype=torch.int16, device="cuda")
    cb = torch.empty(a.shape, dtype=torch.int16, device="cuda")
    sa = torch.empty((nz, ny), dtype=torch.float32, device="cuda")
    sb = torch.empty((nz, ny), dtype=torch.float32, device="cuda")
    _check(lib().prop_ckpt_encode_rows(_dev(a), _dev(b), nx, ny, nz, int(bool(pair)), CKPT[dtype], ca.data_ptr(),
                                       cb.data_ptr(), sa.data_ptr(), sb.data_ptr(), _stream(stream)))
    return ca, cb, sa, sb


def ckpt_decode_rows(ca: torch.Tensor, cb: torch.Tensor, sa: torch.Tensor, sb: torch.Tensor, dtype: str, stream=None):
    """Inverse of the pair codec: (cur, prev) with cur = s_a a, prev = cur - s_b b."""
    nz, ny, nx = ca.shape
    cur = torch.empty(ca.shape, dtype=torch.float32, device="cuda")
    prev = torch.empty(ca.shape, dtype=torch.float32, device="cuda")
    _check(lib().prop_ckpt_decode_rows(ca.data_ptr(), cb.data_ptr(), sa.data_ptr(), sb.data_ptr(), nx, ny, nz,
                                       CKPT[dtype], cur.data_ptr(), prev.data_ptr(), _stream(stream)))
    return cur, prev


class TTIModelling(torch.autograd.Function):
    """d = F(m) for one shot; backward gives grad_m = (dF/dm)^T grad_d through prop_gradient
    (checkpointed forward recomputation + adjoint + imaging condition).

    The forward run keeps its checkpoints (save_ckpt = n_ckpt), so the backward pass reuses them and
    skips a forward sweep, unless the handle's model or checkpoints changed in between (then it runs
    the full checkpointed gradient).  m is the whole-grid model; the gradient of a shot on a window is
    zero outside that window."""

    @staticmethod
    def forward(ctx, m, prop: Propagator, aniso: Sequence[torch.Tensor], shot: Shot, n_ckpt: int = 48,
                ckpt_dtype: str = "f16"):
        model = [m] + list(aniso)
        prop.set_model(model)
        ctx.prop, ctx.shot, ctx.n_ckpt, ctx.ckpt_dtype = prop, shot, n_ckpt, ckpt_dtype
        ctx.model = prop._model
        ctx.m_shape = m.shape
        return prop.forward(shot, save_ckpt=n_ckpt, ckpt_dtype=ckpt_dtype)

    @staticmethod
    def backward(ctx, grad_d):
        prop, shot = ctx.prop, ctx.shot
        res = grad_d.contiguous()
        g = None
        if prop._model is ctx.model:
            try:
                g = prop.gradient(shot, res, 0)   # the forward run's checkpoints
            except PropError as e:
                if e.code != PROP_ESTATE:
                    raise
        if g is None:
            prop.set_model(ctx.model)
            g = prop.gradient(shot, res, ctx.n_ckpt, ctx.ckpt_dtype)
        if any(shot.win_shape):
            (ox, oy, oz), (nx, ny, nz) = shot.win_origin, shot.win_shape
            full = torch.zeros(ctx.m_shape, dtype=g.dtype, device=g.device)
            full[oz:oz + nz, oy:oy + ny, ox:ox + nx] = g
            g = full
        return g, None, None, None, None, None
