"""Pins of the oracle's sparse operators, checkpoint codec, wavelet and damping (no GPU)."""
import math

import numpy as np
import pytest

from paper_2004_10519_amd import inputs

from codec_cases import rows_fixture


@pytest.mark.parametrize("shape", [(9, 7, 6), (12, 1, 10)])
def test_interpolation_exact_on_multilinear_and_injection_is_transpose(orc, shape):
    g = orc.Grid(shape, (10.0, 12.0, 8.0), origin=(5.0, -3.0, 2.0), space_order=4)
    nx, ny, nz = shape
    rng = np.random.default_rng(0)
    npt = 25
    pts = [rng.uniform(g.origin[ax], g.origin[ax] + (g.shape[ax] - 1) * g.spacing[ax], npt) for ax in g.axes()]
    xyz = np.stack(pts, axis=1)
    xyz[0] = [g.origin[ax] + (g.shape[ax] - 1) * g.spacing[ax] for ax in g.axes()]  # last-node clamp
    xyz[1] = [g.origin[ax] for ax in g.axes()]
    sp = orc.sparse_setup(g, xyz)
    Z, Y, X = np.meshgrid(g.origin[2] + np.arange(nz) * g.spacing[2], g.origin[1] + np.arange(ny) * g.spacing[1],
                          g.origin[0] + np.arange(nx) * g.spacing[0], indexing="ij")
    if g.ndim == 3:
        f = (1 + 0.01 * X) * (2 - 0.02 * Y) * (0.5 + 0.03 * Z)
        exact = (1 + 0.01 * xyz[:, 0]) * (2 - 0.02 * xyz[:, 1]) * (0.5 + 0.03 * xyz[:, 2])
    else:
        f = (1 + 0.01 * X) * (0.5 + 0.03 * Z)
        exact = (1 + 0.01 * xyz[:, 0]) * (0.5 + 0.03 * xyz[:, 1])
    assert np.abs(orc.interp(sp, f) - exact).max() < 1e-12
    assert np.allclose(sp.w.sum(axis=1), 1.0) and (sp.w >= 0).all()
    u = rng.standard_normal(g.arr_shape)
    v = rng.standard_normal(npt)
    inj = np.zeros(g.arr_shape)
    orc.inject(sp, inj, v)
    assert abs(np.vdot(orc.interp(sp, u), v) - np.vdot(u, inj)) < 1e-12 * np.abs(v).sum() * np.abs(u).max()
    with pytest.raises(ValueError):
        bad = xyz.copy()
        bad[0, 0] = g.origin[0] + nx * g.spacing[0]
        orc.sparse_setup(g, bad)


def test_staggered_receiver_grid(orc):
    g = orc.Grid((6, 5, 7), (10.0, 10.0, 10.0), space_order=4)
    sp = orc.sparse_setup(g, np.array([[20.0, 10.0, 35.0]]), stagger=orc.VZ_STAGGER)
    f = np.zeros(g.arr_shape)
    f[3, 1, 2] = 1.0  # vz stored at k = 3 lives at z = 35 m
    assert abs(orc.interp(sp, f)[0] - 1.0) < 1e-15


def test_ricker():
    f0, dt, nt = 10.0, 1e-4, 4001
    w = inputs.ricker(f0, dt, nt).astype(np.float64)
    assert abs(w[1000] - 1.0) < 1e-7 and np.argmax(w) == 1000
    # integral over t >= 0 equals -S(0), S(t) = (t - t0) exp(-(pi f0 (t - t0))^2) the antiderivative
    assert abs(np.trapezoid(w, dx=dt) - 0.1 * math.exp(-math.pi ** 2)) < 1e-9
    t = np.arange(nt) * dt - 0.1
    sec = (t ** 2 * (math.pi * f0) ** 2)
    # the Ricker is minus the normalised second derivative of a Gaussian
    g = np.exp(-sec)
    d2 = np.gradient(np.gradient(g, dt), dt)
    assert np.abs(-d2 / (2 * (math.pi * f0) ** 2) - w)[5:-5].max() < 1e-3


def test_damping_profile(orc):
    g = orc.Grid((30, 28, 26), (10.0, 12.0, 8.0), space_order=8, nbl=6, dt=1e-3, vref=2000.0)
    k = orc.damping_kappa(g)
    assert np.abs(k[6:-6, 6:-6, 6:-6]).max() == 0.0
    assert np.allclose(k, k[::-1, ::-1, ::-1])
    kmax = [3 * 2000.0 * math.log(1000) / (2 * 6 * h) for h in g.spacing]
    assert abs(k[13, 14, 0] - kmax[0]) < 1e-9 and abs(k[0, 0, 0] - sum(kmax)) < 1e-9
    g2 = orc.Grid((30, 1, 26), (10.0, 1.0, 8.0), space_order=8, nbl=6, dt=1e-3, vref=2000.0)
    assert orc.damping_kappa(g2)[10, 0, 10] == 0.0  # no y layer in 2D
    assert np.all(orc.elastic_damp(g) <= 1.0) and orc.elastic_damp(g)[13, 14, 15] == 1.0


def _all_f16():
    v = np.arange(0, 0x7C00, dtype=np.uint16).view(np.float16).astype(np.float64)  # finite, >= 0
    return v


def test_codec_f16_is_nearest_even(orc):
    rng = np.random.default_rng(7)
    f = (rng.standard_normal(5000) * 10.0 ** rng.uniform(-6, 2, 5000)).astype(np.float32)
    f[:3] = [0.0, -0.0, 1e-30]
    s, codes = orc.ckpt_encode(f, "f16")
    assert s == 2.0 ** math.ceil(math.log2(np.abs(f).max())) and s / 2 < np.abs(f).max() <= s
    x = np.abs(f.astype(np.float64) / s)
    tab = _all_f16()
    got = np.abs(codes.view(np.float16).astype(np.float64))
    i = np.clip(np.searchsorted(tab, x), 1, len(tab) - 1)
    lo, hi = tab[i - 1], tab[i]
    best = np.where(x - lo < hi - x, lo, hi)
    tie = (x - lo) == (hi - x)
    even = np.where((np.arange(0x7C00)[i - 1] % 2) == 0, lo, hi)
    best = np.where(tie, even, best)
    assert np.array_equal(got, best)
    dec = orc.ckpt_decode(s, codes, "f16")
    assert np.abs(dec - f).max() <= 2.0 ** -12 * s


def test_codec_bf16_is_nearest_even(orc):
    rng = np.random.default_rng(8)
    f = (rng.standard_normal(5000) * 10.0 ** rng.uniform(-3, 3, 5000)).astype(np.float32)
    # exact ties: values halfway between two bf16 numbers
    f[:4] = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.5 + 2 ** -9], dtype=np.float32) * 64
    s, codes = orc.ckpt_encode(f, "bf16")
    x = f.astype(np.float64) / s
    got = (codes.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    # brute force: bf16 neighbours by exponent, nearest with ties to even mantissa
    e = np.floor(np.log2(np.abs(x)))
    ulp = 2.0 ** (e - 7)
    lo = np.floor(np.abs(x) / ulp) * ulp
    hi = lo + ulp
    pick = np.where(np.abs(x) - lo < hi - np.abs(x), lo, hi)
    tie = (np.abs(x) - lo) == (hi - np.abs(x))
    lo_even = (np.round(lo / ulp) % 2) == 0
    pick = np.where(tie, np.where(lo_even, lo, hi), pick) * np.sign(x)
    assert np.array_equal(got, pick)
    assert got[0] == 64 / s * 1.0 and got[1] == 64 / s * (1 + 4 * 2 ** -8)
    assert np.abs(orc.ckpt_decode(s, codes, "bf16") - f).max() <= 2.0 ** -9 * s


def test_codec_zero_field(orc):
    s, codes = orc.ckpt_encode(np.zeros(10, np.float32), "bf16")
    assert s == 1.0 and not codes.any()


def test_codec_subnormal_maximum(orc):
    """A field whose largest magnitude is an FP32 subnormal gets the smallest normal scale 2^-126
    (a subnormal scale would have no finite FP32 reciprocal)."""
    f = np.array([3e-41, -1e-40, 0.0], np.float32)
    for dt in ("f16", "bf16"):
        s, codes = orc.ckpt_encode(f, dt)
        assert s == 2.0 ** -126
        dec = orc.ckpt_decode(s, codes, dt)
        assert np.all(np.isfinite(dec)) and np.abs(dec - f).max() <= 2.0 ** -126 * 2.0 ** -9


def _nearest_even_f16(x):
    """Brute force: the FP16 value nearest to each float64 |x| (all finite FP16 values enumerated), ties to
    the even code; returned with the sign of x."""
    tab = _all_f16()
    ax = np.abs(x)
    i = np.clip(np.searchsorted(tab, ax), 1, len(tab) - 1)
    lo, hi = tab[i - 1], tab[i]
    best = np.where(ax - lo < hi - ax, lo, hi)
    even = np.where((np.arange(0x7C00)[i - 1] % 2) == 0, lo, hi)
    best = np.where((ax - lo) == (hi - ax), even, best)
    return best * np.sign(x)


def _nearest_even_bf16(x):
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    ulp = 2.0 ** (e - 7)
    lo = np.floor(ax / ulp) * ulp
    hi = lo + ulp
    pick = np.where(ax - lo < hi - ax, lo, hi)
    lo_even = (np.round(lo / ulp) % 2) == 0
    pick = np.where((ax - lo) == (hi - ax), np.where(lo_even, lo, hi), pick)
    return np.where(ax > 0, pick, 0.0) * np.sign(x)


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_row_codec_scales_and_nearest_even(orc, dtype):
    f = rows_fixture()
    codes, s = orc.encode_rows(f, dtype)
    mx = np.abs(f).max(axis=-1).astype(np.float64)
    assert s[0, 1] == 1.0 and not codes[0, 1].any()
    assert s[1, 2] == 2.0 ** -126
    nz_ = mx > 0
    # power-of-two scales with max/2 < max|row| <= s (normal maxima)
    assert np.all(np.log2(s) == np.round(np.log2(s)))
    norm = nz_ & (mx >= 2.0 ** -126)
    assert np.all((s[norm] / 2 < mx[norm]) & (mx[norm] <= s[norm]))
    x = f.astype(np.float64) / s[..., None].astype(np.float64)
    want = _nearest_even_f16(x) if dtype == "f16" else _nearest_even_bf16(x)
    got = orc.value16(codes, dtype).astype(np.float64)
    assert np.array_equal(got, want)
    if dtype == "f16":   # the exact ties round to the even FP16 mantissa
        assert got[2, 3, 0] == 1.0 / 2 and got[2, 3, 1] == (1 + 4 * 2 ** -11) / 2


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_checkpoint_pair_codec(orc, dtype):
    """Level + level difference: the difference is coded with its own row scales, so the decoded
    time difference f^c - f^{c-1} carries the 16-bit relative accuracy of the difference itself."""
    rng = np.random.default_rng(23)
    cur = rows_fixture()
    prev = (cur * (1 + 0.05 * rng.standard_normal(cur.shape))).astype(np.float32)
    ca, cb, sa, sb = orc.ckpt_pair_encode_rows(cur, prev, dtype)
    ref_a, ref_sa = orc.encode_rows(cur, dtype)
    ref_b, ref_sb = orc.encode_rows(cur - prev, dtype)
    assert np.array_equal(ca, ref_a) and np.array_equal(cb, ref_b)
    assert np.array_equal(sa, ref_sa) and np.array_equal(sb, ref_sb)
    c2, p2 = orc.ckpt_pair_decode_rows(ca, cb, sa, sb, dtype)
    u = 2.0 ** -11 if dtype == "f16" else 2.0 ** -8   # half an ulp of a value in [1/2, 1), relative to s
    big = np.abs(cur).max(axis=-1) >= 2.0 ** -100    # rows whose codes stay in the normal range
    da = np.abs(c2.astype(np.float64) - cur)
    db = np.abs((c2.astype(np.float64) - p2) - (cur.astype(np.float64) - prev))
    assert np.all(da[big] <= u * sa[big][..., None] * (1 + 1e-6))
    # the decoded difference: its own rounding plus the FP32 roundings of the difference and the decode
    tol_b = u * sb[..., None] + 2.0 ** -23 * (np.abs(cur) + np.abs(prev)) * 2
    assert np.all(db[big] <= tol_b[big])
    # decode is the stated arithmetic: prev = cur - s_b b in FP32
    assert np.array_equal(p2, c2 - sb[..., None] * orc.value16(cb, dtype))
