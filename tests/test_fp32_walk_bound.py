"""The float32 arithmetic of the kernel's DDA walk, emulated in numpy, stays
inside the oracle's decision windows.

The oracle flags a column when two crossing parameters of its walk lie within
a relative 1e-5 of each other (the ray passes a tile corner, Sec. 2.1); on
every other column the kernel must take the same decisions.  That holds when
each float32 crossing parameter is within a relative 5e-6 of the exact one.
The kernel forms each ray component in double and rounds it once to float32,
takes 1/r with the hardware reciprocal (within one ulp), and computes the k-th
crossing as fma(k, |1/r|, t0) with t0 = (X0 - x) / r (X0 - x exact).  This
test emulates those steps (float32 rounding of each operation; the reciprocal
moved one ulp either way as its worst case) over random poses and columns at
the largest map side and frame width, and bounds the relative error of every
crossing parameter a walk of 2N crossings can reach.  CPU only."""
import math

import numpy as np

F32 = np.float32
U = 2.0 ** -24                     # float32 unit roundoff


def _f32(v):
    return np.asarray(v, np.float64).astype(F32)


def _fma32(a, b, c):
    # a*b is exact in double for float32 operands; the sum is rounded twice
    # (to double, then to float32), which can add at most one float32 ulp on
    # rare halfway cases: the bound below allows for it.
    return _f32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def _rays(rng, n, N, Wd, fov=60.0):
    tanH = math.tan(math.radians(fov) / 2)
    th = _f32(rng.uniform(0, 2 * math.pi, n)).astype(np.float64)
    x = _f32(rng.uniform(1.0, N - 1.0, n))
    y = _f32(rng.uniform(1.0, N - 1.0, n))
    col = rng.integers(0, Wd, n)
    k = (2 * col + 1 - Wd) * (tanH / Wd)
    rx = np.cos(th) - k * np.sin(th)          # the exact ray (double)
    ry = np.sin(th) + k * np.cos(th)
    return x, y, rx, ry


def _crossings_rel_err(x, rx, N, ulps):
    """Max relative error over k < 2N of fma(k, |1/r32|, (X0 - x) / r32) where
    1/r32 is the correctly rounded reciprocal moved by `ulps` float32 ulps."""
    r32 = _f32(rx)
    inv = _f32(1.0 / r32.astype(np.float64))
    inv = np.nextafter(inv, F32(np.inf) if ulps > 0 else F32(-np.inf)) if ulps else inv
    X0 = np.where(rx > 0, np.floor(x) + 1, np.floor(x)).astype(F32)
    d = (X0 - x)                                           # exact in float32
    assert (d.astype(np.float64) == X0.astype(np.float64) - x.astype(np.float64)).all()
    t0 = _f32(d.astype(np.float64) * inv.astype(np.float64))
    dt = np.abs(inv)
    worst = 0.0
    for kk in range(0, 2 * N):
        t32 = _fma32(np.full_like(t0, kk), dt, t0).astype(np.float64)
        exact = (d.astype(np.float64) + kk * np.sign(rx)) / rx
        rel = np.abs(t32 - exact) / np.abs(exact)
        # a crossing beyond any walk's reach (t > 2N / |r|... bounded by the map
        # diagonal) is never compared
        reach = exact <= 2.0 * N
        if reach.any():
            worst = max(worst, float(rel[reach].max()))
    return worst


def test_ray_components_rounded_once_from_double():
    rng = np.random.default_rng(3)
    x, y, rx, ry = _rays(rng, 400_000, 64, 128)
    for r in (rx, ry):
        r32 = _f32(r).astype(np.float64)
        nz = r != 0
        assert (np.abs(r32[nz] - r[nz]) <= U * np.abs(r[nz])).all()


def test_float32_formed_components_would_leave_the_window():
    # The same components formed in float32 (cos, sin rounded, then a float
    # multiply-add) lose most digits where dir and the column offset cancel:
    # the relative error then exceeds the oracle's 1e-5 window on some rays,
    # which is why the kernel forms them in double.
    rng = np.random.default_rng(4)
    tanH = math.tan(math.pi / 6)
    n, Wd = 400_000, 64
    th = _f32(rng.uniform(0, 2 * math.pi, n)).astype(np.float64)
    col = rng.integers(0, Wd, n)
    cam = _f32((2 * col + 1 - Wd) / Wd)
    cs, sn = _f32(np.cos(th)), _f32(np.sin(th))
    px = _f32(-sn.astype(np.float64) * F32(tanH))
    rx32 = _fma32(cam, px, cs).astype(np.float64)
    rx = np.cos(th) - ((2 * col + 1 - Wd) / Wd) * tanH * np.sin(th)
    rel = np.abs(rx32 - rx) / np.abs(rx)
    assert rel.max() > 1e-5


def test_crossing_parameters_within_window():
    rng = np.random.default_rng(5)
    N, Wd = 64, 128
    x, y, rx, ry = _rays(rng, 60_000, N, Wd)
    worst = 0.0
    for pos, r in ((x, rx), (y, ry)):
        nz = np.abs(r) > 1e-30
        for ulps in (-1, 0, 1):
            worst = max(worst, _crossings_rel_err(pos[nz], r[nz], N, ulps))
    # derived bound: component 1u, reciprocal 2u, product 1u, fma 1u (+1u for
    # the emulation's double rounding) = 6u ~ 3.6e-7
    assert worst <= 6 * U, worst
    # two parameters each this close cannot swap order outside the 1e-5 window
    assert 2 * worst < 1e-5


def test_column_height_from_float32_distance():
    # hh = (H/2) * rcp(t*): with t* within 6u and the reciprocal within 2u the
    # half-height is within 9u of H / (2 t*): far inside the 1e-5 span window,
    # so the row count ceil(hh - 0.5) matches on every unflagged column
    rng = np.random.default_rng(6)
    t = rng.uniform(0.01, 100.0, 200_000)
    t32 = _f32(t * (1 + rng.uniform(-6, 6, t.size) * U))
    for H in (32, 64, 84, 128):
        inv = _f32(1.0 / t32.astype(np.float64))
        for ulps in (-1, 1):
            inv_w = np.nextafter(inv, F32(np.inf) if ulps > 0 else F32(-np.inf))
            hh = _f32(F32(H / 2) * inv_w.astype(np.float64)).astype(np.float64)
            exact = H / (2 * t)
            rel = np.abs(hh - exact) / exact
            assert rel.max() <= 10 * U
            k = np.floor(exact)               # nearest pixel-centre distance k + 0.5
            near = np.minimum(np.abs(exact - (k + 0.5)), np.abs(exact - (k - 0.5)))
            unflagged = near > 1e-5 * exact
            rows32 = np.clip(np.ceil(hh - 0.5), 0, H // 2)
            rows = np.clip(np.ceil(exact - 0.5), 0, H // 2)
            assert (rows32[unflagged] == rows[unflagged]).all()
