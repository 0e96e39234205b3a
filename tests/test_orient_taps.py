"""Host logic of the orientation stencil (no GPU): the taps the library
computes for side M and width sigma against the oracle's own smoothed
gradient, which is pinned elsewhere.

The oracle's smoothed gradient of a unit impulse at the origin is the
separable kernel pair g_x[y][x] = g(y) d(x), g_y[y][x] = d(y) g(x); the
library returns the correlation weights t_g[j] = g(-j), t_d[j] = d(-j),
truncated where both kernels' tails fall below 2^-26 of their absolute sums
(or kept whole for small grids), so that
  * the weights equal the impulse response's factors up to FP32 rounding,
  * the dropped tails are within the bound and the radius is the smallest
    compiled one that covers what is needed,
  * correlating a test image with them reproduces the oracle's gradient and
    orientation bins.
"""
import ctypes
import os

import numpy as np
import pytest

import oracle as O
from paper_1304_2062_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1304_2062_amd", "libse2n.so")
RADII = (8, 12, 16, 20, 24, 32)
TOL = 2.0 ** -26
RM = 32


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} is not built (run python -m paper_1304_2062_amd.build)")
    L = ctypes.CDLL(LIB)
    L.se2n_last_error.restype = ctypes.c_char_p
    L.se2n_orient_stencil_taps.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                          ctypes.POINTER(ctypes.c_int)]
    return L


def lib_taps(lib, M, sigma):
    g = np.zeros(2 * RM + 1, dtype=np.float32)
    d = np.zeros(2 * RM + 1, dtype=np.float32)
    r = ctypes.c_int(-1)
    rc = lib.se2n_orient_stencil_taps(M, sigma, g.ctypes.data, d.ctypes.data, ctypes.byref(r))
    assert rc == 0, lib.se2n_last_error()
    return g.astype(np.float64), d.astype(np.float64), r.value


def impulse_kernels(M, sigma):
    """(g, d) on [0, M) from the oracle's smoothed gradient of a unit impulse."""
    delta = np.zeros((M, M))
    delta[0, 0] = 1.0
    gx, _ = O.smoothed_gradient(delta, np.zeros((M, M), dtype=np.uint8), sigma)
    d1 = gx[:, 1].sum()  # sum_y g(y) d(1) = d(1): the smoothing kernel sums to 1
    g = gx[:, 1] / d1
    d = gx[0, :] / g[0]
    return g, d


def needed_radius(k):
    M = k.size
    H = M // 2
    dist = np.minimum(np.arange(M), M - np.arange(M))
    total = np.abs(k).sum()
    for R in range(H + 1):
        if np.abs(k[dist > R]).sum() <= TOL * total:
            return R
    return H


CASES = [(16, 2.0), (24, 2.0), (32, 1.0), (64, 2.0), (72, 2.0), (192, 2.0), (512, 2.0), (2048, 2.0),
         (64, 4.0), (256, 3.0), (512, 6.0), (1024, 1.0), (48, 0.5)]


@pytest.mark.parametrize("M,sigma", CASES)
def test_taps_are_the_oracle_kernels_and_the_radius_is_minimal(lib, M, sigma):
    tg, td, rad = lib_taps(lib, M, sigma)
    g, d = impulse_kernels(M, sigma)
    need = max(needed_radius(g), needed_radius(d))
    H = M // 2
    circle = need >= H
    want = next((r for r in RADII if r >= (H if circle else need)), 0)
    assert rad == want, (need, circle)
    if rad == 0:
        return
    js = np.arange(-(H - 1), H + 1) if circle else np.arange(-need, need + 1)
    # every offset the library uses holds the reflected kernel value
    for j in range(-RM, RM + 1):
        if j in js:
            m = (-j) % M
            assert abs(tg[j + RM] - g[m]) <= 6e-8 * np.abs(g).max() + 1e-300
            assert abs(td[j + RM] - d[m]) <= 6e-8 * np.abs(d).max() + 1e-300
        else:
            assert tg[j + RM] == 0.0 and td[j + RM] == 0.0
    # the dropped tails are within the bound
    kept = np.zeros(M, dtype=bool)
    kept[(-js) % M] = True
    assert np.abs(g[~kept]).sum() <= TOL * np.abs(g).sum() * 1.0001
    assert np.abs(d[~kept]).sum() <= TOL * np.abs(d).sum() * 1.0001


def _correlate(img, taps, axis):
    out = np.zeros_like(img)
    for j in range(-RM, RM + 1):
        if taps[j + RM] != 0.0:
            out += taps[j + RM] * np.roll(img, -j, axis=axis)
    return out


@pytest.mark.parametrize("name,M", [("small", 64), ("small", 72), ("medium", 256)])
def test_stencil_gradient_reproduces_the_oracle(lib, name, M):
    case = synth.make_case(name, M=M)
    f, mask, N, sigma = case["f"], case["mask"], case["N"], case["sigma"]
    tg, td, rad = lib_taps(lib, M, sigma)
    assert rad > 0
    fc = f * (1.0 - mask)
    gx = _correlate(_correlate(fc, tg, 0), td, 1)
    gy = _correlate(_correlate(fc, td, 0), tg, 1)
    ox, oy = O.smoothed_gradient(f, mask, sigma)
    scale = np.hypot(ox, oy).max()
    assert np.abs(gx - ox).max() <= 5e-7 * scale
    assert np.abs(gy - oy).max() <= 5e-7 * scale
    rmap, _ = O.bin_angle(gx, gy, N)
    want, tie = O.orient(f, mask, N, sigma)
    mag = np.hypot(ox, oy)
    clear = tie > np.maximum(1e-4, 1e-5 * scale / np.maximum(mag, 1e-300) * N / (2 * np.pi))
    assert np.array_equal(rmap[clear], want[clear])


@pytest.mark.parametrize("M,sigma", [(100, 2.0), (8, 2.0), (64, 0.0), (64, -1.0), (64, float("nan"))])
def test_bad_arguments_are_rejected(lib, M, sigma):
    g = np.zeros(2 * RM + 1, dtype=np.float32)
    r = ctypes.c_int(0)
    assert lib.se2n_orient_stencil_taps(M, sigma, g.ctypes.data, g.ctypes.data, ctypes.byref(r)) == -1
    assert lib.se2n_last_error()
