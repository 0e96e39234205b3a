"""Seeded synthetic images and corruption masks.

This module only draws inputs: it holds none of the diffusion arithmetic and is
shared by the GPU path, the tests and the benchmark.  The paper shows its
results on 256x256 grey-level photographs that are not available; these
generated images stand in for them with the same kind of content (smooth
shading, straight edges, filled shapes) and the corruption patterns of the
paper's experiments (random pixel loss and grids of horizontal/vertical
stripes of width w, Sec. "Heuristic complements", Table 1).

All randomness comes from ``numpy.random.Generator(PCG64(seed))`` so every
image and mask is reproducible from its seed.  Images are float64 in [0, 1],
indexed ``img[y, x]`` (x = column, the fast index); masks are uint8 with 1 for
a missing pixel (the paper's bad set B) and 0 for a known pixel.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "ImageRecipe",
    "RECIPES",
    "make_image",
    "mask_random",
    "mask_stripes",
    "mask_blotches",
    "make_case",
    "BATCH_SIDES",
    "batch_params",
    "make_batch",
    "TABLE1",
    "stripe_period",
    "table1_case",
]


@dataclasses.dataclass(frozen=True)
class ImageRecipe:
    """Shape counts for one synthetic image."""

    sinusoids: int
    lines: int
    polygons: int


# Counts for the workloads: 64^2 FP64 case, 512^2 case, 2048^2 case.
RECIPES = {
    "small": ImageRecipe(sinusoids=6, lines=4, polygons=3),
    "medium": ImageRecipe(sinusoids=10, lines=20, polygons=12),
    "large": ImageRecipe(sinusoids=20, lines=100, polygons=60),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _wrap(d: np.ndarray, M: int) -> np.ndarray:
    """Minimal periodic image of a coordinate difference on a grid of side M."""
    return (d + M / 2.0) % M - M / 2.0


def _sinusoid_background(rng: np.random.Generator, M: int, count: int) -> np.ndarray:
    x = np.arange(M, dtype=np.float64)
    acc = np.zeros((M, M))
    for _ in range(count):
        while True:
            u, v = rng.integers(-8, 9, size=2)
            if u != 0 or v != 0:
                break
        a = rng.uniform(0.2, 1.0)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        # sin(2pi(u x + v y)/M + phi) as a sum of two outer products (rows y, columns x)
        ax = 2.0 * np.pi * u * x / M
        by = 2.0 * np.pi * v * x / M + phi
        acc += a * (np.outer(np.cos(by), np.sin(ax)) + np.outer(np.sin(by), np.cos(ax)))
    return 0.5 + (0.5 / np.sqrt(max(count, 1))) * acc


def _polygon_coverage(rng: np.random.Generator, M: int) -> tuple[np.ndarray, slice, slice, float]:
    """Anti-aliased coverage of one random star-shaped polygon (4x4 supersampling).

    Returns the coverage on a periodic window around the centre plus the
    intensity; the caller composites it with wrap-around indexing.
    """
    nv = int(rng.integers(3, 9))
    cx, cy = rng.uniform(0.0, M, size=2)
    R = rng.uniform(M / 32.0, M / 6.0)
    ang = np.sort(rng.uniform(0.0, 2.0 * np.pi, size=nv))
    rad = R * rng.uniform(0.5, 1.0, size=nv)
    vx = rad * np.cos(ang)
    vy = rad * np.sin(ang)
    inten = rng.uniform(0.0, 1.0)
    half = int(np.ceil(R)) + 2
    offs = np.arange(-half, half + 1)
    W = offs.size
    ix0 = int(np.floor(cx))
    iy0 = int(np.floor(cy))
    # Sub-sample grid (4x4 per pixel) relative to the polygon centre: column q
    # sits at x0 + (q + 0.5)/4, row t at y0 + (t + 0.5)/4.
    x0 = ix0 - half - cx
    y0 = iy0 - half - cy
    py = y0 + (np.arange(4 * W) + 0.5) / 4.0
    # Crossing-number rule along each sub-sample row: a point is inside when an
    # odd number of edge crossings lie strictly to its right, i.e. between the
    # (2i-1)-th and 2i-th sorted crossing.
    xs = np.full((4 * W, nv), np.inf)
    for i in range(nv):
        x1, y1 = vx[i], vy[i]
        x2, y2 = vx[(i + 1) % nv], vy[(i + 1) % nv]
        cond = (y1 > py) != (y2 > py)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = x1 + (py - y1) * (x2 - x1) / (y2 - y1)
        xs[cond, i] = xint[cond]
    xs.sort(axis=1)
    diff = np.zeros((4 * W, 4 * W + 1), dtype=np.int64)
    rows_idx = np.arange(4 * W)
    for j in range(0, nv - 1, 2):
        a_, b_ = xs[:, j], xs[:, j + 1]
        ok = np.isfinite(a_) & np.isfinite(b_)
        qa = np.clip(np.ceil(4.0 * (a_[ok] - x0) - 0.5), 0, 4 * W).astype(np.int64)
        qb = np.clip(np.ceil(4.0 * (b_[ok] - x0) - 0.5), 0, 4 * W).astype(np.int64)
        np.add.at(diff, (rows_idx[ok], qa), 1)
        np.add.at(diff, (rows_idx[ok], qb), -1)
    inside = np.cumsum(diff[:, : 4 * W], axis=1) > 0
    inside = inside.reshape(W, 4, W, 4).transpose(0, 2, 1, 3)
    cov = inside.mean(axis=(2, 3))
    rows = (iy0 + offs) % M
    cols = (ix0 + offs) % M
    return cov, rows, cols, inten


def _draw_line(rng: np.random.Generator, img: np.ndarray) -> None:
    """Composite one anti-aliased straight line in place.

    Coverage is clip(w/2 + 1/2 - d, 0, 1) with d the distance from the pixel
    centre to the line, measured with periodic minimal-image offsets.  Only the
    band of pixels where the coverage can be non-zero is visited.
    """
    M = img.shape[0]
    px, py = rng.uniform(0.0, M, size=2)
    theta = rng.uniform(0.0, np.pi)
    width = rng.uniform(1.0, 4.0)
    inten = rng.uniform(0.0, 1.0)
    c, s = np.cos(theta), np.sin(theta)
    reach = width / 2.0 + 0.5
    idx = np.arange(M, dtype=np.float64)
    if abs(c) >= abs(s):
        # walk the columns; per column the band spans a few rows
        dx = _wrap(idx + 0.5 - px, M)
        centre = s * dx / c
        half = reach / abs(c)
        lo = np.floor(py - 0.5 + centre - half).astype(np.int64)
        span = int(np.ceil(2.0 * half)) + 2
        yy = lo[None, :] + np.arange(span)[:, None]
        xx = np.broadcast_to(np.arange(M)[None, :], yy.shape)
        dy = _wrap(yy + 0.5 - py, M)
        d = np.abs(-s * dx[None, :] + c * dy)
        rows, cols = yy % M, xx
    else:
        dy = _wrap(idx + 0.5 - py, M)
        centre = c * dy / s
        half = reach / abs(s)
        lo = np.floor(px - 0.5 + centre - half).astype(np.int64)
        span = int(np.ceil(2.0 * half)) + 2
        xx = lo[None, :] + np.arange(span)[:, None]
        yy = np.broadcast_to(np.arange(M)[None, :], xx.shape)
        dxx = _wrap(xx + 0.5 - px, M)
        d = np.abs(-s * dxx + c * dy[None, :])
        rows, cols = yy, xx % M
    cov = np.clip(reach - d, 0.0, 1.0)
    hit = cov > 0.0
    r, q, w = rows[hit], cols[hit], cov[hit]
    img[r, q] = img[r, q] * (1.0 - w) + inten * w


def make_image(seed: int, M: int, recipe: ImageRecipe | str = "small") -> np.ndarray:
    """Return a float64 image of side M in [0, 1]: sinusoids, then polygons, then lines."""
    if isinstance(recipe, str):
        recipe = RECIPES[recipe]
    rng = _rng(seed)
    img = _sinusoid_background(rng, M, recipe.sinusoids)
    for _ in range(recipe.polygons):
        cov, rows, cols, inten = _polygon_coverage(rng, M)
        win = img[np.ix_(rows, cols)]
        img[np.ix_(rows, cols)] = win * (1.0 - cov) + inten * cov
    for _ in range(recipe.lines):
        _draw_line(rng, img)
    return np.clip(img, 0.0, 1.0)


def mask_random(seed: int, M: int, rho: float) -> np.ndarray:
    """Bernoulli(rho) pixel loss; 1 = missing."""
    rng = _rng(seed)
    return (rng.uniform(0.0, 1.0, size=(M, M)) < rho).astype(np.uint8)


def mask_stripes(M: int, width: int, period: int) -> np.ndarray:
    """Grid of horizontal and vertical stripes: rows/cols with (i mod period) < width."""
    idx = np.arange(M)
    band = (idx % period) < width
    return (band[:, None] | band[None, :]).astype(np.uint8)


def mask_blotches(seed: int, M: int, count: int, rmin: float, rmax: float) -> np.ndarray:
    """Union of ``count`` filled ellipses with semi-axes in [rmin, rmax], random centre and rotation."""
    rng = _rng(seed)
    y, x = np.mgrid[0:M, 0:M].astype(np.float64)
    out = np.zeros((M, M), dtype=bool)
    for _ in range(count):
        cx, cy = rng.uniform(0.0, M, size=2)
        a, b = rng.uniform(rmin, rmax, size=2)
        rot = rng.uniform(0.0, np.pi)
        dx = _wrap(x + 0.5 - cx, M)
        dy = _wrap(y + 0.5 - cy, M)
        u = np.cos(rot) * dx + np.sin(rot) * dy
        v = -np.sin(rot) * dx + np.cos(rot) * dy
        out |= (u / a) ** 2 + (v / b) ** 2 <= 1.0
    return out.astype(np.uint8)


def make_case(name: str, seed: int | None = None, M: int | None = None) -> dict:
    """Image, mask and diffusion parameters of a named workload.

    ``small``  : 64^2, 30% random loss, N=16, beta=1, T=0.5, 50 steps (FP64 check case)
    ``medium`` : 512^2, 70% random loss + 3-px stripes every 32 px, N=30, beta=1, T=2, 200 steps
    ``large``  : 2048^2, 80% random loss + 5 elliptic blotches (radius 20-80 px), N=32,
                 beta=1, T=4, 400 steps
    ``M`` overrides the side (same recipe), used for cropped samples and size sweeps.
    """
    if name == "small":
        seed = 1 if seed is None else seed
        M = 64 if M is None else M
        img = make_image(seed, M, "small")
        mask = mask_random(seed + 7919, M, 0.30)
        params = dict(N=16, beta=1.0, T=0.5, n_steps=50)
    elif name == "medium":
        seed = 2 if seed is None else seed
        M = 512 if M is None else M
        img = make_image(seed, M, "medium")
        mask = mask_random(seed + 7919, M, 0.70) | mask_stripes(M, 3, 32)
        params = dict(N=30, beta=1.0, T=2.0, n_steps=200)
    elif name == "large":
        seed = 3 if seed is None else seed
        M = 2048 if M is None else M
        img = make_image(seed, M, "large")
        mask = mask_random(seed + 7919, M, 0.80) | mask_blotches(seed + 104729, M, 5, 20.0, 80.0)
        params = dict(N=32, beta=1.0, T=4.0, n_steps=400)
    else:
        raise ValueError(f"unknown case {name!r}")
    return dict(name=name, seed=seed, M=M, f=img, mask=mask.astype(np.uint8), sigma=2.0, **params)


# Sides of the heterogeneous batch workload (all 2^a 3^b, a >= 3).
BATCH_SIDES = (128, 192, 256, 384, 512, 768, 1024)


def batch_params(count: int = 64, seed0: int = 1000, sides=BATCH_SIDES, Ns=(16, 24, 32),
                 tau: float = 0.01) -> list[dict]:
    """Parameters of a heterogeneous batch, image i drawn with seed seed0 + i:
    M uniform over ``sides``, N uniform over ``Ns``, T ~ U[0.5, 4], n_steps =
    round(T / tau), beta = 1, loss rate rho ~ U(0.5, 0.85)."""
    out = []
    for i in range(count):
        rng = _rng(seed0 + i)
        M = int(sides[rng.integers(len(sides))])
        N = int(Ns[rng.integers(len(Ns))])
        T = float(rng.uniform(0.5, 4.0))
        rho = float(rng.uniform(0.5, 0.85))
        out.append(dict(seed=seed0 + i, M=M, N=N, T=T, n_steps=max(1, int(round(T / tau))), beta=1.0,
                        rho=rho, sigma=2.0))
    return out


def make_batch(count: int = 64, seed0: int = 1000, sides=BATCH_SIDES, Ns=(16, 24, 32),
               tau: float = 0.01) -> list[dict]:
    """``batch_params`` plus each image (the medium recipe) and its Bernoulli(rho) mask."""
    out = []
    for p in batch_params(count, seed0, sides, Ns, tau):
        img = make_image(p["seed"], p["M"], "medium")
        mask = mask_random(p["seed"] + 7919, p["M"], p["rho"]).astype(np.uint8)
        out.append(dict(p, f=img, mask=mask))
    return out


# Rows of Appendix A, Table 1 (reconstructions of 256^2 images whose corrupted
# part is a grid of vertical and horizontal lines of width w): the diffusion
# weight alpha and time T of the paper's clock, the number n of restoration
# steps, the mixing weight eps, the line width w in pixels, the corruption in
# percent, and whether the figure used the dynamic (DR) or the static (SR)
# procedure (Fig. 2: SR; Fig. 3 and the appendix figures: DR).
TABLE1 = {
    "fig2_up": (2.0, 0.8, 200, 0.5, 3, 37, False),
    "fig2_down": (3.0, 0.2, 200, 0.5, 3, 37, False),
    "fig3_up": (4.0, 0.2, 200, 0.5, 3, 37, True),
    "fig3_down": (0.30, 4.0, 160, 0.5, 3, 37, True),
    "figE1": (0.30, 4.0, 160, 0.5, 3, 67, True),
    "figE2": (0.30, 4.0, 160, 0.5, 4, 58, True),
    "figE3": (0.30, 4.0, 160, 0.5, 5, 65, True),
    "figE4": (0.40, 4.0, 120, 0.5, 5, 69, True),
    "figE5": (0.35, 5.0, 160, 0.5, 6, 67, True),
    "figE6": (0.33, 6.0, 180, 0.5, 7, 68, True),
    "figE7": (0.33, 6.0, 250, 0.5, 8, 43, True),
    "figE8": (0.33, 6.0, 250, 0.5, 8, 53, True),
    "figE9": (0.33, 6.0, 250, 0.5, 10, 41, True),
}


def stripe_period(width: int, corruption: float) -> int:
    """Period p of a w-pixel stripe grid whose corrupted share 1 - (1 - w/p)^2 is
    closest to ``corruption`` (a fraction)."""
    return int(round(width / (1.0 - np.sqrt(1.0 - corruption))))


def table1_case(name: str, seed: int = 7, M: int = 256, N: int = 30) -> dict:
    """Input of one Table-1 reconstruction: a seeded image (the medium recipe)
    mapped to [0.1, 1] -- the restoration heuristics assume f > 0 on the good
    set -- and the stripe grid of the row's width and corruption (random
    offset).  The paper's weight alpha and time T_p map to beta = alpha
    (N / 2 pi)^2 and T = T_p / 2 on the clock of the diffusion here; n is the
    number of restoration intervals and eps the mixing weight."""
    alpha, Tp, n, eps, w, pct, dynamic = TABLE1[name]
    rng = _rng(seed + 31)
    p = stripe_period(w, pct / 100.0)
    oy, ox = (int(v) for v in rng.integers(0, p, size=2))
    idx = np.arange(M)
    rows = ((idx + oy) % p) < w
    cols = ((idx + ox) % p) < w
    mask = (rows[:, None] | cols[None, :]).astype(np.uint8)
    f = 0.1 + 0.9 * make_image(seed, M, "medium")
    beta = alpha * (N / (2.0 * np.pi)) ** 2
    return dict(name=name, seed=seed, M=M, N=N, f=f, mask=mask, alpha=alpha, beta=beta, T=Tp / 2.0,
                T_paper=Tp, n=n, eps=eps, width=w, period=p, corruption=float(mask.mean()),
                dynamic=dynamic, sigma=2.0)
