"""FP64 CPU oracle of the paper's restoration heuristics: static restoration (SR)
and dynamic restoration (DR), Sec. "Heuristic complements", subsections
"Static restoration (SR)" and "Dynamic restoration (DR)".

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may call this module.  It uses the plain oracle of the
diffusion (``se2n_oracle``) for every integration interval and shares no code
with the GPU library.

What the paper defines
----------------------
The pixels split into a good set G (not corrupted) and a bad set B (f = 0 on
B).  [0, T] is cut into n intervals of tau = T/n with mesh points t_i = i tau.
The equation is integrated over [t_i, t_{i+1}] starting from the state at t_i
"mixed" with the initial lift on G:

    psi(x, y, theta, t_i)  <-  sigma(x, y, t_i) psi(x, y, theta, t_i)  on G,
    sigma = (eps h(x, y, 0) + (1 - eps) h(x, y, t_i)) / h(x, y, t_i),
    h(x, y, t) = max_theta psi(x, y, theta, t),

and left unchanged on B.  DR lets G grow: G_i holds G_{i-1} and every point p
of the boundary of B_{i-1} whose image value f_{i-1}(p) exceeds the mean of
f_{i-1} over the points of B_{i-1} in the 9-point neighbourhood of p;
B_i is the complement of G_i.

Readings taken where the paper is silent
----------------------------------------
* Clock and integrator: the diffusion of ``se2n_oracle`` (its time-scale
  reading), each interval integrated by ``substeps`` Crank-Nicolson steps of
  tau/substeps (default 1) or exactly.
* The mix happens at t_1 .. t_{n-1}; at t_0 sigma is 1 by definition, and the
  state at t_n is projected without a final mix.
* Where h(x, y, t_i) <= 0 on G (possible because the central differences and
  Crank-Nicolson do not preserve positivity) sigma is undefined; the state is
  left unchanged there (sigma = 1).
* DR: the "image at step i-1" is the max projection h(., t_i) of the state that
  the (i-1)-th interval produced, so G_i is formed at t_i from h(., t_i) and
  used for the mix at t_i.  The boundary of B_{i-1} is the set of its points
  with at least one of their 8 neighbours in G_{i-1}; the mean runs over the
  points of B_{i-1} in the 3x3 neighbourhood (the point itself included);
  "larger" is strict; neighbourhoods wrap around (periodic images).  A point
  that joins G at t_i is mixed from then on towards its own value h(p, t_i)
  at the moment it joined (for the initially good points the reference is
  h(p, 0), as in SR): the paper asks that the diffusion stop mattering at a
  point once it is good, and h(p, 0) = 0 on B would pull it to zero instead.
"""
from __future__ import annotations

import numpy as np

from . import se2n_oracle as O


def mix(psi: np.ndarray, href: np.ndarray, good: np.ndarray, eps: float):
    """One mixing step on the good set.  Returns ``(mixed, h)`` with h = max_theta psi.

    On good pixels with h > 0 every orientation is multiplied by
    sigma = (eps href + (1 - eps) h) / h; elsewhere psi is left unchanged.
    """
    psi = np.asarray(psi, dtype=np.float64)
    h = psi.max(axis=0)
    sig = np.ones_like(h)
    m = np.asarray(good, dtype=bool) & (h > 0.0)
    sig[m] = (eps * href[m] + (1.0 - eps) * h[m]) / h[m]
    return psi * sig[None, :, :], h


def _shift(a: np.ndarray, dy: int, dx: int) -> np.ndarray:
    """a[(y + dy) mod M, (x + dx) mod M]."""
    return np.roll(np.roll(a, -dy, axis=0), -dx, axis=1)


def grow(good: np.ndarray, h: np.ndarray):
    """One update of DR's good set.  Returns ``(new, margin)``.

    new[p] is True where p is bad, has a good 8-neighbour, and h[p] is larger
    than the mean of h over the bad points of its 3x3 neighbourhood.  margin is
    h[p] minus that mean on the boundary points of B whose neighbourhood holds
    another bad point (NaN elsewhere): how far each decision is from its tie.
    A boundary point with no other bad point in its neighbourhood is its own
    mean and never joins, in any precision.
    """
    good = np.asarray(good, dtype=bool)
    bad = ~good
    h = np.asarray(h, dtype=np.float64)
    near_good = np.zeros_like(good)
    s = np.zeros_like(h)
    c = np.zeros_like(h)
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            b = _shift(bad, dy, dx)
            s += np.where(b, _shift(h, dy, dx), 0.0)
            c += b
            if dy or dx:
                near_good |= _shift(good, dy, dx)
    boundary = bad & near_good
    mean = np.where(c > 0, s / np.maximum(c, 1.0), 0.0)  # c >= 1 on B: p itself is bad
    new = boundary & (h > mean)
    margin = np.full_like(h, np.nan)
    real = boundary & (c > 1)
    margin[real] = h[real] - mean[real]
    return new, margin


def restore(f, mask, N: int, T: float, beta: float, n: int, eps: float, dynamic: bool = False,
            substeps: int = 1, sigma: float = 2.0, scheme: str = "cn", proj: str = "max", rmap=None,
            join_in=None):
    """SR (``dynamic=False``) or DR of the image f with bad set mask == 1.

    Returns ``(out, rmap, join, info)``: the projected image at T, the
    orientation map used, the mesh index at which each pixel became good
    (0 for the initially good ones, -1 for never; SR: 0 or -1), and, for DR,
    ``info["min_margin"]`` (the smallest |h - mean| over all decisions taken)
    and ``info["flips"]`` (decisions where the oracle's own rule disagrees with
    ``join_in``, with their largest |margin|).

    ``join_in`` (DR only) imposes the good-set updates instead of deciding them:
    pixel p joins at mesh point join_in[p].  This lets the rest of the method
    be compared with another implementation whose decisions were taken in a
    different precision.
    """
    if rmap is None:
        rmap, _ = O.orient(f, mask, N, sigma)
    psi = O.lift(f, mask, rmap, N)
    good = np.asarray(mask) == 0
    href = psi.max(axis=0)  # h(x, y, 0)
    join = np.where(good, 0, -1).astype(np.int32)
    tau = T / n
    min_margin = np.inf
    flips, flip_margin = 0, 0.0
    for i in range(n):
        if i > 0:
            h = psi.max(axis=0)
            if dynamic:
                own, margin = grow(good, h)
                fin = margin[np.isfinite(margin)]
                if fin.size:
                    min_margin = min(min_margin, float(np.abs(fin).min()))
                if join_in is None:
                    new = own
                else:
                    new = (np.asarray(join_in) == i) & ~good
                    diff = new != own
                    if diff.any():
                        flips += int(diff.sum())
                        flip_margin = max(flip_margin, float(np.nanmax(np.abs(margin[diff]))))
                href = np.where(new, h, href)
                join[new] = i
                good = good | new
            psi, _ = mix(psi, href, good, eps)
        psi = O.diffuse(psi, tau, beta, substeps, scheme)
    info = {"min_margin": min_margin, "flips": flips, "flip_max_margin": flip_margin}
    return O.project(psi, proj), rmap, join, info
