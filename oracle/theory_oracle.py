"""FP64 references for the paper's theoretical statements about the
semi-discrete diffusion, used to cross-check the grid path.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``ap_solve``: the almost-periodic reduction (Sec. "A view through almost
  periodic functions", equations (redap)/(elem), Theorem 1).  A trigonometric
  polynomial sum_s a^s_r exp(i(lambda_s x + mu_s y)) stays one under the
  semi-discrete equation, and each coefficient vector evolves by
      dA/dt = (beta L - diag_r (lambda cos e_r + mu sin e_r)^2) A,
  here on the clock of the grid path (the paper's factor 1/2 dropped, as the
  diffusion oracle does).  The grid path replaces lambda by the central-
  difference symbol sqrt(M) sin(lambda / sqrt(M)), which tends to lambda as M
  grows: the grid result must converge to this one.
* ``theta_continuum``: the N -> infinity limit at one spatial frequency
  (Sec. "The weighting of the metric", equation (contdif-weight) with the
  relation alpha = beta_N (2 pi / N)^2): the coefficient a(theta, t) obeys
      da/dt = -(lambda cos theta + mu sin theta)^2 a + alpha d^2 a / d theta^2,
  solved in the Fourier basis exp(i m theta), |m| <= K, where the potential
  couples m to m +- 2 only.
* ``heat_kernel_trace_form``: the semi-discrete heat kernel in the form of
  (Discrker) (one propagator per rotation orbit of the frequency, read along
  its shifted diagonal against the rotated point), on the square grid with
  the rotations it shares with the orientations; the appendix's proof makes
  it equal to the form of (new2), the plain inverse FFT of e^{tA} delta.
"""
from __future__ import annotations

import numpy as np

from . import se2n_oracle as O


def ap_generator(lam: float, mu: float, N: int, beta: float) -> np.ndarray:
    """beta L - diag_r (lam cos e_r + mu sin e_r)^2 (equation (elem), grid clock)."""
    e = O.orientation_angles(N)
    w = (lam * np.cos(e) + mu * np.sin(e)) ** 2
    return beta * O.cyclic_laplacian(N) - np.diag(w)


def ap_solve(lam: float, mu: float, a0: np.ndarray, N: int, beta: float, T: float) -> np.ndarray:
    """A(T) = exp(T A_{lam,mu}) A(0) by a symmetric eigen-decomposition."""
    lamb, Q = np.linalg.eigh(ap_generator(lam, mu, N, beta))
    return Q @ (np.exp(T * lamb) * (Q.T @ np.asarray(a0, dtype=np.complex128)))


def theta_generator(lam: float, mu: float, alpha: float, K: int) -> np.ndarray:
    """Generator of the continuous-angle equation on the coefficients c_m,
    m = -K .. K, of a(theta) = sum_m c_m exp(i m theta).

    (lam cos + mu sin)^2 = (lam^2 + mu^2)/2 + (lam^2 - mu^2)/2 cos 2 theta
    + lam mu sin 2 theta; multiplying exp(i m theta) by cos 2 theta gives
    (exp(i(m+2)theta) + exp(i(m-2)theta))/2, by sin 2 theta gives
    (exp(i(m+2)theta) - exp(i(m-2)theta))/(2i); d^2/dtheta^2 gives -m^2.
    """
    m = np.arange(-K, K + 1)
    n = m.size
    G = np.zeros((n, n), dtype=np.complex128)
    c0 = 0.5 * (lam * lam + mu * mu)
    cc = 0.5 * (lam * lam - mu * mu)
    cs = lam * mu
    for j in range(n):
        G[j, j] -= c0 + alpha * m[j] ** 2
        if j + 2 < n:  # coefficient m+2 receives from m
            G[j + 2, j] -= 0.5 * cc + cs / 2j
        if j - 2 >= 0:
            G[j - 2, j] -= 0.5 * cc - cs / 2j
    return G


def theta_continuum(lam: float, mu: float, alpha: float, a_fun, T: float, thetas: np.ndarray,
                    K: int = 64, P: int = 1024) -> np.ndarray:
    """a(theta, T) at the given angles for the initial function a_fun(theta)
    (smooth, 2 pi periodic), truncated to |m| <= K Fourier modes."""
    th = 2.0 * np.pi * np.arange(P) / P
    c = np.fft.fft(a_fun(th)) / P
    m = np.arange(-K, K + 1)
    c0 = c[m % P]
    lamb, V = np.linalg.eig(theta_generator(lam, mu, alpha, K))
    cT = V @ (np.exp(T * lamb) * np.linalg.solve(V, c0))
    return (np.exp(1j * np.outer(np.asarray(thetas), m)) @ cT).real


# ---------------------------------------------------------------------------
# The semi-discrete heat kernel two ways (Sec. "The semi-discrete heat kernel
# via the GFT", equation (Discrker); Sec. "A direct way to compute the
# semi-discrete heat kernel", equation (new2); the identity is proved in the
# appendix "Proof that expressions (2.10) and (2.12) are identical").
# ---------------------------------------------------------------------------

def _rotation_group(N: int) -> int:
    """Order of the rotation group shared by the orientations and the square
    frequency grid: quarter turns when 4 | N, the half turn when N is even,
    else the identity only."""
    return 4 if N % 4 == 0 else (2 if N % 2 == 0 else 1)


def _rotate(M: int, g: int, a, b):
    """(a, b) in Z_M^2 turned by 2 pi / g (the same map for frequencies and
    for pixels: (a, b) -> (-b, a), or -(a, b) for the half turn)."""
    a = np.asarray(a)
    b = np.asarray(b)
    if g == 4:
        return (-b) % M, a % M
    if g == 2:
        return (-a) % M, (-b) % M
    return a % M, b % M


def _orbit_representatives(M: int, g: int):
    """One frequency (k, l) per orbit of the g rotations, and |orbit| / g."""
    code = np.arange(M * M)
    a, b = code // M, code % M
    codes = [code]
    for _ in range(g - 1):
        a, b = _rotate(M, g, a, b)
        codes.append(a * M + b)
    codes = np.stack(codes)              # [g, M*M]: the orbit of every frequency
    rep = codes.min(axis=0) == code      # the smallest code of its orbit
    size = np.array([np.unique(c).size for c in codes[:, rep].T])
    return code[rep] // M, code[rep] % M, size / g


def heat_kernel_trace_form(M: int, N: int, beta: float, T: float, r, scheme: str = "exact",
                           n_steps: int = 0, pixels=None) -> np.ndarray:
    """Orientation(s) r of the grid heat kernel (the solution from a unit
    mass at pixel (0, 0) and orientation 0, on the clock of the grid path) in
    the form of (Discrker): instead of one vector e^{tA} delta per frequency,
    one propagator P per orbit of the frequency under the rotations R_n shared
    by the orientations and the grid (n = 0, N/g, 2N/g, ...), read along its
    shifted diagonal and paired with the rotated pixel:

        D_r(z) = (1/M^2) sum_{orbits k} w_k sum_n P_k[r + n, n] e^{2 pi i <k, R_n z> / M},

    w_k = |orbit| / g.  This is the appendix's reindexing
    (S^{-n} P S^n = P at the rotated frequency) on the grid, where the grid
    symbol rotates with the frequency.  Equal to the plain inverse FFT of
    (P_k delta)_r over all frequencies, the grid form of (new2).

    r: one orientation or a sequence (then a leading axis).  pixels:
    optional (ys, xs) to evaluate at; default every pixel ([M, M], rows y).
    scheme 'exact' (e^{TA}) or 'cn' (n_steps Crank-Nicolson steps).
    """
    from . import se2n_oracle as O

    g = _rotation_group(N)
    step = N // g
    ks, ls, w = _orbit_representatives(M, g)
    rs = np.atleast_1d(np.asarray(r))
    if pixels is None:
        ys, xs = np.mgrid[0:M, 0:M]
        shape = (M, M)
    else:
        ys, xs = (np.asarray(p) for p in pixels)
        shape = ys.shape
    ys = ys.reshape(-1)
    xs = xs.reshape(-1)
    out = np.zeros((rs.size, ys.size), dtype=np.complex128)
    xq, yq = xs, ys
    for q in range(g):
        c = q * step  # column n of P, read at rows r + n
        X = np.zeros((ks.size, N), dtype=np.complex128)
        X[:, c] = 1.0
        if scheme == "exact":
            col = O.diffuse_modes_exact(X, M, ks, ls, beta, T)
        else:
            col = O.diffuse_modes_cn(X, M, ks, ls, beta, T, n_steps)
        coef = w[None, :] * col[:, (rs + c) % N].T  # [len(r), orbits]
        phase = np.exp(2j * np.pi * (np.outer(ks, xq) + np.outer(ls, yq)) / M)
        out += coef @ phase
        xq, yq = _rotate(M, g, xq, yq)  # the pixel turned q + 1 times
    out = out / (M * M)
    return out.reshape(shape) if np.ndim(r) == 0 else out.reshape((rs.size,) + shape)
