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
