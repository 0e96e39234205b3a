"""Pins of the theory references (oracle/theory_oracle.py): closed forms of
the almost-periodic reduction (equation (redap), Theorem 1) and of the
continuous-angle limit (equation (contdif-weight)), the rotation theorem of
Sec. "A view through almost periodic functions", and the correspondence
between the reduction and the grid's per-mode systems (Theorem 2)."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import theory_oracle as TH  # noqa: E402


def test_ap_zero_frequency_orientation_modes_decay_in_closed_form():
    """lambda = mu = 0: A = beta L, so the orientation DFT mode m decays by
    exp(-4 beta sin^2(pi m / N) T)."""
    N, beta, T = 12, 1.7, 0.8
    r = np.arange(N)
    for m in range(N):
        a0 = np.exp(2j * np.pi * m * r / N)
        got = TH.ap_solve(0.0, 0.0, a0, N, beta, T)
        np.testing.assert_allclose(got, np.exp(-4 * beta * np.sin(np.pi * m / N) ** 2 * T) * a0, atol=1e-13)


def test_ap_without_coupling_decays_by_the_potential():
    N, lam, mu, T = 10, 1.3, -0.7, 0.9
    a0 = np.linspace(1.0, 2.0, N)
    e = 2 * np.pi * np.arange(N) / N
    got = TH.ap_solve(lam, mu, a0, N, 0.0, T)
    np.testing.assert_allclose(got, np.exp(-((lam * np.cos(e) + mu * np.sin(e)) ** 2) * T) * a0, rtol=1e-13)


@pytest.mark.parametrize("j", [1, 3, 5])
def test_rotation_theorem(j):
    """If omega' = R_j omega then the solution for omega' started from
    S^j A(0) is S^j A(t): one resolvent per rotation orbit suffices."""
    N, beta, T = 16, 2.0, 0.6
    lam, mu = 1.1, 0.4
    e = 2 * np.pi * j / N
    lam2, mu2 = lam * np.cos(e) - mu * np.sin(e), lam * np.sin(e) + mu * np.cos(e)
    rng = np.random.default_rng(j)
    a0 = rng.normal(size=N) + 1j * rng.normal(size=N)
    A = TH.ap_solve(lam, mu, a0, N, beta, T)
    A2 = TH.ap_solve(lam2, mu2, np.roll(a0, j), N, beta, T)
    np.testing.assert_allclose(A2, np.roll(A, j), atol=1e-12)


def test_grid_mode_is_the_reduction_at_the_central_difference_symbol():
    """Theorem 2's per-mode system at grid frequency (k, l) is the almost-periodic
    system with lambda = sqrt(M) sin(2 pi k / M), mu = sqrt(M) sin(2 pi l / M)."""
    M, N, beta, T = 64, 8, 1.5, 0.4
    rng = np.random.default_rng(3)
    for k, l in ((1, 3), (5, 0), (17, 40)):
        a0 = rng.normal(size=N) + 1j * rng.normal(size=N)
        grid = O.diffuse_modes_exact(a0[None, :], M, [k], [l], beta, T)[0]
        s = np.sqrt(M) * np.sin(2 * np.pi * np.array([k, l]) / M)
        np.testing.assert_allclose(grid, TH.ap_solve(s[0], s[1], a0, N, beta, T), atol=1e-13)


def test_continuum_pure_angular_diffusion():
    alpha, T = 0.3, 0.7
    th = np.linspace(0, 2 * np.pi, 13, endpoint=False)
    got = TH.theta_continuum(0.0, 0.0, alpha, lambda t: np.cos(3 * t) + 0.5 * np.sin(t), T, th)
    want = np.exp(-9 * alpha * T) * np.cos(3 * th) + 0.5 * np.exp(-alpha * T) * np.sin(th)
    np.testing.assert_allclose(got, want, atol=1e-13)


def test_continuum_without_angular_diffusion_is_pointwise():
    """alpha = 0: a(theta, T) = exp(-(lam cos theta + mu sin theta)^2 T) a(theta, 0)."""
    lam, mu, T = 1.2, -0.8, 0.5
    g = lambda t: np.exp(np.cos(t - 0.4))
    th = np.linspace(0, 2 * np.pi, 17, endpoint=False)
    got = TH.theta_continuum(lam, mu, 0.0, g, T, th)
    want = np.exp(-((lam * np.cos(th) + mu * np.sin(th)) ** 2) * T) * g(th)
    np.testing.assert_allclose(got, want, rtol=1e-11)


def test_semi_discrete_tends_to_the_continuum_at_second_order():
    """beta_N = alpha (N / 2 pi)^2: the N-orientation system converges to the
    continuous-angle equation as N grows, the error falling like 1/N^2
    (the cyclic second difference is a second-order approximation)."""
    lam, mu, alpha, T = 1.0, 0.5, 0.4, 0.6
    g = lambda t: np.exp(0.8 * np.cos(t - 0.3))
    errs = []
    for N in (16, 32, 64, 128):
        e = 2 * np.pi * np.arange(N) / N
        beta = O.beta_from_alpha(alpha, N)
        semi = TH.ap_solve(lam, mu, g(e), N, beta, T).real
        errs.append(np.abs(semi - TH.theta_continuum(lam, mu, alpha, g, T, e)).max())
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.6 < r < 4.4 for r in ratios), (errs, ratios)


@pytest.mark.parametrize("N", [8, 12, 32])
def test_swapped_frequency_is_the_reflected_orientation(N):
    """Swapping kx and ky is the reflection e_r -> pi/2 - e_r of the
    orientations, r -> N/4 - r (mod N), when 4 | N: started from the reflected
    vector, the mode (l, k) evolves into the reflected evolution of (k, l).
    (One propagator thus serves both frequency classes.)  Checked on the
    oracle's Crank-Nicolson steps and exact exponential, mirrored frequencies
    (ky > M/2) included.  For N = 2 mod 4 no orientation index is N/4 and the
    relation has no grid form (next test)."""
    M, beta, T = 64, 1.3, 0.5
    rng = np.random.default_rng(N)
    refl = (N // 4 - np.arange(N)) % N
    for k, l in ((3, 11), (1, 30), (7, 64 - 5), (0, 9)):
        a0 = rng.normal(size=N) + 1j * rng.normal(size=N)
        for evolve in (lambda X, kk, ll: O.diffuse_modes_cn(X, M, [kk], [ll], beta, T, 40),
                       lambda X, kk, ll: O.diffuse_modes_exact(X, M, [kk], [ll], beta, T)):
            A = evolve(a0[None, :], k, l)[0]
            B = evolve(a0[refl][None, :], l, k)[0]
            np.testing.assert_allclose(B, A[refl], rtol=0, atol=1e-12 * np.abs(A).max())


def test_swapped_frequency_has_no_reflection_when_4_does_not_divide_N():
    M, N, beta, T = 64, 10, 1.3, 0.5
    a0 = np.random.default_rng(1).normal(size=N).astype(complex)
    A = O.diffuse_modes_exact(a0[None, :], M, [3], [11], beta, T)[0]
    B = O.diffuse_modes_exact(a0[None, :], M, [11], [3], beta, T)[0]
    # the potentials of the two classes are not orientation permutations of each other
    pa = np.sort(O.mode_potential(M, N, np.array([3]), np.array([11])).ravel())
    pb = np.sort(O.mode_potential(M, N, np.array([11]), np.array([3])).ravel())
    assert np.abs(pa - pb).max() > 1e-3
    assert np.abs(A - B).max() > 1e-6


@pytest.mark.parametrize("M,N,scheme", [(16, 8, "exact"), (24, 12, "cn"), (16, 10, "exact"), (12, 7, "cn")])
def test_trace_form_of_the_heat_kernel_is_the_inverse_fft(M, N, scheme):
    """(Discrker) against (new2) on the grid: the trace form over rotation
    orbits (quarter turns for 4 | N, the half turn for N = 2 mod 4, nothing
    for odd N) equals the plain diffusion of a unit mass at pixel (0, 0),
    orientation 0, to rounding -- and is real."""
    beta, T, n = 1.7, 0.35, 12
    psi = np.zeros((N, M, M))
    psi[0, 0, 0] = 1.0
    ref = O.diffuse(psi, T, beta, n, scheme)
    for r in (0, 1, N // 2, N - 1):
        got = TH.heat_kernel_trace_form(M, N, beta, T, r, scheme, n)
        assert np.abs(got.imag).max() < 1e-14
        np.testing.assert_allclose(got.real, ref[r], rtol=0, atol=1e-14)


def test_trace_form_needs_the_rotation_of_the_orientations():
    """Pairing each orbit's rotated pixels with the unshifted entry P[r, 0]
    (dropping the shift S^n of the proof) gives a different field: the pin
    above would catch a wrong orientation index in the trace form."""
    M, N, beta, T, r = 16, 8, 1.7, 0.35, 1
    psi = np.zeros((N, M, M))
    psi[0, 0, 0] = 1.0
    ref = O.diffuse(psi, T, beta, 0, "exact")[r]
    good = TH.heat_kernel_trace_form(M, N, beta, T, r).real
    np.testing.assert_allclose(good, ref, atol=1e-14)
    # the same orbit representatives and weights, no orientation shift
    g, seen, reps, w = 4, np.zeros((M, M), bool), [], []
    for k in range(M):
        for l in range(M):
            if seen[k, l]:
                continue
            orb, a, b = {(k, l)}, k, l
            for _ in range(g - 1):
                a, b = (-b) % M, a % M
                orb.add((a, b))
            for (a, b) in orb:
                seen[a, b] = True
            reps.append((k, l))
            w.append(len(orb) / g)
    ks, ls = np.array(reps).T
    X = np.zeros((ks.size, N))
    X[:, 0] = 1.0
    coef = np.array(w) * O.diffuse_modes_exact(X, M, ks, ls, beta, T)[:, r]
    ys, xs = np.mgrid[0:M, 0:M]
    wrong = np.zeros((M, M), dtype=complex)
    xq, yq = xs, ys
    for _ in range(g):
        wrong += np.tensordot(coef, np.exp(2j * np.pi * (ks[:, None, None] * xq + ls[:, None, None] * yq) / M), 1)
        xq, yq = (-yq) % M, xq % M
    wrong = wrong.real / (M * M)
    assert np.abs(wrong - ref).max() > 1e-3 * np.abs(ref).max()
