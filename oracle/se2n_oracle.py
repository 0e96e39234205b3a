"""FP64 CPU oracle: lift -> diffuse -> project, step by step as the paper states it.

TEST INFRASTRUCTURE ONLY (see the package docstring): only the tests, the smoke
check and the benchmark's CPU-baseline leg may call this module.

Notation (paper, Sec. "Numerical treatment of the diffusion equation"):

* The image is an M x M periodic grid, ``f[y, x]``; x is the column index.
* Orientations are e_r = 2*pi*r/N, r in Z_N (the rotation angles of SE(2,N),
  Sec. "The group of discrete motions SE(2,N)").
* D_x psi = (sqrt(M)/2) (psi[x+1] - psi[x-1]) and likewise D_y; their Fourier
  symbols are i*sqrt(M)*s_k with s_k = sin(2*pi*k/M) (proof of Theorem 2).
* The totally discrete operator is
      D psi^r = (cos e_r D_x + sin e_r D_y)^2 psi^r
                + beta (psi^{r-1} - 2 psi^r + psi^{r+1})   (equation FTE).

Readings of the paper taken where it is silent or inconsistent:

* Time scale.  The paper writes d psi/dt = D psi / 2 in (FTE) but the per-mode
  matrix it derives, A = (Lambda_N - M diag(a^2))/2 with Lambda_N = beta/2 * L,
  halves the angular rate once more.  The oracle integrates d psi/dt = D psi,
  i.e. per mode A_{k,l} = beta*L - M*diag_r((a^r_{k,l})^2), which is the weighted
  operator Delta^(N) of Sec. "The weighting of the metric" and gives the zero
  frequency orientation modes the decay exp(-4 beta sin^2(pi m / N) t).
  A paper time T_p corresponds to T = T_p/2.
* Lift direction.  theta = arg(grad f_sigma) + pi/2, the level-line direction,
  binned to the nearest e_r with ties rounded up: r = floor(theta N/(2 pi) + 1/2)
  mod N.  The gradient uses the same central-difference symbol as D_x, D_y and a
  Gaussian of sigma pixels applied in Fourier space; it is taken on the
  corrupted image f*(1-mask) as the paper does.  The lifted value is the
  unsmoothed f*(1-mask) at the selected orientation and 0 elsewhere.
* Crank-Nicolson is the implicit trapezoidal rule, tau = T/n.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cn_core.c")
_LIB = os.path.join(_HERE, "liboracle_cn.so")
_lib = None


def build_core(force: bool = False) -> str:
    """Compile the plain-C Crank-Nicolson core (gcc, OpenMP) next to this file."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c99", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _core():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build_core())
        dp = ctypes.POINTER(ctypes.c_double)
        lib.oracle_cn_modes.argtypes = [
            ctypes.c_int, ctypes.c_long, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp,
        ]
        lib.oracle_cn_modes.restype = ctypes.c_int
        lib.oracle_cyclic_solve.argtypes = [ctypes.c_int, dp, ctypes.c_double, dp, dp]
        lib.oracle_cyclic_solve.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        lib.oracle_set_num_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def num_threads() -> int:
    """Threads the C core uses for its mode loop."""
    return int(_core().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the C core's mode loop from now on."""
    _core().oracle_set_num_threads(int(n))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------------
# The model: angles, symbols, generator (Sec. "The semi-discrete diffusion
# operator", Sec. "Numerical treatment of the diffusion equation").
# --------------------------------------------------------------------------

def orientation_angles(N: int) -> np.ndarray:
    """e_r = 2*pi*r/N, the rotation angles of SE(2,N)."""
    return 2.0 * np.pi * np.arange(N) / N


def symbol(M: int) -> np.ndarray:
    """s_k = sin(2*pi*k/M): the central difference D_x has symbol i*sqrt(M)*s_k."""
    return np.sin(2.0 * np.pi * np.arange(M) / M)


def cyclic_laplacian(N: int) -> np.ndarray:
    """L: the cyclic second difference over Z_N (jump generator up to the rate beta)."""
    L = -2.0 * np.eye(N)
    for r in range(N):
        L[r, (r + 1) % N] += 1.0
        L[r, (r - 1) % N] += 1.0
    return L


def mode_potential(M: int, N: int, k, l) -> np.ndarray:
    """M * (a^r_{k,l})^2 with a^r_{k,l} = cos(e_r) s_k + sin(e_r) s_l (proof of Theorem 2).

    k is the x frequency and l the y frequency; both may be arrays, the
    orientation axis is appended last.
    """
    e = orientation_angles(N)
    s = symbol(M)
    sk = np.asarray(s[np.asarray(k) % M])[..., None]
    sl = np.asarray(s[np.asarray(l) % M])[..., None]
    a = np.cos(e) * sk + np.sin(e) * sl
    return M * a * a


def generator_matrix(M: int, N: int, beta: float, k: int, l: int) -> np.ndarray:
    """A_{k,l} = beta*L - M*diag_r((a^r_{k,l})^2), real symmetric (equation deceq, time scale above)."""
    return beta * cyclic_laplacian(N) - np.diag(mode_potential(M, N, k, l))


def beta_from_alpha(alpha: float, N: int) -> float:
    """The weight relation alpha = beta_N (2*pi/N)^2 solved for beta_N."""
    return alpha * (N / (2.0 * np.pi)) ** 2


# --------------------------------------------------------------------------
# Lift (Sec. "A final inpainting algorithm...": smoothing and gradient at the
# level of the FFT, nearest angle).
# --------------------------------------------------------------------------

def smoothed_gradient(f: np.ndarray, mask: np.ndarray, sigma: float = 2.0):
    """(g_x, g_y) = (D_x, D_y) applied to the Gaussian-smoothed corrupted image.

    Both the smoothing (multiplier exp(-2 pi^2 sigma^2 (kbar^2 + lbar^2) / M^2),
    frequencies wrapped to [-M/2, M/2)) and the central differences (symbol
    i*sqrt(M)*s_k) act on the FFT of f_c = f*(1-mask).
    """
    f = np.asarray(f, dtype=np.float64)
    M = f.shape[0]
    fc = f * (1.0 - np.asarray(mask, dtype=np.float64))
    F = np.fft.fft2(fc)  # F[l, k]: l = y frequency, k = x frequency
    kbar = (np.arange(M) + M // 2) % M - M // 2
    gauss = np.exp(-2.0 * np.pi**2 * sigma**2 * (kbar[None, :] ** 2 + kbar[:, None] ** 2) / M**2)
    s = symbol(M)
    Gx = F * (1j * np.sqrt(M) * s[None, :]) * gauss
    Gy = F * (1j * np.sqrt(M) * s[:, None]) * gauss
    return np.fft.ifft2(Gx).real, np.fft.ifft2(Gy).real


def bin_angle(gx: np.ndarray, gy: np.ndarray, N: int):
    """Nearest orientation of the level line theta = atan2(g_y, g_x) + pi/2.

    Returns ``(rmap, tie)`` with rmap = floor(theta N/(2 pi) + 1/2) mod N and tie
    the distance of theta N/(2 pi) + 1/2 to the nearest bin edge.
    """
    theta = np.arctan2(gy, gx) + np.pi / 2.0
    t = theta * N / (2.0 * np.pi) + 0.5
    fl = np.floor(t)
    rmap = (fl.astype(np.int64) % N).astype(np.uint8)
    frac = t - fl
    return rmap, np.minimum(frac, 1.0 - frac)


def orient(f: np.ndarray, mask: np.ndarray, N: int, sigma: float = 2.0):
    """Orientation map of the corrupted image.

    Returns ``(rmap, tie)``: rmap[y, x] in [0, N) is the orientation bin and
    tie[y, x] is the distance of theta*N/(2 pi) + 1/2 to the nearest bin edge
    (0 means an exact tie), used to exclude near-tie pixels from comparisons.
    """
    gx, gy = smoothed_gradient(f, mask, sigma)
    return bin_angle(gx, gy, N)


def lift(f: np.ndarray, mask: np.ndarray, rmap: np.ndarray, N: int) -> np.ndarray:
    """psi^r(x,y) = f_c(x,y) [rmap(x,y) = r] with f_c = f*(1-mask); shape [N, M, M]."""
    fc = np.asarray(f, dtype=np.float64) * (1.0 - np.asarray(mask, dtype=np.float64))
    r = np.arange(N)[:, None, None]
    return np.where(np.asarray(rmap)[None, :, :] == r, fc[None, :, :], 0.0)


# --------------------------------------------------------------------------
# Diffusion (Theorem 2: FFT over (Z/MZ)^2, M^2 independent N-dimensional
# systems, inverse FFT; remark 2: Crank-Nicolson; (soleq): exact exponential).
# --------------------------------------------------------------------------

def diffuse_modes_cn(X: np.ndarray, M: int, k, l, beta: float, T: float, n_steps: int) -> np.ndarray:
    """Crank-Nicolson for a list of modes.

    X: complex [nmodes, N] initial spectra of modes (k[i], l[i]); returns the
    spectra at time T after ``n_steps`` steps of tau = T/n_steps.
    """
    X = np.asarray(X, dtype=np.complex128)
    nm, N = X.shape
    pot = np.ascontiguousarray(mode_potential(M, N, np.asarray(k), np.asarray(l)).reshape(nm, N))
    re = np.ascontiguousarray(X.real)
    im = np.ascontiguousarray(X.imag)
    tau = T / n_steps if n_steps > 0 else 0.0
    rc = _core().oracle_cn_modes(int(N), int(nm), _dptr(pot), float(beta), float(tau),
                                 int(n_steps), _dptr(re), _dptr(im))
    if rc != 0:
        raise RuntimeError(f"oracle CN core failed ({rc})")
    return re + 1j * im


def diffuse_modes_exact(X: np.ndarray, M: int, k, l, beta: float, T: float,
                        chunk: int = 16384) -> np.ndarray:
    """Exact propagator e^{T A_{k,l}} (equation soleq) via a symmetric eigen-decomposition."""
    X = np.asarray(X, dtype=np.complex128)
    nm, N = X.shape
    k = np.asarray(k).reshape(-1)
    l = np.asarray(l).reshape(-1)
    L = cyclic_laplacian(N)
    out = np.empty_like(X)
    for a in range(0, nm, chunk):
        b = min(nm, a + chunk)
        pot = mode_potential(M, N, k[a:b], l[a:b])
        A = beta * L[None, :, :] - pot[:, :, None] * np.eye(N)[None, :, :]
        lam, Q = np.linalg.eigh(A)
        c = np.einsum("mji,mj->mi", Q, X[a:b])
        c = c * np.exp(T * lam)
        out[a:b] = np.einsum("mij,mj->mi", Q, c)
    return out


def diffuse(psi: np.ndarray, T: float, beta: float, n_steps: int, scheme: str = "cn") -> np.ndarray:
    """Integrate d psi/dt = D psi from psi (shape [N, M, M], real) to time T.

    FFT of every orientation slice, per-mode Crank-Nicolson (or the exact
    exponential), inverse FFT.  Returns the real part; the imaginary part
    vanishes because every A_{k,l} is real and A_{-k,-l} = A_{k,l}.
    """
    psi = np.asarray(psi, dtype=np.float64)
    N, M, M2 = psi.shape
    assert M == M2
    Psi = np.fft.fft2(psi, axes=(1, 2))  # Psi[r, l, k]
    X = Psi.reshape(N, M * M).T  # [mode = l*M + k, r]
    ll, kk = np.divmod(np.arange(M * M), M)
    if scheme == "cn":
        Y = diffuse_modes_cn(X, M, kk, ll, beta, T, n_steps)
    elif scheme == "exact":
        Y = diffuse_modes_exact(X, M, kk, ll, beta, T)
    else:
        raise ValueError(scheme)
    out = np.fft.ifft2(Y.T.reshape(N, M, M), axes=(1, 2))
    scale = max(np.abs(out.real).max(), 1e-300)
    if np.abs(out.imag).max() > 1e-9 * scale:
        raise AssertionError("diffused field is not real")
    return out.real


def project(psi: np.ndarray, mode: str = "max") -> np.ndarray:
    """Back to the plane: maximum (the paper's choice) or mean over orientations."""
    psi = np.asarray(psi, dtype=np.float64)
    if mode == "max":
        return psi.max(axis=0)
    if mode == "mean":
        return psi.mean(axis=0)
    raise ValueError(mode)


def inpaint(f, mask, N: int, T: float, beta: float, n_steps: int, sigma: float = 2.0,
            scheme: str = "cn", proj: str = "max", rmap=None):
    """Whole path: orient, lift, diffuse, project.  Returns ``(out, rmap)``.

    Pass ``rmap`` to lift with a given orientation map (used to compare the
    downstream steps with another implementation on an identical lift).
    """
    if rmap is None:
        rmap, _ = orient(f, mask, N, sigma)
    psi = lift(f, mask, rmap, N)
    psi = diffuse(psi, T, beta, n_steps, scheme)
    return project(psi, proj), rmap


def cyclic_solve(diag: np.ndarray, off: float, rhs: np.ndarray) -> np.ndarray:
    """Solve the cyclic tridiagonal system of the CN step with the C core's solver."""
    diag = np.ascontiguousarray(diag, dtype=np.float64)
    rhs = np.ascontiguousarray(rhs, dtype=np.float64)
    x = np.empty_like(rhs)
    rc = _core().oracle_cyclic_solve(int(diag.size), _dptr(diag), float(off), _dptr(rhs), _dptr(x))
    if rc != 0:
        raise RuntimeError(f"cyclic solve failed ({rc})")
    return x
