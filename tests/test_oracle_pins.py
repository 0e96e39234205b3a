"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test checks the oracle against something the paper or the mathematics
fixes independently of the oracle's own code path: the real-space operator of
(FTE) built from its stencils and integrated densely, closed-form decays,
symmetries of the grid, and library routines for the small dense problems.
"""
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from paper_1304_2062_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# helpers: the real-space operator of (FTE) from its stencils
# ---------------------------------------------------------------------------

def _central_difference_matrix(M):
    """(D v)[i] = sqrt(M)/2 (v[i+1] - v[i-1]) on a periodic line."""
    fwd = np.roll(np.eye(M), 1, axis=1)  # (fwd v)[i] = v[i+1]
    return np.sqrt(M) / 2.0 * (fwd - fwd.T)


def _dense_operator(M, N, beta):
    """D = blockdiag_r (cos e_r D_x + sin e_r D_y)^2 + beta * (cyclic 2nd difference in r).

    Flattening order is [r][y][x]; D_x acts on x, D_y on y.  The squares are
    matrix products of the stencil matrices, the angular coupling is written
    out entry by entry.
    """
    d1 = _central_difference_matrix(M)
    I = np.eye(M)
    Dx = np.kron(I, d1)
    Dy = np.kron(d1, I)
    blocks = []
    for r in range(N):
        e = 2.0 * np.pi * r / N
        G = np.cos(e) * Dx + np.sin(e) * Dy
        blocks.append(G @ G)
    D = sla.block_diag(*blocks)
    P = M * M
    for r in range(N):
        for rr in ((r + 1) % N, (r - 1) % N):
            D[r * P:(r + 1) * P, rr * P:(rr + 1) * P] += beta * np.eye(P)
        D[r * P:(r + 1) * P, r * P:(r + 1) * P] -= 2.0 * beta * np.eye(P)
    return D


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


# ---------------------------------------------------------------------------
# Theorem 2: the FFT decoupling reproduces the real-space system exactly
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("M,N,beta,T", [(8, 8, 1.3, 0.37), (6, 4, 0.7, 0.5), (12, 6, 2.0, 0.2)])
def test_exact_scheme_matches_dense_expm(M, N, beta, T):
    rng = np.random.default_rng(M * 100 + N)
    psi0 = rng.standard_normal((N, M, M))
    D = _dense_operator(M, N, beta)
    want = (sla.expm(T * D) @ psi0.reshape(-1)).reshape(N, M, M)
    got = O.diffuse(psi0, T, beta, 1, "exact")
    assert _rel(got, want) < 1e-12


@pytest.mark.parametrize("M,N,beta,T,n", [(16, 8, 1.0, 0.5, 20), (12, 4, 3.0, 0.3, 7)])
def test_cn_scheme_matches_dense_real_space_cn(M, N, beta, T, n):
    """n steps of (I - tau D/2) x' = (I + tau D/2) x on the full real-space system."""
    rng = np.random.default_rng(7 + M)
    psi0 = rng.standard_normal((N, M, M))
    D = _dense_operator(M, N, beta)
    tau = T / n
    I = np.eye(D.shape[0])
    lu = sla.lu_factor(I - 0.5 * tau * D)
    B = I + 0.5 * tau * D
    x = psi0.reshape(-1).copy()
    for _ in range(n):
        x = sla.lu_solve(lu, B @ x)
    got = O.diffuse(psi0, T, beta, n, "cn")
    assert _rel(got, x.reshape(N, M, M)) < 1e-12


# ---------------------------------------------------------------------------
# per-mode solver
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N", [3, 4, 5, 8, 16, 30, 64])
def test_cyclic_solve_matches_dense_solve(N):
    rng = np.random.default_rng(N)
    off = -0.37
    diag = 1.0 + 2 * abs(off) + rng.uniform(0.0, 5.0, size=N)
    B = np.diag(diag)
    for r in range(N):
        B[r, (r + 1) % N] += off
        B[r, (r - 1) % N] += off
    rhs = rng.standard_normal(N)
    assert _rel(O.cyclic_solve(diag, off, rhs), np.linalg.solve(B, rhs)) < 1e-13


@pytest.mark.parametrize("M,N,beta,T,n", [(64, 16, 1.0, 0.5, 50), (512, 30, 1.0, 2.0, 200), (64, 8, 0.0, 0.3, 10)])
def test_cn_modes_match_dense_matrix_power(M, N, beta, T, n):
    rng = np.random.default_rng(3)
    ks = rng.integers(0, M, size=12)
    ls = rng.integers(0, M, size=12)
    X = rng.standard_normal((12, N)) + 1j * rng.standard_normal((12, N))
    got = O.diffuse_modes_cn(X, M, ks, ls, beta, T, n)
    tau = T / n
    for i in range(12):
        A = O.generator_matrix(M, N, beta, ks[i], ls[i])
        I = np.eye(N)
        C = np.linalg.solve(I - 0.5 * tau * A, I + 0.5 * tau * A)
        want = np.linalg.matrix_power(C, n) @ X[i]
        assert _rel(got[i], want) < 1e-12


@pytest.mark.parametrize("N", [4, 8])
def test_exact_modes_match_expm(N):
    M, beta, T = 32, 1.7, 0.9
    rng = np.random.default_rng(N)
    ks = rng.integers(0, M, size=10)
    ls = rng.integers(0, M, size=10)
    X = rng.standard_normal((10, N)) + 1j * rng.standard_normal((10, N))
    got = O.diffuse_modes_exact(X, M, ks, ls, beta, T)
    for i in range(10):
        want = sla.expm(T * O.generator_matrix(M, N, beta, ks[i], ls[i])) @ X[i]
        # strongly damped modes: measure the error against the initial size
        assert np.linalg.norm(got[i] - want) < 1e-12 * np.linalg.norm(X[i])


def test_generator_is_symmetric_negative_semidefinite():
    for (M, N, k, l) in [(64, 16, 3, 5), (48, 30, 0, 7), (64, 32, 16, 16)]:
        A = O.generator_matrix(M, N, 1.0, k, l)
        assert np.array_equal(A, A.T)
        assert np.linalg.eigvalsh(A).max() <= 1e-12


def test_cn_converges_at_second_order_to_exact():
    """Halving tau cuts the CN error by ~4 on a non-stiff mode."""
    M, N, beta, T = 64, 16, 1.0, 0.5
    X = np.cos(2 * np.pi * 3 * np.arange(N) / N)[None, :] + 0j
    want = O.diffuse_modes_exact(X, M, [1], [2], beta, T)
    errs = [_rel(O.diffuse_modes_cn(X, M, [1], [2], beta, T, n), want) for n in (40, 80, 160)]
    assert 3.8 < errs[0] / errs[1] < 4.2
    assert 3.8 < errs[1] / errs[2] < 4.2


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", ["exact", "cn"])
@pytest.mark.parametrize("kx,ky", [(0, 0), (1, 0), (0, 1), (1, 1)])  # 1 means the Nyquist index M/2
def test_zero_symbol_modes_decay_in_closed_form(scheme, kx, ky):
    """Where s_k = s_l = 0 (k, l in {0, M/2}) the potential vanishes and A = beta L:
    orientation Fourier mode m decays by exp(-4 beta sin^2(pi m/N) T) (exact) or
    ((1 - 2 beta tau sin^2)/(1 + 2 beta tau sin^2))^n (Crank-Nicolson)."""
    M, N, beta, T, n = 16, 16, 1.0, 0.5, 50
    y, x = np.mgrid[0:M, 0:M]
    spatial = ((-1.0) ** x) ** kx * ((-1.0) ** y) ** ky
    r = np.arange(N)
    for m in (0, 1, 3, N // 2):
        psi0 = np.cos(2 * np.pi * m * r / N)[:, None, None] * spatial[None]
        s2 = np.sin(np.pi * m / N) ** 2
        if scheme == "exact":
            g = np.exp(-4.0 * beta * s2 * T)
        else:
            tau = T / n
            g = ((1.0 - 2.0 * beta * tau * s2) / (1.0 + 2.0 * beta * tau * s2)) ** n
        got = O.diffuse(psi0, T, beta, n, scheme)
        assert np.abs(got - g * psi0).max() < 1e-13


@pytest.mark.parametrize("scheme", ["exact", "cn"])
def test_uncoupled_plane_wave_decays_by_its_potential(scheme):
    """beta = 0: each orientation evolves alone; a plane wave of frequency (k,l)
    in slice r decays by exp(-M a^2 T) with a = cos(e_r) s_k + sin(e_r) s_l."""
    M, N, T, n = 32, 8, 0.05, 25
    y, x = np.mgrid[0:M, 0:M]
    for (k, l, r) in [(1, 0, 0), (0, 3, 2), (5, 2, 1), (7, 11, 3)]:
        psi0 = np.zeros((N, M, M))
        psi0[r] = np.cos(2 * np.pi * (k * x + l * y) / M)
        e = 2 * np.pi * r / N
        lam = M * (np.cos(e) * np.sin(2 * np.pi * k / M) + np.sin(e) * np.sin(2 * np.pi * l / M)) ** 2
        if scheme == "exact":
            g = np.exp(-lam * T)
        else:
            tau = T / n
            g = ((1 - 0.5 * tau * lam) / (1 + 0.5 * tau * lam)) ** n
        got = O.diffuse(psi0, T, 0.0, n, scheme)
        assert np.abs(got - g * psi0).max() < 1e-13


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------

def _small_lifted(seed=1, M=32, N=16):
    f = synth.make_image(seed, M, "small")
    mask = synth.mask_random(seed + 1, M, 0.3)
    rmap, _ = O.orient(f, mask, N)
    return O.lift(f, mask, rmap, N), f, mask


@pytest.mark.parametrize("scheme", ["exact", "cn"])
def test_total_mass_is_conserved(scheme):
    psi0, _, _ = _small_lifted()
    got = O.diffuse(psi0, 0.8, 1.5, 40, scheme)
    assert abs(got.sum() - psi0.sum()) < 1e-13 * abs(psi0).sum()


def test_linearity():
    psi_a, _, _ = _small_lifted(1)
    psi_b, _, _ = _small_lifted(2)
    lhs = O.diffuse(2.0 * psi_a - 0.5 * psi_b, 0.4, 1.0, 20)
    rhs = 2.0 * O.diffuse(psi_a, 0.4, 1.0, 20) - 0.5 * O.diffuse(psi_b, 0.4, 1.0, 20)
    assert _rel(lhs, rhs) < 1e-13


def test_translation_equivariance():
    psi0, _, _ = _small_lifted()
    a = O.diffuse(np.roll(psi0, (3, -5), axis=(1, 2)), 0.5, 1.0, 25)
    b = np.roll(O.diffuse(psi0, 0.5, 1.0, 25), (3, -5), axis=(1, 2))
    assert _rel(a, b) < 1e-13


def test_reflection_equivariance():
    """y -> -y with orientation r -> -r."""
    psi0, _, _ = _small_lifted()
    N, M = psi0.shape[0], psi0.shape[1]
    refl = lambda p: p[(-np.arange(N)) % N][:, (-np.arange(M)) % M, :]
    a = O.diffuse(refl(psi0), 0.5, 1.0, 25)
    b = refl(O.diffuse(psi0, 0.5, 1.0, 25))
    assert _rel(a, b) < 1e-13


def _rot90(img):
    """f'[y][x] = f[(-x) mod M][y]: rotation of the periodic grid by +90 degrees."""
    M = img.shape[-1]
    idx = (-np.arange(M)) % M
    return np.swapaxes(img, -1, -2)[..., :, idx] if img.ndim == 2 else np.swapaxes(img, -1, -2)[..., :, idx]


@pytest.mark.parametrize("scheme", ["exact", "cn"])
def test_rotation_equivariance_of_diffusion(scheme):
    """Rotating the plane by 90 degrees and shifting orientations by N/4 commutes with the diffusion."""
    psi0, _, _ = _small_lifted(N=16)
    N = psi0.shape[0]
    rot = lambda p: np.roll(_rot90(p), N // 4, axis=0)
    a = O.diffuse(rot(psi0), 0.6, 1.0, 30, scheme)
    b = rot(O.diffuse(psi0, 0.6, 1.0, 30, scheme))
    assert _rel(a, b) < 1e-13


def test_rotation_equivariance_of_whole_pipeline():
    """Orient + lift + diffuse + project commutes with the 90-degree rotation,
    except where an orientation bin is decided by a rounding-level tie."""
    M, N = 32, 16
    f = synth.make_image(4, M, "small")
    mask = synth.mask_random(5, M, 0.3)
    out, rmap = O.inpaint(f, mask, N, 0.5, 1.0, 25)
    out_r, rmap_r = O.inpaint(_rot90(f), _rot90(mask), N, 0.5, 1.0, 25)
    _, tie = O.orient(f, mask, N)
    flips = (rmap_r != ((_rot90(rmap).astype(int) + N // 4) % N)) & (_rot90(tie) > 1e-9)
    assert flips.sum() == 0
    assert _rel(out_r, _rot90(out)) < 1e-12


# ---------------------------------------------------------------------------
# lift
# ---------------------------------------------------------------------------

def test_gradient_matches_real_space_stencils():
    """The FFT gradient equals sqrt(M)/2 (h[x+1] - h[x-1]) of the image convolved
    with the periodised sampled Gaussian (real-space, separable), up to the
    aliasing of the sampled Gaussian (< 1e-8 for sigma = 2)."""
    M, sigma = 64, 2.0
    f = synth.make_image(9, M, "small")
    mask = synth.mask_random(10, M, 0.3)
    fc = f * (1 - mask)
    xs = np.arange(M)
    d = (xs[:, None] - xs[None, :] + M // 2) % M - M // 2
    g1 = np.zeros((M, M))
    for j in range(-3, 4):
        g1 += np.exp(-((d + j * M) ** 2) / (2 * sigma**2))
    g1 /= np.sqrt(2 * np.pi) * sigma
    h = g1 @ fc @ g1.T
    gx_ref = np.sqrt(M) / 2 * (np.roll(h, -1, axis=1) - np.roll(h, 1, axis=1))
    gy_ref = np.sqrt(M) / 2 * (np.roll(h, -1, axis=0) - np.roll(h, 1, axis=0))
    gx, gy = O.smoothed_gradient(f, mask, sigma)
    scale = np.abs(gx_ref).max()
    assert np.abs(gx - gx_ref).max() < 1e-8 * scale
    assert np.abs(gy - gy_ref).max() < 1e-8 * scale


@pytest.mark.parametrize("N", [16, 30, 32])
@pytest.mark.parametrize("u,v", [(1, 0), (0, 2), (3, 1), (-2, 5)])
def test_plane_wave_lifts_to_two_level_line_bins(N, u, v):
    """f = 0.5 + 0.4 sin(2 pi (u x + v y)/M): the smoothed central-difference
    gradient is cos(phase) * (s_u, s_v) times a positive factor, so theta takes
    the two values atan2(s_v, s_u) + pi/2 and that + pi."""
    M = 64
    y, x = np.mgrid[0:M, 0:M]
    phase = 2 * np.pi * (u * x + v * y) / M
    f = 0.5 + 0.4 * np.sin(phase)
    mask = np.zeros((M, M), np.uint8)
    rmap, tie = O.orient(f, mask, N)
    su, sv = np.sin(2 * np.pi * u / M), np.sin(2 * np.pi * v / M)
    base = np.arctan2(sv, su) + np.pi / 2
    expect = np.where(np.cos(phase) > 0, base, base + np.pi)
    t = expect * N / (2 * np.pi) + 0.5
    want = (np.floor(t).astype(int) % N).astype(np.uint8)
    crest = np.abs(np.cos(phase)) > 1e-6
    # Where the closed-form angle sits exactly on a bin edge (e.g. a horizontal
    # gradient when N = 2 mod 4) either neighbouring bin is a correct rounding.
    at_edge = np.abs(t - np.round(t)) < 1e-9
    lower = ((np.round(t).astype(int) - 1) % N).astype(np.uint8)
    upper = (np.round(t).astype(int) % N).astype(np.uint8)
    assert crest.sum() > M * M // 2
    clear = crest & ~at_edge
    assert np.array_equal(rmap[clear], want[clear])
    edge = crest & at_edge
    assert np.all((rmap[edge] == lower[edge]) | (rmap[edge] == upper[edge]))
    assert len(np.unique(want[crest])) <= 2


def test_lift_places_the_corrupted_image_in_one_slice():
    M, N = 32, 16
    f = synth.make_image(3, M, "small")
    mask = synth.mask_random(4, M, 0.4)
    rmap, _ = O.orient(f, mask, N)
    psi = O.lift(f, mask, rmap, N)
    fc = f * (1 - mask)
    assert np.array_equal(psi.sum(axis=0), fc)
    assert ((psi != 0).sum(axis=0) <= 1).all()
    assert np.all(psi[:, mask == 1] == 0)
    yy, xx = np.nonzero(fc)
    assert np.array_equal(psi[rmap[yy, xx], yy, xx], fc[yy, xx])


# ---------------------------------------------------------------------------
# project
# ---------------------------------------------------------------------------

def test_projection_max_and_mean():
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((8, 16, 16))
    mx, mn = O.project(psi, "max"), O.project(psi, "mean")
    assert np.all(mx >= mn)
    single = np.zeros_like(psi)
    single[3] = np.abs(psi[3])
    assert np.array_equal(O.project(single, "max"), np.abs(psi[3]))
    assert np.allclose(O.project(single, "mean"), np.abs(psi[3]) / 8)


# ---------------------------------------------------------------------------
# printed parameters (Appendix A, Table 1; Sec. "The weighting of the metric")
# ---------------------------------------------------------------------------

def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_parameters.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, alpha, T, n, eps, w, pct = line.split()
            rows.append((name, float(alpha), float(T), int(n), float(eps), int(w), int(pct)))
    return rows


def test_alpha_beta_relation_on_table1():
    """alpha = beta_N (2 pi / N)^2; at N = 30 the printed alphas 0.3..4 map to beta 6.8..91."""
    rows = _table1()
    assert len(rows) == 13
    for (_, alpha, *_rest) in rows:
        beta = O.beta_from_alpha(alpha, 30)
        assert abs(beta * (2 * np.pi / 30) ** 2 - alpha) < 1e-14
    assert abs(O.beta_from_alpha(1.0, 2 * np.pi) - 1.0) < 1e-15


def test_stripe_masks_reach_table1_corruption():
    """A w-pixel stripe grid removes 1 - (1 - w/p)^2 of the pixels; at 256^2 the
    printed 37% for w = 3 is reached with a period of about 15 px."""
    rows = _table1()
    w3 = [r for r in rows if r[5] == 3 and r[6] == 37]
    assert w3
    m = synth.mask_stripes(256, 3, 15)
    assert abs(m.mean() - 0.36) < 0.01
