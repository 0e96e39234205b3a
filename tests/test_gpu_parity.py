"""GPU parity: the gfx950 library against the FP64 oracle, element by element.

Tolerances (rel-L2 over the whole result): 1e-10 for FP64 runs, 2e-5 for FP32
runs.  The orientation map is a discontinuous function of the gradient, so the
downstream steps are compared on the GPU's own map (the oracle lifts with it),
and the map itself is compared bin for bin away from rounding-level ties.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1304_2062_amd import synth

pytestmark = pytest.mark.gpu

TOL = {torch.float64: 1e-10, torch.float32: 2e-5}
TIE = {torch.float64: 1e-9, torch.float32: 1e-4}
# Absolute error of the FFT-computed gradient relative to its maximum: the
# angle of a pixel whose gradient is smaller than this floor is rounding noise.
GRAD_FLOOR = {torch.float64: 1e-13, torch.float32: 1e-5}


def _decided(f, mask, N, sigma, dtype):
    """Pixels whose orientation bin the given precision determines: away from a
    bin edge by more than the angle's rounding uncertainty (in bins)."""
    gx, gy = O.smoothed_gradient(f, mask, sigma)
    mag = np.hypot(gx, gy)
    _, tie = O.orient(f, mask, N, sigma)
    unc = GRAD_FLOOR[dtype] * mag.max() / np.maximum(mag, 1e-300) * N / (2 * np.pi)
    return tie > np.maximum(TIE[dtype], unc)


@pytest.fixture(scope="module")
def se2n():
    from paper_1304_2062_amd import se2n as mod
    return mod


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _say(msg):
    print(msg, flush=True)


# ---------------------------------------------------------------------------
# diffusion of a real-space volume
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("M,N", [(64, 16), (48, 4), (24, 6), (96, 30), (72, 8), (16, 64)])
def test_zero_time_is_identity(se2n, dtype, M, N):
    """T = 0: the propagator is the identity, so diffuse = inverse FFT of forward FFT."""
    _say(f"identity M={M} N={N} {dtype}")
    rng = np.random.default_rng(M + N)
    psi0 = rng.standard_normal((N, M, M))
    plan = se2n.Plan(M, N, dtype)
    psi = _dev(psi0, dtype)
    plan.diffuse(psi, 0.0, 1.0, 1)
    torch.cuda.synchronize()
    ref = psi0.astype(np.float32).astype(np.float64) if dtype == torch.float32 else psi0
    assert _rel(psi.cpu().numpy(), ref) < (1e-14 if dtype == torch.float64 else 2e-6)
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("scheme", ["cn", "exact"])
@pytest.mark.parametrize("M,N,beta,T,n", [
    (64, 16, 1.0, 0.5, 50),
    (48, 4, 2.0, 0.3, 7),
    (24, 6, 0.0, 0.2, 5),
    (96, 30, 1.0, 2.0, 200),
    (72, 8, 4.0, 1.0, 33),
    (16, 64, 0.25, 4.0, 400),
])
def test_diffuse_matches_oracle(se2n, dtype, scheme, M, N, beta, T, n):
    _say(f"diffuse M={M} N={N} beta={beta} T={T} n={n} {scheme} {dtype}")
    rng = np.random.default_rng(7 * M + N)
    psi0 = rng.standard_normal((N, M, M))
    if dtype == torch.float32:
        psi0 = psi0.astype(np.float32).astype(np.float64)
    want = O.diffuse(psi0, T, beta, n, scheme)
    plan = se2n.Plan(M, N, dtype)
    psi = _dev(psi0, dtype)
    plan.diffuse(psi, T, beta, n, scheme)
    torch.cuda.synchronize()
    err = _rel(psi.cpu().numpy(), want)
    _say(f"  rel-L2 {err:.3e}")
    assert err < TOL[dtype]
    plan.close()


# ---------------------------------------------------------------------------
# orient / lift / project
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("name,M", [("small", 64), ("medium", 512), ("small", 192)])
def test_orient_matches_oracle(se2n, dtype, name, M):
    case = synth.make_case(name, M=M)
    N = case["N"]
    f = case["f"].astype(np.float32).astype(np.float64) if dtype == torch.float32 else case["f"]
    _say(f"orient {name} M={M} N={N} {dtype}")
    want, _ = O.orient(f, case["mask"], N, case["sigma"])
    plan = se2n.Plan(M, N, dtype)
    got = plan.orient(_dev(f, dtype), _dev(case["mask"]), case["sigma"]).cpu().numpy()
    clear = _decided(f, case["mask"], N, case["sigma"], dtype)
    mism = (got != want) & clear
    _say(f"  undecided pixels {int((~clear).sum())} ({(~clear).mean():.2e}), "
         f"mismatches elsewhere {int(mism.sum())}, mismatches in total {int((got != want).sum())}")
    assert mism.sum() == 0
    assert (~clear).mean() < 1e-2
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_lift_and_project_are_exact(se2n, dtype):
    M, N = 64, 16
    case = synth.make_case("small")
    f = case["f"].astype(np.float32).astype(np.float64) if dtype == torch.float32 else case["f"]
    rmap, _ = O.orient(f, case["mask"], N)
    plan = se2n.Plan(M, N, dtype)
    psi = plan.lift(_dev(f, dtype), _dev(case["mask"]), _dev(rmap))
    want = O.lift(f, case["mask"], rmap, N)
    assert np.array_equal(psi.cpu().numpy(), want)
    rng = np.random.default_rng(2)
    vol = rng.standard_normal((N, M, M))
    if dtype == torch.float32:
        vol = vol.astype(np.float32).astype(np.float64)
    vd = _dev(vol, dtype)
    assert np.array_equal(plan.project(vd, "max").cpu().numpy(), O.project(vol, "max"))
    mean = plan.project(vd, "mean").cpu().numpy()
    assert _rel(mean, O.project(vol, "mean")) < (1e-15 if dtype == torch.float64 else 1e-6)
    plan.close()


# ---------------------------------------------------------------------------
# whole path
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("proj", ["max", "mean"])
def test_inpaint_small_case(se2n, dtype, proj):
    """64^2, 30% loss, N=16, beta=1, T=0.5, 50 CN steps."""
    case = synth.make_case("small")
    f = case["f"].astype(np.float32).astype(np.float64) if dtype == torch.float32 else case["f"]
    _say(f"inpaint small {dtype} {proj}")
    plan = se2n.Plan(case["M"], case["N"], dtype)
    out, rmap = plan.inpaint(_dev(f, dtype), _dev(case["mask"]), case["T"], case["beta"], case["n_steps"],
                             sigma=case["sigma"], proj=proj)
    torch.cuda.synchronize()
    rmap = rmap.cpu().numpy()
    want, _ = O.inpaint(f, case["mask"], case["N"], case["T"], case["beta"], case["n_steps"], proj=proj,
                        rmap=rmap)
    err = _rel(out.cpu().numpy(), want)
    _say(f"  rel-L2 {err:.3e}")
    assert err < TOL[dtype]
    own, rmap_o = O.inpaint(f, case["mask"], case["N"], case["T"], case["beta"], case["n_steps"], proj=proj)
    _say(f"  with independent orientation maps: {int((rmap_o != rmap).sum())} bins differ, "
         f"rel-L2 {_rel(out.cpu().numpy(), own):.3e}")
    plan.close()


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_inpaint_medium_case(se2n, dtype):
    """512^2, 70% loss + 3 px stripes every 32 px, N=30, beta=1, T=2, 200 CN steps."""
    case = synth.make_case("medium")
    f = case["f"].astype(np.float32).astype(np.float64) if dtype == torch.float32 else case["f"]
    _say(f"inpaint medium {dtype}")
    plan = se2n.Plan(case["M"], case["N"], dtype)
    out, rmap = plan.inpaint(_dev(f, dtype), _dev(case["mask"]), case["T"], case["beta"], case["n_steps"],
                             sigma=case["sigma"])
    torch.cuda.synchronize()
    rmap = rmap.cpu().numpy()
    want, _ = O.inpaint(f, case["mask"], case["N"], case["T"], case["beta"], case["n_steps"], rmap=rmap)
    err = _rel(out.cpu().numpy(), want)
    _say(f"  rel-L2 {err:.3e}")
    assert err < TOL[dtype]
    plan.close()


def test_rmap_in_is_used_and_copied(se2n):
    case = synth.make_case("small")
    M, N = case["M"], case["N"]
    rng = np.random.default_rng(5)
    rmap = rng.integers(0, N, size=(M, M)).astype(np.uint8)
    plan = se2n.Plan(M, N, torch.float64)
    out, rmap_out = plan.inpaint(_dev(case["f"]), _dev(case["mask"]), case["T"], case["beta"], case["n_steps"],
                                 rmap_in=_dev(rmap))
    torch.cuda.synchronize()
    assert np.array_equal(rmap_out.cpu().numpy(), rmap)
    want, _ = O.inpaint(case["f"], case["mask"], N, case["T"], case["beta"], case["n_steps"], rmap=rmap)
    assert _rel(out.cpu().numpy(), want) < 1e-10
    plan.close()


# ---------------------------------------------------------------------------
# full size: properties and sampled modes
# ---------------------------------------------------------------------------

def _plane_wave_volume(M, N, waves):
    """Sum of cos(2 pi (k x + l y)/M + phi) placed in orientation slices."""
    y, x = np.mgrid[0:M, 0:M]
    psi = np.zeros((N, M, M))
    for (k, l, r, amp, phi) in waves:
        psi[r] += amp * np.cos(2 * np.pi * (k * x + l * y) / M + phi)
    return psi


def _plane_wave_solution(M, N, waves, beta, T, n):
    """Exact discrete solution: each wave excites modes (k,l) and (-k,-l) of one slice;
    the oracle's per-mode CN propagates them, then the waves are summed on the grid."""
    y, x = np.mgrid[0:M, 0:M]
    out = np.zeros((N, M, M))
    for (k, l, r, amp, phi) in waves:
        e = np.zeros((1, N), dtype=np.complex128)
        e[0, r] = 1.0
        v = O.diffuse_modes_cn(e, M, [k], [l], beta, T, n)[0].real  # real propagator column
        ph = 2 * np.pi * (k * x + l * y) / M + phi
        out += amp * v[:, None, None] * np.cos(ph)[None]
    return out


@pytest.mark.parametrize("dtype", [torch.float32])
def test_full_size_sampled_modes(se2n, dtype):
    """2048^2, N=32, T=4, 400 steps, beta in {0.25, 1, 4}: plane waves at sampled
    frequencies (including the class mirrors kx -> M/2-kx, ky -> -ky) are
    propagated exactly as the oracle's per-mode Crank-Nicolson says."""
    M, N, T, n = 2048, 32, 4.0, 400
    waves = [(1, 0, 0, 1.0, 0.0), (3, 5, 7, 0.5, 0.3), (1021, 17, 12, 0.7, 1.1), (17, 2031, 12, 0.7, -0.4),
             (0, 1024, 5, 0.2, 0.0), (512, 512, 31, 0.3, 0.5), (700, 1500, 20, 0.4, 2.0), (2, 1, 16, 1.0, 0.7)]
    psi0 = _plane_wave_volume(M, N, waves)
    plan = se2n.Plan(M, N, dtype)
    for beta in (0.25, 1.0, 4.0):
        _say(f"full-size sampled modes beta={beta}")
        want = _plane_wave_solution(M, N, waves, beta, T, n)
        psi = _dev(psi0, dtype)
        plan.diffuse(psi, T, beta, n)
        torch.cuda.synchronize()
        got = psi.cpu().numpy()
        err = np.abs(got - want).max() / np.abs(psi0).max()
        _say(f"  max error / max input {err:.3e}")
        assert err < 2e-5
    plan.close()


def test_full_size_inpaint_properties(se2n):
    """2048^2, N=32, T=4, 400 steps on the large synthetic case: the lifted mass
    is conserved by the diffusion and the FP32 result agrees with the FP64 run."""
    case = synth.make_case("large")
    M, N = case["M"], case["N"]
    f32 = case["f"].astype(np.float32)
    res = {}
    for dtype in (torch.float32, torch.float64):
        plan = se2n.Plan(M, N, dtype)
        fd = _dev(f32.astype(np.float64), dtype)
        md = _dev(case["mask"])
        rmap = plan.orient(fd, md, case["sigma"]) if dtype == torch.float32 else res["rmap"]
        psi = plan.lift(fd, md, rmap)
        mass0 = psi.double().sum().item()
        plan.diffuse(psi, case["T"], case["beta"], case["n_steps"])
        mass1 = psi.double().sum().item()
        _say(f"  {dtype}: mass {mass0:.9e} -> {mass1:.9e}")
        assert abs(mass1 - mass0) < (1e-5 if dtype == torch.float32 else 1e-11) * abs(mass0)
        out, _ = plan.inpaint(fd, md, case["T"], case["beta"], case["n_steps"], rmap_in=rmap)
        proj = plan.project(psi, "max")
        torch.cuda.synchronize()
        assert _rel(out.cpu().numpy(), proj.cpu().numpy()) < TOL[dtype]
        res[dtype] = out.cpu().numpy()
        res["rmap"] = rmap
        plan.close()
    err = _rel(res[torch.float32], res[torch.float64])
    _say(f"  FP32 vs FP64 rel-L2 {err:.3e}")
    assert err < 2e-5
