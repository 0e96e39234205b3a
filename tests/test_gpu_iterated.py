"""The iterated Crank-Nicolson schedule (remark 2 after Theorem 2: n steps per
mode with a cyclic tridiagonal solver) against the FP64 oracle, which also
steps Crank-Nicolson per mode (Thomas + Sherman-Morrison on the full N-cycle;
the GPU solves the two N/2 blocks of the p/q split).

Tolerances: 1e-10 (FP64 plans) and 2e-5 (FP32) rel-L2, as for the collapsed
propagator.  The downstream comparison runs on the GPU's orientation map.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1304_2062_amd import se2n, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _inpaint_iter(case, dtype, schedule="iterated", **over):
    c = dict(case)
    c.update(over)
    plan = se2n.Plan(c["M"], c["N"], dtype)
    plan.set_schedule(schedule)
    f = torch.from_numpy(c["f"]).to(DEV, dtype)
    m = torch.from_numpy(c["mask"]).to(DEV)
    out, rmap = plan.inpaint(f, m, c["T"], c["beta"], c["n_steps"], sigma=c["sigma"], proj=c.get("proj", "max"))
    torch.cuda.synchronize()
    used = plan.last_schedule()
    res = out.double().cpu().numpy(), rmap.cpu().numpy(), used
    plan.close()
    return res


def test_small_case_fp64_matches_oracle():
    """64^2, N = 16, beta = 1, T = 0.5, 50 steps, FP64."""
    case = synth.make_case("small")
    print("iterated: 64^2 N=16 FP64", flush=True)
    got, rmap, used = _inpaint_iter(case, torch.float64)
    assert used == "iterated"
    want, _ = O.inpaint(case["f"], case["mask"], case["N"], case["T"], case["beta"], case["n_steps"], rmap=rmap)
    assert _rel(got, want) < 1e-10


def test_medium_case_fp32_matches_oracle():
    """512^2, N = 30, beta = 1, T = 2, 200 steps, FP32 against FP64."""
    case = synth.make_case("medium")
    case["f"] = case["f"].astype(np.float32).astype(np.float64)
    print("iterated: 512^2 N=30 FP32", flush=True)
    got, rmap, used = _inpaint_iter(case, torch.float32)
    assert used == "iterated"
    want, _ = O.inpaint(case["f"], case["mask"], case["N"], case["T"], case["beta"], case["n_steps"], rmap=rmap)
    rel = _rel(got, want)
    print(f"  rel-L2 {rel:.2e}", flush=True)
    assert rel < 2e-5


@pytest.mark.parametrize("M,N,beta,T,n", [(48, 4, 3.0, 0.4, 7), (32, 6, 1.0, 0.3, 1), (32, 64, 2.0, 0.2, 9),
                                          (96, 10, 0.0, 0.5, 12), (24, 8, 50.0, 0.1, 30)])
def test_block_sizes_and_edges_fp64(M, N, beta, T, n):
    """Blocks of 2 (N = 4: the corners coincide with the neighbours), 3 and 32
    (N = 64), one step, beta = 0 (no angular coupling), a stiff coupling, and
    sides with a factor 3 -- diffusion of a random volume, FP64."""
    print(f"iterated: diffuse M={M} N={N} beta={beta} n={n} FP64", flush=True)
    rng = np.random.default_rng(M * 100 + N)
    psi = rng.normal(size=(N, M, M))
    plan = se2n.Plan(M, N, torch.float64)
    plan.set_schedule("iterated")
    t = torch.from_numpy(psi).to(DEV)
    plan.diffuse(t, T, beta, n)
    torch.cuda.synchronize()
    assert plan.last_schedule() == "iterated"
    got = t.cpu().numpy()
    plan.close()
    want = O.diffuse(psi, T, beta, n, "cn")
    assert _rel(got, want) < 1e-10


def test_iterated_and_collapsed_schedules_agree_fp32():
    """The two schedules compute the same CN result; 1024^2, N = 32, FP32."""
    case = synth.make_case("large", M=1024)
    case["f"] = case["f"].astype(np.float32).astype(np.float64)
    print("iterated vs propagator: 1024^2 N=32 FP32, 400 steps", flush=True)
    a, rmap, ua = _inpaint_iter(case, torch.float32, "iterated")
    b, _, ub = _inpaint_iter(case, torch.float32, "propagator")
    assert (ua, ub) == ("iterated", "propagator")
    assert _rel(a, b) < 2e-5


def test_auto_schedule_choice():
    """AUTO: an uncached key cheap to iterate runs the iterated steps once; the
    second request builds the table; EXACT always uses the table."""
    case = synth.make_case("small")
    plan = se2n.Plan(64, 16, torch.float32)
    assert plan.last_schedule() == "auto"  # nothing run yet
    plan.set_schedule("auto")
    f = torch.from_numpy(case["f"]).to(DEV, torch.float32)
    m = torch.from_numpy(case["mask"]).to(DEV)
    a, _ = plan.inpaint(f, m, 0.5, 1.0, 10)
    assert plan.last_schedule() == "iterated"
    b, _ = plan.inpaint(f, m, 0.5, 1.0, 10)
    assert plan.last_schedule() == "propagator"
    c, _ = plan.inpaint(f, m, 0.5, 1.0, 10)
    assert plan.last_schedule() == "propagator"
    plan.inpaint(f, m, 0.5, 1.0, 10, scheme="exact")
    assert plan.last_schedule() == "propagator"
    torch.cuda.synchronize()
    assert _rel(a.double().cpu().numpy(), b.double().cpu().numpy()) < 2e-5
    assert torch.equal(b, c)
    plan.close()
