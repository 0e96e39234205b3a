"""The 2048^2, N = 32, T = 4, 400-step inpaint (the timed configuration) at
every beta in {0.25, 1, 4} against the FP64 oracle.

The oracle's outputs at 16384 fixed pixels are stored in
tests/golden/c3_oracle_samples.npz, written by tests/golden/make_c3_samples.py
(which calls only the oracle and the input generator; a 2048^2 oracle run
takes minutes).  Both sides lift with the oracle's FP64 orientation map: the
GPU's FP64 orientation route must reproduce it bin for bin (its SHA-256 is
stored), and that map is passed to every GPU run as rmap_in.

Tolerances: rel-L2 over the samples <= 2e-5 for FP32 plans, <= 1e-10 for FP64.
"""
import hashlib
import os

import numpy as np
import pytest
import torch

from paper_1304_2062_amd import se2n, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_oracle_samples.npz")


@pytest.fixture(scope="module")
def c3():
    g = np.load(GOLDEN, allow_pickle=False)
    case = synth.make_case("large")
    f64 = case["f"].astype(np.float32).astype(np.float64)
    M, N = case["M"], case["N"]
    assert (M, N, case["T"], case["n_steps"]) == (int(g["M"]), int(g["N"]), float(g["T"]), int(g["n_steps"]))
    p64 = se2n.Plan(M, N, torch.float64)
    ft64 = torch.from_numpy(f64).to(DEV)
    mt = torch.from_numpy(case["mask"]).to(DEV)
    rmap = p64.orient(ft64, mt, case["sigma"])
    torch.cuda.synchronize()
    sha = hashlib.sha256(rmap.cpu().numpy().tobytes()).hexdigest()
    yield dict(g=g, case=case, p64=p64, f64=ft64, f32=ft64.float(), mask=mt, rmap=rmap, sha=sha,
               idx=torch.from_numpy(g["idx"]).to(DEV))
    p64.close()


def _rel_samples(c3, out, beta):
    want = torch.from_numpy(c3["g"][f"beta_{beta:g}_samples"]).to(DEV)
    got = out.reshape(-1).index_select(0, c3["idx"]).double()
    return float(torch.linalg.norm(got - want) / torch.linalg.norm(want))


def test_gpu_fp64_orientation_equals_the_oracle_map(c3):
    """Bin-exact: the oracle's closest bin edge is far above FP64 rounding."""
    assert float(c3["g"]["rmap_min_tie"]) > 1e-12
    assert c3["sha"] == str(c3["g"]["rmap_sha256"])


@pytest.mark.parametrize("beta", [0.25, 1.0, 4.0])
def test_fp32_inpaint_matches_oracle(c3, beta):
    case = c3["case"]
    print(f"C3 FP32 beta={beta}", flush=True)
    plan = se2n.Plan(case["M"], case["N"], torch.float32)
    out, _ = plan.inpaint(c3["f32"], c3["mask"], case["T"], beta, case["n_steps"], rmap_in=c3["rmap"])
    torch.cuda.synchronize()
    neg = float(plan.propagator_flags(case["T"], beta, case["n_steps"]).mean())
    rel = _rel_samples(c3, out, beta)
    print(f"  rel-L2 vs oracle {rel:.3e}, negligible classes {neg:.3f}", flush=True)
    assert rel < 2e-5
    plan.close()


def test_fp64_inpaint_matches_oracle(c3):
    case = c3["case"]
    print("C3 FP64 beta=1", flush=True)
    out, _ = c3["p64"].inpaint(c3["f64"], c3["mask"], case["T"], 1.0, case["n_steps"], rmap_in=c3["rmap"])
    torch.cuda.synchronize()
    rel = _rel_samples(c3, out, 1.0)
    print(f"  rel-L2 vs oracle {rel:.3e}", flush=True)
    assert rel < 1e-10


def test_fp32_without_the_negligible_skip_matches_oracle(c3, monkeypatch):
    """The plan option that keeps every class (the timing without the skip)
    computes the same result."""
    case = c3["case"]
    print("C3 FP32 beta=1, no class skipped", flush=True)
    monkeypatch.setenv("SE2N_KEEP_NEGLIGIBLE", "1")
    plan = se2n.Plan(case["M"], case["N"], torch.float32)
    monkeypatch.delenv("SE2N_KEEP_NEGLIGIBLE")
    out, _ = plan.inpaint(c3["f32"], c3["mask"], case["T"], 1.0, case["n_steps"], rmap_in=c3["rmap"])
    torch.cuda.synchronize()
    assert float(plan.propagator_flags(case["T"], 1.0, case["n_steps"]).mean()) == 0.0
    assert _rel_samples(c3, out, 1.0) < 2e-5
    plan.close()


def test_fp32_iterated_schedule_matches_oracle(c3):
    """The 400 Crank-Nicolson steps taken one by one on every mode."""
    case = c3["case"]
    print("C3 FP32 beta=1, iterated schedule", flush=True)
    plan = se2n.Plan(case["M"], case["N"], torch.float32)
    plan.set_schedule("iterated")
    out, _ = plan.inpaint(c3["f32"], c3["mask"], case["T"], 1.0, case["n_steps"], rmap_in=c3["rmap"])
    torch.cuda.synchronize()
    assert plan.last_schedule() == "iterated"
    rel = _rel_samples(c3, out, 1.0)
    print(f"  rel-L2 vs oracle {rel:.3e}", flush=True)
    assert rel < 2e-5
    plan.close()
