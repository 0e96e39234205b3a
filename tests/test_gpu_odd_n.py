"""Odd orientation counts (no p/q block split: one N x N propagator per
frequency class) against the FP64 oracle: FP64 at 1e-10, FP32 at 2e-5
rel-L2, lift on the GPU's orientation map."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1304_2062_amd import se2n, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("M,N,dtype,scheme,T,n", [
    (36, 5, torch.float64, "cn", 0.5, 30), (36, 5, torch.float64, "exact", 0.5, 1),
    (108, 7, torch.float32, "cn", 1.0, 50), (64, 63, torch.float64, "cn", 0.3, 20),
    (512, 31, torch.float32, "cn", 2.0, 200), (96, 9, torch.float32, "exact", 1.5, 1),
])
def test_inpaint_matches_oracle(M, N, dtype, scheme, T, n):
    print(f"odd N: M={M} N={N} {dtype} {scheme}", flush=True)
    f = synth.make_image(60 + N, M, "medium")
    if dtype == torch.float32:
        f = f.astype(np.float32).astype(np.float64)
    mask = (synth.mask_random(61 + N, M, 0.6) | synth.mask_stripes(M, 3, 21)).astype(np.uint8)
    beta = 1.3
    plan = se2n.Plan(M, N, dtype)
    out, rmap = plan.inpaint(torch.from_numpy(f).to(DEV, dtype), torch.from_numpy(mask).to(DEV), T, beta, n,
                             scheme=scheme)
    torch.cuda.synchronize()
    got = out.double().cpu().numpy()
    plan.close()
    want, _ = O.inpaint(f, mask, N, T, beta, n, scheme=scheme, rmap=rmap.cpu().numpy())
    assert _rel(got, want) < (2e-5 if dtype == torch.float32 else 1e-10)


def test_negligible_skip_with_odd_n_at_2048(monkeypatch):
    """2048^2, N = 31, T = 4: a large share of the classes is negligible and
    their modes are neither stored nor read by the column passes (a compiled
    size); the result equals the run that keeps every class."""
    case = synth.make_case("large")
    M, N, T, n = 2048, 31, 4.0, 400
    f = torch.from_numpy(case["f"].astype(np.float32)).to(DEV)
    m = torch.from_numpy(case["mask"]).to(DEV)
    plan = se2n.Plan(M, N, torch.float32)
    a, rmap = plan.inpaint(f, m, T, 1.0, n)
    neg = float(plan.propagator_flags(T, 1.0, n).mean())
    monkeypatch.setenv("SE2N_KEEP_NEGLIGIBLE", "1")
    keep = se2n.Plan(M, N, torch.float32)
    monkeypatch.delenv("SE2N_KEEP_NEGLIGIBLE")
    b, _ = keep.inpaint(f, m, T, 1.0, n, rmap_in=rmap)
    torch.cuda.synchronize()
    print(f"  negligible classes {neg:.3f}", flush=True)
    assert neg > 0.1
    assert _rel(a.double().cpu().numpy(), b.double().cpu().numpy()) < 2e-5
    plan.close()
    keep.close()


def test_diffuse_and_restore_with_odd_n():
    from oracle import restore_oracle as RO
    M, N = 48, 11
    rng = np.random.default_rng(11)
    psi = rng.normal(size=(N, M, M))
    plan = se2n.Plan(M, N, torch.float64)
    t = torch.from_numpy(psi).to(DEV)
    plan.diffuse(t, 0.4, 2.0, 15)
    torch.cuda.synchronize()
    assert _rel(t.cpu().numpy(), O.diffuse(psi, 0.4, 2.0, 15, "cn")) < 1e-10
    f = 0.1 + 0.9 * synth.make_image(3, M, "small")
    mask = synth.mask_stripes(M, 2, 7)
    out, rmap, join = plan.restore(torch.from_numpy(f).to(DEV), torch.from_numpy(mask).to(DEV), 0.3, 2.0, 6, 0.5,
                                   dynamic=True)
    torch.cuda.synchronize()
    want, _, wjoin, info = RO.restore(f, mask, N, 0.3, 2.0, 6, 0.5, dynamic=True, rmap=rmap.cpu().numpy())
    assert info["min_margin"] > 1e-9 and np.array_equal(join.cpu().numpy(), wjoin)
    assert _rel(out.cpu().numpy(), want) < 1e-10
    with pytest.raises(se2n.Se2nError) as e:
        plan.set_schedule("iterated")
    assert e.value.code == -2
    plan.close()
