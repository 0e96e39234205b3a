"""GPU parity of the corrector network's BF16 MFMA kernels against the FP64
reference (oracle/cnn_oracle.py) with bfloat16 rounding at the same points:
forward, loss, gradients and Adam; and the corrected inpainting path."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C
from paper_1304_2062_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def se2n():
    from paper_1304_2062_amd import se2n as mod
    return mod


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _say(msg):
    print(msg, flush=True)


def _params(N, seed):
    """Oracle-initialised layers 1-2, a random nonzero layer 3 and random biases
    (padded entries zero), rounded to float32 (what the GPU holds)."""
    rng = np.random.default_rng(seed)
    p = C.init_params(N, seed)
    L = C.unpack(p)
    w3 = 0.05 * rng.standard_normal((C.CP, C.CP, 3, 3))
    w3[N:] = 0.0
    b = [0.05 * rng.standard_normal(C.CP) for _ in range(3)]
    b[2][N:] = 0.0
    p = C.pack([(L[0][0], b[0]), (L[1][0], b[1]), (w3, b[2])])
    return p.astype(np.float32).astype(np.float64)


# Tolerances: both sides round the same values to bfloat16; what remains is
# FP32 accumulation order and the bfloat16 rounding decisions that a last-bit
# FP32/FP64 difference flips.  A flip moves one stored activation by one bf16
# ulp (2^-8 relative) and reaches every output within two pixels through the
# following layers; a few flips per 32x32x32 volume give ~1e-4.  The bounds
# are an order of magnitude below the difference between the bfloat16 network
# and the same network in FP64 (~5e-3), so a result inside them follows the
# rounding points of the reference, not merely the network.
TOL_FWD = 1e-3
TOL_GRAD = 5e-3


@pytest.mark.parametrize("N,M,B", [(8, 32, 2), (32, 48, 1), (5, 16, 3)])
def test_forward_matches_the_reference(se2n, N, M, B):
    rng = np.random.default_rng(100 + N)
    p = _params(N, 7 + N)
    net = se2n.Corrector(N, seed=1)
    net.set_params(p)
    x = rng.standard_normal((B, N, M, M)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    out = net.forward(xt).cpu().numpy().astype(np.float64)
    for b in range(B):
        ref = C.forward(x[b].astype(np.float64), p, bf16=True)
        exact = C.forward(x[b].astype(np.float64), p, bf16=False)
        r_gpu = out[b] - x[b]
        rel = _rel(r_gpu, ref["out"] - x[b])
        gap = _rel(r_gpu, exact["out"] - x[b])
        _say(f"forward N={N} M={M} b={b}: rel vs bf16 reference {rel:.2e}, vs FP64 network {gap:.2e}")
        assert rel < TOL_FWD and rel < 0.1 * gap
    net.close()


@pytest.mark.parametrize("N,M,B", [(8, 32, 2), (32, 32, 1)])
def test_gradients_and_loss_match_the_reference(se2n, N, M, B):
    rng = np.random.default_rng(200 + N)
    p = _params(N, 11 + N)
    net = se2n.Corrector(N, seed=2)
    net.set_params(p)
    x = rng.standard_normal((B, N, M, M)).astype(np.float32)
    t = (x + 0.3 * rng.standard_normal(x.shape)).astype(np.float32)
    g, loss = net.gradients(torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda())
    g = g.cpu().numpy().astype(np.float64)
    xs = [xi.astype(np.float64) for xi in x]
    ts = [ti.astype(np.float64) for ti in t]
    ref_loss, ref_g = C.loss_and_grads(xs, ts, p, bf16=True)
    _, exact_g = C.loss_and_grads(xs, ts, p, bf16=False)
    # the loss moves with the forward pass's rounding flips (bounded by TOL_FWD
    # on r); its FP32 summation alone agrees to ~1e-7
    assert abs(float(loss.item()) - ref_loss) <= 1e-4 * ref_loss
    for l in range(3):
        for name, sl in (("W", slice(l * C.NL, l * C.NL + C.NW)), ("b", slice(l * C.NL + C.NW, (l + 1) * C.NL))):
            rel = _rel(g[sl], ref_g[sl])
            gap = _rel(g[sl], exact_g[sl])
            _say(f"grad N={N} layer {l + 1} {name}: rel vs bf16 reference {rel:.2e}, vs FP64 network {gap:.2e}")
            assert rel < TOL_GRAD
    # padded entries receive no gradient
    L = C.unpack(g)
    assert np.all(L[0][0][:, N:] == 0.0) and np.all(L[2][0][N:] == 0.0) and np.all(L[2][1][N:] == 0.0)
    net.close()


def test_adam_step_matches_the_reference(se2n):
    rng = np.random.default_rng(300)
    N = 16
    p = _params(N, 3)
    net = se2n.Corrector(N, seed=3)
    net.set_params(p)
    g1 = rng.standard_normal(C.NPARAM).astype(np.float32).astype(np.float64)
    g2 = rng.standard_normal(C.NPARAM).astype(np.float32).astype(np.float64)
    net.adam_step(torch.from_numpy(g1.astype(np.float32)).cuda(), 1e-3)
    net.adam_step(torch.from_numpy(g2.astype(np.float32)).cuda(), 1e-3)
    got = net.params().astype(np.float64)
    q, m, v = C.adam(p, g1, np.zeros_like(p), np.zeros_like(p), 1, 1e-3)
    q, m, v = C.adam(q, g2, m, v, 2, 1e-3)
    assert np.max(np.abs(got - q)) < 1e-6
    net.close()


def test_params_roundtrip_and_padding(se2n, tmp_path):
    N = 6
    net = se2n.Corrector(N, seed=4)
    p0 = net.params()
    assert p0.size == C.NPARAM
    L = C.unpack(p0.astype(np.float64))
    assert np.all(L[2][0] == 0.0) and np.all(L[0][0][:, N:] == 0.0)
    q = np.random.default_rng(5).standard_normal(C.NPARAM).astype(np.float32)
    net.set_params(q)
    got = C.unpack(net.params().astype(np.float64))
    want = C.unpack(q.astype(np.float64))
    assert np.array_equal(got[1][0], want[1][0])
    assert np.all(got[0][0][:, N:] == 0.0) and np.all(got[2][0][N:] == 0.0)
    path = str(tmp_path / "w.npz")
    net.save(path)
    other = se2n.Corrector(N, seed=9)
    other.load(path)
    assert np.array_equal(other.params(), net.params())
    net.close()
    other.close()


def test_corrected_path_with_an_identity_network_is_the_plain_path(se2n):
    """Layer 3 is zero at creation, so the corrected path equals the plain
    inpainting with the same (coarse) step count."""
    case = synth.make_case("small", M=64)
    N = case["N"]
    plan = se2n.Plan(64, N, torch.float32)
    plan.set_schedule("propagator")  # the same schedule for the calls compared bit for bit
    net = se2n.Corrector(N, seed=6)
    f = torch.from_numpy(case["f"].astype(np.float32)).cuda()
    m = torch.from_numpy(case["mask"]).cuda()
    # a record licenses the network in this regime (the identity's error against
    # the 64-step solve is the coarse solve's own)
    net.set_validation(64, case["T"], case["beta"], 8, 64, 0.01)
    out_c, rmap_c, fb = se2n.inpaint_corrected(plan, net, f, m, case["T"], case["beta"], 8, 64, max_rel_l2=0.02)
    out_p, rmap_p = plan.inpaint(f, m, case["T"], case["beta"], 8)
    torch.cuda.synchronize()
    assert not fb
    assert torch.equal(rmap_c, rmap_p)
    assert _rel(out_c.cpu().numpy(), out_p.cpu().numpy()) < 1e-6
    # above the recorded error, or without a record, the fine-step plain path runs
    out_f, _, fb = se2n.inpaint_corrected(plan, net, f, m, case["T"], case["beta"], 8, 64, max_rel_l2=0.005)
    ref_f, _ = plan.inpaint(f, m, case["T"], case["beta"], 64)
    torch.cuda.synchronize()
    assert fb and torch.equal(out_f, ref_f)
    _, _, fb = se2n.inpaint_corrected(plan, net, f, m, case["T"], case["beta"], 8, 32, max_rel_l2=1.0)
    assert fb
    net.close()
    plan.close()


def test_corrected_call_meets_the_bar_at_1024(se2n):
    """The committed network at 1024^2, N = 32 (25 coarse steps to T = 2 against
    the 200-step solve): whichever path the call takes, its output is within
    1e-3 of the fine-step FP64 solve (the network's recorded error there is
    far above the bar, so the call must fall back)."""
    import os
    from paper_1304_2062_amd import corrector
    M, N, T, beta = 1024, 32, 2.0, 1.0
    net = se2n.Corrector(N)
    net.load(os.path.join(os.path.dirname(corrector.__file__), "corrector_N32.npz"))
    plan = se2n.Plan(M, N, torch.float32)
    p64 = se2n.Plan(M, N, torch.float64)
    (f, m), = corrector.images([corrector.EVAL_SEED0 + 100], M, workers=1)
    ft, mt = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
    out, rmap, fb = se2n.inpaint_corrected(plan, net, ft, mt, T, beta, 25, 200, max_rel_l2=1e-3)
    ref, _ = p64.inpaint(ft.double(), mt, T, beta, 200, rmap_in=rmap)
    torch.cuda.synchronize()
    rel = _rel(out.double().cpu().numpy(), ref.cpu().numpy())
    _say(f"corrected call at 1024^2: fallback={fb}, rel-L2 vs fine FP64 {rel:.2e}")
    assert fb
    assert rel < 1e-3
    net.close()
    plan.close()
    p64.close()


def _pairs(se2n, M, N, seeds, n_coarse=25, n_fine=200, T=2.0):
    from paper_1304_2062_amd import corrector
    plan = se2n.Plan(M, N, torch.float32)
    C_, F_ = corrector.pairs(plan, corrector.images(seeds, M, workers=4), T, 1.0, n_coarse, n_fine)
    torch.cuda.synchronize()
    plan.close()
    return C_, F_


def _rel_t(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def test_training_on_the_gpu_reduces_the_coarse_step_error(se2n):
    """A short training run (library kernels only: forward, loss, backward,
    Adam) on coarse/fine pairs the method generates; the held-out error of the
    corrected volumes against the fine-step solve falls well below the
    coarse-step error."""
    M, N = 256, 32
    C_, F_ = _pairs(se2n, M, N, range(30000, 30000 + 160))
    Ch, Fh = C_[128:].contiguous(), F_[128:].contiguous()
    net = se2n.Corrector(N, seed=0)
    base = _rel_t(Ch, Fh)
    gen = torch.Generator().manual_seed(0)
    for ep in range(12):
        perm = torch.randperm(128, generator=gen)
        for k in range(0, 128, 16):
            idx = perm[k:k + 16].cuda()
            net.train_step(C_.index_select(0, idx), F_.index_select(0, idx), 3e-4)
    out = net.forward(Ch)
    rel = _rel_t(out, Fh)
    _say(f"trained 12 epochs at {M}^2 N={N}: held-out rel-L2 {rel:.3e} vs coarse {base:.3e} ({rel / base:.3f})")
    assert rel < 0.7 * base
    net.close()


def test_committed_network_gains_on_held_out_images(se2n):
    """The committed network (trained on 2000 pairs of 256^2, N = 32, 25 vs 200
    steps to T = 2) on held-out 256^2 images."""
    import os
    from paper_1304_2062_amd import corrector
    path = os.path.join(os.path.dirname(corrector.__file__), "corrector_N32.npz")
    net = se2n.Corrector(32)
    net.load(path)
    C_, F_ = _pairs(se2n, 256, 32, range(corrector.EVAL_SEED0, corrector.EVAL_SEED0 + 4))
    base = _rel_t(C_, F_)
    out = net.forward(C_.contiguous())
    rel = _rel_t(out, F_)
    _say(f"committed network at 256^2: rel-L2 {rel:.3e} vs coarse {base:.3e} ({rel / base:.3f})")
    assert rel < 0.3 * base
    net.close()


def test_training_resumes_bit_for_bit_from_a_checkpoint(se2n, tmp_path):
    """Training checkpoint = parameters + Adam moments + step counter: 3 steps,
    save, 3 more steps; a fresh network loaded from the checkpoint and taking
    the same 3 steps ends with identical parameters (training is deterministic)."""
    torch.manual_seed(0)
    M, N = 64, 8
    c = torch.randn((4, N, M, M), device="cuda")
    f = c + 0.05 * torch.randn_like(c)
    a = se2n.Corrector(N, seed=3)
    for _ in range(3):
        a.train_step(c, f, 1e-3)
    path = str(tmp_path / "ckpt.npz")
    a.save(path, with_optimizer=True)
    for _ in range(3):
        a.train_step(c, f, 1e-3)
    b = se2n.Corrector(N, seed=99)
    b.load(path)
    assert b.adam_state()[2] == 3
    for _ in range(3):
        b.train_step(c, f, 1e-3)
    torch.cuda.synchronize()
    assert np.array_equal(a.params(), b.params())
    ma, va, ta = a.adam_state()
    mb, vb, tb = b.adam_state()
    assert ta == tb == 6 and np.array_equal(ma, mb) and np.array_equal(va, vb)
    a.close()
    b.close()
