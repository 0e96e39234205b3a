"""GPU parity of the batched path: many heterogeneous images in one graph
launch, against the FP64 oracle (small images) and against the single-image
FP32 path (every size), across schedules, graph replays and buffer changes."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1304_2062_amd import synth

pytestmark = pytest.mark.gpu

TOL32 = 2e-5


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


def _items(se2n, params):
    out = []
    for p in params:
        f = torch.from_numpy(p["f"].astype(np.float32)).cuda()
        m = torch.from_numpy(p["mask"]).cuda()
        out.append(se2n.BatchItem(f, m, p["N"], p["T"], p["beta"], p["n_steps"], sigma=p["sigma"],
                                  scheme=p.get("scheme", "cn"), proj=p.get("proj", "max")))
    return out


# small heterogeneous images: sides of every size class path (generic, 2^a 3^b)
SMALL = [
    dict(M=16, N=4, T=0.3, n_steps=7, scheme="cn", proj="max", beta=1.0),
    dict(M=24, N=6, T=1.0, n_steps=20, scheme="exact", proj="max", beta=0.5),
    dict(M=48, N=8, T=0.5, n_steps=50, scheme="cn", proj="mean", beta=2.0),
    dict(M=64, N=16, T=0.5, n_steps=50, scheme="cn", proj="max", beta=1.0),
    dict(M=72, N=10, T=2.0, n_steps=40, scheme="cn", proj="max", beta=1.0),
    dict(M=96, N=12, T=1.5, n_steps=30, scheme="exact", proj="mean", beta=1.0),
]


# sigma = 6 at M = 72 and 96 takes the FFT route of the orientation step, the
# others the separable stencil: one batch holds both routes
SIGMAS = [2.0, 2.0, 2.0, 2.0, 6.0, 6.0]


def _small_params():
    out = []
    for k, p in enumerate(SMALL):
        seed = 500 + k
        out.append(dict(p, seed=seed, sigma=SIGMAS[k], f=synth.make_image(seed, p["M"], "small"),
                        mask=synth.mask_random(seed + 7919, p["M"], 0.4).astype(np.uint8)))
    return out


def test_small_batch_matches_the_fp64_oracle(se2n):
    """Each item against the oracle lifting with the batch's orientation map."""
    params = _small_params()
    items = _items(se2n, params)
    _say("batch small: " + " ".join(f"{p['M']}/{p['N']}" for p in params))
    se2n.inpaint_batched(items)
    torch.cuda.synchronize()
    for p, it in zip(params, items):
        rmap = it.rmap_out.cpu().numpy()
        assert rmap.max() < p["N"]
        f32 = p["f"].astype(np.float32).astype(np.float64)
        ref, _ = O.inpaint(f32, p["mask"], p["N"], p["T"], p["beta"], p["n_steps"], sigma=p["sigma"],
                           scheme=p["scheme"], proj=p["proj"], rmap=rmap)
        rel = _rel(it.out.cpu().numpy(), ref)
        _say(f"  M={p['M']} N={p['N']} {p['scheme']} {p['proj']}: rel {rel:.2e}")
        assert rel < TOL32


def test_small_batch_orientation_matches_the_oracle_where_decided(se2n):
    params = _small_params()
    items = _items(se2n, params)
    se2n.inpaint_batched(items)
    torch.cuda.synchronize()
    for p, it in zip(params, items):
        want, tie = O.orient(p["f"].astype(np.float32).astype(np.float64), p["mask"], p["N"], p["sigma"])
        gx, gy = O.smoothed_gradient(p["f"].astype(np.float32).astype(np.float64), p["mask"], p["sigma"])
        mag = np.hypot(gx, gy)
        unc = 1e-5 * mag.max() / np.maximum(mag, 1e-300) * p["N"] / (2 * np.pi)
        decided = tie > np.maximum(1e-4, unc)
        got = it.rmap_out.cpu().numpy()
        assert decided.mean() > 0.9
        assert np.array_equal(got[decided], want[decided])


def _single(se2n, p, rmap):
    plan = se2n.Plan(p["M"], p["N"], torch.float32)
    f = torch.from_numpy(p["f"].astype(np.float32)).cuda()
    m = torch.from_numpy(p["mask"]).cuda()
    out, rm = plan.inpaint(f, m, p["T"], p["beta"], p["n_steps"], sigma=p["sigma"], scheme=p.get("scheme", "cn"),
                           proj=p.get("proj", "max"))
    torch.cuda.synchronize()
    res = out.cpu().numpy(), rm.cpu().numpy()
    plan.close()
    return res


@pytest.mark.parametrize("tune", [None, (0, 1, 1), (1, 0, 4), (4, 1, 2)])
def test_schedules_agree_with_the_single_image_path(se2n, tune):
    """Same items under several schedules (persistent or one workgroup per tile,
    both tile orders, 1-4 slice groups) against se2n_inpaint, per item."""
    params = _small_params() + [dict(p, proj="max") for p in synth.make_batch(3, seed0=1000, sides=(512, 1024, 192))]
    items = _items(se2n, params)
    if tune is not None:
        se2n.batch_set_tune(items, *tune)
        assert se2n.batch_get_tune(items) == dict(zip(("wg_per_cu", "order", "row_groups"), tune))
    _say(f"schedule {tune}")
    se2n.inpaint_batched(items)
    torch.cuda.synchronize()
    for p, it in zip(params, items):
        ref, rref = _single(se2n, p, None)
        got = it.rmap_out.cpu().numpy()
        assert np.array_equal(got, rref), p["M"]
        rel = _rel(it.out.cpu().numpy(), ref)
        assert rel < 1e-6, (p["M"], p["N"], rel)


def test_graph_replays_and_new_buffers(se2n):
    """Replays of the captured graph with eager work between them give the
    same bits; a call with other output buffers (same shapes) writes there."""
    params = _small_params()
    items = _items(se2n, params)
    ws = se2n.batch_workspace(items)
    se2n.inpaint_batched(items, ws)
    torch.cuda.synchronize()
    first = [it.out.clone() for it in items]
    for r in range(3):
        junk = torch.randn(1 << 20, device="cuda")
        (junk * 2).sum().item()
        for it in items:
            it.out.fill_(float("nan"))
        se2n.inpaint_batched(items, ws)
        torch.cuda.synchronize()
        for a, it in zip(first, items):
            assert torch.equal(a, it.out), r
    fresh = [se2n.BatchItem(it.f, it.mask, it.N, it.T, it.beta, it.n_steps, sigma=it.sigma, scheme=it.scheme,
                            proj=it.proj) for it in items]
    ws2 = se2n.batch_workspace(fresh)
    se2n.inpaint_batched(fresh, ws2)
    torch.cuda.synchronize()
    for a, it in zip(first, fresh):
        assert torch.equal(a, it.out)


def test_autotune_keeps_results_and_writes_the_table(se2n, tmp_path):
    params = _small_params()
    items = _items(se2n, params)
    path = str(tmp_path / "tune.jsonl")
    best, ms = se2n.batch_autotune(items, reps=1, table_path=path)
    _say(f"autotune best {best} {ms:.3f} ms")
    assert ms > 0 and best["wg_per_cu"] in (0, 1, 2, 4) and best["row_groups"] in (1, 2, 4)
    text = open(path).read()
    assert '"wg_per_cu": %d' % best["wg_per_cu"] in text
    assert se2n.batch_get_tune(items) == best
    se2n.inpaint_batched(items)
    torch.cuda.synchronize()
    for p, it in zip(params, items):
        ref, _ = O.inpaint(p["f"].astype(np.float32).astype(np.float64), p["mask"], p["N"], p["T"], p["beta"],
                           p["n_steps"], sigma=p["sigma"], scheme=p["scheme"], proj=p["proj"],
                           rmap=it.rmap_out.cpu().numpy())
        assert _rel(it.out.cpu().numpy(), ref) < TOL32
    se2n.batch_clear()


def test_profiled_batch_times_every_pass(se2n):
    params = _small_params()
    items = _items(se2n, params)
    se2n.batch_profile(True)
    se2n.inpaint_batched(items)
    stats = se2n.batch_profile_stats()
    se2n.batch_profile(False)
    for name in ("b_orient_row_fwd", "b_orient_col", "b_orient_row_inv", "b_lift_row_fwd", "b_col_fft_fwd",
                 "b_col_fft_inv", "b_row_inv_max", "b_row_inv_mean", "b_solve_N16"):
        assert name in stats and stats[name][1] > 0, name


def test_full_heterogeneous_batch_against_single_images(se2n):
    """The 64-image workload (sides 128..1024, N in {16, 24, 32}, T in [0.5, 4],
    tau = 0.01): every orientation map and output finite and in range; a
    sample of 8 items against the single-image path."""
    params = synth.make_batch(64, seed0=1000)
    items = _items(se2n, params)
    _say("full batch 64")
    se2n.inpaint_batched(items)
    torch.cuda.synchronize()
    for p, it in zip(params, items):
        assert int(it.rmap_out.max()) < p["N"]
        assert torch.isfinite(it.out).all()
    for k in (0, 7, 13, 21, 34, 42, 55, 63):
        p = params[k]
        ref, rref = _single(se2n, p, None)
        assert np.array_equal(items[k].rmap_out.cpu().numpy(), rref)
        rel = _rel(items[k].out.cpu().numpy(), ref)
        _say(f"  item {k} M={p['M']} N={p['N']}: rel vs single {rel:.2e}")
        assert rel < 1e-6
    se2n.batch_clear()


def test_poisoned_workspace_leaks_nothing(se2n):
    """Long diffusion times (many negligible classes, whose modes the solve
    sets to zero without reading them, or, at sides 512 and 1024, neither
    stores nor the inverse column pass reads) with the batch workspace filled
    with NaN bytes: every item still equals the single-image path."""
    large = synth.make_batch(2, seed0=1000, sides=(512, 1024))
    large = [dict(p, M=m, f=synth.make_image(p["seed"], m, "medium"),
                  mask=synth.mask_random(p["seed"] + 7919, m, p["rho"]).astype(np.uint8))
             for p, m in zip(large, (512, 1024))]
    params = [dict(p, T=4.0, n_steps=400) for p in _small_params() + large]
    items = _items(se2n, params)
    ws = se2n.batch_workspace(items)
    ws.fill_(255)
    se2n.inpaint_batched(items, ws)
    torch.cuda.synchronize()
    for p, it in zip(params, items):
        got = it.out.cpu().numpy()
        assert np.all(np.isfinite(got)), p["M"]
        ref, rref = _single(se2n, p, None)
        assert np.array_equal(it.rmap_out.cpu().numpy(), rref)
        assert _rel(got, ref) < 1e-6, (p["M"], p["N"])
    se2n.batch_clear()
