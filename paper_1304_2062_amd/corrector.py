"""Training and evaluation of the learned corrector (coarse-step diffusion ->
fine-step diffusion) with the library's own kernels.

The training pairs come from the method itself: a synthetic image is
orientation-mapped and lifted on the GPU, then diffused to T with n_coarse
and with n_fine Crank-Nicolson steps (FP32); the network learns the
difference.  Evaluation compares, on larger held-out images, the coarse
result, the corrected result and plain solves with several step counts
against the fine-step FP64 solve.

    python -m paper_1304_2062_amd.corrector train --out paper_1304_2062_amd/corrector_N32.npz
    python -m paper_1304_2062_amd.corrector eval --weights paper_1304_2062_amd/corrector_N32.npz

Defaults: 2000 training images of 256^2, N = 32, beta = 1, T = 2, 25 vs 200
steps (tau = 0.08 vs 0.01), 60% random pixel loss; evaluation on 16 images of
1024^2 with the same parameters.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_1304_2062_amd import synth  # noqa: E402

TRAIN_SEED0 = 10000
EVAL_SEED0 = 20000
LOSS_RATE = 0.6


def _image(args):
    seed, M = args
    f = synth.make_image(seed, M, "medium").astype(np.float32)
    m = synth.mask_random(seed + 7919, M, LOSS_RATE).astype(np.uint8)
    return f, m


def images(seeds, M, workers: int | None = None):
    """Seeded images and masks, generated on the host in parallel."""
    workers = workers or min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(_image, [(s, M) for s in seeds], chunksize=8))


def pairs(plan, imgs, T, beta, n_coarse, n_fine):
    """(coarse, fine) real-space volumes [count][N][M][M] on the GPU."""
    import torch
    M, N = plan.M, plan.N
    C = torch.empty((len(imgs), N, M, M), dtype=torch.float32, device="cuda")
    F = torch.empty_like(C)
    for i, (f, m) in enumerate(imgs):
        ft = torch.from_numpy(f).cuda()
        mt = torch.from_numpy(m).cuda()
        psi = plan.lift(ft, mt, plan.orient(ft, mt))
        C[i].copy_(psi)
        plan.diffuse(C[i], T, beta, n_coarse)
        plan.diffuse(psi, T, beta, n_fine)
        F[i].copy_(psi)
    return C, F


def train(N=32, M=256, count=2000, T=2.0, beta=1.0, n_coarse=25, n_fine=200, batch=16, epochs=40, lr=3e-4,
          seed=0, holdout=64, log=print):
    """Train a corrector on `count` pairs; returns (network, history)."""
    import torch

    from paper_1304_2062_amd import se2n
    t0 = time.time()
    imgs = images(range(TRAIN_SEED0, TRAIN_SEED0 + count + holdout), M)
    plan = se2n.Plan(M, N, torch.float32)
    C, F = pairs(plan, imgs, T, beta, n_coarse, n_fine)
    torch.cuda.synchronize()
    Ch, Fh = C[count:].contiguous(), F[count:].contiguous()
    C, F = C[:count], F[:count]
    log(f"[corrector] {count}+{holdout} pairs of {M}^2 N={N} in {time.time() - t0:.1f} s")
    net = se2n.Corrector(N, seed=seed)

    def holdout_rel():
        out = torch.empty_like(Ch)
        for k in range(0, holdout, batch):
            net.forward(Ch[k:k + batch].contiguous(), out[k:k + batch])
        return float(torch.linalg.norm(out - Fh) / torch.linalg.norm(Fh))

    base = float(torch.linalg.norm(Ch - Fh) / torch.linalg.norm(Fh))
    gen = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = count // batch
    total = epochs * steps_per_epoch
    history = []
    step = 0
    t1 = time.time()
    loss = torch.zeros(1, device="cuda")
    for ep in range(epochs):
        perm = torch.randperm(count, generator=gen)
        for k in range(steps_per_epoch):
            # cosine decay of the step size to 5% of lr
            rate = lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * step / total)))
            idx = perm[k * batch:(k + 1) * batch].cuda()
            net.train_step(C.index_select(0, idx), F.index_select(0, idx), rate, loss)
            step += 1
        rel = holdout_rel()
        history.append(dict(epoch=ep + 1, loss=float(loss.item()), holdout_rel=rel, coarse_rel=base))
        log(f"[corrector] epoch {ep + 1}/{epochs} loss {loss.item():.3e} holdout rel-L2 {rel:.3e} "
            f"({rel / base:.3f} of coarse {base:.3e}) {time.time() - t1:.1f} s")
    plan.close()
    return net, history


def evaluate(net, M=1024, count=16, T=2.0, beta=1.0, n_coarse=25, n_fine=200, plain_steps=(25, 50, 100, 200),
             log=print):
    """Held-out comparison at side M against the fine-step FP64 solve."""
    import torch

    from paper_1304_2062_amd import se2n
    N = net.N
    p32 = se2n.Plan(M, N, torch.float32)
    p64 = se2n.Plan(M, N, torch.float64)
    imgs = images(range(EVAL_SEED0, EVAL_SEED0 + count), M)
    acc = {"coarse": [], "corrected": []}
    acc.update({f"plain_{n}": [] for n in plain_steps})
    img_acc = {k: [] for k in acc}
    cws = net.workspace(M, 1, False)

    def rel(a, b):
        return float(torch.linalg.norm(a.double() - b) / torch.linalg.norm(b))

    for i, (f, m) in enumerate(imgs):
        ft = torch.from_numpy(f).cuda()
        mt = torch.from_numpy(m).cuda()
        rmap = p32.orient(ft, mt)
        lifted = p32.lift(ft, mt, rmap)
        ref = p64.diffuse(lifted.double(), T, beta, n_fine)
        ref_img = p64.project(ref)
        vol = p32.diffuse(lifted.clone(), T, beta, n_coarse)
        acc["coarse"].append(rel(vol, ref))
        img_acc["coarse"].append(rel(p32.project(vol), ref_img))
        net.forward(vol, vol)
        acc["corrected"].append(rel(vol, ref))
        img_acc["corrected"].append(rel(p32.project(vol), ref_img))
        for n in plain_steps:
            v = p32.diffuse(lifted.clone(), T, beta, n)
            acc[f"plain_{n}"].append(rel(v, ref))
            img_acc[f"plain_{n}"].append(rel(p32.project(v), ref_img))
        log(f"[corrector] eval image {i}: coarse {acc['coarse'][-1]:.3e} corrected {acc['corrected'][-1]:.3e}")
    res = {k: float(np.mean(v)) for k, v in acc.items()}
    res_img = {k: float(np.mean(v)) for k, v in img_acc.items()}
    # the network's licence in this regime: its measured error against the
    # fine-step FP64 solve (se2n_inpaint_corrected falls back above the bar)
    net.set_validation(M, T, beta, n_coarse, n_fine, max(acc["corrected"]))

    # timings (warm, per image): plain fused inpaint vs coarse + corrector
    f, m = imgs[0]
    ft, mt = torch.from_numpy(f).cuda(), torch.from_numpy(m).cuda()
    cws_all = torch.empty(int(se2n._lib.se2n_corrected_workspace_bytes(p32._h, net._h)), dtype=torch.uint8,
                          device="cuda")

    def timed(fn, k=10):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(k):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / k * 1e3

    times = {
        "plain_fused_ms": {n: timed(lambda n=n: p32.inpaint(ft, mt, T, beta, n)) for n in (n_coarse, n_fine)},
        # the network path itself (a bar it always meets, so no fallback) ...
        "corrected_ms": timed(lambda: se2n.inpaint_corrected(p32, net, ft, mt, T, beta, n_coarse, n_fine,
                                                             max_rel_l2=float("inf"), workspace=cws_all)),
        # ... and what the call does at the 1e-3 bar (the fine-step fallback where the network misses it)
        "corrected_at_bar_ms": timed(lambda: se2n.inpaint_corrected(p32, net, ft, mt, T, beta, n_coarse, n_fine,
                                                                    max_rel_l2=1e-3, workspace=cws_all)),
    }
    times["fallback_at_bar"] = se2n.inpaint_corrected(p32, net, ft, mt, T, beta, n_coarse, n_fine, max_rel_l2=1e-3,
                                                      workspace=cws_all)[2]
    # cold propagator computation for each step count (the only cost that depends on n)
    cold = {}
    for n in (n_coarse, n_fine):
        fresh = se2n.Plan(M, N, torch.float32)
        fresh.profile(True)
        fresh.precompute(T, beta, n)
        cold[n] = fresh.profile_stats().get("precompute", (0, 0.0))[1]
        fresh.close()
    times["precompute_ms"] = cold
    p32.close()
    p64.close()
    del cws
    return dict(M=M, N=N, images=count, T=T, beta=beta, n_coarse=n_coarse, n_fine=n_fine, volume_rel_l2=res,
                image_rel_l2=res_img, times=times)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("train")
    a.add_argument("--out", required=True)
    a.add_argument("--count", type=int, default=2000)
    a.add_argument("--M", type=int, default=256)
    a.add_argument("--epochs", type=int, default=40)
    a.add_argument("--batch", type=int, default=16)
    a.add_argument("--lr", type=float, default=3e-4)
    a.add_argument("--seed", type=int, default=0)
    a.add_argument("--history")
    b = sub.add_parser("eval")
    b.add_argument("--weights", required=True)
    b.add_argument("--M", type=int, default=1024)
    b.add_argument("--count", type=int, default=16)
    b.add_argument("--json")
    b.add_argument("--record", help="write the weights with this evaluation's validation record here")
    args = ap.parse_args(argv)
    import torch  # noqa: F401

    from paper_1304_2062_amd import se2n
    if args.cmd == "train":
        net, hist = train(M=args.M, count=args.count, epochs=args.epochs, batch=args.batch, lr=args.lr,
                          seed=args.seed)
        net.save(args.out)
        if args.history:
            with open(args.history, "w") as fh:
                json.dump(hist, fh, indent=1)
        return 0
    with np.load(args.weights, allow_pickle=False) as z:
        N = int(z["N"])
    net = se2n.Corrector(N)
    net.load(args.weights)
    res = evaluate(net, M=args.M, count=args.count)
    if args.record:
        net.save(args.record)
    print(json.dumps(res))
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(res, fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
