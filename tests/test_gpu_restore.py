"""GPU parity of static and dynamic restoration (se2n_restore) against the
FP64 oracle (Sec. "Heuristic complements", subsections "Static restoration
(SR)" and "Dynamic restoration (DR)"; Appendix A, Table 1).

Tolerances: FP64 plans 1e-10 and FP32 plans 2e-5 rel-L2 against the FP64
oracle, as for the plain path.  The downstream comparison runs on the GPU's
orientation map (the oracle lifts with it).  DR's growth decisions compare h
with a neighbourhood mean: in FP64 the decisions are identical (the test
checks that the oracle's closest decision is far above FP64 rounding); an
FP32 run may decide near-ties the other way, so the oracle is then run on
the GPU's decisions (join map), and every decision where the two rules
disagree must be a near-tie of the FP64 rule (|h - mean| below 1e-5 of the
largest |h|).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import restore_oracle as RO
from paper_1304_2062_amd import se2n, synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _inputs(M, seed, dtype, rho=0.5, stripes=(3, 13)):
    f = 0.1 + 0.9 * synth.make_image(seed, M, "medium")
    mask = (synth.mask_random(seed + 1, M, rho) | synth.mask_stripes(M, *stripes)).astype(np.uint8)
    if dtype == torch.float32:
        f = f.astype(np.float32).astype(np.float64)
    return f, mask


def _gpu_restore(f, mask, N, dtype, **kw):
    M = f.shape[0]
    plan = se2n.Plan(M, N, dtype)
    ft = torch.from_numpy(f).to(DEV, dtype)
    mt = torch.from_numpy(mask).to(DEV)
    out, rmap, join = plan.restore(ft, mt, **kw)
    torch.cuda.synchronize()
    res = out.double().cpu().numpy(), rmap.cpu().numpy(), join.cpu().numpy().astype(np.int32)
    plan.close()
    return res


@pytest.mark.parametrize("dynamic", [False, True])
@pytest.mark.parametrize("scheme,substeps,proj", [("cn", 1, "max"), ("cn", 3, "mean"), ("exact", 1, "max")])
def test_fp64_matches_oracle(dynamic, scheme, substeps, proj):
    print(f"restore FP64 64^2 N=16 dynamic={dynamic} {scheme} x{substeps} {proj}", flush=True)
    f, mask = _inputs(64, 21, torch.float64)
    kw = dict(T=0.4, beta=2.0, n_intervals=12, eps=0.5, dynamic=dynamic, substeps=substeps, scheme=scheme, proj=proj)
    got, rmap, join = _gpu_restore(f, mask, 16, torch.float64, **kw)
    want, _, wjoin, info = RO.restore(f, mask, 16, kw["T"], kw["beta"], kw["n_intervals"], kw["eps"],
                                      dynamic=dynamic, substeps=substeps, scheme=scheme, proj=proj, rmap=rmap)
    if dynamic:
        assert info["min_margin"] > 1e-9
        assert (wjoin > 0).any()
    assert np.array_equal(join, wjoin)
    assert _rel(got, want) < 1e-10


@pytest.mark.parametrize("dynamic", [False, True])
def test_fp32_matches_oracle(dynamic):
    """96^2 (a side with a factor 3 and a ragged last row block of the row
    passes' geometry) and N = 30 (4 does not divide N)."""
    print(f"restore FP32 96^2 N=30 dynamic={dynamic}", flush=True)
    f, mask = _inputs(96, 22, torch.float32)
    kw = dict(T=0.6, beta=5.0, n_intervals=20, eps=0.5, dynamic=dynamic)
    got, rmap, join = _gpu_restore(f, mask, 30, torch.float32, **kw)
    want, _, wjoin, info = RO.restore(f, mask, 30, 0.6, 5.0, 20, 0.5, dynamic=dynamic, rmap=rmap,
                                      join_in=join if dynamic else None)
    assert np.array_equal(join, wjoin)
    if dynamic:
        assert info["flip_max_margin"] <= 1e-5 * np.abs(want).max()
        print(f"  decisions taken the other way by FP32: {info['flips']}", flush=True)
    assert _rel(got, want) < 2e-5


@pytest.mark.parametrize("name", ["fig2_up", "fig3_down"])
def test_table1_rows_at_full_size(name):
    """A Table-1 reconstruction at its own size: 256^2, N = 30, stripe grid of
    the printed width and corruption, alpha -> beta, T -> T_p/2, the printed n
    and eps; FP32 against the FP64 oracle (SR for Fig. 2, DR for Fig. 3).
    The rows with 58-69 % corruption grow without bound under this
    discretisation (see test_heavy_corruption_row_before_it_diverges)."""
    c = synth.table1_case(name)
    print(f"restore Table 1 {name}: 256^2 N=30 n={c['n']} dynamic={c['dynamic']}", flush=True)
    f = c["f"].astype(np.float32).astype(np.float64)
    kw = dict(T=c["T"], beta=c["beta"], n_intervals=c["n"], eps=c["eps"], dynamic=c["dynamic"])
    got, rmap, join = _gpu_restore(f, c["mask"], c["N"], torch.float32, **kw)
    want, _, wjoin, info = RO.restore(f, c["mask"], c["N"], c["T"], c["beta"], c["n"], c["eps"],
                                      dynamic=c["dynamic"], rmap=rmap, join_in=join if c["dynamic"] else None)
    assert np.array_equal(join, wjoin)
    if c["dynamic"]:
        assert info["flip_max_margin"] <= 1e-5 * np.abs(want).max()
        assert (join > 0).sum() > 0.05 * c["mask"].sum()
    assert _rel(got, want) < 2e-5
    # the restoration changes the plain diffusion's result
    plain, _ = O.inpaint(f, c["mask"], c["N"], c["T"], c["beta"], c["n"], rmap=rmap)
    assert _rel(want, plain) > 1e-3


@pytest.mark.parametrize("dynamic", [False, True])
def test_heavy_corruption_row_before_it_diverges(dynamic):
    """figE4 (69 % corruption, alpha 0.4, n = 120): the mixing factor reaches
    ~20 at good pixels whose orientation maximum the first intervals drive
    close to zero, and from about the tenth interval the state grows without
    bound in the oracle and on the GPU alike.  Its first 8 intervals (same
    tau, T scaled by 8/120) are compared in FP64, where factors up to ~20
    are already applied."""
    c = synth.table1_case("figE4")
    k = 8
    T = c["T"] * k / c["n"]
    print(f"restore figE4 first {k} intervals FP64 dynamic={dynamic}", flush=True)
    got, rmap, join = _gpu_restore(c["f"], c["mask"], c["N"], torch.float64, T=T, beta=c["beta"], n_intervals=k,
                                   eps=c["eps"], dynamic=dynamic)
    want, _, wjoin, info = RO.restore(c["f"], c["mask"], c["N"], T, c["beta"], k, c["eps"], dynamic=dynamic,
                                      rmap=rmap)
    if dynamic:
        assert info["min_margin"] > 1e-9
    assert np.array_equal(join, wjoin)
    assert _rel(got, want) < 1e-10


def test_eps_zero_is_the_plain_path_on_gpu():
    """eps = 0: the mixes are the identity, so n single-step intervals equal the
    fused plain path with n steps (FP32, 512^2, a size with compiled kernels
    and column skipping)."""
    print("restore eps=0 vs inpaint, 512^2 N=32 FP32", flush=True)
    f, mask = _inputs(512, 23, torch.float32)
    ft = torch.from_numpy(f).to(DEV, torch.float32)
    mt = torch.from_numpy(mask).to(DEV)
    plan = se2n.Plan(512, 32, torch.float32)
    a, rmap, _ = plan.restore(ft, mt, 1.0, 1.0, 40, 0.0)
    b, _ = plan.inpaint(ft, mt, 1.0, 1.0, 40, rmap_in=rmap)
    torch.cuda.synchronize()
    assert _rel(a.double().cpu().numpy(), b.double().cpu().numpy()) < 2e-5
    plan.close()


def test_edge_cases():
    print("restore edge cases FP64 48^2 N=8", flush=True)
    M, N = 48, 8
    f, mask = _inputs(M, 24, torch.float64, stripes=(2, 9))
    # one interval: no mesh point to mix at -> the plain path with `substeps` steps
    got, rmap, join = _gpu_restore(f, mask, N, torch.float64, T=0.3, beta=1.0, n_intervals=1, eps=0.9, dynamic=True,
                                   substeps=7)
    want, _ = O.inpaint(f, mask, N, 0.3, 1.0, 7, rmap=rmap)
    assert _rel(got, want) < 1e-12
    assert np.array_equal(join, np.where(mask == 0, 0, -1))
    # nothing missing: DR has no bad pixel to grow into and equals SR
    none = np.zeros_like(mask)
    a, _, ja = _gpu_restore(f, none, N, torch.float64, T=0.3, beta=1.0, n_intervals=5, eps=1.0, dynamic=True)
    b, _, _ = _gpu_restore(f, none, N, torch.float64, T=0.3, beta=1.0, n_intervals=5, eps=1.0, dynamic=False)
    assert _rel(a, b) < 1e-14 and (ja == 0).all()
    # everything missing: the lift is zero and stays zero
    allm = np.ones_like(mask)
    z, _, jz = _gpu_restore(f, allm, N, torch.float64, T=0.3, beta=1.0, n_intervals=4, eps=0.5, dynamic=True)
    assert np.abs(z).max() == 0.0 and (jz == -1).all()


def test_bad_arguments_are_rejected():
    plan = se2n.Plan(64, 16, torch.float32)
    f = torch.zeros((64, 64), device=DEV)
    m = torch.zeros((64, 64), dtype=torch.uint8, device=DEV)
    for kw in (dict(eps=1.5), dict(eps=-0.1), dict(n_intervals=0), dict(n_intervals=40000), dict(substeps=0),
               dict(T=-1.0), dict(beta=-2.0)):
        args = dict(T=1.0, beta=1.0, n_intervals=4, eps=0.5)
        args.update(kw)
        with pytest.raises(se2n.Se2nError) as e:
            plan.restore(f, m, **args)
        assert e.value.code == -1
    plan.close()
