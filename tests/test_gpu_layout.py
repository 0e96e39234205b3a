"""The row-blocked layout of the inverse passes against the in-place one.

For FP32 plans of the compiled sides the inverse column pass writes its
result into a second spectrum in row blocks of 16, which the inverse row
pass reads contiguously; a plan created with SE2N_NO_ROW_BLOCKS keeps both
passes in place on one spectrum.  Only the addresses differ, so every result
must be bit-identical.  The oracle parity of the default (blocked) plans is
covered by the parity, edge and restoration tests.
"""
import numpy as np
import pytest
import torch

from paper_1304_2062_amd import se2n, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _plans(monkeypatch, M, N):
    blocked = se2n.Plan(M, N, torch.float32)
    monkeypatch.setenv("SE2N_NO_ROW_BLOCKS", "1")
    flat = se2n.Plan(M, N, torch.float32)
    monkeypatch.delenv("SE2N_NO_ROW_BLOCKS")
    spec = N * (M // 2 + 1) * M * 8
    # the blocked plan's workspace holds one more spectrum
    assert blocked.workspace_bytes - flat.workspace_bytes >= spec
    return blocked, flat


def _image(M, seed):
    f = torch.from_numpy(synth.make_image(seed, M, "medium")).to(DEV, torch.float32)
    mask = torch.from_numpy(synth.mask_random(seed + 1, M, 0.6)).to(DEV)
    return f, mask


@pytest.mark.parametrize("M,N,proj", [(2048, 32, "max"), (1024, 16, "mean"), (512, 31, "max")])
def test_inpaint_is_identical_in_both_layouts(monkeypatch, M, N, proj):
    print(f"layout: inpaint {M}^2 N={N} {proj}", flush=True)
    blocked, flat = _plans(monkeypatch, M, N)
    f, mask = _image(M, 3)
    a, ra = blocked.inpaint(f, mask, 4.0, 1.0, 400, proj=proj)
    b, rb = flat.inpaint(f, mask, 4.0, 1.0, 400, proj=proj)
    torch.cuda.synchronize()
    assert torch.equal(ra, rb)
    assert torch.isfinite(a).all()
    assert torch.equal(a, b), float((a - b).abs().max())
    blocked.close()
    flat.close()


def test_iterated_schedule_and_diffuse_are_identical_in_both_layouts(monkeypatch):
    M, N = 1024, 16
    print(f"layout: iterated inpaint and diffuse {M}^2 N={N}", flush=True)
    blocked, flat = _plans(monkeypatch, M, N)
    f, mask = _image(M, 5)
    for p in (blocked, flat):
        p.set_schedule("iterated")
    a, _ = blocked.inpaint(f, mask, 1.0, 2.0, 40)
    b, _ = flat.inpaint(f, mask, 1.0, 2.0, 40)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    for p in (blocked, flat):
        p.set_schedule("propagator")
    rng = np.random.default_rng(2)
    psi = torch.from_numpy(rng.standard_normal((N, M, M)).astype(np.float32)).to(DEV)
    pa = blocked.diffuse(psi.clone(), 0.7, 1.5, 30)
    pb = flat.diffuse(psi.clone(), 0.7, 1.5, 30)
    torch.cuda.synchronize()
    assert torch.equal(pa, pb)
    blocked.close()
    flat.close()


@pytest.mark.parametrize("dynamic", [False, True])
def test_restoration_is_identical_in_both_layouts(monkeypatch, dynamic):
    M, N = 512, 30
    print(f"layout: restoration {M}^2 N={N} dynamic={dynamic}", flush=True)
    blocked, flat = _plans(monkeypatch, M, N)
    f, _ = _image(M, 7)
    mask = torch.from_numpy(synth.mask_stripes(M, 6, 24)).to(DEV)
    kw = dict(T=2.0, beta=1.0, n_intervals=6, substeps=10, eps=0.5, dynamic=dynamic)
    a, ra, ja = blocked.restore(f, mask, **kw)
    b, rb, jb = flat.restore(f, mask, **kw)
    torch.cuda.synchronize()
    assert torch.equal(ra, rb)
    assert (ja is None and jb is None) or torch.equal(ja, jb)
    assert torch.equal(a, b)
    blocked.close()
    flat.close()
