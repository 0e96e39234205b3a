"""The FP64 propagator build on the matrix cores (blocks of 9..16, even
N = 18..32: column-wise cyclic tridiagonal inverse, binary powering on
v_mfma_f64_16x16x4) against the scalar build (Gauss-Jordan, LDS products)
and against the oracle's per-mode solutions."""
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1304_2062_amd import se2n, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _diffuse(psi, M, N, T, beta, n, scheme, scalar, monkeypatch):
    if scalar:
        monkeypatch.setenv("SE2N_SCALAR_PRECOMPUTE", "1")
    else:
        monkeypatch.delenv("SE2N_SCALAR_PRECOMPUTE", raising=False)
    plan = se2n.Plan(M, N, torch.float64)
    t = torch.from_numpy(psi).to(DEV)
    plan.diffuse(t, T, beta, n, scheme)
    torch.cuda.synchronize()
    flags = plan.propagator_flags(T, beta, n, scheme)
    plan.close()
    monkeypatch.delenv("SE2N_SCALAR_PRECOMPUTE", raising=False)
    return t.cpu().numpy(), flags


@pytest.mark.parametrize("N", [4, 16, 18, 24, 30, 32])
@pytest.mark.parametrize("scheme,T,n", [("cn", 0.6, 1), ("cn", 0.8, 37), ("cn", 2.0, 400), ("exact", 0.7, 1)])
def test_matrix_core_build_matches_scalar_build_and_oracle(N, scheme, T, n, monkeypatch):
    print(f"precompute N={N} {scheme} T={T} n={n}", flush=True)
    M, beta = 48, 1.7
    rng = np.random.default_rng(N)
    psi = rng.normal(size=(N, M, M))
    a, fa = _diffuse(psi, M, N, T, beta, n, scheme, False, monkeypatch)
    b, fb = _diffuse(psi, M, N, T, beta, n, scheme, True, monkeypatch)
    assert _rel(a, b) < 1e-12
    assert np.array_equal(fa, fb)
    want = O.diffuse(psi, T, beta, n, scheme)
    assert _rel(a, want) < 1e-10


def test_flags_agree_at_2048(monkeypatch):
    """The negligible-class flags of the timed configuration (2048^2, N = 32,
    T = 4, 400 steps) from both builds; FP32 tables."""
    M, N, T, n = 2048, 32, 4.0, 400
    flags = []
    for scalar in (False, True):
        if scalar:
            monkeypatch.setenv("SE2N_SCALAR_PRECOMPUTE", "1")
        plan = se2n.Plan(M, N, torch.float32)
        flags.append(plan.propagator_flags(T, 1.0, n))
        plan.close()
        monkeypatch.delenv("SE2N_SCALAR_PRECOMPUTE", raising=False)
    diff = int((flags[0] != flags[1]).sum())
    print(f"  negligible {flags[0].mean():.4f}, differing flags {diff}", flush=True)
    assert diff <= 0.001 * flags[0].size
