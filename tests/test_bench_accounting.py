"""Host logic of bench.py's roofline accounting (no GPU): the solve's bytes as a
function of the negligible-class flags.  The members of the frequency classes
must tile the half spectrum exactly once, checked here by brute force."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def fold(k, M):
    H, M4 = M // 2, M // 4
    return k if k <= M4 else (H - k if k <= H else (k - H if k <= 3 * M4 else M - k))


@pytest.mark.parametrize("M", [16, 24, 48, 64, 72, 128])
def test_class_members_tile_the_half_spectrum(M):
    """Every (kx, ky) of the half spectrum belongs to exactly one class, and the
    member counts the accounting uses (2 or 1 columns, 4 or 2 rows) add up."""
    Q = M // 4 + 1
    count = np.zeros((Q, Q), dtype=np.int64)
    for kx in range(M // 2 + 1):
        for ky in range(M):
            count[fold(kx, M), fold(ky, M)] += 1
    nkx = np.full(Q, 2)
    nkx[M // 4] = 1
    nky = np.full(Q, 4)
    nky[0] = 2
    nky[M // 4] = 2
    assert np.array_equal(count, np.outer(nkx, nky))


@pytest.mark.parametrize("M,N", [(64, 8), (128, 16), (2048, 32)])
def test_solve_bytes_limits_and_monotonicity(M, N):
    Q = M // 4 + 1
    K = M // 2 + 1
    V = N * K * M * 8
    full = bench.algorithmic_bytes(M, N, 4)["solve"]
    assert bench.solve_bytes(M, N, np.zeros((Q, Q), np.uint8), 4) == full
    assert bench.solve_bytes(M, N, np.ones((Q, Q), np.uint8), 4) == V  # only the zeros are written
    rng = np.random.default_rng(M)
    flags = (rng.random((Q, Q)) < 0.5).astype(np.uint8)
    b = bench.solve_bytes(M, N, flags, 4)
    assert V < b < full
    # one more negligible class removes exactly its members' reads and its table entries
    i, j = np.argwhere(flags == 0)[0]
    more = flags.copy()
    more[i, j] = 1
    nk = (1 if i == M // 4 else 2) * (2 if j in (0, M // 4) else 4)
    h = N // 2
    assert b - bench.solve_bytes(M, N, more, 4) == N * nk * 8 + h * (h + 1) * 4


@pytest.mark.parametrize("M,N", [(64, 8), (2048, 32)])
def test_forward_column_bytes_limits(M, N):
    """No negligible class: the whole spectrum is read and written; all
    negligible: it is only read; one class more negligible removes exactly
    its members' writes."""
    Q = M // 4 + 1
    V = N * (M // 2 + 1) * M * 8
    assert bench.col_fwd_bytes(M, N, np.zeros((Q, Q), np.uint8)) == bench.algorithmic_bytes(M, N, 4)["col_fft_fwd"]
    assert bench.col_fwd_bytes(M, N, np.ones((Q, Q), np.uint8)) == V
    flags = np.zeros((Q, Q), np.uint8)
    flags[0, M // 4] = 1  # columns kx in {0, M/2}, rows ky in {M/4, 3M/4}
    assert bench.col_fwd_bytes(M, N, np.zeros((Q, Q), np.uint8)) - bench.col_fwd_bytes(M, N, flags) == N * 2 * 2 * 8


@pytest.mark.parametrize("M,N", [(64, 8), (2048, 32)])
def test_skipping_solve_and_inverse_bytes(M, N):
    """With the column passes leaving negligible modes out, the solve writes
    only live modes (nothing when every class is negligible; the full figure
    when none is), and the inverse pass reads only live modes."""
    Q = M // 4 + 1
    V = N * (M // 2 + 1) * M * 8
    none, every = np.zeros((Q, Q), np.uint8), np.ones((Q, Q), np.uint8)
    assert bench.solve_bytes(M, N, none, 4, True) == bench.solve_bytes(M, N, none, 4, False)
    assert bench.solve_bytes(M, N, every, 4, True) == 0
    assert bench.col_inv_bytes(M, N, none) == 2 * V
    assert bench.col_inv_bytes(M, N, every) == V
    rng = np.random.default_rng(M + N)
    flags = (rng.random((Q, Q)) < 0.5).astype(np.uint8)
    # skipping removes exactly the writes of the negligible modes
    neg_modes = N * (bench.live_modes(M, none) - bench.live_modes(M, flags)) * 8
    assert bench.solve_bytes(M, N, flags, 4, False) - bench.solve_bytes(M, N, flags, 4, True) == neg_modes


def test_measured_traffic_takes_the_workload_instance(tmp_path, monkeypatch):
    """The counter record lists every instance that matches a pass's name
    prefix (the warm-up plan's run once); the lookup takes the one the
    profiled run dispatched most, and nothing once the sources changed."""
    import json

    from paper_1304_2062_amd.profile_summary import kernel_source_hash

    rec = {"source_hash": kernel_source_hash(), "kernels": {
        "k_col_inv_paired<float,8,0,false,false>": {"fetch_bytes": 7.0e5, "write_bytes": 5.0e5, "dispatches": 1},
        "k_col_inv_paired<float,8,2048,true,true>": {"fetch_bytes": 3.24e8, "write_bytes": 5.37e8, "dispatches": 12},
    }}
    (tmp_path / "profiles").mkdir()
    path = tmp_path / "profiles" / "traffic_inpaint_2048_N32.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("col_fft_inv") == pytest.approx(8.61e8)
    assert bench.measured_traffic("solve") is None
    rec["source_hash"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("col_fft_inv") is None
