"""Write the FP64 oracle's outputs of the 2048^2, N = 32, T = 4, 400-step
inpaint at beta in {0.25, 1, 4}, sampled at fixed pixels, to
``c3_oracle_samples.npz`` next to this file.

Calls only the oracle and the input generator.  The image is rounded to FP32
first (the GPU's FP32 runs read that image), and the orientation map is the
oracle's own FP64 map; the GPU test passes the same map (recomputed by the
oracle, checked against the stored SHA-256) as rmap_in, so both sides lift
identically.

    python tests/golden/make_c3_samples.py      (about 2-3 minutes per beta on 8 cores)
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_1304_2062_amd import synth  # noqa: E402

BETAS = (0.25, 1.0, 4.0)
SAMPLES = 16384
SAMPLE_SEED = 2048


def main() -> None:
    case = synth.make_case("large")
    M, N, T, n, sigma = case["M"], case["N"], case["T"], case["n_steps"], case["sigma"]
    f = case["f"].astype(np.float32).astype(np.float64)
    mask = case["mask"]
    rmap, tie = O.orient(f, mask, N, sigma)
    rng = np.random.Generator(np.random.PCG64(SAMPLE_SEED))
    idx = np.sort(rng.choice(M * M, size=SAMPLES, replace=False)).astype(np.int64)
    rec = {"idx": idx, "betas": np.array(BETAS), "rmap_sha256": np.array(hashlib.sha256(rmap.tobytes()).hexdigest()),
           "rmap_min_tie": np.array(float(tie.min())), "M": np.int64(M), "N": np.int64(N), "T": np.float64(T),
           "n_steps": np.int64(n), "sigma": np.float64(sigma), "seed": np.int64(case["seed"])}
    for beta in BETAS:
        t0 = time.time()
        out, _ = O.inpaint(f, mask, N, T, beta, n, sigma=sigma, rmap=rmap)
        key = f"beta_{beta:g}"
        rec[key + "_samples"] = out.reshape(-1)[idx]
        rec[key + "_norm"] = np.float64(np.linalg.norm(out))
        rec[key + "_max"] = np.float64(np.abs(out).max())
        print(f"beta={beta}: {time.time() - t0:.1f} s, |out| = {rec[key + '_norm']:.6e}", flush=True)
    np.savez(os.path.join(HERE, "c3_oracle_samples.npz"), **rec)


if __name__ == "__main__":
    main()
