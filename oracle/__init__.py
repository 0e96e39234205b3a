"""FP64 CPU oracle for the semi-discrete SE(2,N) hypoelliptic diffusion inpainting.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU library never
imports, links or calls it, and the two share no code: the only common module
is the seeded input generator, which holds none of the method's arithmetic.

The oracle is written from the paper (Boscain, Chertovskih, Gauthier, Remizov,
"Hypoelliptic diffusion and human vision: a semi-discrete new twist") and is
deliberately plain: full complex FFTs from numpy, an explicit per-mode
Crank-Nicolson loop in C (``cn_core.c``), and dense eigen-decompositions for the
exact propagator.  ``restore_oracle`` adds the paper's static and dynamic
restoration heuristics on top of that diffusion.
"""
from .se2n_oracle import (  # noqa: F401
    orientation_angles,
    symbol,
    cyclic_laplacian,
    mode_potential,
    generator_matrix,
    beta_from_alpha,
    smoothed_gradient,
    bin_angle,
    orient,
    lift,
    diffuse,
    diffuse_modes_cn,
    diffuse_modes_exact,
    project,
    inpaint,
    cyclic_solve,
)
