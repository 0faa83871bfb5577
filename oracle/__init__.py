"""FP64 CPU oracle for pMMF — test infrastructure only.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this package.  The
library under ``paper_1507_04396_amd`` never imports or calls it, and it imports nothing from the
library: the two share no code.
"""
from .pmmf_oracle import (  # noqa: F401
    Factorization,
    Rotation,
    mix64,
    chain_hash,
    mulhi,
    stage_schedule,
    cluster_sizes,
    boundary_cuts,
    cut_cluster_sizes,
    allocate_rotations,
    rotation_k2,
    rotation_k3,
    TIE,
    KAPPA,
    TINY32,
    U32,
    score_error,
    near_tie,
    partner_decision,
    rotation_decision,
    elimination_decision,
    factor,
    apply_U,
    apply_Ut,
    apply,
    apply_inverse,
    apply_inverse_sqrt,
    backward,
    rot3_generators,
    rot3_param_matrix,
    rot3_param_jacobian,
    with_params3,
    dense_U,
    dense_reconstruction,
)
