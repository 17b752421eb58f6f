"""FP64 CPU oracle for Fast Local Regression.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check in
``__graft_entry__.py`` and the CPU-baseline leg of ``bench.py``, never by the
library. It shares no code with the HIP path.
"""
from . import brute, flr_adjoint, flr_lowres, flr_ref, net_adjoint
from .flr_ref import (apply_model, average_coefficients, central_moment_planes,
                      coefficient_planes, coefficients_from_planes, flr_reference,
                      flr_reference_block, moments_from_central_planes, solve_coefficients,
                      solve_normalised, window_count, window_moments, window_sum)

__all__ = [
    "brute", "flr_adjoint", "flr_lowres", "flr_ref", "net_adjoint", "apply_model", "average_coefficients", "central_moment_planes",
    "coefficient_planes", "coefficients_from_planes", "flr_reference", "flr_reference_block",
    "moments_from_central_planes", "solve_coefficients", "solve_normalised", "window_count",
    "window_moments", "window_sum",
]
