"""MI355X (gfx950) Gaussian Multipole (GMP) features: HIP kernels behind a
small C ABI (include/gmp.h), with a thin Python binding.

The compute path is libgmp.so only; importing this package does not load
it until a plan is created, and a missing library raises instead of falling
back to any CPU implementation.
"""
from .gmp import (GMPPlan, DeviceBatch, Neighbors, Workspace, build_neighbors, features,  # noqa: F401
                  features_backward, GMPFunction, feature_labels, profile, GMPError, rebuild_neighbors_nosync,
                  check_status, CapturedStep, build_reverse, feature_jacobian, pair_centres, pairs_by_centre)
from ._lib import LIB_PATH, EXPORTS, load  # noqa: F401
