"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package holds no arithmetic of the method itself: it produces volumes
(dense float32 grids), initial network parameters, feature-mapping
frequencies and epoch permutations, i.e. the data and the random draws that
both sides take as inputs.  None of the paper's datasets is available, so the
procedural volumes here stand in for its scanned level sets, density clouds
and simulated sequences.
"""
from .volumes import (sphere_sdf, two_spheres_sdf, noise_sphere_sdf, fbm_cloud, water_frame,  # noqa: F401
                      saturated_fog, gradient_noise, fbm)
from .params import init_params, ffm_matrix, pe_matrix, epoch_permutation, net_shapes  # noqa: F401
