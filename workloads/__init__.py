"""Seeded synthetic problem data (geometry, masks, fields, initial states).

Holds no solver arithmetic; both the CPU oracle and the HIP path consume it.
"""
from .grids import (Box, runs_from_predicate, runs_from_mask, mask_from_runs, site_ijk,
                    site_coords, site_linear_index, complex_noise, normalise_input)
from . import configs

__all__ = ["Box", "runs_from_predicate", "runs_from_mask", "mask_from_runs", "site_ijk",
           "site_coords", "site_linear_index", "complex_noise", "normalise_input", "configs"]
