"""Seeded synthetic inputs of the repeated-pattern FETI hot path (problem statements only)."""
from .structures import (BASE_SEED, Pattern, Problem, config, grid_structure, mirror_row_heat, random_spd_ring,
                         ring_elast, ring_heat, small_elast, small_heat, uneven_three, mortar_row,
                         mortar_weights_1d)

__all__ = ["BASE_SEED", "Pattern", "Problem", "config", "grid_structure", "mirror_row_heat", "random_spd_ring",
           "ring_elast", "ring_heat",
           "small_elast", "small_heat", "uneven_three", "mortar_row", "mortar_weights_1d"]
