"""Seeded synthetic inputs for the THC-oo-K exchange build.

This package builds cells, Gaussian Bloch basis functions on the real-space
grid and orthonormal occupied orbitals. It is input preparation only: it
holds none of the exchange method's arithmetic (no pair densities, no fit,
no Coulomb kernel, no k-convolution). Both the FP64 oracle and the HIP path
take their inputs from here.
"""

from .cells import (  # noqa: F401
    Cell,
    Shell,
    make_config,
    make_batch_cells,
    make_random_cell,
    make_ring_cell,
    make_ring_series_cell,
    make_config5_coarse,
    ao_on_grid,
    ao_at_points,
    ao_overlap,
    orbital_coeffs,
    orbitals_on_grid,
    point_coords,
    grid_coords,
    smooth_grid_size,
)
