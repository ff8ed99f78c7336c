"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and bench.py.

This package holds grids, initial fields and parameter sets only. It contains none of
the solver's arithmetic (no metrics, fluxes, boundary conditions or time stepping), so
that the oracle and the GPU library stay independent of each other.
"""
from .grids import (cartesian_periodic_grid, skewed_periodic_grid, jet_grid,
                    jet_axial_map, jet_radial_map)
from .fields import (tgv_field, jet_field, uniform_field, conserved_from_primitive)
from .configs import (Params, BC_PERIODIC, BC_AXIS, BC_JET_INFLOW, BC_FARFIELD,
                      BC_EXIT, tgv_params, jet_params, box_params, make_case,
                      make_ensemble, ENSEMBLE_SHAPES)

__all__ = [
    "cartesian_periodic_grid", "skewed_periodic_grid", "jet_grid", "jet_axial_map",
    "jet_radial_map", "tgv_field", "jet_field", "uniform_field",
    "conserved_from_primitive", "Params", "BC_PERIODIC", "BC_AXIS", "BC_JET_INFLOW",
    "BC_FARFIELD", "BC_EXIT", "tgv_params", "jet_params", "box_params", "make_case",
    "make_ensemble", "ENSEMBLE_SHAPES",
]
