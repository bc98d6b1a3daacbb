"""Seeded synthetic inputs for the boundary-integral water-wave solve.

This package only *describes* boundaries: it samples closed-form curves and
their exact alpha-derivatives on uniform grids and draws seeded parameters.
It holds none of the method's arithmetic (no kernels, no layer potentials,
no solver), so both the FP64 CPU oracle and the GPU path may consume it.
"""
from .geometry import Geometry, fourier_surface, graph_bottom, ellipse, trig_potential
from .configs import (make_config, paper_problem, tiny_config, ragged_config, CONFIG_NAMES,
                      large_adjoint_draws)

__all__ = [
    "Geometry", "fourier_surface", "graph_bottom", "ellipse", "trig_potential",
    "make_config", "paper_problem", "tiny_config", "ragged_config", "CONFIG_NAMES",
]
