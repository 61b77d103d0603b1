"""Seeded synthetic least-squares problems (input generators only).

This module builds inputs; it holds none of the solver's arithmetic.  Both the
CPU oracle tests and the GPU path take their inputs from here.
"""
from .problems import (CONFIGS, Problem, draw_batch_shapes, make_batch, make_problem, pack_batch,
                       sigma_geometric, sigma_half_ones_loguniform)

__all__ = ["CONFIGS", "Problem", "draw_batch_shapes", "make_batch", "make_problem", "pack_batch",
           "sigma_geometric", "sigma_half_ones_loguniform"]
