"""Seeded synthetic inputs (point clouds, flow conditions) for the q-LSKUM solver.

Holds geometry, connectivity and random streams only; none of the method's
arithmetic.  Both the HIP solver's tests and the CPU oracle draw their
inputs from here.
"""
from .naca import (Cloud, KIND_INTERIOR, KIND_OUTER, KIND_WALL, five_point_cloud,
                   naca_ocloud, naca_ocloud_cached, naca_thickness, radius_neighbours, random_cloud,
                   rotate_cloud)
from .conditions import glorot_weights, sample_conditions, warm_features
from .rng import splitmix64, uniform, uniform01

__all__ = ["Cloud", "KIND_INTERIOR", "KIND_WALL", "KIND_OUTER", "naca_ocloud", "naca_ocloud_cached",
           "naca_thickness", "five_point_cloud", "random_cloud", "rotate_cloud",
           "radius_neighbours", "splitmix64", "uniform", "uniform01",
           "sample_conditions", "warm_features", "glorot_weights"]
