"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package draws random numbers and lays out initial conditions. It
holds none of the lattice Boltzmann arithmetic: no equilibria, no
collision, no boundary scheme. Both sides of every parity check take
their inputs from here, so a test never feeds one side's output to the
other.

All randomness is numpy ``default_rng(seed)`` (PCG64).
"""
from .fields import (HitSpectrum, hit_spectrum, hit_field, hit_field_at,
                     pipe_initial_velocity, random_density, random_velocity)
from .particles import random_spheres
from .weights import mlp_initial_params

__all__ = ["HitSpectrum", "hit_spectrum", "hit_field", "hit_field_at",
           "pipe_initial_velocity", "random_density", "random_velocity", "random_spheres",
           "mlp_initial_params"]
