"""Seeded initial parameters of the gradient-corrector network.

Draws only: every weight matrix W[out][in] is iid normal with variance
1/in, every bias zero, packed as W1 (64x85), b1, W2 (64x64), b2, W3 (9x64),
b3 into one float64 vector of 10,249 entries. Both the reference network
and the GPU training take their starting point from here.
"""
import numpy as np

LAYERS = ((64, 85), (64, 64), (9, 64))


def mlp_initial_params(seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    parts = []
    for n_out, n_in in LAYERS:
        parts.append(rng.normal(0.0, 1.0 / np.sqrt(n_in), size=(n_out, n_in)).ravel())
        parts.append(np.zeros(n_out))
    return np.concatenate(parts)
