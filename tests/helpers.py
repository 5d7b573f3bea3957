"""Shared helpers for the parity tests (comparison metrics, GPU lattice
construction). Holds no method arithmetic."""
import numpy as np


def rel_l2(a, b, mask=None):
    """||a - b|| / ||b|| over the masked entries (mask over the trailing
    spatial axes)."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    if mask is not None:
        a = a[..., mask]
        b = b[..., mask]
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu_config(**kw):
    from paper_1906_05448_amd import lbm
    return lbm.Config(**kw)


def gpu_lattice(cfg):
    from paper_1906_05448_amd import lbm
    return lbm.Lattice(cfg)
