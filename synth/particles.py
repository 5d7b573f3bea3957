"""Seeded sphere placement.

Random sequential addition in a periodic box: candidate centres are drawn
uniformly and accepted when their minimum-image distance to every accepted
centre is at least ``min_dist``. A cell grid keeps each test local.
"""
import numpy as np


def random_spheres(n: int, shape, min_dist: float, seed: int,
                   max_tries: int = 10_000_000) -> np.ndarray:
    """Return (n, 3) float64 centres (x, y, z) in [0, L) per axis."""
    L = np.asarray(shape, np.float64)
    rng = np.random.default_rng(seed)
    ncell = np.maximum(1, np.floor(L / min_dist).astype(int))
    csize = L / ncell
    cells = {}
    out = np.empty((n, 3))
    placed = 0
    tries = 0
    d2min = min_dist * min_dist
    while placed < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"placed only {placed} of {n} spheres")
        p = rng.uniform(0.0, 1.0, 3) * L
        ci = np.floor(p / csize).astype(int) % ncell
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    key = tuple((ci + (dx, dy, dz)) % ncell)
                    for j in cells.get(key, ()):
                        d = p - out[j]
                        d -= L * np.round(d / L)
                        if d @ d < d2min:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            out[placed] = p
            cells.setdefault(tuple(ci), []).append(placed)
            placed += 1
    return out
