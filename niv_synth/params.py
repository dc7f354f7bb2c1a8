"""Seeded parameter values for a model whose layout the caller states.

The caller passes the number of grid values and the list of weight-matrix
shapes (out, in); this module only draws numbers.  Grid latents are uniform
in [lo, hi]; weights are Xavier-uniform (Glorot & Bengio 2010), i.e. uniform
in [-a, a] with a = sqrt(6 / (fan_in + fan_out)).
"""
import numpy as np


def xavier_bound(fan_out: int, fan_in: int) -> float:
    return float(np.sqrt(6.0 / (fan_in + fan_out)))


def make_params(n_grid_values: int, mat_shapes, seed: int, grid_lo: float,
                grid_hi: float) -> np.ndarray:
    """Flat float32 vector: [grid values][W_0 row-major][W_1]...[W_H]."""
    rng = np.random.default_rng(seed)
    parts = [rng.uniform(grid_lo, grid_hi, size=int(n_grid_values))]
    for (n_out, n_in) in mat_shapes:
        a = xavier_bound(n_out, n_in)
        parts.append(rng.uniform(-a, a, size=int(n_out) * int(n_in)))
    return np.concatenate(parts).astype(np.float32)
