"""Seeded query points for workloads that are not G-buffers."""
import numpy as np


def uniform_unit_normals(rng, n: int) -> np.ndarray:
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v.astype(np.float32)


def unit_cube_queries(n: int, seed: int):
    """Positions uniform in [0,1]^3, normals uniform on the sphere (float32)."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, size=(n, 3)).astype(np.float32)
    nrm = uniform_unit_normals(rng, n)
    return pos, nrm
