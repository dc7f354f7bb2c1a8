"""Dynamic objects of the 4K scene-variable workload: icospheres subdivided
five times (20,480 triangles) with seeded radial displacement, standing in
for the moving meshes the paper places inside its volumes (Sec. 6)."""
import numpy as np


def icosphere(subdiv: int):
    """Unit icosphere: (vertices [V,3], faces [F,3] int), 20 * 4^subdiv faces."""
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0), (0, -1, t), (0, 1, t), (0, -1, -t),
         (0, 1, -t), (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.asarray(p, float) / np.linalg.norm(p) for p in v]
    faces = np.asarray(f, np.int64)
    for _ in range(subdiv):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces.tolist():
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = np.asarray(nf, np.int64)
    return np.asarray(verts), faces


def displaced_sphere(seed: int, center, radius=0.6, subdiv=5, lo=0.8, hi=1.2, albedo=None):
    """Triangle soup of an icosphere whose vertices are pushed along their
    direction by a seeded factor U(lo, hi)."""
    rng = np.random.default_rng(seed)
    v, f = icosphere(subdiv)
    v = v * (radius * rng.uniform(lo, hi, size=(len(v), 1)))
    v = v + np.asarray(center, float)[None, :]
    alb = rng.uniform(0.2, 0.8, size=3) if albedo is None else np.asarray(albedo, float)
    return {"v0": v[f[:, 0]], "v1": v[f[:, 1]], "v2": v[f[:, 2]],
            "center": np.asarray(center, float), "radius": radius * hi, "albedo": alb}
