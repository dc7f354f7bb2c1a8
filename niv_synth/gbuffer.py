"""Synthetic G-buffers: primary rays from a pinhole camera cast into a scene.

Primary visibility is input preparation, not part of the method (the paper
excludes buffer generation from its timings, Sec. 5.2 and App. F).  The output
is what a rasteriser would hand the irradiance query: per pixel a position, a
surface normal, an albedo and a coverage mask (0 where the ray leaves the room
through the opening, i.e. sky).
"""
from dataclasses import dataclass

import numpy as np

from .scene import PRIM_BOX, PRIM_RECT, PRIM_DISK, make_room


@dataclass
class Camera:
    pos: tuple
    target: tuple
    hfov_deg: float
    width: int
    height: int


def default_camera(width: int, height: int) -> Camera:
    return Camera(pos=(5.0, 3.2, 0.4), target=(5.0, 2.6, 10.0), hfov_deg=80.0,
                  width=width, height=height)


def camera_basis(cam: Camera):
    """Origin, forward, right and up unit vectors and the half-extents of the
    image plane at unit distance."""
    o = np.asarray(cam.pos, dtype=np.float64)
    fwd = np.asarray(cam.target, dtype=np.float64) - o
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    tx = np.tan(np.radians(cam.hfov_deg) * 0.5)
    ty = tx * cam.height / cam.width
    return o, fwd, right, up, tx, ty


def primary_rays(cam: Camera):
    o, fwd, right, up, tx, ty = camera_basis(cam)
    xs = (2.0 * (np.arange(cam.width) + 0.5) / cam.width - 1.0) * tx
    ys = (1.0 - 2.0 * (np.arange(cam.height) + 0.5) / cam.height) * ty
    d = (fwd[None, None, :] + xs[None, :, None] * right[None, None, :]
         + ys[:, None, None] * up[None, None, :])
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    return o, d.reshape(-1, 3)


def _safe_inv(d):
    d = np.where(d == 0.0, 1e-300, d)
    return 1.0 / d


def _cast_chunk(prims, o, d):
    n = d.shape[0]
    best_t = np.full(n, np.inf)
    best_n = np.zeros((n, 3))
    best_alb = np.zeros((n, 3))
    best_id = np.full(n, -1, dtype=np.int64)
    best_ax = np.full(n, -1, dtype=np.int64)
    best_c = np.zeros(n)
    inv = _safe_inv(d)
    tmin = 1e-6
    for k, r in enumerate(prims):
        kind = int(r["kind"])
        if kind == PRIM_BOX:
            lo = np.asarray(r["p"], float)
            hi = np.asarray(r["q"], float)
            t1 = (lo[None, :] - o[None, :]) * inv
            t2 = (hi[None, :] - o[None, :]) * inv
            tn = np.minimum(t1, t2)
            tf = np.maximum(t1, t2)
            ax = np.argmax(tn, axis=1)
            tnear = tn[np.arange(n), ax]
            tfar = tf.min(axis=1)
            hit = (tnear <= tfar) & (tnear > tmin) & (tnear < best_t)
            if not hit.any():
                continue
            nn = np.zeros((n, 3))
            nn[np.arange(n), ax] = -np.sign(d[np.arange(n), ax])
            best_t = np.where(hit, tnear, best_t)
            best_ax = np.where(hit, ax, best_ax)
            best_c = np.where(hit, np.where(d[np.arange(n), ax] > 0, lo[ax], hi[ax]), best_c)
            best_n = np.where(hit[:, None], nn, best_n)
            best_alb = np.where(hit[:, None], np.asarray(r["albedo"], float)[None, :], best_alb)
            best_id = np.where(hit, k, best_id)
        elif kind == PRIM_RECT:
            a = int(r["axis"])
            u, v = (a + 1) % 3, (a + 2) % 3
            c = np.asarray(r["p"], float)
            t = (c[a] - o[a]) * inv[:, a]
            hu = o[u] + t * d[:, u]
            hv = o[v] + t * d[:, v]
            hit = ((t > tmin) & (t < best_t) & (np.abs(hu - c[u]) <= r["q"][0])
                   & (np.abs(hv - c[v]) <= r["q"][1]))
            if not hit.any():
                continue
            nn = np.zeros(3)
            nn[a] = r["sign"]
            best_t = np.where(hit, t, best_t)
            best_ax = np.where(hit, a, best_ax)
            best_c = np.where(hit, c[a], best_c)
            best_n = np.where(hit[:, None], nn[None, :], best_n)
            best_alb = np.where(hit[:, None], np.asarray(r["albedo"], float)[None, :], best_alb)
            best_id = np.where(hit, k, best_id)
        elif kind == PRIM_DISK:
            c = np.asarray(r["p"], float)
            nd = np.asarray(r["q"], float)
            den = d @ nd
            den = np.where(den == 0.0, 1e-300, den)
            t = ((c - o) @ nd) / den
            ph = o[None, :] + t[:, None] * d - c[None, :]
            hit = (t > tmin) & (t < best_t) & (np.sum(ph * ph, axis=1) <= r["radius"] ** 2)
            if not hit.any():
                continue
            best_t = np.where(hit, t, best_t)
            best_ax = np.where(hit, -1, best_ax)
            best_n = np.where(hit[:, None], nd[None, :], best_n)
            best_alb = np.where(hit[:, None], np.asarray(r["albedo"], float)[None, :], best_alb)
            best_id = np.where(hit, k, best_id)
    return best_t, best_n, best_alb, best_id, best_ax, best_c


def _mesh_hits(cam: Camera, d, meshes, max_pairs=1 << 22):
    """Nearest triangle hit per pixel for triangle soups: each triangle's
    projected bounding box gives candidate pixels, and every candidate is
    tested exactly against the pixel's primary ray (Moller-Trumbore).
    Returns t [n] (inf = no hit), normal [n,3] facing the camera, albedo
    [n,3], mesh index [n] (-1 = none)."""
    o, fwd, right, up, tx, ty = camera_basis(cam)
    W, H = cam.width, cam.height
    n = W * H
    best_t = np.full(n, np.inf)
    best_n = np.zeros((n, 3))
    best_alb = np.zeros((n, 3))
    best_id = np.full(n, -1, np.int64)
    for mi, mesh in enumerate(meshes):
        v = [np.asarray(mesh[k], float) for k in ("v0", "v1", "v2")]
        rel = [x - o[None, :] for x in v]
        z = np.stack([r @ fwd for r in rel], 1)
        front = (z > 1e-3).all(axis=1)
        px = np.stack([((r @ right) / (zz * tx) + 1.0) * W / 2 - 0.5
                       for r, zz in zip(rel, z.T)], 1)
        py = np.stack([(1.0 - (r @ up) / (zz * ty)) * H / 2 - 0.5
                       for r, zz in zip(rel, z.T)], 1)
        i0 = np.clip(np.floor(px.min(1)), 0, W - 1).astype(np.int64)
        i1 = np.clip(np.ceil(px.max(1)), 0, W - 1).astype(np.int64)
        j0 = np.clip(np.floor(py.min(1)), 0, H - 1).astype(np.int64)
        j1 = np.clip(np.ceil(py.max(1)), 0, H - 1).astype(np.int64)
        bw, bh = i1 - i0 + 1, j1 - j0 + 1
        cnt = np.where(front & (px.max(1) >= 0) & (px.min(1) <= W - 1) & (py.max(1) >= 0)
                       & (py.min(1) <= H - 1), bw * bh, 0)
        e1, e2 = v[1] - v[0], v[2] - v[0]
        fn = np.cross(e1, e2)
        fn /= np.linalg.norm(fn, axis=1, keepdims=True)
        alb = np.asarray(mesh["albedo"], float)
        tri = 0
        while tri < len(cnt):
            c = np.cumsum(cnt[tri:])
            stop = tri + max(1, int(np.searchsorted(c, max_pairs, side="right")))
            sel = np.arange(tri, stop)
            tri = stop
            cs = cnt[sel]
            tot = int(cs.sum())
            if tot == 0:
                continue
            ti = np.repeat(sel, cs)
            k = np.arange(tot) - np.repeat(np.cumsum(cs) - cs, cs)
            pix = (j0[ti] + k // bw[ti]) * W + (i0[ti] + k % bw[ti])
            dr = d[pix]
            pv = np.cross(dr, e2[ti])
            det = np.sum(e1[ti] * pv, 1)
            ok = np.abs(det) > 1e-14
            inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
            tv = o[None, :] - v[0][ti]
            uu = np.sum(tv * pv, 1) * inv
            qv = np.cross(tv, e1[ti])
            vv = np.sum(dr * qv, 1) * inv
            tt = np.sum(e2[ti] * qv, 1) * inv
            hit = ok & (uu >= 0) & (vv >= 0) & (uu + vv <= 1) & (tt > 1e-6)
            if not hit.any():
                continue
            pix, tt, ti, dr = pix[hit], tt[hit], ti[hit], dr[hit]
            order = np.lexsort((tt, pix))
            pix, tt, ti, dr = pix[order], tt[order], ti[order], dr[order]
            first = np.ones(len(pix), bool)
            first[1:] = pix[1:] != pix[:-1]
            pix, tt, ti, dr = pix[first], tt[first], ti[first], dr[first]
            better = tt < best_t[pix]
            pix, tt, ti, dr = pix[better], tt[better], ti[better], dr[better]
            nn = fn[ti]
            nn = np.where((np.sum(nn * dr, 1) > 0)[:, None], -nn, nn)
            best_t[pix] = tt
            best_n[pix] = nn
            best_alb[pix] = alb[None, :]
            best_id[pix] = mi
    return best_t, best_n, best_alb, best_id


def cast_gbuffer(prims, cam: Camera, tris=None, chunk: int = 1 << 18):
    """Returns dict of pos/nrm/albedo [H,W,3] float32, mask [H,W] uint8 and
    prim id [H,W] int32 (-1 = sky)."""
    o, d = primary_rays(cam)
    n = d.shape[0]
    pos = np.zeros((n, 3), np.float32)
    nrm = np.zeros((n, 3), np.float32)
    alb = np.zeros((n, 3), np.float32)
    pid = np.full(n, -1, np.int32)
    if tris:
        mt, mn, ma, mid = _mesh_hits(cam, d, tris)
    for s in range(0, n, chunk):
        t, nn, aa, ii, ax, cc = _cast_chunk(prims, o, d[s:s + chunk])
        if tris:
            sl = slice(s, s + chunk)
            m = mt[sl] < t
            t = np.where(m, mt[sl], t)
            nn = np.where(m[:, None], mn[sl], nn)
            aa = np.where(m[:, None], ma[sl], aa)
            ii = np.where(m, len(prims) + mid[sl], ii)
            ax = np.where(m, -1, ax)
        hit = np.isfinite(t)
        p = o[None, :] + np.where(hit, t, 0.0)[:, None] * d[s:s + chunk]
        # put hits on axis-aligned faces exactly on their plane
        rows = np.nonzero(ax >= 0)[0]
        p[rows, ax[rows]] = cc[rows]
        pos[s:s + chunk] = np.where(hit[:, None], p, 0.0)
        nrm[s:s + chunk] = np.where(hit[:, None], nn, 0.0)
        alb[s:s + chunk] = np.where(hit[:, None], aa, 0.0)
        pid[s:s + chunk] = ii
    H, W = cam.height, cam.width
    mask = (pid >= 0).astype(np.uint8)
    return {"pos": pos.reshape(H, W, 3), "nrm": nrm.reshape(H, W, 3),
            "albedo": alb.reshape(H, W, 3), "mask": mask.reshape(H, W),
            "prim": pid.reshape(H, W)}


def _sky_fraction(seed, n_boxes, scale, w=240, h=135):
    room = make_room(seed, n_boxes=n_boxes, n_lights=0, opening_scale=scale)
    g = cast_gbuffer(room["prims_no_lights"], default_camera(w, h))
    return 1.0 - g["mask"].mean()


def fit_opening(seed, n_boxes=32, target=0.05, iters=18):
    """Bisection on the opening size until the low-resolution sky fraction
    meets `target` (monotone in the size)."""
    lo, hi = 0.02, 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if _sky_fraction(seed, n_boxes, mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def make_room_gbuffer(seed: int, width: int, height: int, n_boxes: int = 32,
                      sky_target: float = 0.05, n_lights: int = 2, meshes=None):
    """Room + G-buffer for a workload; returns (room, gbuffer)."""
    scale = fit_opening(seed, n_boxes, sky_target)
    room = make_room(seed, n_boxes=n_boxes, n_lights=n_lights, opening_scale=scale)
    g = cast_gbuffer(room["prims_no_lights"], default_camera(width, height), tris=meshes)
    return room, g


def workload_meshes(w):
    """The dynamic meshes of a workload (displaced icospheres)."""
    from .mesh import displaced_sphere
    return [displaced_sphere(seed, centre) for seed, centre in w.meshes]


def mesh_triangles(meshes):
    """All triangles of the meshes as one float32 array [m, 3, 3]."""
    if not meshes:
        return np.zeros((0, 3, 3), np.float32)
    return np.concatenate([np.stack([m["v0"], m["v1"], m["v2"]], axis=1) for m in meshes]).astype(np.float32)


def make_workload_gbuffer(w, frame: int = 0, size=None):
    """Room + G-buffer of a workload's frame (or of `size` = (W, H) pixels of
    the same scene and camera), with its dynamic meshes."""
    meshes = workload_meshes(w) or None
    W, H = size if size is not None else w.frames[frame]
    return make_room_gbuffer(w.scene_seeds[frame], W, H, meshes=meshes)
