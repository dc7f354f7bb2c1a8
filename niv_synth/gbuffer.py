"""Synthetic G-buffers: primary rays from a pinhole camera cast into a scene.

Primary visibility is input preparation, not part of the method (the paper
excludes buffer generation from its timings, Sec. 5.1 and App. F).  The output
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


def primary_rays(cam: Camera):
    o = np.asarray(cam.pos, dtype=np.float64)
    fwd = np.asarray(cam.target, dtype=np.float64) - o
    fwd /= np.linalg.norm(fwd)
    right = np.cross(fwd, np.array([0.0, 1.0, 0.0]))
    right /= np.linalg.norm(right)
    up = np.cross(right, fwd)
    tx = np.tan(np.radians(cam.hfov_deg) * 0.5)
    ty = tx * cam.height / cam.width
    xs = (2.0 * (np.arange(cam.width) + 0.5) / cam.width - 1.0) * tx
    ys = (1.0 - 2.0 * (np.arange(cam.height) + 0.5) / cam.height) * ty
    d = (fwd[None, None, :] + xs[None, :, None] * right[None, None, :]
         + ys[:, None, None] * up[None, None, :])
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    return o, d.reshape(-1, 3)


def _safe_inv(d):
    d = np.where(d == 0.0, 1e-300, d)
    return 1.0 / d


def _cast_chunk(prims, o, d, tris=None):
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
    if tris is not None:
        best_t, best_n, best_alb, best_id, best_ax = _cast_tris(
            tris, o, d, best_t, best_n, best_alb, best_id, best_ax, len(prims))
    return best_t, best_n, best_alb, best_id, best_ax, best_c


def _cast_tris(tris, o, d, best_t, best_n, best_alb, best_id, best_ax, id_base):
    """Moller-Trumbore over a triangle soup, vectorised over rays; only rays
    that hit a mesh's bounding sphere are tested against its triangles."""
    for mi, mesh in enumerate(tris):
        v0, v1, v2 = mesh["v0"], mesh["v1"], mesh["v2"]
        c, rad = mesh["center"], mesh["radius"]
        oc = o - c
        b = d @ oc
        disc = b * b - (oc @ oc - rad * rad)
        cand = np.nonzero(disc > 0.0)[0]
        if cand.size == 0:
            continue
        dc = d[cand]
        e1 = v1 - v0
        e2 = v2 - v0
        tri_best = best_t[cand].copy()
        tri_n = np.zeros((cand.size, 3))
        tri_hit = np.zeros(cand.size, dtype=bool)
        fn = np.cross(e1, e2)
        fn /= np.linalg.norm(fn, axis=1, keepdims=True)
        step = 512
        for s0 in range(0, v0.shape[0], step):
            E1, E2, V0, FN = e1[s0:s0 + step], e2[s0:s0 + step], v0[s0:s0 + step], fn[s0:s0 + step]
            pv = np.cross(dc[:, None, :], E2[None, :, :])
            det = np.einsum("tk,rtk->rt", E1, pv)
            ok = np.abs(det) > 1e-12
            inv_det = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
            tv = (o - V0)[None, :, :]
            uu = np.einsum("rtk,rtk->rt", np.broadcast_to(tv, pv.shape), pv) * inv_det
            qv = np.cross(np.broadcast_to(tv, pv.shape), E1[None, :, :])
            vv = np.einsum("rk,rtk->rt", dc, qv) * inv_det
            tt = np.einsum("tk,rtk->rt", E2, qv) * inv_det
            valid = ok & (uu >= 0) & (vv >= 0) & (uu + vv <= 1) & (tt > 1e-6)
            tt = np.where(valid, tt, np.inf)
            j = np.argmin(tt, axis=1)
            tj = tt[np.arange(cand.size), j]
            better = tj < tri_best
            if better.any():
                tri_best = np.where(better, tj, tri_best)
                nsel = FN[j]
                nsel = np.where((np.sum(nsel * dc, axis=1) > 0)[:, None], -nsel, nsel)
                tri_n = np.where(better[:, None], nsel, tri_n)
                tri_hit |= better
        idx = cand[tri_hit]
        best_t[idx] = tri_best[tri_hit]
        best_n[idx] = tri_n[tri_hit]
        best_alb[idx] = np.asarray(mesh["albedo"], float)[None, :]
        best_id[idx] = id_base + mi
        best_ax[idx] = -1
    return best_t, best_n, best_alb, best_id, best_ax


def cast_gbuffer(prims, cam: Camera, tris=None, chunk: int = 1 << 18):
    """Returns dict of pos/nrm/albedo [H,W,3] float32, mask [H,W] uint8 and
    prim id [H,W] int32 (-1 = sky)."""
    o, d = primary_rays(cam)
    n = d.shape[0]
    pos = np.zeros((n, 3), np.float32)
    nrm = np.zeros((n, 3), np.float32)
    alb = np.zeros((n, 3), np.float32)
    pid = np.full(n, -1, np.int32)
    for s in range(0, n, chunk):
        t, nn, aa, ii, ax, cc = _cast_chunk(prims, o, d[s:s + chunk], tris)
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
