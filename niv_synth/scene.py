"""Seeded synthetic scenes as flat primitive records.

A scene is a numpy structured array of 64-byte records (the binary layout
both the oracle and the GPU library read):

    int32 kind        0 = solid axis-aligned box, 1 = axis-aligned rectangle,
                      2 = disk
    int32 axis        rectangle: index of its normal axis
    float32 sign      rectangle: +1 / -1, the side its front face looks at
    float32 p[3]      box: min corner; rectangle and disk: centre
    float32 q[3]      box: max corner; rectangle: half extents along axes
                      (axis+1)%3 and (axis+2)%3 in q[0], q[1]; disk: unit normal
    float32 radius    disk radius
    float32 albedo[3] diffuse reflectance
    float32 emission[3] radiance leaving the front face

Box faces look outward, room walls look inward.  Any primitive with non-zero
emission is a light.
"""
import numpy as np

from .workloads import ROOM_LO, ROOM_HI

PRIM_BOX, PRIM_RECT, PRIM_DISK = 0, 1, 2

PRIM_DTYPE = np.dtype([
    ("kind", "<i4"), ("axis", "<i4"), ("sign", "<f4"), ("p", "<f4", (3,)),
    ("q", "<f4", (3,)), ("radius", "<f4"), ("albedo", "<f4", (3,)),
    ("emission", "<f4", (3,)),
])
assert PRIM_DTYPE.itemsize == 64


def _rec():
    return np.zeros(1, dtype=PRIM_DTYPE)[0]


def box_prim(lo, hi, albedo, emission=(0, 0, 0)):
    r = _rec()
    r["kind"] = PRIM_BOX
    r["p"], r["q"] = lo, hi
    r["albedo"], r["emission"] = albedo, emission
    return r


def rect_prim(axis, sign, center, half_u, half_v, albedo, emission=(0, 0, 0)):
    r = _rec()
    r["kind"], r["axis"], r["sign"] = PRIM_RECT, axis, sign
    r["p"] = center
    r["q"] = (half_u, half_v, 0.0)
    r["albedo"], r["emission"] = albedo, emission
    return r


def disk_prim(center, normal, radius, albedo=(0, 0, 0), emission=(0, 0, 0)):
    r = _rec()
    n = np.asarray(normal, dtype=np.float64)
    r["kind"] = PRIM_DISK
    r["p"], r["q"] = center, n / np.linalg.norm(n)
    r["radius"] = radius
    r["albedo"], r["emission"] = albedo, emission
    return r


def _uv_axes(axis):
    return (axis + 1) % 3, (axis + 2) % 3


def _wall_rects(lo, hi, axis, side, albedo, emission, opening=None):
    """Inward-looking wall of the box [lo, hi] on the `side` (0 = min, 1 = max)
    face of `axis`; `opening` = (umin, umax, vmin, vmax) cuts a hole."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    u, v = _uv_axes(axis)
    coord = lo[axis] if side == 0 else hi[axis]
    sign = 1.0 if side == 0 else -1.0
    pieces = []
    if opening is None:
        pieces.append((lo[u], hi[u], lo[v], hi[v]))
    else:
        u0, u1, v0, v1 = opening
        pieces += [(lo[u], u0, lo[v], hi[v]), (u1, hi[u], lo[v], hi[v]),
                   (u0, u1, lo[v], v0), (u0, u1, v1, hi[v])]
    out = []
    for (a0, a1, b0, b1) in pieces:
        c = np.zeros(3)
        c[axis] = coord
        c[u], c[v] = 0.5 * (a0 + a1), 0.5 * (b0 + b1)
        out.append(rect_prim(axis, sign, c, 0.5 * (a1 - a0), 0.5 * (b1 - b0),
                             albedo, emission))
    return out


def enclosure_prims(lo, hi, albedo, emission):
    """Closed box of six inward-looking walls, all with the same albedo and
    emission (used for the uniform-radiance and furnace closed forms)."""
    out = []
    for axis in range(3):
        for side in range(2):
            out += _wall_rects(lo, hi, axis, side, albedo, emission)
    return np.array(out, dtype=PRIM_DTYPE)


def room_prims(room, include_lights=True):
    return room["prims"] if include_lights else room["prims_no_lights"]


def scene_bounds(prims):
    """Axis-aligned bounds of every primitive (float64)."""
    lo = np.full(3, np.inf)
    hi = np.full(3, -np.inf)
    for r in prims:
        if r["kind"] == PRIM_BOX:
            a, b = np.asarray(r["p"], float), np.asarray(r["q"], float)
        elif r["kind"] == PRIM_RECT:
            u, v = _uv_axes(int(r["axis"]))
            a = np.asarray(r["p"], float).copy()
            b = a.copy()
            a[u] -= r["q"][0]
            b[u] += r["q"][0]
            a[v] -= r["q"][1]
            b[v] += r["q"][1]
        else:
            c = np.asarray(r["p"], float)
            a, b = c - r["radius"], c + r["radius"]
        lo, hi = np.minimum(lo, a), np.maximum(hi, b)
    return lo, hi


def make_room(seed: int, n_boxes: int = 32, n_lights: int = 2,
              light_radiance: float = 20.0, opening_scale: float = None,
              camera_pos=(5.0, 3.2, 0.4), clear_depth: float = 2.0):
    """A 10x4x10 m room with `n_boxes` seeded solid boxes (sizes U(0.3,1.5) m
    per axis, fully inside, overlaps allowed, none closer to the camera wall
    than `clear_depth` beyond the camera),
    per-surface albedo U(0.2,0.8)^3, a rectangular opening in the far wall
    (z = 10) and `n_lights` 1x1 m ceiling lights facing down.

    `opening_scale` s in (0, 1] sets the opening's half size (4.6 s by 1.9 s
    metres, centred on the wall); None leaves the wall closed."""
    rng = np.random.default_rng(seed)
    lo, hi = np.array(ROOM_LO), np.array(ROOM_HI)
    wall_albedo = rng.uniform(0.2, 0.8, size=(6, 3))
    boxes = []
    cam = np.asarray(camera_pos, float)
    while len(boxes) < n_boxes:
        size = rng.uniform(0.3, 1.5, size=3)
        blo = lo + rng.uniform(0.0, 1.0, size=3) * (hi - lo - size)
        bhi = blo + size
        alb = rng.uniform(0.2, 0.8, size=3)
        if blo[2] < cam[2] + clear_depth:
            continue
        boxes.append((blo, bhi, alb))
    light_xz = []
    for _ in range(n_lights):
        light_xz.append(rng.uniform(1.5, 8.5, size=2))
    prims = []
    opening = None
    if opening_scale is not None:
        s = float(opening_scale)
        opening = (5.0 - 4.6 * s, 5.0 + 4.6 * s, 2.0 - 1.9 * s, 2.0 + 1.9 * s)
    face = 0
    for axis in range(3):
        for side in range(2):
            op = opening if (axis == 2 and side == 1) else None
            prims += _wall_rects(lo, hi, axis, side, wall_albedo[face], (0, 0, 0), op)
            face += 1
    for (blo, bhi, alb) in boxes:
        prims.append(box_prim(blo, bhi, alb))
    prims_no_lights = np.array(prims, dtype=PRIM_DTYPE)
    for (x, z) in light_xz:
        prims.append(rect_prim(1, -1.0, (x, hi[1] - 1e-3, z), 0.5, 0.5, (0, 0, 0),
                               (light_radiance,) * 3))
    return {
        "seed": seed, "lo": lo, "hi": hi, "boxes": boxes, "opening": opening,
        "wall_albedo": wall_albedo, "camera_pos": cam,
        "prims": np.array(prims, dtype=PRIM_DTYPE),
        "prims_no_lights": prims_no_lights,
    }


def room_motion(room, light_dx: float = 3.0, box_dz: float = 1.5):
    """Motion vectors for a room that changes with a scene variable t in
    [0, 1] (Sec. 6): each ceiling light slides along x by light_dx towards the
    middle of the room, and the first box moves along z by box_dz (a moving
    occluder).  Returns [n_prims, 3] float32 (zero for static primitives)."""
    prims = room["prims"]
    motion = np.zeros((len(prims), 3), np.float32)
    mid = 0.5 * (room["lo"][0] + room["hi"][0])
    for k in range(len(prims)):
        if prims["emission"][k].max() > 0:
            motion[k, 0] = light_dx if prims["p"][k][0] < mid else -light_dx
    boxes = np.nonzero(prims["kind"] == 0)[0]
    if len(boxes):
        motion[boxes[0], 2] = box_dz
    return motion
