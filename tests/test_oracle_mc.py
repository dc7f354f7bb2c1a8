"""Pins of the oracle's random numbers, Monte Carlo irradiance estimator and
training-point sampler: a library generator, closed forms of Eq. 1 and
statistical identities.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O
from niv_synth import enclosure_prims, disk_prim, rect_prim, make_room, box_prim, PRIM_DTYPE


def _rand_dirs(rng, n):
    v = rng.standard_normal((n, 3))
    return (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)


# ------------------------------------------------------------ Philox
@pytest.mark.parametrize("ctr,key", [([0, 0, 0, 0], [0, 0]), ([5, 7, 0, 0], [123, 0]),
                                     ([2**64 - 2, 2**63, 17, 1], [2**64 - 1, 99]),
                                     ([12345, 67, 3, 0], [0xDEADBEEF, 0])])
def test_philox_matches_numpy(ctr, key):
    """numpy's Philox bit generator is Philox4x64-10; it increments the
    counter before each block."""
    bg = np.random.Philox(counter=np.array(ctr, dtype=np.uint64),
                          key=np.array(key, dtype=np.uint64))
    want = [int(x) for x in bg.random_raw(4)]
    c1 = list(ctr)
    c1[0] = (c1[0] + 1) % 2**64
    if c1[0] == 0:
        c1[1] = (c1[1] + 1) % 2**64
    assert O.philox4x64(c1, key) == want


def test_uniform_mapping():
    seed, a, b, stream = 77, 1234, 56, 0
    blk = O.philox4x64([a, b, 0, stream], [seed, 0]) + O.philox4x64([a, b, 1, stream], [seed, 0])
    for dim in range(16):
        w = blk[dim // 2]
        u32 = (w >> 32) if dim & 1 else (w & 0xFFFFFFFF)
        assert O.uniform(seed, a, b, stream, dim) == (u32 >> 8) * 2.0 ** -24


# ------------------------------------------------------------ closed forms of Eq. 1
def test_uniform_enclosure_gives_pi_L():
    """Inside a closed box whose walls all emit L (albedo 0), every direction
    sees radiance L, so E = int L cos = pi L with zero variance."""
    L = np.array([0.7, 1.3, 2.1])
    prims = enclosure_prims((0, 0, 0), (2, 1, 3), albedo=(0, 0, 0), emission=L)
    rng = np.random.default_rng(0)
    x = rng.uniform([0.1, 0.1, 0.1], [1.9, 0.9, 2.9], size=(40, 3)).astype(np.float32)
    n = _rand_dirs(rng, 40)
    E, var, bf, valid = O.mc_irradiance(prims, x, n, 64, 3, O.MC_INCLUDE_DIRECT, 5)
    L32 = L.astype(np.float32).astype(np.float64)
    np.testing.assert_allclose(E, np.tile(math.pi * L32, (40, 1)), rtol=1e-12)
    assert np.abs(var).max() < 1e-20
    assert (bf == 0).all() and valid.all()


@pytest.mark.parametrize("B", [1, 2, 3, 5])
def test_furnace_emit_on_hit_bounce_count(B):
    """Walls emit L and reflect rho: light reflected exactly k times before
    reaching x carries pi L rho^k, so the indirect part with B bounces is
    pi L sum_{k=1..B} rho^k, every sample exactly."""
    L = np.array([1.0, 2.0, 0.5], np.float32).astype(np.float64)
    rho = np.array([0.3, 0.5, 0.7], np.float32).astype(np.float64)
    prims = enclosure_prims((0, 0, 0), (1, 1, 1), albedo=rho, emission=L)
    rng = np.random.default_rng(B)
    x = rng.uniform(0.05, 0.95, size=(30, 3)).astype(np.float32)
    n = _rand_dirs(rng, 30)
    want = math.pi * L * sum(rho ** k for k in range(1, B + 1))
    E, var, _, _ = O.mc_irradiance(prims, x, n, 32, B, O.MC_EMIT_ON_HIT, 9)
    np.testing.assert_allclose(E, np.tile(want, (30, 1)), rtol=1e-12)
    E2, _, _, _ = O.mc_irradiance(prims, x, n, 32, B, O.MC_EMIT_ON_HIT | O.MC_INCLUDE_DIRECT, 9)
    np.testing.assert_allclose(E2, np.tile(want + math.pi * L, (30, 1)), rtol=1e-12)


def test_furnace_nee_expectation():
    """Same furnace with next-event estimation to every emitting wall: each
    vertex gathers rho/pi * (pi L), unbiased but not zero-variance."""
    L = np.array([1.0, 1.0, 1.0])
    rho = np.array([0.4, 0.6, 0.8], np.float32).astype(np.float64)
    prims = enclosure_prims((0, 0, 0), (1, 1, 1), albedo=rho, emission=L)
    rng = np.random.default_rng(21)
    x = rng.uniform(0.2, 0.8, size=(6, 3)).astype(np.float32)
    n = _rand_dirs(rng, 6)
    want = math.pi * L * sum(rho ** k for k in range(1, 4))
    E, var, _, _ = O.mc_irradiance(prims, x, n, 20000, 3, O.MC_NEE, 3)
    z = (E - want) / np.sqrt(var)
    assert np.abs(z).max() < 4.5, z


def _disk_case(h=1.5, r=0.8, L=3.0):
    prims = np.array([disk_prim((0.2, 0.1, 0.3 + h), (0, 0, -1), r, emission=(L, L, L))],
                     dtype=PRIM_DTYPE)
    x = np.float32([[0.2, 0.1, 0.3]])
    n = np.float32([[0, 0, 1]])
    return prims, x, n, math.pi * L * r * r / (r * r + h * h)


@pytest.mark.parametrize("flags", [O.MC_INCLUDE_DIRECT, O.MC_DIRECT_AT_ORIGIN])
def test_disk_light_closed_form(flags):
    """On-axis disk of radius r at distance h: E = pi L sin^2(alpha),
    sin^2(alpha) = r^2 / (r^2 + h^2).  Tests the cosine sampler (hit mode)
    and light sampling (direct mode)."""
    prims, x, n, want = _disk_case()
    E, var, _, _ = O.mc_irradiance(prims, x, n, 200000, 1, flags, 11)
    z = (E[0] - want) / np.sqrt(var[0])
    assert np.abs(z).max() < 4.0, (E[0], want, z)
    assert np.abs(E[0] / want - 1).max() < 0.01


def _lambert_polygon(x, n, verts, L):
    """Lambert's formula for a uniformly emitting polygon seen entirely
    above the horizon: E = (L/2) |sum_i Theta_i n . g_i|, g_i the unit normal
    of the plane through x and edge i, Theta_i the angle the edge subtends."""
    s = 0.0
    k = len(verts)
    for i in range(k):
        a = verts[i] - x
        b = verts[(i + 1) % k] - x
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        th = math.acos(np.clip(a @ b, -1, 1))
        g = np.cross(a, b)
        g /= np.linalg.norm(g)
        s += th * (n @ g)
    return 0.5 * L * abs(s)


@pytest.mark.parametrize("flags", [O.MC_INCLUDE_DIRECT, O.MC_DIRECT_AT_ORIGIN])
def test_rect_light_lambert_formula(flags):
    L = 2.5
    c = np.array([0.7, 2.0, -0.4])
    hu, hv = 0.6, 0.35  # axis 1 (y): u = z, v = x
    prims = np.array([rect_prim(1, -1.0, c, hu, hv, (0, 0, 0), (L, L, L))], dtype=PRIM_DTYPE)
    x = np.array([0.1, 0.2, 0.3])
    nn = np.array([0.3, 0.9, -0.2])
    nn /= np.linalg.norm(nn)
    cf = np.float32(c).astype(np.float64)
    verts = [cf + np.array([dx, 0, dz]) for dx, dz in
             [(-hv, -hu), (hv, -hu), (hv, hu), (-hv, hu)]]
    xf = np.float32(x).astype(np.float64)
    nf = np.float32(nn).astype(np.float64)
    nf /= np.linalg.norm(nf)
    want = _lambert_polygon(xf, nf, verts, L)
    E, var, _, _ = O.mc_irradiance(prims, x[None].astype(np.float32), nn[None].astype(np.float32),
                                   200000, 1, flags, 13)
    z = (E[0] - want) / np.sqrt(var[0])
    assert np.abs(z).max() < 4.0, (E[0], want)


# ------------------------------------------------------------ culling and rejection
def test_point_inside_box_is_culled():
    room = make_room(2001)
    prims = room["prims"]
    blo, bhi, _ = room["boxes"][0]
    x = np.float32([0.5 * (blo + bhi)])
    n = np.float32([[0, 1, 0]])
    E, _, bf, valid = O.mc_irradiance(prims, x, n, 64, 3, O.MC_NEE, 1)
    assert bf[0] == 64 and valid[0] == 0 and (E == 0).all()


def test_dark_room_rejects_null_irradiance():
    room = make_room(2001, n_lights=0)
    x = np.float32([[5.0, 2.0, 5.0]])
    n = np.float32([[0, -1, 0]])
    E, _, bf, valid = O.mc_irradiance(room["prims"], x, n, 64, 3, O.MC_NEE, 1)
    assert (E == 0).all() and valid[0] == 0


def test_validity_rule_majority_backfacing_and_null():
    """Culling reading: a point is invalid when more than half of its first
    hits are back faces (exactly half is kept) or when every channel of E is
    zero.  Points near box faces give partial back-face counts."""
    room = make_room(2001)
    rng = np.random.default_rng(17)
    pts, nrms = [], []
    for (blo, bhi, _) in room["boxes"][:8]:
        c = 0.5 * (blo + bhi)
        for _ in range(4):
            p = c.copy()
            p[1] = bhi[1] + rng.uniform(-0.05, 0.05)  # straddling the top face
            pts.append(p)
            nrms.append(_rand_dirs(rng, 1)[0])
    x = np.array(pts, np.float32)
    n = np.array(nrms, np.float32)
    S = 64
    E, _, bf, valid = O.mc_irradiance(room["prims"], x, n, S, 3, O.MC_NEE, 2)
    want = (2 * bf <= S) & (E > 0).any(1)
    np.testing.assert_array_equal(valid.astype(bool), want)
    assert ((bf > 0) & (bf < S)).any()


# ------------------------------------------------------------ estimator consistency
def test_nee_and_emit_on_hit_agree_in_room():
    """Next-event estimation and emission-on-hit estimate the same indirect
    irradiance (light reflected 1..B times); they agree within noise."""
    room = make_room(2001)
    rng = np.random.default_rng(31)
    x = rng.uniform([1, 0.5, 3], [9, 3.5, 9], size=(6, 3)).astype(np.float32)
    n = _rand_dirs(rng, 6)
    Ea, va, _, vda = O.mc_irradiance(room["prims"], x, n, 6000, 3, O.MC_NEE, 4)
    Eb, vb, _, vdb = O.mc_irradiance(room["prims"], x, n, 60000, 3, O.MC_EMIT_ON_HIT, 5)
    ok = vda.astype(bool) & vdb.astype(bool)
    assert ok.sum() >= 3
    z = (Ea - Eb)[ok] / np.sqrt(va + vb)[ok]
    assert np.abs(z).max() < 4.5, z


def test_replay_is_deterministic():
    room = make_room(2001)
    x = np.float32([[3, 2, 6], [6, 1, 7]])
    n = np.float32([[0, 1, 0], [1, 0, 0]])
    a = O.mc_irradiance(room["prims"], x, n, 128, 3, O.MC_NEE, 42)
    b = O.mc_irradiance(room["prims"], x, n, 128, 3, O.MC_NEE, 42)
    c = O.mc_irradiance(room["prims"], x, n, 128, 3, O.MC_NEE, 43)
    np.testing.assert_array_equal(a[0], b[0])
    assert not np.array_equal(a[0], c[0])


# ------------------------------------------------------------ training-point sampler
def test_sampler_volume_and_surface_points():
    prims = enclosure_prims((0, 0, 0), (1, 2, 3), (0.5, 0.5, 0.5), (0, 0, 0))
    lo, hi = np.zeros(3), np.array([1.0, 2.0, 3.0])
    n_total, n_surf = 60000, 30000
    x, n = O.sample_points(prims, lo, hi, n_total, n_surf, 7)
    xv, nv = x[:n_total - n_surf], n[:n_total - n_surf]
    assert (xv >= lo).all() and (xv <= hi).all()
    np.testing.assert_allclose(np.linalg.norm(nv, axis=1), 1, atol=1e-6)
    # uniform on the sphere: mean ~ 0, second moment ~ I/3
    assert np.abs(nv.mean(0)).max() < 0.02
    np.testing.assert_allclose((nv.T @ nv) / len(nv), np.eye(3) / 3, atol=0.01)
    np.testing.assert_allclose(xv.mean(0), hi / 2, rtol=0.02)
    xs, ns = x[n_total - n_surf:], n[n_total - n_surf:]
    # each surface point lies on its wall and looks inward
    counts = np.zeros(6)
    for axis in range(3):
        for side in range(2):
            sel = ns[:, axis] == (1.0 if side == 0 else -1.0)
            plane = 0.0 if side == 0 else hi[axis]
            assert (xs[sel, axis] == np.float32(plane)).all()
            counts[2 * axis + side] = sel.sum()
    assert counts.sum() == n_surf
    areas = np.array([6, 6, 3, 3, 2, 2], float)
    np.testing.assert_allclose(counts / n_surf, areas / areas.sum(), atol=0.01)


# ------------------------------------------------------------ scenes that change with t (Sec. 6)
@pytest.mark.parametrize("flags", [O.MC_INCLUDE_DIRECT, O.MC_DIRECT_AT_ORIGIN])
def test_moving_disk_closed_form(flags):
    """A disk light moving away along its axis: at scene variable t it sits
    at distance h + t, and E = pi L r^2 / (r^2 + (h + t)^2) on the axis."""
    h, r, L = 1.0, 0.8, 3.0
    prims, x, n, _ = _disk_case(h=h, r=r, L=L)
    motion = np.float32([[0.0, 0.0, 1.0]])
    ts = np.float32([0.0, 0.5, 1.0])
    E, var, _, _ = O.mc_irradiance(prims, np.repeat(x, 3, 0), np.repeat(n, 3, 0), 200000, 1,
                                   flags, 12, motion=motion, t=ts)
    for k, tv in enumerate(ts):
        want = math.pi * L * r * r / (r * r + (h + tv) ** 2)
        z = (E[k] - want) / np.sqrt(var[k])
        assert np.abs(z).max() < 4.0, (tv, E[k], want)
        assert np.abs(E[k] / want - 1).max() < 0.01


def test_motion_equals_translated_scene():
    """Translating primitives by t * motion inside the estimator gives the
    estimate of the scene built already translated (same random streams)."""
    room = make_room(2001)
    prims = np.array(room["prims"], copy=True)
    motion = np.zeros((len(prims), 3), np.float32)
    lights = np.nonzero(prims["emission"].max(axis=1) > 0)[0]
    motion[lights] = [0.5, 0.0, -0.25]      # both ceiling lights slide
    motion[-1] = [0.0, 0.0, 0.5]            # and the last box moves
    tv = 0.5
    moved = np.array(prims, copy=True)
    for k in np.nonzero(np.abs(motion).sum(1))[0]:
        off = (tv * motion[k]).astype(np.float32)
        moved["p"][k] += off
        if prims["kind"][k] == 0:
            moved["q"][k] += off
    rng = np.random.default_rng(41)
    x = rng.uniform([1, 0.5, 3], [9, 3.5, 9], size=(8, 3)).astype(np.float32)
    nn = _rand_dirs(rng, 8)
    a = O.mc_irradiance(prims, x, nn, 256, 3, O.MC_NEE, 9, motion=motion,
                        t=np.full(8, tv, np.float32))
    b = O.mc_irradiance(moved, x, nn, 256, 3, O.MC_NEE, 9)
    np.testing.assert_allclose(a[0], b[0], rtol=1e-9, atol=1e-12)
    np.testing.assert_array_equal(a[2], b[2])
    np.testing.assert_array_equal(a[3], b[3])
    # t = 0 is the static scene, and t changes the answer
    c = O.mc_irradiance(prims, x, nn, 256, 3, O.MC_NEE, 9, motion=motion, t=np.zeros(8, np.float32))
    d = O.mc_irradiance(prims, x, nn, 256, 3, O.MC_NEE, 9)
    np.testing.assert_array_equal(c[0], d[0])
    assert not np.allclose(a[0], d[0])


def test_sampler_scene_variable():
    """The scene variable drawn with each training point is uniform on
    [0, 1) (dimension 7 of the point's stream) and leaves the points as they
    were."""
    prims = enclosure_prims((0, 0, 0), (1, 2, 3), (0.5, 0.5, 0.5), (0, 0, 0))
    lo, hi = np.zeros(3), np.array([1.0, 2.0, 3.0])
    x0, n0 = O.sample_points(prims, lo, hi, 20000, 4000, 11)
    x, n, t = O.sample_points(prims, lo, hi, 20000, 4000, 11, with_t=True)
    np.testing.assert_array_equal(x, x0)
    np.testing.assert_array_equal(n, n0)
    assert (t >= 0).all() and (t < 1).all()
    from scipy.stats import kstest
    assert kstest(t, "uniform").pvalue > 1e-3
    assert t[5] == np.float32(O.uniform(11, 5, 0, 1, 7))
