"""Pins of the FP64 oracle's model arithmetic against things other than
itself: numbers printed in the paper, closed forms, library routines and
brute force.  CPU only."""
import math
import os

import numpy as np
import pytest
import scipy.special as sps
from scipy.interpolate import RegularGridInterpolator

import oracle as O
from niv_synth import get_workload, make_params

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _cfg(**kw):
    base = dict(n_levels=2, log2_T=12, n_features=2, base_res=2.0, per_level_scale=2.0,
                sh_bands=4, n_extra=0, extra_bands=0, width=16, n_hidden=2, n_out=3,
                aabb_min=(0.0, 0.0, 0.0), aabb_max=(1.0, 1.0, 1.0))
    base.update(kw)
    return O.make_config(**base)


# ------------------------------------------------------------ level table
def test_level_lists_unit_cube_and_room():
    c1 = O.config_from_workload(get_workload("unit_cube_16k"))
    t1 = O.level_table(c1)
    assert t1["res"].tolist() == [4, 6, 9, 13, 20, 30, 45, 68]
    assert t1["dense"].tolist() == [True] * 5 + [False] * 3
    assert t1["size"].tolist()[:5] == [125, 343, 1000, 2744, 9261]
    assert t1["total"] == 62625
    c2 = O.config_from_workload(get_workload("room_1080p"))
    t2 = O.level_table(c2)
    assert t2["res"].tolist() == [16, 22, 32, 45, 64, 90, 128, 181, 256, 362, 512, 724,
                                  1024, 1448, 2048, 2896]
    assert t2["dense"].tolist() == [True] * 4 + [False] * 12
    assert t2["size"].tolist()[:4] == [4913, 12167, 35937, 97336]


def test_table1_memory_column():
    """Half-precision sizes from the level rule reproduce the memory column
    of Table 1 and the ~10 MB of the doubled table (Sec. 6); which rows count
    the network is stated in the fixture."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_memory.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 5
    for width, levels, log2T, mb, digits, counted in rows:
        c = O.make_config(n_levels=int(levels), log2_T=int(log2T), n_features=4,
                          base_res=16.0, per_level_scale=math.sqrt(2.0), sh_bands=4,
                          n_extra=0, extra_bands=0, width=int(width), n_hidden=3, n_out=3,
                          aabb_min=(0, 0, 0), aabb_max=(1, 1, 1))
        nbytes = 2 * (O.n_params(c) if counted == "grid+mlp" else O.n_grid_values(c))
        assert round(nbytes / 1e6, int(digits)) == pytest.approx(float(mb)), (levels, nbytes)


def test_level_rule_alternatives_do_not_fit():
    """The printed 1.20 MB (4 levels) rules out an N^3 dense rule and a
    ceiling rounding of the resolutions."""
    res = [math.floor(16 * math.sqrt(2) ** l + 1e-9) for l in range(4)]
    n3 = sum(min(r ** 3, 1 << 17) for r in res) * 8
    ceil_res = [math.ceil(16 * math.sqrt(2) ** l - 1e-9) for l in range(4)]
    ceil = sum(min((r + 1) ** 3, 1 << 17) for r in ceil_res) * 8
    assert round(n3 / 1e6, 2) != 1.20 and round(ceil / 1e6, 2) != 1.20


# ------------------------------------------------------------ hash / dense index
def test_hash_brute_force():
    rng = np.random.default_rng(0)
    for _ in range(2000):
        x, y, z = (int(v) for v in rng.integers(0, 1 << 20, size=3))
        log2T = int(rng.integers(4, 24))
        want = ((x * 1) ^ ((y * 2654435761) & 0xFFFFFFFF) ^ ((z * 805459861) & 0xFFFFFFFF)) \
            & 0xFFFFFFFF & ((1 << log2T) - 1)
        assert O.hash_index(x, y, z, log2T) == want


def test_hash_x_pairs_adjacent():
    """With the first prime equal to 1, the corner at x+1 of an even x sits
    next to the corner at x: idx(x+1) = idx(x) ^ 1."""
    rng = np.random.default_rng(1)
    for _ in range(500):
        x = 2 * int(rng.integers(0, 1 << 15))
        y, z = (int(v) for v in rng.integers(0, 1 << 16, size=2))
        assert O.hash_index(x + 1, y, z, 17) == O.hash_index(x, y, z, 17) ^ 1


def test_dense_index_matches_ravel():
    for N in (1, 4, 16, 45):
        side = N + 1
        rng = np.random.default_rng(N)
        for _ in range(200):
            v = rng.integers(0, side, size=3)
            want = np.ravel_multi_index(tuple(int(a) for a in v), (side,) * 3, order="F")
            assert O.dense_index(int(v[0]), int(v[1]), int(v[2]), N) == want


# ------------------------------------------------------------ trilinear interpolation
def _dense_cfg():
    # every level dense: N = 2, 4, 8 with T = 2^12 (9^3 = 729 <= 4096)
    return _cfg(n_levels=3, log2_T=12, base_res=2.0, per_level_scale=2.0)


def test_trilinear_matches_library_interpolator():
    c = _dense_cfg()
    tab = O.level_table(c)
    assert tab["dense"].all()
    rng = np.random.default_rng(2)
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), 7, -1, 1).astype(np.float64)
    grid = O.split_params(c, params)[0]
    pos = rng.uniform(0, 1, size=(300, 3)).astype(np.float32)
    nrm = np.tile(np.float32([0, 0, 1]), (300, 1))
    _, _, _, x0 = O.query(c, params, pos, nrm, want_x0=True)
    for l in range(c.n_levels):
        N = int(tab["res"][l])
        side = N + 1
        lat = grid[tab["offset"][l]:tab["offset"][l] + side ** 3]
        ax = np.arange(side, dtype=np.float64)
        for j in range(c.n_features):
            vol = lat[:, j].reshape(side, side, side, order="F")  # [x, y, z]
            f = RegularGridInterpolator((ax, ax, ax), vol, method="linear")
            want = f(pos.astype(np.float64) * N)
            np.testing.assert_allclose(x0[:, l * c.n_features + j], want, rtol=0, atol=1e-12)


def test_trilinear_reproduces_affine_latents():
    c = _dense_cfg()
    tab = O.level_table(c)
    params = np.zeros(O.n_params(c))
    grid = O.split_params(c, params)[0]
    a = np.array([0.3, -1.1, 0.7])
    for l in range(c.n_levels):
        N = int(tab["res"][l])
        side = N + 1
        zz, yy, xx = np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij")
        v = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1)  # x fastest
        grid[tab["offset"][l]:tab["offset"][l] + side ** 3, 0] = v @ a + 0.25
        grid[tab["offset"][l]:tab["offset"][l] + side ** 3, 1] = v @ (-a) - 1.0
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 1, size=(200, 3)).astype(np.float32)
    nrm = np.tile(np.float32([1, 0, 0]), (200, 1))
    _, _, _, x0 = O.query(c, params, pos, nrm, want_x0=True)
    for l in range(c.n_levels):
        s = pos.astype(np.float64) * tab["res"][l]
        np.testing.assert_allclose(x0[:, 2 * l], s @ a + 0.25, atol=1e-12)
        np.testing.assert_allclose(x0[:, 2 * l + 1], s @ (-a) - 1.0, atol=1e-12)


def test_trilinear_reproduces_affine_latents_in_world_coordinates_on_a_box():
    """The room's 10 x 4 x 10 m box (non-cubic, offset from the origin):
    latents that are an affine function of each vertex's WORLD position,
    lo + i (hi - lo) / N per axis, are reproduced exactly at any world
    point.  An axis mapped with another axis' extent, a missing offset or a
    transposed cell index breaks this."""
    lo, hi = np.array([-2.0, 0.5, 3.0]), np.array([8.0, 4.5, 13.0])
    c = _cfg(n_levels=3, log2_T=14, base_res=3.0, per_level_scale=2.0,
             aabb_min=tuple(lo), aabb_max=tuple(hi))
    tab = O.level_table(c)
    assert tab["dense"].all()
    params = np.zeros(O.n_params(c))
    grid = O.split_params(c, params)[0]
    a = np.array([0.3, -1.1, 0.7])
    for l in range(c.n_levels):
        N = int(tab["res"][l])
        side = N + 1
        zz, yy, xx = np.meshgrid(np.arange(side), np.arange(side), np.arange(side), indexing="ij")
        v = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], 1).astype(np.float64)   # x fastest
        world = lo + v * (hi - lo) / N
        grid[tab["offset"][l]:tab["offset"][l] + side ** 3, 0] = world @ a + 0.25
        grid[tab["offset"][l]:tab["offset"][l] + side ** 3, 1] = world @ (-a) - 1.0
    rng = np.random.default_rng(31)
    pos = rng.uniform(lo, hi, size=(400, 3)).astype(np.float32)
    nrm = np.tile(np.float32([0, 1, 0]), (400, 1))
    _, _, _, x0 = O.query(c, params, pos, nrm, want_x0=True)
    p64 = pos.astype(np.float64)
    for l in range(c.n_levels):
        np.testing.assert_allclose(x0[:, 2 * l], p64 @ a + 0.25, atol=1e-11)
        np.testing.assert_allclose(x0[:, 2 * l + 1], p64 @ (-a) - 1.0, atol=1e-11)


def test_fp32_error_bar_reading_on_the_room_network():
    """The reading of the FP32 bar (max relative error 1e-5): relative to
    the output, or under cancellation to the magnitude of the terms summed
    into it.  A plain numpy FP32 evaluation of the room_1080p network (same
    FP64 encoded inputs rounded to FP32, sequential FP32 matrix products)
    meets 1e-5 on that scale, while the error relative to a floor of 1e-3
    of the largest output exceeds 1e-5: that floored form is not a bar any
    FP32 evaluation of this network can meet."""
    from niv_metrics import term_scale, max_rel_floored
    w = get_workload("room_1080p")
    c = O.config_from_workload(w)
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), w.param_seed, *w.grid_init)
    p64 = params.astype(np.float64)
    rng = np.random.default_rng(5)
    n = 1 << 16
    pos = rng.uniform(w.aabb_min, w.aabb_max, size=(n, 3)).astype(np.float32)
    v = rng.standard_normal((n, 3))
    nrm = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    E, _, _, x0 = O.query(c, p64, pos, nrm, want_x0=True)
    mats = O.split_params(c, p64)[1:]
    h = x0.astype(np.float32)
    for k, Wm in enumerate(mats):
        h = h @ Wm.astype(np.float32).T
        if k < len(mats) - 1:
            h = np.maximum(h, np.float32(0))
    scale = term_scale(mats, x0)
    err = np.abs(h.astype(np.float64) - E)
    term = float(np.max(err / np.maximum(np.abs(E), scale)))
    floored = max_rel_floored(h.astype(np.float64), E)
    print(f"numpy FP32 on {n} points: term-scale {term:.2e}, floored {floored:.2e}")
    assert term <= 1e-5
    assert floored > 1e-5


def test_init_params_follow_their_stream_and_xavier_bounds():
    """Seeded start: value k is lo + (hi - lo) u_k on the grid and a (2 u_k
    - 1) in weight matrix m, a = sqrt(6 / (fan_in + fan_out)), where u_k is
    the low 32 bits of the first word of Philox4x64-10 at counter (k, 0, 0,
    3), key (seed, 0), cut to 24 bits (recomputed here with numpy's Philox).
    The moments follow: grid mean (lo + hi) / 2; weight variance
    2 / (fan_in + fan_out) (Xavier)."""
    w = get_workload("room_1080p")
    c = O.config_from_workload(w)
    seed, lo, hi = 4242, -1e-4, 1e-4
    p = O.init_params(c, seed, lo, hi)
    assert p.dtype == np.float32 and p.size == O.n_params(c)
    n_grid = O.n_grid_values(c)

    def u_k(k):   # numpy increments its counter before a block: start one below (k, 0, 0, 3)
        bg = np.random.Philox(counter=np.array([k - 1, 0, 0, 3], dtype=np.uint64),
                              key=np.array([seed, 0], dtype=np.uint64))
        return (int(bg.random_raw(1)[0]) & 0xFFFFFFFF) >> 8

    from fractions import Fraction
    rng = np.random.default_rng(8)
    ks = list(rng.integers(1, n_grid, 40)) + list(rng.integers(n_grid, p.size, 40)) + [1, n_grid]
    shapes = O.mat_shapes(c)
    ends = np.cumsum([o * i for o, i in shapes]) + n_grid
    for k in ks:
        u = u_k(int(k)) * 2.0 ** -24
        if k < n_grid:   # one rounding of the exact lo + (hi - lo) u to double, then to float
            want = np.float32(float(Fraction(hi - lo) * Fraction(u) + Fraction(lo)))
        else:
            m = int(np.searchsorted(ends, k, side="right"))
            o, i = shapes[m]
            want = np.float32(math.sqrt(6.0 / (o + i)) * (2.0 * u - 1.0))
        assert p[k] == want, (k, p[k], want)
    g = p[:n_grid].astype(np.float64)
    assert g.min() >= lo and g.max() < hi
    assert abs(g.mean()) < 1e-6
    k = n_grid
    for (o, i) in shapes:
        wm = p[k:k + o * i].astype(np.float64)
        a = math.sqrt(6.0 / (o + i))
        assert wm.min() >= -a and wm.max() < a
        assert wm.var() == pytest.approx(2.0 / (o + i), rel=0.35 if o * i < 500 else 0.06)
        k += o * i
    assert not np.array_equal(p, O.init_params(c, seed + 1, lo, hi))


def test_weights_partition_of_unity_and_corner_range():
    c = O.config_from_workload(get_workload("room_1080p"))
    tab = O.level_table(c)
    rng = np.random.default_rng(4)
    for _ in range(50):
        p = rng.uniform([0, 0, 0], [10, 4, 10]).astype(np.float32)
        idx, w = O.corners(c, p)
        np.testing.assert_allclose(w.sum(1), 1.0, atol=1e-13)
        assert (w >= 0).all()
        assert (idx >= 0).all() and (idx < tab["size"][:, None]).all()


def test_interpolation_continuous_across_cell_faces():
    c = O.config_from_workload(get_workload("unit_cube_16k"))
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), 5, -0.5, 0.5).astype(np.float64)
    base = np.array([0.3, 0.6, 0.2])
    eps = 1e-9
    for N in (4, 13, 68):
        face = 7.0 / N  # an interior cell face of this level on the x axis
        p0 = base.copy(); p0[0] = face - eps
        p1 = base.copy(); p1[0] = face + eps
        pos = np.array([p0, p1]).astype(np.float32)
        if pos[0, 0] == pos[1, 0]:
            pos[1, 0] = np.nextafter(pos[0, 0], np.float32(2))
        nrm = np.float32([[0, 1, 0], [0, 1, 0]])
        _, _, _, x0 = O.query(c, params, pos, nrm, want_x0=True)
        assert np.abs(x0[0] - x0[1]).max() < 1e-4


def test_outside_box_is_clamped_and_flagged():
    c = O.config_from_workload(get_workload("unit_cube_16k"))
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), 5, -0.5, 0.5).astype(np.float64)
    pos = np.float32([[1.5, 0.5, 0.5], [1.0, 0.5, 0.5], [0.5, -0.1, 0.5]])
    nrm = np.float32([[0, 0, 1]] * 3)
    E, _, fl = O.query(c, params, pos, nrm)
    assert (fl & (0xff ^ O.FLAG_NEG_OUTPUT)).tolist() == [O.FLAG_OUTSIDE, 0, O.FLAG_OUTSIDE]
    np.testing.assert_array_equal(E[0], E[1])


def test_negative_output_flag():
    """Bit 4 marks a finite output with a negative channel, nothing else."""
    c = O.config_from_workload(get_workload("unit_cube_16k"))
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), 5, -0.5, 0.5).astype(np.float64)
    rng = np.random.default_rng(3)
    pos = rng.uniform(0, 1, (500, 3)).astype(np.float32)
    nrm = rng.standard_normal((500, 3)).astype(np.float32)
    E, _, fl = O.query(c, params, pos, nrm)
    neg = (E < 0).any(axis=1)
    assert 0 < neg.sum() < 500
    np.testing.assert_array_equal((fl & O.FLAG_NEG_OUTPUT) != 0, neg)
    # flipping the sign of the output layer swaps which channels are negative
    p2 = params.copy()
    shapes = O.mat_shapes(c)
    p2[-shapes[-1][0] * shapes[-1][1]:] *= -1
    E2, _, fl2 = O.query(c, p2, pos, nrm)
    np.testing.assert_array_equal(E2, -E)
    np.testing.assert_array_equal((fl2 & O.FLAG_NEG_OUTPUT) != 0, (E > 0).any(axis=1))


# ------------------------------------------------------------ SH and frequency encoding
def test_sh_y00_and_addition_theorem():
    rng = np.random.default_rng(6)
    for _ in range(100):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        y = O.sh(4, n)
        assert y[0] == pytest.approx(0.5 / math.sqrt(math.pi), abs=1e-15)
        for l in range(4):
            assert np.sum(y[l * l:(l + 1) * (l + 1)] ** 2) == pytest.approx(
                (2 * l + 1) / (4 * math.pi), rel=1e-12)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi: exact for these degrees.
    xg, wg = np.polynomial.legendre.leggauss(16)
    nphi = 32
    G = np.zeros((16, 16))
    for x, w in zip(xg, wg):
        s = math.sqrt(1 - x * x)
        for k in range(nphi):
            phi = 2 * math.pi * k / nphi
            y = O.sh(4, np.array([s * math.cos(phi), s * math.sin(phi), x]))
            G += np.outer(y, y) * w * (2 * math.pi / nphi)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_matches_scipy_complex_harmonics():
    """Real SH with the Condon-Shortley phase: sqrt(2) Re Y_l^m for m > 0,
    sqrt(2) Im Y_l^|m| for m < 0, Y_l^0 for m = 0 (scipy includes the phase)."""
    rng = np.random.default_rng(7)
    for _ in range(50):
        n = rng.standard_normal(3)
        n /= np.linalg.norm(n)
        theta = math.acos(n[2])
        phi = math.atan2(n[1], n[0])
        y = O.sh(4, n)
        for l in range(4):
            for m in range(-l, l + 1):
                Y = complex(sps.sph_harm_y(l, abs(m), theta, phi))
                want = (math.sqrt(2) * Y.real if m > 0 else
                        math.sqrt(2) * Y.imag if m < 0 else Y.real)
                assert y[l * l + l + m] == pytest.approx(want, abs=1e-12)


def test_legendre_matches_scipy():
    for l in range(5):
        for m in range(l + 1):
            for x in (-0.9, -0.3, 0.0, 0.45, 0.99):
                assert O.legendre(l, m, x) == pytest.approx(float(sps.lpmv(m, l, x)), abs=1e-12)


def test_frequency_encoding_closed_form():
    g = O.freq(8, 0.25)
    for k in range(8):
        ang = (2 ** k) * math.pi * 0.25
        assert g[2 * k] == pytest.approx(math.sin(ang), abs=1e-12)
        assert g[2 * k + 1] == pytest.approx(math.cos(ang), abs=1e-12)
    g = O.freq(3, 0.5)  # sin(pi/2), cos(pi/2), sin(pi), cos(pi), sin(2pi), cos(2pi)
    np.testing.assert_allclose(g, [1, 0, 0, -1, 0, 1], atol=1e-12)


# ------------------------------------------------------------ MLP and Eq. 2
@pytest.mark.parametrize("wname", ["unit_cube_16k", "room_4k_6d"])
def test_mlp_matches_numpy_matmul(wname):
    w = get_workload(wname)
    c = O.config_from_workload(w)
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), 9, -0.5, 0.5).astype(np.float64)
    rng = np.random.default_rng(8)
    lo, hi = np.array(w.aabb_min), np.array(w.aabb_max)
    pos = rng.uniform(lo, hi, size=(64, 3)).astype(np.float32)
    nrm = rng.standard_normal((64, 3)).astype(np.float32)
    extra = rng.uniform(0, 1, size=(64, c.n_extra)).astype(np.float32) if c.n_extra else None
    alb = rng.uniform(0.2, 0.8, size=(64, 3)).astype(np.float32)
    E, L, fl, x0 = O.query(c, params, pos, nrm, extra=extra, albedo=alb, want_x0=True)
    mats = O.split_params(c, params)[1:]
    h = x0.T
    for Wm in mats[:-1]:
        h = np.maximum(Wm @ h, 0.0)
    want = (mats[-1] @ h).T
    np.testing.assert_allclose(E, want, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(L, alb.astype(np.float64) * want / math.pi, rtol=1e-12, atol=1e-14)
    assert ((fl & (0xff ^ O.FLAG_NEG_OUTPUT)) == 0).all()
    np.testing.assert_array_equal((fl & O.FLAG_NEG_OUTPUT) != 0, (E < 0).any(axis=1))
    if c.n_extra:
        for q in range(4):
            np.testing.assert_allclose(x0[q, -16:], O.freq(8, float(extra[q, 0])), atol=1e-12)


def test_masked_and_degenerate_points_write_zero():
    c = O.config_from_workload(get_workload("unit_cube_16k"))
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), 5, -0.5, 0.5).astype(np.float64)
    pos = np.float32([[0.5, 0.5, 0.5], [0.2, 0.2, 0.2], [np.nan, 0.1, 0.1], [0.3, 0.3, 0.3]])
    nrm = np.float32([[0, 0, 1], [0, 0, 1], [0, 0, 1], [0, 0, 0]])
    mask = np.uint8([1, 0, 1, 1])
    E, L, fl = O.query(c, params, pos, nrm, albedo=np.ones((4, 3), np.float32), mask=mask)
    assert np.abs(E[0]).sum() > 0
    assert (E[1:] == 0).all() and (L[1:] == 0).all()
    assert fl[2] & O.FLAG_BAD_INPUT and fl[3] & O.FLAG_BAD_INPUT


# ------------------------------------------------------------ Eq. 3 and its gradient
def _small_train_case(n=24, seed=10):
    c = _cfg(n_levels=3, log2_T=6, base_res=2.0, per_level_scale=2.0, width=8,
             n_hidden=2)  # level 2 (N=8, 729 > 64) is hashed
    tab = O.level_table(c)
    assert tab["dense"].tolist() == [True, False, False]
    rng = np.random.default_rng(seed)
    params = make_params(O.n_grid_values(c), O.mat_shapes(c), seed, -0.5, 0.5).astype(np.float64)
    pos = rng.uniform(0, 1, size=(n, 3)).astype(np.float32)
    nrm = rng.standard_normal((n, 3)).astype(np.float32)
    tgt = rng.uniform(0, 2, size=(n, 3)).astype(np.float32)
    return c, params, pos, nrm, tgt


def test_loss_matches_eq3_directly():
    c, params, pos, nrm, tgt = _small_train_case()
    E, _, _ = O.query(c, params, pos, nrm)
    want = np.mean((E - tgt) ** 2 / (E ** 2 + 0.01))
    assert O.loss(c, params, pos, nrm, tgt) == pytest.approx(want, rel=1e-13)
    l2, _ = O.loss_grad(c, params, pos, nrm, tgt)
    assert l2 == pytest.approx(want, rel=1e-12)


def test_gradient_matches_central_differences():
    """d loss / d theta with the Eq. 3 denominator held fixed (stop-gradient):
    compared with central differences of a loss whose denominator is frozen
    at the current prediction."""
    c, params, pos, nrm, tgt = _small_train_case()
    E0, _, _ = O.query(c, params, pos, nrm)
    den = E0 ** 2 + 0.01
    _, g = O.loss_grad(c, params, pos, nrm, tgt)

    def frozen_loss(p):
        E, _, _ = O.query(c, p, pos, nrm)
        return np.mean((E - tgt) ** 2 / den)

    rng = np.random.default_rng(11)
    n_grid = O.n_grid_values(c)
    touched = np.nonzero(g[:n_grid])[0]
    picks = list(rng.choice(touched, 25, replace=False)) + list(
        rng.choice(np.arange(n_grid, params.size), 40, replace=False))
    h = 1e-6
    for k in picks:
        p1 = params.copy(); p1[k] += h
        p2 = params.copy(); p2[k] -= h
        fd = (frozen_loss(p1) - frozen_loss(p2)) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k
    # untouched grid entries get exactly zero gradient
    assert np.count_nonzero(g[:n_grid]) == touched.size


def test_gradient_of_output_is_closed_form():
    """For the last layer: dl/dW_H[o,k] = sum_b 2 (E-y)/(E^2+eps)/(3B) x_H[k]."""
    c, params, pos, nrm, tgt = _small_train_case()
    E, _, _, x0 = O.query(c, params, pos, nrm, want_x0=True)
    mats = O.split_params(c, params)[1:]
    h = x0.T
    for Wm in mats[:-1]:
        h = np.maximum(Wm @ h, 0.0)
    dE = 2 * (E - tgt) / (E ** 2 + 0.01) / E.size
    want = dE.T @ h.T
    _, g = O.loss_grad(c, params, pos, nrm, tgt)
    gH = g[-3 * c.width:].reshape(3, c.width)
    np.testing.assert_allclose(gH, want, rtol=1e-11, atol=1e-15)


def test_invalid_samples_contribute_nothing():
    c, params, pos, nrm, tgt = _small_train_case()
    valid = np.ones(len(pos), np.uint8)
    valid[::3] = 0
    l_mask, g_mask = O.loss_grad(c, params, pos, nrm, tgt, valid=valid)
    keep = valid.astype(bool)
    l_sub, g_sub = O.loss_grad(c, params, pos[keep], nrm[keep], tgt[keep])
    scale = keep.sum() / len(pos)
    assert l_mask == pytest.approx(l_sub * scale, rel=1e-12)
    np.testing.assert_allclose(g_mask, g_sub * scale, rtol=1e-10, atol=1e-16)


# ------------------------------------------------------------ Adam and schedule
def test_adam_first_step_closed_form():
    rng = np.random.default_rng(12)
    p0 = rng.standard_normal(100)
    g = rng.standard_normal(100)
    g[:5] = 0.0
    p = p0.copy(); m = np.zeros(100); v = np.zeros(100)
    O.adam(p, g, m, v, lr=1e-2, step=1)
    np.testing.assert_allclose(p, p0 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-17)
    np.testing.assert_array_equal(p[:5], p0[:5])


def test_adam_matches_torch_optimizer():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    p0 = rng.standard_normal(257)
    tp = torch.nn.Parameter(torch.tensor(p0, dtype=torch.float64))
    opt = torch.optim.Adam([tp], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    p = p0.copy(); m = np.zeros_like(p); v = np.zeros_like(p)
    for step in range(1, 8):
        g = rng.standard_normal(257)
        tp.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        O.adam(p, g.copy(), m, v, lr=3e-3, step=step)
    np.testing.assert_allclose(p, tp.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_lr_schedule_endpoints():
    assert O.lr_at(1, 1000, 5000) == 1e-2
    assert O.lr_at(1000, 1000, 5000) == 1e-2
    assert O.lr_at(3000, 1000, 5000) == pytest.approx(1e-3, rel=1e-12)
    assert O.lr_at(5000, 1000, 5000) == pytest.approx(1e-4, rel=1e-12)
    assert O.lr_at(9000, 1000, 5000) == pytest.approx(1e-4, rel=1e-12)


# ------------------------------------------------------------ positional code (grid-free models)
def _pe_cfg(width=16, **kw):
    base = dict(n_levels=0, log2_T=17, n_features=2, base_res=16.0,
                per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=0, extra_bands=0,
                width=width, n_hidden=3, n_out=3, aabb_min=(0.0, 0.0, 0.0),
                aabb_max=(10.0, 4.0, 10.0), pos_bands=8)
    base.update(kw)
    return O.make_config(**base)


def test_table1_memory_grid_free_rows():
    """Half-precision parameter bytes of the grid-free networks reproduce the
    first three memory entries of Table 1, which pins the input width (67)."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "table1_memory_pe.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for width, mb, digits in rows:
        c = _pe_cfg(int(width))
        assert O.input_dim(c) == 67
        assert O.n_grid_values(c) == 0
        nbytes = 2 * O.n_params(c)
        assert round(nbytes / 1e6, int(digits)) == pytest.approx(float(mb)), (width, nbytes)
    # the alternatives named in the fixture do not fit the width-64 row
    for din in (64, 51):
        nbytes = 2 * (64 * din + 2 * 64 * 64 + 3 * 64)
        assert round(nbytes / 1e6, 2) != 0.03


def test_positional_code_closed_form():
    """At u = 1/2 and u = 1/4 on every axis, sin and cos of 2^k pi u take
    exact values; the code is [u, per band three sines then three cosines]
    followed by the SH of the normal."""
    c = _pe_cfg()
    lo, hi = np.array([0.0, 0.0, 0.0]), np.array([10.0, 4.0, 10.0])
    params = np.zeros(O.n_params(c))
    for frac in (0.5, 0.25):
        pos = (lo + frac * (hi - lo)).astype(np.float32)[None]
        nrm = np.array([[0.0, 0.0, 1.0]], np.float32)
        _, _, fl, x0 = O.query(c, params, pos, nrm, want_x0=True)
        assert fl[0] == 0
        x0 = x0[0]
        np.testing.assert_allclose(x0[:3], frac, rtol=0, atol=1e-15)
        for k in range(8):
            # angle 2^k pi frac: multiples of pi/2 for frac = 1/2, pi/4 for 1/4
            q = (2 ** k) * frac * 2          # angle in units of pi/2
            if frac == 0.5:
                s = [0.0, 1.0, 0.0, -1.0][int(q) % 4]
                co = [1.0, 0.0, -1.0, 0.0][int(q) % 4]
            else:
                if k == 0:
                    s = co = math.sqrt(0.5)   # pi/4
                else:
                    s = [0.0, 1.0, 0.0, -1.0][int(q) % 4]
                    co = [1.0, 0.0, -1.0, 0.0][int(q) % 4]
            np.testing.assert_allclose(x0[3 + 6 * k: 6 + 6 * k], s, atol=1e-12)
            np.testing.assert_allclose(x0[6 + 6 * k: 9 + 6 * k], co, atol=1e-12)
        # SH of +z: Y00, Y1-1 = 0, Y10 = sqrt(3/(4 pi)), ...
        np.testing.assert_allclose(x0[51], 0.5 / math.sqrt(math.pi), atol=1e-15)
        np.testing.assert_allclose(x0[53], math.sqrt(3.0 / (4 * math.pi)), atol=1e-15)


def test_positional_code_outside_box_clamps_and_flags():
    c = _pe_cfg()
    params = np.zeros(O.n_params(c))
    pos = np.array([[-1.0, 2.0, 11.0], [5.0, 2.0, 5.0]], np.float32)
    nrm = np.array([[0.0, 1.0, 0.0]] * 2, np.float32)
    _, _, fl, x0 = O.query(c, params, pos, nrm, want_x0=True)
    assert fl.tolist() == [1, 0]
    np.testing.assert_allclose(x0[0, :3], [0.0, 0.5, 1.0], atol=1e-15)
    np.testing.assert_allclose(x0[1, :3], [0.5, 0.5, 0.5], atol=1e-15)


def test_positional_code_pairs_on_unit_circle():
    """Every (sin, cos) pair lies on the unit circle, and band k + 1 follows
    band k by the double-angle formulas."""
    c = _pe_cfg()
    rng = np.random.default_rng(11)
    pos = (rng.random((64, 3)) * [10.0, 4.0, 10.0]).astype(np.float32)
    nrm = rng.normal(size=(64, 3)).astype(np.float32)
    _, _, _, x0 = O.query(c, np.zeros(O.n_params(c)), pos, nrm, want_x0=True)
    s = np.stack([x0[:, 3 + 6 * k: 6 + 6 * k] for k in range(8)], 1)
    co = np.stack([x0[:, 6 + 6 * k: 9 + 6 * k] for k in range(8)], 1)
    np.testing.assert_allclose(s ** 2 + co ** 2, 1.0, atol=1e-14)
    np.testing.assert_allclose(s[:, 1:], 2 * s[:, :-1] * co[:, :-1], atol=1e-12)
    np.testing.assert_allclose(co[:, 1:], 1 - 2 * s[:, :-1] ** 2, atol=1e-12)
    # band 0 recovers u: u = atan2(sin, cos) / pi on [0, 1]
    np.testing.assert_allclose(np.arctan2(s[:, 0], co[:, 0]) / np.pi, x0[:, :3], atol=1e-12)


def test_grid_free_mlp_matches_numpy():
    """The grid-free network is the plain matrix chain on the code."""
    c = _pe_cfg(32)
    rng = np.random.default_rng(12)
    params = make_params(0, O.mat_shapes(c), 5, 0.0, 0.0).astype(np.float64)
    pos = (rng.random((50, 3)) * [10.0, 4.0, 10.0]).astype(np.float32)
    nrm = rng.normal(size=(50, 3)).astype(np.float32)
    E, _, _, x0 = O.query(c, params, pos, nrm, want_x0=True)
    mats = O.split_params(c, params)[1:]
    h = x0
    for W in mats[:-1]:
        h = np.maximum(h @ W.T, 0.0)
    np.testing.assert_allclose(E, h @ mats[-1].T, rtol=1e-12, atol=1e-14)


def test_corners_many_equals_brute_force():
    """The batched corner indices (used for the GPU's bit-exact index check)
    against the per-point routine and a brute-force Python formula: cell
    floor((p - lo) N / (hi - lo)) clamped to N - 1, dense x + (N+1)(y +
    (N+1) z) or the 32-bit XOR hash of the primes 1, 2654435761, 805459861
    masked to T - 1; room box (dense and hashed levels) and T = 2^19."""
    for name in ("room_1080p", "room_4k_6d"):
        c = O.config_from_workload(get_workload(name))
        tab = O.level_table(c)
        lo = np.array(c.aabb_min[:3]); hi = np.array(c.aabb_max[:3])
        rng = np.random.default_rng(17)
        pts = rng.uniform(lo - 0.5, hi + 0.5, size=(300, 3)).astype(np.float32)
        pts[:4] = [lo, hi, [hi[0], lo[1], hi[2]], (lo + hi) / 2]
        many = O.corners_many(c, pts)
        T = 1 << c.log2_T
        for q, p in enumerate(pts):
            idx, _ = O.corners(c, p)
            np.testing.assert_array_equal(many[q], idx)
            pc = np.clip(p.astype(np.float64), lo, hi)
            for l in (0, 3, 4, 9, 15):
                N = int(tab["res"][l])
                s = (pc - lo) * N / (hi - lo)
                i = np.minimum(np.floor(s).astype(np.int64), N - 1)
                for k in range(8):
                    v = [int(i[a]) + ((k >> a) & 1) for a in range(3)]
                    if tab["dense"][l]:
                        want = v[0] + (N + 1) * (v[1] + (N + 1) * v[2])
                    else:
                        h = ((v[0] * 1) ^ (v[1] * 2654435761) ^ (v[2] * 805459861)) & 0xFFFFFFFF
                        want = h & (T - 1)
                    assert many[q, l, k] == want, (name, q, l, k)


def test_four_feature_levels_are_two_two_feature_grids():
    """Four features per entry (Table 1's grid networks, Sec. 4.1): each
    level's four interpolated features equal those of two-feature grids on the
    same levels that hold the entries' first and second feature pairs."""
    kw = dict(n_levels=4, log2_T=10, base_res=4.0, per_level_scale=math.sqrt(2.0),
              width=16, n_hidden=2)
    c4, c2 = _cfg(n_features=4, **kw), _cfg(n_features=2, **kw)
    rng = np.random.default_rng(44)
    g4 = rng.uniform(-1, 1, (O.n_grid_values(c4) // 4, 4))
    m4 = np.zeros(O.n_params(c4) - g4.size)
    m2 = np.zeros(O.n_params(c2) - g4.size // 2)
    pos = rng.uniform(-0.1, 1.1, (500, 3)).astype(np.float32)
    nrm = rng.normal(size=(500, 3)).astype(np.float32)
    _, _, fl4, x4 = O.query(c4, np.concatenate([g4.ravel(), m4]), pos, nrm, want_x0=True)
    halves = []
    for h in range(2):
        p2 = np.concatenate([np.ascontiguousarray(g4[:, 2 * h:2 * h + 2]).ravel(), m2])
        _, _, fl2, x2 = O.query(c2, p2, pos, nrm, want_x0=True)
        assert (fl2 == fl4).all()
        halves.append(x2)
    L = kw["n_levels"]
    assert x4.shape[1] == 4 * L + 16 and halves[0].shape[1] == 2 * L + 16
    for l in range(L):
        np.testing.assert_array_equal(x4[:, 4 * l:4 * l + 2], halves[0][:, 2 * l:2 * l + 2])
        np.testing.assert_array_equal(x4[:, 4 * l + 2:4 * l + 4], halves[1][:, 2 * l:2 * l + 2])
    np.testing.assert_array_equal(x4[:, 4 * L:], halves[0][:, 2 * L:])
