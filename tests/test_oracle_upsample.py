"""Pins of the oracle's half-resolution rendering (joint bilateral
upsampling, Sec. 4.4) against closed forms and limiting cases.  CPU only."""
import math

import numpy as np
import pytest

import oracle as O


def _cfg():
    return O.make_config(n_levels=0, log2_T=17, n_features=2, base_res=16.0,
                         per_level_scale=math.sqrt(2.0), sh_bands=4, n_extra=0,
                         extra_bands=0, width=16, n_hidden=3, n_out=3,
                         aabb_min=(-100.0, -100.0, -100.0), aabb_max=(100.0, 100.0, 100.0),
                         pos_bands=8)


def _plane(W, H, spacing=0.01, normal=(0.0, 0.0, 1.0)):
    """A fronto-parallel plane z = 0 seen pixel by pixel."""
    X, Y = np.meshgrid(np.arange(W), np.arange(H))
    pos = np.stack([X * spacing, Y * spacing, np.zeros_like(X, float)], -1).reshape(-1, 3)
    nrm = np.tile(np.array(normal, np.float32), (W * H, 1))
    return pos.astype(np.float32), nrm


def test_constant_field_is_reproduced():
    W, H = 17, 12
    pos, nrm = _plane(W, H)
    hE = np.tile([0.3, 1.7, 2.5], (((H + 1) // 2) * ((W + 1) // 2), 1))
    E, L, fl = O.upsample(_cfg(), W, H, pos, nrm, hE)
    np.testing.assert_allclose(E, np.tile([0.3, 1.7, 2.5], (W * H, 1)), rtol=1e-14)
    assert (fl == 0).all()


def test_linear_field_on_a_plane_with_flat_guides():
    """Guides that do not discriminate (one normal, sigma_pos huge): in the
    interior the symmetric spatial window reproduces a linear field at the
    pixel exactly, odd pixels included."""
    W, H = 20, 14
    pos, nrm = _plane(W, H)
    hw, hh = W // 2, H // 2
    y, x = np.meshgrid(np.arange(hh), np.arange(hw), indexing="ij")
    a, b, c = 0.5, 0.07, -0.03
    hE = np.stack([a + b * 2 * x + c * 2 * y] * 3, -1).reshape(-1, 3)
    E, _, _ = O.upsample(_cfg(), W, H, pos, nrm, hE, sigma_pos=1e6)
    Y, X = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    want = (a + b * X + c * Y).reshape(-1)
    inner = ((X >= 2) & (X <= W - 3) & (Y >= 2) & (Y <= H - 3)).reshape(-1)
    np.testing.assert_allclose(E[inner, 0], want[inner], rtol=0, atol=1e-12)


def test_step_edge_keeps_each_side():
    """Left half faces +z, right half faces +x: a pixel never takes samples
    of the other side (normal term zero), so each side keeps its value."""
    W, H = 16, 10
    pos, nrm = _plane(W, H)
    X = np.tile(np.arange(W), H)
    nrm[X >= 7] = [1.0, 0.0, 0.0]
    hw, hh = W // 2, H // 2
    hx = np.tile(np.arange(hw), hh)
    hE = np.where((2 * hx >= 7)[:, None], 5.0, 1.0) * np.ones((hh * hw, 3))
    E, _, fl = O.upsample(_cfg(), W, H, pos, nrm, hE)
    np.testing.assert_allclose(E[X < 7], 1.0, rtol=1e-14)
    np.testing.assert_allclose(E[X >= 7], 5.0, rtol=1e-14)
    assert (fl == 0).all()


def test_nearest_neighbour_limit():
    """With a tiny spatial sigma each even-even pixel takes its own sample,
    and the weights stay finite (log-domain normalisation)."""
    W, H = 10, 8
    pos, nrm = _plane(W, H)
    rng = np.random.default_rng(3)
    hE = rng.random(((H // 2) * (W // 2), 3))
    E, _, fl = O.upsample(_cfg(), W, H, pos, nrm, hE, sigma_px=1e-3)
    ee = O.half_samples(W, H, np.arange(W * H))[0]
    np.testing.assert_allclose(E[ee], hE, rtol=1e-14)
    assert np.isfinite(E).all() and (fl == 0).all()


def test_weights_match_formula_at_one_pixel():
    """One odd-odd pixel with two usable samples of different normals and
    depths: the average equals the three-factor weights written out."""
    W, H = 4, 4
    pos, nrm = _plane(W, H, spacing=0.05)
    nrm[2] = [0.0, 0.6, 0.8]          # sample (1, 0) tilted
    pos[2 * W + 2, 2] = 0.07          # sample (1, 1) displaced in depth
    hE = np.array([[1.0] * 3, [2.0] * 3, [3.0] * 3, [4.0] * 3])
    E, _, _ = O.upsample(_cfg(), W, H, pos, nrm, hE, sigma_px=1.0, sigma_pos=0.1, normal_power=8)
    i = 1 * W + 1                      # pixel (1, 1): samples at (0,0), (2,0), (0,2), (2,2)
    ws = []
    for (sx, sy), e in zip([(0, 0), (2, 0), (0, 2), (2, 2)], [1.0, 2.0, 3.0, 4.0]):
        s = sy * W + sx
        n1 = nrm[i].astype(float) / np.linalg.norm(nrm[i].astype(float))
        n2 = nrm[s].astype(float) / np.linalg.norm(nrm[s].astype(float))
        w = math.exp(-2 / 2.0) * float(n1 @ n2) ** 8 * \
            math.exp(-float(np.sum((pos[i].astype(float) - pos[s]) ** 2)) / (2 * 0.01))
        ws.append((w, e))
    want = sum(w * e for w, e in ws) / sum(w for w, _ in ws)
    assert E[i, 0] == pytest.approx(want, rel=1e-12)


def test_fallback_and_empty_window_flags():
    W, H = 6, 6
    pos, nrm = _plane(W, H)
    mask = np.ones(W * H, np.uint8)
    # pixel (3, 3): every window sample faces away -> nearest sample, flag 32
    nrm[3 * W + 3] = [0.0, 0.0, -1.0]
    hE = np.arange((H // 2) * (W // 2) * 3, dtype=float).reshape(-1, 3)
    # pixel (5, 5) region: mask out samples (4,4) and its window -> no sample, flag 64
    for (x, y) in [(4, 4)]:
        mask[y * W + x] = 0
    E, _, fl = O.upsample(_cfg(), W, H, pos, nrm, hE, mask=mask)
    # nearest usable sample of (3,3): (2,2) (d2 = 2, first in row-major order) -> half index (1,1)
    assert fl[3 * W + 3] == 32
    np.testing.assert_allclose(E[3 * W + 3], hE[1 * (W // 2) + 1])
    assert fl[5 * W + 5] == 64 and (E[5 * W + 5] == 0).all()
    assert fl[4 * W + 4] == 0 and (E[4 * W + 4] == 0).all()   # masked pixel


def test_bad_inputs_and_outside_flags():
    W, H = 6, 4
    pos, nrm = _plane(W, H)
    pos[1] = [np.nan, 0.0, 0.0]
    nrm[7] = [0.0, 0.0, 0.0]
    pos[9] = [500.0, 0.0, 0.0]
    hE = np.ones(((H // 2) * (W // 2), 3))
    E, L, fl = O.upsample(_cfg(), W, H, pos, nrm, hE, albedo=np.full((W * H, 3), 0.5))
    assert fl[1] == 2 and fl[7] == 2 and (fl[9] & 1)
    assert (E[[1, 7]] == 0).all()
    np.testing.assert_allclose(L[0], 0.5 * E[0] / np.pi)


def test_depth_edge_keeps_each_side():
    """Two parallel planes 1 m apart, same normal: the position term (sigma
    0.1) leaves each side with its own value to within exp(-50)."""
    W, H = 16, 10
    pos, nrm = _plane(W, H)
    X = np.tile(np.arange(W), H)
    pos[X >= 9, 2] = 1.0
    hw, hh = W // 2, H // 2
    hx = np.tile(np.arange(hw), hh)
    hE = np.where((2 * hx >= 9)[:, None], 5.0, 1.0) * np.ones((hh * hw, 3))
    E, _, _ = O.upsample(_cfg(), W, H, pos, nrm, hE, sigma_pos=0.1)
    np.testing.assert_allclose(E[X < 9], 1.0, rtol=1e-15, atol=1e-18)
    np.testing.assert_allclose(E[X >= 9], 5.0, rtol=1e-15, atol=1e-18)
