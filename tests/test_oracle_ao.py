"""Pins of the dynamic ambient-occlusion oracle (Sec. 4.4): closed forms of
the cosine-weighted obstruction of a hemisphere, the radius cut-off and the
exact special cases."""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def quad(x0, x1, y0, y1, z, flip=False):
    """Two triangles covering [x0,x1] x [y0,y1] at height z."""
    a, b, c, d = (x0, y0, z), (x1, y0, z), (x1, y1, z), (x0, y1, z)
    t = [[a, b, c], [a, c, d]]
    if flip:
        t = [[a, c, b], [a, d, c]]
    return np.array(t, np.float32)


def corner_form_factor(a, b, c):
    """Point to a parallel a x b rectangle at distance c whose corner lies on
    the point's normal (the classic differential-area form factor)."""
    X, Y = a / c, b / c
    sx, sy = math.sqrt(1 + X * X), math.sqrt(1 + Y * Y)
    return (X / sx * math.atan(Y / sx) + Y / sy * math.atan(X / sy)) / (2 * math.pi)


ORIGIN = np.zeros((1, 3), np.float32)
UP = np.array([[0, 0, 1]], np.float32)


def test_corner_form_factor_limits():
    # the whole plane above is the whole hemisphere: four corners of 1/4
    assert 4 * corner_form_factor(1e7, 1e7, 1.0) == pytest.approx(1.0, abs=1e-6)
    # a small rectangle: F ~ A cos^2 / (pi c^2) for a point straight below
    a = 1e-3
    assert 4 * corner_form_factor(a / 2, a / 2, 1.0) == pytest.approx(a * a / math.pi, rel=1e-5)


@pytest.mark.parametrize("a,b,c", [(2.0, 2.0, 1.0), (1.0, 3.0, 0.5), (0.6, 0.6, 1.0)])
def test_parallel_rectangle_matches_form_factor(a, b, c):
    rays = 40000
    tris = quad(-a / 2, a / 2, -b / 2, b / 2, c)
    vis = oracle.dynamic_ao(tris, ORIGIN, UP, rays, 1e3, 0.0, seed=11)[0]
    F = 4 * corner_form_factor(a / 2, b / 2, c)
    sigma = math.sqrt(F * (1 - F) / rays)
    assert abs((1 - vis) - F) < 5 * sigma + 1e-12


def test_radius_keeps_the_cone_it_reaches():
    # plane at height 2, radius 2.5: hits need cos(theta) >= 0.8, a cone whose
    # cosine-weighted share of the hemisphere is sin^2 = 0.36 (the 4 x 4 quad
    # covers the cone's footprint of radius 1.5)
    rays = 40000
    tris = quad(-2, 2, -2, 2, 2.0)
    vis = oracle.dynamic_ao(tris, ORIGIN, UP, rays, 2.5, 0.0, seed=5)[0]
    sigma = math.sqrt(0.36 * 0.64 / rays)
    assert abs((1 - vis) - 0.36) < 5 * sigma
    # out of reach entirely: exactly visible
    assert oracle.dynamic_ao(tris, ORIGIN, UP, 512, 1.5, 0.0, seed=5)[0] == 1.0


def test_exact_special_cases():
    # geometry behind the tangent plane never occludes
    assert oracle.dynamic_ao(quad(-5, 5, -5, 5, -1.0), ORIGIN, UP, 512, 1e3, 0.0, seed=1)[0] == 1.0
    # a plane above that reaches every direction but the last 1e-8 of the
    # cosine-weighted hemisphere occludes all rays
    assert oracle.dynamic_ao(quad(-1e4, 1e4, -1e4, 1e4, 1.0), ORIGIN, UP, 512, 1e6, 0.0, seed=1)[0] == 0.0
    # the offset along the normal lifts the origin over a coplanar triangle
    assert oracle.dynamic_ao(quad(-1, 1, -1, 1, 0.0), ORIGIN, UP, 512, 1e3, 1e-4, seed=1)[0] == 1.0
    # no triangles: visible
    empty = np.zeros((0, 3, 3), np.float32)
    assert oracle.dynamic_ao(empty, ORIGIN, UP, 64, 1.0, 0.0, seed=1)[0] == 1.0


def test_two_sided_and_keyed_by_point():
    tris = quad(-0.7, 0.4, -0.3, 0.9, 0.8)
    pos = np.repeat(ORIGIN, 3, 0)
    nrm = np.array([[0, 0, 1], [0, 0, 2], [0, 0, 1]], np.float32)   # the normal is normalised
    v = oracle.dynamic_ao(tris, pos, nrm, 4096, 1e3, 0.0, seed=3, point_id=[7, 7, 8])
    vf = oracle.dynamic_ao(quad(-0.7, 0.4, -0.3, 0.9, 0.8, flip=True), pos, nrm, 4096, 1e3, 0.0,
                           seed=3, point_id=[7, 7, 8])
    assert np.array_equal(v, vf)          # winding does not matter
    assert v[0] == v[1]                   # same stream, same estimate
    assert v[0] != v[2]                   # another point id draws other directions
