"""Dynamic ambient occlusion (Sec. 4.4) on the GPU against the FP64 oracle,
through the C interface.  Both sides draw the same directions (the pixel's
stream 2), so the hit counts agree ray for ray except where FP32 and FP64
decide a ray that grazes a triangle edge, the radius or the horizon
differently: per pixel at most one ray, over all pixels at most 0.5 % of
them.  E and L are scaled by exactly the returned visibility."""
import numpy as np
import pytest
import torch

import oracle as O
from niv_synth import get_workload, make_workload_gbuffer, workload_meshes, mesh_triangles

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
RADIUS, EPS = 1.0, 1e-3


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _ao(tris):
    from paper_2602_12949_amd.niv import DynamicAO
    return DynamicAO(tris)


def _near(pos, mask, meshes, reach):
    """Valid pixels whose position lies within `reach` of a mesh's bound."""
    near = np.zeros(len(pos), bool)
    for m in meshes:
        d = np.linalg.norm(pos - m["center"][None, :], axis=1)
        near |= d <= m["radius"] + reach
    return np.flatnonzero(near & (mask != 0))


def _compare(vis_gpu, vis_orc, rays):
    hg = np.rint((1.0 - vis_gpu.astype(np.float64)) * rays).astype(np.int64)
    ho = np.rint((1.0 - vis_orc) * rays).astype(np.int64)
    diff = np.abs(hg - ho)
    print(f"[ao] {len(hg)} pixels, occluded {np.mean(ho > 0):.3f}, differing {np.mean(diff > 0):.5f}, "
          f"max |dhits| {diff.max() if len(diff) else 0}", flush=True)
    assert diff.max(initial=0) <= 1
    assert np.mean(diff > 0) <= 0.005
    return hg, ho


@pytest.fixture(scope="module")
def scene():
    w = get_workload("room_4k_6d")
    _, g = make_workload_gbuffer(w, size=(480, 270))
    meshes = workload_meshes(w)
    return w, g, meshes, mesh_triangles(meshes)


@pytest.mark.parametrize("rays", [16, 64])
def test_mesh_pixels_match_oracle(scene, rays):
    w, g, meshes, tris = scene
    pos = g["pos"].reshape(-1, 3).astype(np.float32)
    nrm = g["nrm"].reshape(-1, 3).astype(np.float32)
    mask = g["mask"].reshape(-1).astype(np.uint8)
    ao = _ao(tris)
    nodes, depth = ao.info()
    assert depth <= 20 and nodes >= len(tris) // 4 - 1   # inner nodes; leaves hold <= 4
    vis = ao.apply(_t(pos), _t(nrm), rays, RADIUS, EPS, seed=17, mask=_t(mask)).cpu().numpy()
    # masked pixels and pixels out of reach are visible
    assert np.all(vis[mask == 0] == 1.0)
    near = _near(pos, mask, meshes, RADIUS + 0.1)
    far = np.setdiff1d(np.flatnonzero(mask), near)
    assert np.all(vis[far] == 1.0)
    sel = near[:: max(1, len(near) // 1500)]
    ref = O.dynamic_ao(tris, pos[sel], nrm[sel], rays, RADIUS, EPS, 17, point_id=sel)
    hg, ho = _compare(vis[sel], ref, rays)
    assert np.mean(ho > 0) > 0.3            # the sample does test occlusion
    # a few far pixels through the oracle too (no triangle within reach)
    fs = far[:: max(1, len(far) // 50)]
    assert np.all(O.dynamic_ao(tris, pos[fs], nrm[fs], 8, RADIUS, EPS, 17, point_id=fs) == 1.0)


def test_scales_E_and_L_in_place(scene):
    w, g, meshes, tris = scene
    pos = _t(g["pos"].reshape(-1, 3).astype(np.float32))
    nrm = _t(g["nrm"].reshape(-1, 3).astype(np.float32))
    mask = g["mask"].reshape(-1).astype(np.uint8)
    n = pos.shape[0]
    rng = np.random.default_rng(3)
    E0 = rng.uniform(0.1, 2.0, (n, 3)).astype(np.float32)
    L0 = rng.uniform(0.1, 2.0, (n, 3)).astype(np.float32)
    E, L = _t(E0), _t(L0)
    ao = _ao(tris)
    vis = ao.apply(pos, nrm, 16, RADIUS, EPS, seed=5, mask=_t(mask), E=E, L=L).cpu().numpy()
    assert np.array_equal(E.cpu().numpy(), E0 * vis[:, None])
    assert np.array_equal(L.cpu().numpy(), L0 * vis[:, None])
    m0 = mask == 0
    assert np.array_equal(E.cpu().numpy()[m0], E0[m0])
    assert (vis < 1).sum() > 100


def test_closed_form_quad_and_special_cases():
    """One pixel under a parallel quad: the GPU's count agrees with the
    oracle's, whose estimate the CPU tests pin to the form factor."""
    quad = np.array([[[-1, -1, 1], [1, -1, 1], [1, 1, 1]],
                     [[-1, -1, 1], [1, 1, 1], [-1, 1, 1]]], np.float32)
    pos = np.zeros((4, 3), np.float32)
    nrm = np.array([[0, 0, 1], [0, 0, 1], [0, 0, -1], [0, 0, 0]], np.float32)
    pos[1] = [0, 0, np.nan]
    ao = _ao(quad)
    vis = ao.apply(_t(pos), _t(nrm), 4096, 10.0, 0.0, seed=9).cpu().numpy()
    ref = O.dynamic_ao(quad, pos[:1], nrm[:1], 4096, 10.0, 0.0, 9)
    _compare(vis[:1], ref, 4096)
    assert vis[1] == 1.0 and vis[2] == 1.0 and vis[3] == 1.0   # non-finite, facing away, zero normal
    # out of reach
    assert ao.apply(_t(pos[:1]), _t(nrm[:1]), 256, 0.9, 0.0, seed=9).item() == 1.0


def test_no_triangles_and_empty_frames():
    ao = _ao(np.zeros((0, 3, 3), np.float32))
    pos = _t(np.random.default_rng(1).uniform(0, 1, (1000, 3)).astype(np.float32))
    nrm = _t(np.tile(np.array([[0, 1, 0]], np.float32), (1000, 1)))
    E0 = torch.ones((1000, 3), device=DEV)
    E = E0.clone()
    vis = ao.apply(pos, nrm, 8, 1.0, 0.0, seed=1, E=E)
    assert torch.all(vis == 1.0) and torch.equal(E, E0)
    assert ao.apply(pos[:0], nrm[:0], 8, 1.0, 0.0, seed=1).numel() == 0


@pytest.mark.parametrize("rays", [16])
def test_room_4k_6d_full_size(rays, workload_gbuffer):
    """The 3840x2160 frame of the field workload: sampled pixels near the
    meshes against the oracle, at the bench's settings."""
    w = get_workload("room_4k_6d")
    _, g = workload_gbuffer("room_4k_6d")
    meshes = workload_meshes(w)
    tris = mesh_triangles(meshes)
    pos = g["pos"].reshape(-1, 3).astype(np.float32)
    nrm = g["nrm"].reshape(-1, 3).astype(np.float32)
    mask = g["mask"].reshape(-1).astype(np.uint8)
    vis = _ao(tris).apply(_t(pos), _t(nrm), rays, RADIUS, EPS, seed=23, mask=_t(mask)).cpu().numpy()
    near = _near(pos, mask, meshes, RADIUS + 0.1)
    sel = near[:: max(1, len(near) // 800)]
    ref = O.dynamic_ao(tris, pos[sel], nrm[sel], rays, RADIUS, EPS, 23, point_id=sel)
    _compare(vis[sel], ref, rays)
    far = np.setdiff1d(np.flatnonzero(mask), near)
    assert np.all(vis[far] == 1.0)
