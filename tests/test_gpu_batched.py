"""Many frames in one launch, the Monte Carlo fallback, graph replay and the
launch autotuner, through the C interface on the GPU.

Per pixel the batched launch does the same arithmetic as a launch of that
frame alone, so batched outputs must equal single-frame outputs bit for bit;
both are held to the oracle's bars (FP16/BF16: per-frame relative L2 2e-3
against the oracle on the same rounded parameters).  Fallback pixels carry
the Monte Carlo estimate of Eq. 1 keyed by (frame << 28) | pixel, checked
against the oracle's estimator on the same random streams."""
import numpy as np
import pytest
import torch

import oracle as O
from niv_synth import (get_workload, make_params, make_room, make_room_gbuffer,
                       make_room_gbuffers)
from niv_metrics import rel_l2, term_scale, assert_flags, sign_margin

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _round(p, prec):
    if prec == "fp16":
        return p.astype(np.float16).astype(np.float64)
    if prec == "bf16":
        return torch.from_numpy(p).to(torch.bfloat16).to(torch.float64).numpy()
    return p.astype(np.float64)


def _models(w, oc, k, seed0):
    return [make_params(O.n_grid_values(oc), O.mat_shapes(oc), seed0 + i, *w.grid_init)
            for i in range(k)]


def _room_points(n, seed, lo=(0.0, 0.0, 0.0), hi=(10.0, 4.0, 10.0)):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    v = rng.standard_normal((n, 3))
    nrm = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    alb = rng.uniform(0.2, 0.8, size=(n, 3)).astype(np.float32)
    mask = (rng.uniform(size=n) > 0.05).astype(np.uint8)
    return pos, nrm, alb, mask


class Frames:
    """Device buffers of several frames and their niv_frame records."""

    def __init__(self, m, data, prepared, which, extras=None, in_flags=None, scenes=None):
        self.m = m
        self.dev = []
        self.frames = []
        self.outs = []
        for i, (pos, nrm, alb, mask) in enumerate(data):
            d = dict(pos=_t(pos), nrm=_t(nrm), alb=_t(alb), mask=_t(mask),
                     inf=_t(in_flags[i]) if in_flags is not None else None)
            f, outs = m.frame(d["pos"], d["nrm"], prepared[which[i]], albedo=d["alb"],
                              mask=d["mask"], extra=extras[i] if extras else (),
                              in_flags=d["inf"],
                              scene=scenes[i] if scenes is not None else None)
            self.dev.append(d)
            self.frames.append(f)
            self.outs.append(outs)

    def host(self):
        torch.cuda.synchronize()
        return [tuple(o.cpu().numpy() for o in outs) for outs in self.outs]


def _single(m, data, prepared, which, prec, extras=None):
    res = []
    for i in range(len(data)):
        fr = Frames(m, [data[i]], prepared, [which[i]], [extras[i]] if extras else None)
        m.query_frames(fr.frames, prec)
        res.append(fr.host()[0])
    return res


def _oracle_frame(oc, params, prec, pos, nrm, alb, mask, extra=()):
    pr = _round(params, prec)
    ex = None
    if oc.n_extra:
        ex = np.tile(np.float32(extra[:oc.n_extra]), (len(pos), 1))
    E, L, fl, x0 = O.query(oc, pr, pos, nrm, extra=ex, albedo=alb, mask=mask, want_x0=True)
    sc = term_scale(O.split_params(oc, pr)[1:], x0)
    return E, L, fl, sc


COUNTS = [0, 1, 63, 64, 65, 4097, 3000, 129]


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_uneven_frames_one_launch(prec):
    """Empty, single-pixel, ragged and multi-tile frames over three models
    in one launch: equal to single-frame launches, and to the oracle."""
    from paper_2602_12949_amd import NIV
    w = get_workload("room_1080p")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 3, 700)
    prepared = [m.prepare(_t(p), prec) for p in params]
    data = [_room_points(n, 100 + i) for i, n in enumerate(COUNTS)]
    which = [i % 3 for i in range(len(COUNTS))]
    print(f"{prec}: {len(COUNTS)} frames {COUNTS}", flush=True)
    fr = Frames(m, data, prepared, which)
    m.query_frames(fr.frames, prec)
    got = fr.host()
    ref = _single(m, data, prepared, which, prec)
    for i, n in enumerate(COUNTS):
        for a, b in zip(got[i], ref[i]):
            np.testing.assert_array_equal(a, b)
        if n == 0:
            continue
        pos, nrm, alb, mask = data[i]
        E_ref, L_ref, fl_ref, sc = _oracle_frame(oc, params[which[i]], prec, pos, nrm, alb, mask)
        E, L, fl = got[i]
        ok = mask.astype(bool)
        assert (E[~ok] == 0).all()
        assert_flags(fl, fl_ref, E_ref, sign_margin(prec, E_ref, sc))
        if not ok.any():
            continue
        if prec == "fp32":
            err = np.max(np.abs(E[ok] - E_ref[ok]) / np.maximum(np.abs(E_ref[ok]), sc[ok]))
            assert err <= 1e-5, (i, err)
        elif n >= 64:   # relative L2 over a handful of pixels is noise
            err = rel_l2(E[ok], E_ref[ok])
            assert err <= 2e-3, (i, err)


def test_more_frames_than_one_launch_holds():
    """20 frames go out as two launches (16 + 4) with identical results."""
    from paper_2602_12949_amd import NIV
    w = get_workload("room_1080p")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 2, 800)
    prepared = [m.prepare(_t(p), "fp16") for p in params]
    counts = [(37 * i * i + 11) % 900 for i in range(20)]
    data = [_room_points(n, 200 + i) for i, n in enumerate(counts)]
    which = [i % 2 for i in range(20)]
    fr = Frames(m, data, prepared, which)
    m.query_frames(fr.frames, "fp16")
    got = fr.host()
    ref = _single(m, data, prepared, which, "fp16")
    for i in range(20):
        for a, b in zip(got[i], ref[i]):
            np.testing.assert_array_equal(a, b)


def test_scene_variable_per_frame_bf16():
    """The 6-D field (position, normal, scene variable t) at BF16: three
    frames with t = 0, 0.37, 1 and one model in one launch."""
    from paper_2602_12949_amd import NIV
    w = get_workload("room_4k_6d")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 1, w.param_seed)
    prepared = [m.prepare(_t(params[0]), "bf16")]
    counts = [3000, 1777, 4096]
    data = [_room_points(n, 300 + i) for i, n in enumerate(counts)]
    extras = [(t,) for t in w.extra_values]
    fr = Frames(m, data, prepared, [0, 0, 0], extras=extras)
    m.query_frames(fr.frames, "bf16")
    got = fr.host()
    ref = _single(m, data, prepared, [0, 0, 0], "bf16", extras=extras)
    for i in range(3):
        for a, b in zip(got[i], ref[i]):
            np.testing.assert_array_equal(a, b)
        pos, nrm, alb, mask = data[i]
        E_ref, L_ref, fl_ref, sc = _oracle_frame(oc, params[0], "bf16", pos, nrm, alb, mask,
                                                 extra=extras[i])
        E, L, fl = got[i]
        ok = mask.astype(bool)
        err = rel_l2(E[ok], E_ref[ok])
        print(f"  t={extras[i][0]}: rel-L2 {err:.2e}", flush=True)
        assert err <= 2e-3
        assert_flags(fl, fl_ref, E_ref, sign_margin("bf16", E_ref, sc))
    # the scene variable matters: frames at different t differ
    fr2 = Frames(m, [data[0]], prepared, [0], extras=[(0.5,)])
    m.query_frames(fr2.frames, "bf16")
    assert not np.array_equal(fr2.host()[0][0], got[0][0])


# ------------------------------------------------------------ Monte Carlo fallback
@pytest.fixture(scope="module")
def small_rooms():
    """Two small G-buffers of two rooms with planted special pixels."""
    out = []
    for k, seed in enumerate((2001, 4003)):
        room, g = make_room_gbuffer(seed, 96 + 32 * k, 54 + 18 * k)
        pos = g["pos"].reshape(-1, 3).copy()
        nrm = g["nrm"].reshape(-1, 3).copy()
        alb = g["albedo"].reshape(-1, 3).copy()
        mask = g["mask"].reshape(-1).copy()
        rng = np.random.default_rng(seed)
        valid = np.nonzero(mask)[0]
        pick = rng.choice(valid, size=40, replace=False)
        pos[pick[:10], 1] = 4.25          # above the ceiling: outside the volume
        pos[pick[10]] = [np.nan, 1.0, 1.0]  # non-finite input: no estimate at all
        inf = np.zeros(len(pos), np.uint8)
        inf[pick[11:30]] = 1              # caller's requests
        inf[np.nonzero(mask == 0)[0][:3]] = 1  # requests on sky pixels are ignored
        out.append((room, (pos, nrm, alb, mask), inf))
    return out


def _fallback_run(m, rooms, prepared, prec, fb, ws):
    from paper_2602_12949_amd import McScene
    scenes = [McScene(r[0]["prims"]) for r in rooms]
    fr = Frames(m, [r[1] for r in rooms], prepared, list(range(len(rooms))),
                in_flags=[r[2] for r in rooms], scenes=scenes)
    m.query_fallback(fr.frames, prec, fb, ws)
    return fr, scenes


def test_fallback_pixels_get_monte_carlo_estimates(small_rooms):
    from paper_2602_12949_amd import NIV, niv as N
    w = get_workload("batched_8_rooms")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 2, w.param_seed)
    prepared = [m.prepare(_t(p), "fp16") for p in params]
    fb = NIV.fallback(flag_mask=N.FLAG_OUTSIDE | N.FLAG_BAD_OUTPUT, spp=32, bounces=2,
                      mc_flags=N.MC_NEE, seed=91)
    ws = m.fallback_workspace(4096)
    fr, scenes = _fallback_run(m, small_rooms, prepared, "fp16", fb, ws)
    got = fr.host()
    count = int(ws[:4].view(torch.int32).item())
    plain = _single(m, [r[1] for r in small_rooms], prepared, [0, 1], "fp16")
    total = 0
    for fi, (room, (pos, nrm, alb, mask), inf) in enumerate(small_rooms):
        E, L, fl = got[fi]
        E0, L0, fl0 = plain[fi]
        on = mask.astype(bool)
        want = on & ((fl0 & 2) == 0) & (((fl0 & (N.FLAG_OUTSIDE | N.FLAG_BAD_OUTPUT)) != 0) | (inf != 0))
        taken = (fl & 8) != 0
        np.testing.assert_array_equal(taken, want)
        assert want.sum() >= 25
        np.testing.assert_array_equal(fl & 0xF7, fl0)
        # untouched pixels keep the network's answer
        np.testing.assert_array_equal(E[~taken], E0[~taken])
        np.testing.assert_array_equal(L[~taken], L0[~taken])
        idx = np.nonzero(taken)[0]
        total += idx.size
        ids = (np.uint64(fi) << np.uint64(28)) | idx.astype(np.uint64)
        Eo, varo, _, _ = O.mc_irradiance(room["prims"], pos[idx], nrm[idx], 32, 2, O.MC_NEE, 91,
                                         point_id=ids)
        scale = np.maximum(np.abs(Eo).max(1, keepdims=True), 1e-3)
        close = (np.abs(E[idx] - Eo) / scale).max(1) <= 1e-4
        print(f"  frame {fi}: {idx.size} fallback pixels, {close.mean():.3f} agree to 1e-4",
              flush=True)
        assert close.mean() >= 0.99
        d = ~close
        if d.any():
            z = (E[idx][d] - Eo[d]) / np.sqrt(2 * varo[d] + 1e-30)
            assert np.abs(z).max() < 6
        np.testing.assert_allclose(L[idx], alb[idx] * E[idx] / np.float32(np.pi), rtol=1e-6,
                                   atol=1e-7)
    assert count == total


def test_fallback_list_capacity(small_rooms):
    """A list shorter than the flagged set: the first `cap` entries are
    estimated, the rest keep the network's answer."""
    from paper_2602_12949_amd import NIV, niv as N
    w = get_workload("batched_8_rooms")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 2, w.param_seed)
    prepared = [m.prepare(_t(p), "fp16") for p in params]
    fb = NIV.fallback(flag_mask=N.FLAG_OUTSIDE, spp=8, bounces=1, seed=5)
    ws = m.fallback_workspace(7)
    fr, _ = _fallback_run(m, small_rooms, prepared, "fp16", fb, ws)
    got = fr.host()
    count = int(ws[:4].view(torch.int32).item())
    taken = sum(int(((g[2] & 8) != 0).sum()) for g in got)
    assert count > 7 and taken == 7


def test_fallback_argument_checks(small_rooms):
    from paper_2602_12949_amd import NIV, niv as N
    w = get_workload("batched_8_rooms")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    prepared = [m.prepare(_t(p), "fp16") for p in _models(w, oc, 2, 1)]
    ws = m.fallback_workspace(16)
    for bad in (NIV.fallback(spp=0), NIV.fallback(flag_mask=2), NIV.fallback(bounces=-1),
                NIV.fallback(mc_flags=N.MC_NEE | N.MC_EMIT_ON_HIT)):
        with pytest.raises(N.NivError):
            _fallback_run(m, small_rooms, prepared, "fp16", bad, ws)
    with pytest.raises(N.NivError):
        _fallback_run(m, small_rooms, prepared, "fp16", NIV.fallback(), ws[:200])


# ------------------------------------------------------------ graph and autotuner
def test_graph_replays_follow_new_inputs(small_rooms):
    """A captured query + fallback replayed three times, with new G-buffer
    contents and unrelated eager work between replays: every replay equals
    an eager call on the same inputs."""
    from paper_2602_12949_amd import NIV, niv as N
    w = get_workload("batched_8_rooms")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 2, w.param_seed)
    prepared = [m.prepare(_t(p), "fp16") for p in params]
    fb = NIV.fallback(flag_mask=N.FLAG_OUTSIDE | N.FLAG_BAD_OUTPUT, spp=8, bounces=2, seed=3)
    ws = m.fallback_workspace(4096)
    fr, scenes = _fallback_run(m, small_rooms, prepared, "fp16", fb, ws)
    g = m.capture(fr.frames, "fp16", fb, ws)
    rng = np.random.default_rng(12)
    for rep in range(3):
        # new contents in the same buffers
        for d, (room, (pos, nrm, alb, mask), inf) in zip(fr.dev, small_rooms):
            jit = rng.uniform(-0.05, 0.05, size=pos.shape).astype(np.float32)
            d["pos"].copy_(torch.from_numpy(np.where(np.isfinite(pos), pos + jit, pos)))
        for outs in fr.outs:
            for o in outs:
                o.fill_(0xff if o.dtype == torch.uint8 else float("nan"))
        junk = torch.randn(1 << 20, device=DEV)
        junk = (junk * 2).sum()  # eager work between replays
        g.launch()
        torch.cuda.synchronize()
        replay = fr.host()
        for outs in fr.outs:
            for o in outs:
                o.zero_()
        m.query_fallback(fr.frames, "fp16", fb, ws)
        eager = fr.host()
        for a3, b3 in zip(replay, eager):
            for a, b in zip(a3, b3):
                np.testing.assert_array_equal(a, b)
        print(f"  replay {rep}: ok", flush=True)
    del g


def test_autotune_keeps_results():
    from paper_2602_12949_amd import NIV
    w = get_workload("room_1080p")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 1, 900)
    prepared = [m.prepare(_t(params[0]), "fp16")]
    data = [_room_points(200000, 7), _room_points(70001, 8)]
    fr = Frames(m, data, prepared, [0, 0])
    m.query_frames(fr.frames, "fp16")
    before = fr.host()
    r = m.autotune(fr.frames, "fp16")
    print(f"  candidates {r['candidates']}; chosen {r['block']}x{r['blocks_per_cu']} "
          f"order {r['xcd_order']}", flush=True)
    assert len(r["candidates"]) == 12
    assert (r["block"], r["blocks_per_cu"], r["xcd_order"]) in [c[:3] for c in r["candidates"]]
    assert r["ms"] == min(c[3] for c in r["candidates"])
    for outs in fr.outs:
        for o in outs:
            o.zero_()
    m.query_frames(fr.frames, "fp16")
    after = fr.host()
    for a3, b3 in zip(before, after):
        for a, b in zip(a3, b3):
            np.testing.assert_array_equal(a, b)
    # every shape gives the same pixels
    from paper_2602_12949_amd import niv as N
    for blk, per_cu, order, _ in r["candidates"][::3]:
        m.set_tune("fp16", blk, per_cu, order)
        for outs in fr.outs:
            for o in outs:
                o.zero_()
        m.query_frames(fr.frames, "fp16")
        for a3, b3 in zip(before, fr.host()):
            for a, b in zip(a3, b3):
                np.testing.assert_array_equal(a, b)
    with pytest.raises(N.NivError):
        m.set_tune("fp16", 384, 0, 0)


# ------------------------------------------------------------ full-size batch
@pytest.fixture(scope="module")
def eight_rooms():
    w = get_workload("batched_8_rooms")
    return w, make_room_gbuffers(w.scene_seeds, w.frames)


def test_batched_8_rooms_full_size(eight_rooms):
    """The eight uneven G-buffers (16.3 M pixels) with eight models in one
    launch; 4096 sampled pixels per frame against the oracle, two frames
    in full against their single-frame launches."""
    from paper_2602_12949_amd import NIV
    w, rooms = eight_rooms
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 8, w.param_seed)
    prepared = [m.prepare(_t(p), "fp16") for p in params]
    data = [(g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3), g["albedo"].reshape(-1, 3),
             g["mask"].reshape(-1)) for _, g in rooms]
    fr = Frames(m, data, prepared, list(range(8)))
    m.query_frames(fr.frames, "fp16")
    got = fr.host()
    print(f"  {sum(len(d[0]) for d in data)} pixels", flush=True)
    rng = np.random.default_rng(4242)
    for i, (pos, nrm, alb, mask) in enumerate(data):
        s = rng.choice(len(pos), size=4096, replace=False)
        E_ref, L_ref, fl_ref, sc = _oracle_frame(oc, params[i], "fp16", pos[s], nrm[s], alb[s],
                                                 mask[s])
        E, L, fl = (x[s] for x in got[i])
        ok = mask[s].astype(bool)
        err = rel_l2(E[ok], E_ref[ok])
        print(f"  frame {i} {w.frames[i]}: sampled rel-L2 {err:.2e}", flush=True)
        assert err <= 2e-3
        assert_flags(fl, fl_ref, E_ref, sign_margin("fp16", E_ref, sc))
    for i in (0, 7):
        ref = _single(m, [data[i]], [prepared[i]], [0], "fp16")[0]
        for a, b in zip(got[i], ref):
            np.testing.assert_array_equal(a, b)


# ------------------------------------------------------------ 4K scene-variable field
@pytest.fixture(scope="module")
def room_4k(workload_gbuffer):
    return get_workload("room_4k_6d"), workload_gbuffer("room_4k_6d")


def test_room_4k_6d_full_size(room_4k):
    """The 3840x2160 G-buffer with two displaced icospheres (general
    normals), three frames t = 0, 0.37, 1 in one BF16 launch: every covered
    pixel of every frame against the oracle (per-frame relative L2), and the
    flags of 8192 sampled pixels per frame, mesh pixels included."""
    from paper_2602_12949_amd import NIV
    w, (room, g) = room_4k
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = _models(w, oc, 1, w.param_seed)
    prepared = [m.prepare(_t(params[0]), "bf16")]
    d = (g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3), g["albedo"].reshape(-1, 3),
         g["mask"].reshape(-1))
    extras = [(t,) for t in w.extra_values]
    fr = Frames(m, [d, d, d], prepared, [0, 0, 0], extras=extras)
    m.query_frames(fr.frames, "bf16")
    got = fr.host()
    rng = np.random.default_rng(99)
    on_mesh = np.nonzero(g["prim"].reshape(-1) >= len(room["prims_no_lights"]))[0]
    s = np.concatenate([rng.choice(len(d[0]), 8192 - 1024, replace=False),
                        rng.choice(on_mesh, 1024, replace=False)])
    pr = _round(params[0], "bf16")
    ok_all = d[3].astype(bool)
    for i, ex in enumerate(extras):
        # whole frame
        exa = np.full((len(d[0]), 1), np.float32(ex[0]))
        E_all, _, _ = O.query(oc, pr, d[0], d[1], extra=exa, albedo=d[2], mask=d[3])
        err_all = rel_l2(got[i][0][ok_all], E_all[ok_all])
        del E_all
        # flags on a sample (their margin needs the terms of the oracle's pass)
        E_ref, L_ref, fl_ref, sc = _oracle_frame(oc, params[0], "bf16", d[0][s], d[1][s], d[2][s],
                                                 d[3][s], extra=ex)
        E, L, fl = (x[s] for x in got[i])
        ok = d[3][s].astype(bool)
        err = rel_l2(E[ok], E_ref[ok])
        print(f"  t={ex[0]}: whole-frame rel-L2 {err_all:.2e} over {int(ok_all.sum())} pixels, "
              f"sampled {err:.2e}", flush=True)
        assert err_all <= 2e-3 and err <= 2e-3
        assert_flags(fl, fl_ref, E_ref, sign_margin("bf16", E_ref, sc))


def test_fallback_in_a_scene_that_moves(small_rooms):
    """Frames of a field with a scene variable (Sec. 6) whose scene moves
    with it: the Monte Carlo fallback estimates each flagged pixel in the
    scene at its frame's variable (extra value 0)."""
    from paper_2602_12949_amd import NIV, McScene, niv as N
    from niv_synth import room_motion
    w = get_workload("room_train_6d")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), w.param_seed, -0.5, 0.5)
    prepared = [m.prepare(_t(params), "fp16")]
    room, data, inf = small_rooms[0]
    motion = room_motion(room)
    scene = McScene(room["prims"])
    scene.set_motion(motion)
    ts = (0.25, 0.75)
    fr = Frames(m, [data, data], prepared, [0, 0], extras=[(ts[0],), (ts[1],)],
                in_flags=[inf, inf], scenes=[scene, scene])
    fb = NIV.fallback(flag_mask=N.FLAG_OUTSIDE, spp=32, bounces=2, mc_flags=N.MC_NEE, seed=93)
    ws = m.fallback_workspace(4096)
    m.query_fallback(fr.frames, "fp16", fb, ws)
    got = fr.host()
    pos, nrm, alb, mask = data
    for fi in range(2):
        E, L, fl = got[fi]
        idx = np.nonzero((fl & 8) != 0)[0]
        assert idx.size >= 20
        ids = (np.uint64(fi) << np.uint64(28)) | idx.astype(np.uint64)
        Eo, varo, _, _ = O.mc_irradiance(room["prims"], pos[idx], nrm[idx], 32, 2, O.MC_NEE, 93,
                                         point_id=ids, motion=motion,
                                         t=np.full(idx.size, ts[fi], np.float32))
        scale = np.maximum(np.abs(Eo).max(1, keepdims=True), 1e-3)
        close = (np.abs(E[idx] - Eo) / scale).max(1) <= 1e-4
        print(f"  frame {fi} (t = {ts[fi]}): {idx.size} fallback pixels, {close.mean():.3f} agree",
              flush=True)
        assert close.mean() >= 0.99
