"""End-to-end baking on the GPU (Sec. 4.5): points from the sampler, targets
from the Monte Carlo estimator, Adam steps on Eq. 3, then the trained
network is judged against a high-sample Monte Carlo reference on held-out
points, and compared with Monte Carlo at equal query time."""
import time

import numpy as np
import pytest
import torch

import oracle as O
from niv_synth import get_workload, make_params, make_room, room_motion

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_bake_room_learns_irradiance():
    from paper_2602_12949_amd import NIV
    from paper_2602_12949_amd.bake import Baker, held_out_error
    w = get_workload("room_train")
    oc = O.config_from_workload(w)
    room = make_room(w.scene_seeds[0])
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), w.param_seed, *w.grid_init)
    niv = NIV(w.model_dict())
    p = torch.from_numpy(params).to(DEV)
    steps, batch = 400, 1 << 15
    bk = Baker(niv, p, room["prims"], room["lo"], room["hi"], prec="fp16", batch=batch, spp=64,
               bounces=3, seed=7)
    # held-out points and a 1024-spp reference
    from paper_2602_12949_amd import McScene
    # held out: 2^16 points against 4096-spp Monte Carlo
    hx, hn = bk.scene.sample_points(room["lo"], room["hi"], 1 << 16, 13107, seed=3003)
    Eh, varh, bfh, vh = bk.scene.irradiance(hx, hn, 4096, 3, 1, 99)
    Eh = Eh.float()
    err0 = held_out_error(niv, bk.trainer.model, "fp16", hx, hn, Eh, vh)
    t0 = time.perf_counter()
    bk.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err1 = held_out_error(niv, bk.trainer.model, "fp16", hx, hn, Eh, vh)
    print(f"  {steps} steps x {batch} in {dt:.1f}s; held-out rel-L2 {err0[0]:.3f} -> {err1[0]:.3f}, "
          f"relMSE {err0[1]:.3e} -> {err1[1]:.3e}; valid {float(vh.float().mean()):.3f}", flush=True)
    assert err1[0] < 0.5 * err0[0]
    assert err1[0] < 0.35

    # Monte Carlo at (at least) the network's query time: 1 sample per point
    t1 = time.perf_counter()
    for _ in range(10):
        niv.query(hx, hn, bk.trainer.model, "fp16")
    torch.cuda.synchronize()
    t_niv = (time.perf_counter() - t1) / 10
    t2 = time.perf_counter()
    E1, _, _, _ = bk.scene.irradiance(hx, hn, 1, 3, 1, 12345)
    torch.cuda.synchronize()
    t_mc = time.perf_counter() - t2
    v = vh.bool()
    mc_err = float(torch.linalg.norm((E1.float() - Eh)[v]) / torch.linalg.norm(Eh[v]))
    print(f"  equal-time: network {t_niv * 1e3:.3f} ms rel-L2 {err1[0]:.3f}; "
          f"MC 1 spp {t_mc * 1e3:.3f} ms rel-L2 {mc_err:.3f}", flush=True)
    assert err1[0] < mc_err


def test_bake_field_with_scene_variable():
    """Sec. 6: the room's lights slide and a box moves with t; every training
    point draws its own t.  The trained field is judged at t = 0, 0.5 and 1
    against 1024-spp Monte Carlo in the scene at that t, and it must follow
    t: against the t = 1 reference the query at t = 1 beats the query at
    t = 0, and the other way round (a network that ignored t would tie)."""
    from paper_2602_12949_amd import NIV
    from paper_2602_12949_amd.bake import Baker, held_out_error
    w = get_workload("room_train_6d")
    oc = O.config_from_workload(w)
    room = make_room(w.scene_seeds[0])
    motion = room_motion(room)
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), w.param_seed, *w.grid_init)
    niv = NIV(w.model_dict())
    steps, batch = 4000, 1 << 15
    bk = Baker(niv, torch.from_numpy(params).to(DEV), room["prims"], room["lo"], room["hi"],
               prec="fp16", batch=batch, spp=64, bounces=3, seed=8, motion=motion)
    hx, hn = bk.scene.sample_points(room["lo"], room["hi"], 4096, 819, seed=6003)
    refs = {}
    for tv in w.extra_values:
        tt = torch.full((4096,), tv, dtype=torch.float32, device=DEV)
        E, _, _, v = bk.scene.irradiance(hx, hn, 1024, 3, 1, 199, t=tt)
        refs[tv] = (E.float(), v)
    err0 = {tv: held_out_error(niv, bk.trainer.model, "fp16", hx, hn, *refs[tv], extra=(tv,))[0]
            for tv in w.extra_values}
    v = (refs[0.0][1].bool() & refs[1.0][1].bool())
    signal = float(torch.linalg.norm((refs[1.0][0] - refs[0.0][0])[v]) / torch.linalg.norm(refs[1.0][0][v]))
    print(f"  references at t = 0 and t = 1 differ by rel-L2 {signal:.3f}", flush=True)
    t0 = time.perf_counter()
    bk.run(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err1 = {tv: held_out_error(niv, bk.trainer.model, "fp16", hx, hn, *refs[tv], extra=(tv,))[0]
            for tv in w.extra_values}
    cross = held_out_error(niv, bk.trainer.model, "fp16", hx, hn, *refs[1.0], extra=(0.0,))[0]
    cross0 = held_out_error(niv, bk.trainer.model, "fp16", hx, hn, *refs[0.0], extra=(1.0,))[0]
    print(f"  {steps} steps x {batch} in {dt:.1f}s; held-out rel-L2 by t: "
          + ", ".join(f"t={tv}: {err0[tv]:.3f} -> {err1[tv]:.3f}" for tv in w.extra_values)
          + f"; t=1 reference with the t=0 query {cross:.3f}, t=0 reference with the t=1 query "
            f"{cross0:.3f}", flush=True)
    for tv in w.extra_values:
        assert err1[tv] < 0.5 * err0[tv]
        assert err1[tv] < 0.4
    assert err1[1.0] < 0.95 * cross and err1[0.0] < 0.95 * cross0
