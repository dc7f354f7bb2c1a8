"""Benchmark of the Neural Irradiance Volume hot path on one MI355X.

Headline workload (room_1080p): one 1920x1080 G-buffer of a 10x4x10 m room
with 32 boxes (seeded, ~5 % sky pixels masked), model of 16 hash-grid levels
(T = 2^17, F = 2), 16 SH of the normal, MLP 48-64-64-64-3.  A step is one
fused query of the whole frame (G-buffer read, encoding, MLP, E and
albedo * E / pi written), inputs resident in HBM.  The headline is the
FP16-MFMA path; FP32 and BF16 are timed on the same inputs and weights, each
with its error against the FP64 oracle.

Also measured, as extra fields of the same JSON line:
  train       room_train: niv_train_step at B = 2^18 (FP16), the Monte Carlo
              targets (256 spp, 3 bounces, NEE) and the sampler, and the whole
              baking step (samples/s); the FP16 gradient of that batch against
              the FP64 oracle per parameter block; then a model baked on the
              GPU judged against 4096-spp Monte Carlo on 2^16 held-out points;
  batched     batched_8_rooms: eight uneven G-buffers (16.3 M pixels), eight
              models, one persistent launch replayed from a HIP graph, after
              the autotuner; with and without the Monte Carlo fallback (64 spp);
  field_4k    room_4k_6d: 3840x2160 G-buffer with two displaced icospheres,
              scene variable t in {0, 0.37, 1}, MLP 64-128^4-3, BF16; then the
              dynamic ambient occlusion pass over the frame (Sec. 4.4: the
              icospheres' 40,960 triangles, 16 rays per pixel within 1 m);
  table1      room_1080p_pe16/32/64 and room_1080p_g2/4/6/8: the same 1080p
              G-buffer under the networks of Table 1: grid-free (eight-band
              positional code of x, three hidden layers of width 16, 32 or
              64) and grid (2, 4, 6 or 8 levels of four features, T = 2^17,
              three hidden layers of width 64), FP16;
  half        half-resolution rendering of the 1080p G-buffer (Table 1's
              "half" column): the query at a quarter of the pixels, joint
              bilateral upsampling with the G-buffer as guide, full-resolution
              albedo; for the room model and every network of Table 1, FP16.

Kernel times come from HIP events recorded on the stream the kernels are
launched on (torch's current stream).  Prints one JSON line on stdout;
progress goes to stderr.

`--profile CASE` runs only that case's kernel a few times (for rocprofv3
counter and trace runs): query_fp16, query_fp32, query_bf16, field_4k,
train_step, mc, pe16, pe32, pe64, g2, g4, g6, g8, half, gather (the gather-rate probes), copy (a 1 GiB device copy that calibrates
the HBM byte counters).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp32": 157.3}
# Vector ALU issue rate: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# (non-packed) operation per lane per clock.
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# Algorithmic vector work per query of a 16-level grid: ~640 integer
# operations for corner indices and hashing, ~1000 FP32 operations for cell
# coordinates, weights and trilinear blends.
ALU_OPS_PER_QUERY = 1640
# Compulsory HBM bytes per pixel: pos, nrm, albedo (3 x 12), mask 1, E and L
# (2 x 12), flags 1.
HBM_BYTES_PER_PX = 12 * 3 + 1 + 12 * 2 + 1


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mlp_flops(cfg):
    pb = cfg.get("pos_bands", 0)
    din = cfg["n_levels"] * cfg["n_features"] + (3 + 6 * pb if pb > 0 else 0) + \
        cfg["sh_bands"] ** 2 + cfg["n_extra"] * 2 * cfg["extra_bands"]
    W = cfg["width"]
    macs = W * din + (cfg["n_hidden"] - 1) * W * W + cfg["n_out"] * W
    return 2 * macs


def term_scale(mats, x0):
    """Magnitude of the terms summed into each output: |W_H|..|W_0||x0| along
    the ReLU units active in the FP64 pass (the scale FP32 rounding is
    relative to)."""
    h = x0.T
    a = np.abs(x0).T
    for Wm in mats[:-1]:
        z = Wm @ h
        act = z > 0
        h = np.where(act, z, 0.0)
        a = (np.abs(Wm) @ a) * act
    return (np.abs(mats[-1]) @ a).T


def time_steps(fn, steps, warmup):
    """Per-step times (ms) from event pairs on the current stream, and the
    whole timed region (ms per step)."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    per = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(steps)])
    total = ev[0].elapsed_time(ev[-1]) / steps
    return total, per


def stats(total, per):
    return {"ms": total, "p10": float(np.percentile(per, 10)), "p50": float(np.median(per)),
            "p90": float(np.percentile(per, 90))}


def round_params(p, prec):
    import torch
    if prec == "fp16":
        return p.astype(np.float16).astype(np.float64)
    if prec == "bf16":
        return torch.from_numpy(p).to(torch.bfloat16).to(torch.float64).numpy()
    return p.astype(np.float64)


def kernel_source_hash():
    """Hash of the library sources and build flags: a counter summary taken
    from another build does not describe this one."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2602_12949_amd", "csrc")
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode() + f.read())
    with open(os.path.join(ROOT, "paper_2602_12949_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary, if it was taken from the current sources; else None."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"source hash: `([0-9a-f]+)`", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    m = re.search(r"\| " + re.escape(kernel_key) + r" \|[^\n]*\| ([0-9.eE+]+) \|\s*$", txt, re.M)
    return float(m.group(1)) if m else None


# ---------------------------------------------------------------- workloads
def setup_1080p(dev):
    import torch
    from niv_synth import get_workload, make_params, make_room_gbuffer
    from paper_2602_12949_amd import NIV
    w = get_workload("room_1080p")
    Wd, Ht = w.frames[0]
    log(f"[bench] G-buffer {Wd}x{Ht} seed {w.scene_seeds[0]}")
    # profiling runs start many processes: the G-buffer is kept in /tmp for them
    cache = os.path.join(os.environ.get("TMPDIR", "/tmp"),
                         f"niv_bench_room_1080p_{w.scene_seeds[0]}_{Wd}x{Ht}.npz")
    if os.path.exists(cache):
        with np.load(cache) as z:
            g = {k: z[k] for k in z.files}
    else:
        _, g = make_room_gbuffer(w.scene_seeds[0], Wd, Ht)
        try:
            np.savez(cache + ".tmp.npz", **{k: g[k] for k in ("pos", "nrm", "albedo", "mask")})
            os.replace(cache + ".tmp.npz", cache)
        except OSError:
            pass
    m = NIV(w.model_dict())
    params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    d = dict(pos=t(g["pos"]), nrm=t(g["nrm"]), alb=t(g["albedo"]), mask=t(g["mask"]),
             params=t(params))
    return w, g, m, params, d


def bench_1080p(args, dev, precs):
    import torch
    w, g, m, params, d = setup_1080p(dev)
    cfg = w.model_dict()
    Wd, Ht = w.frames[0]
    Q = Wd * Ht
    n_valid = int(g["mask"].sum())
    results, outputs = {}, {}
    for prec in precs:
        prepared = m.prepare(d["params"], prec)
        frame, outs = m.frame(d["pos"], d["nrm"], prepared, albedo=d["alb"], mask=d["mask"])
        if args.tune:
            b_, c_, x_ = (int(v) for v in args.tune.split(","))
            m.set_tune(prec, b_, c_, x_)
            tune = {"block": b_, "blocks_per_cu": c_, "xcd_order": x_, "candidates": "fixed (--tune)"}
        else:
            tune = m.autotune([frame], prec)
        log(f"[bench] room_1080p {prec} autotune: block {tune['block']} x {tune['blocks_per_cu']}"
            f" per CU, xcd order {tune['xcd_order']}: {tune['candidates']}")
        total, per = time_steps(lambda: m.query_frames([frame], prec), args.steps, args.warmup)
        graph = m.capture([frame], prec)
        gtotal, gper = time_steps(graph.launch, args.steps, args.warmup)
        torch.cuda.synchronize()
        outputs[prec] = outs[0].reshape(-1, 3).cpu().numpy().astype(np.float64)
        ms = min(total, gtotal)
        results[prec] = {"ms_per_frame": ms, "launch": stats(total, per),
                         "autotune": {k: tune[k] for k in ("block", "blocks_per_cu", "xcd_order")},
                         "graph": stats(gtotal, gper),
                         "queries_per_s": n_valid / (ms * 1e-3),
                         "mlp_tflops": mlp_flops(cfg) * n_valid / (ms * 1e-3) / 1e12,
                         "alu_tops": ALU_OPS_PER_QUERY * n_valid / (ms * 1e-3) / 1e12,
                         "hbm_compulsory_GBs": HBM_BYTES_PER_PX * Q / (ms * 1e-3) / 1e9}
        log(f"[bench] room_1080p {prec}: {ms:.4f} ms/frame (launch p50 {np.median(per):.4f}, "
            f"graph p50 {np.median(gper):.4f}), {n_valid / (ms * 1e-3) / 1e9:.3f} G queries/s")
        del graph
        # the encoding stage alone at the same launch shape: a floor for the query
        pframe, pouts = m.frame(d["pos"], d["nrm"], prepared, albedo=d["alb"], mask=d["mask"])
        etotal, eper = time_steps(lambda: m.probe_encode(pframe, prec), args.steps, args.warmup)
        results[prec]["encode_only"] = {**stats(etotal, eper), "frac_of_query": etotal / ms}
        log(f"[bench] room_1080p {prec}: encoding stage alone {etotal:.4f} ms ({etotal / ms:.2f} of the query)")
        del pframe, pouts
    return w, g, params, results, outputs, n_valid, Q


def errors_1080p(w, g, params, outputs):
    import oracle as O
    oc = O.config_from_workload(w)
    pos, nrm, mask = g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3), g["mask"].reshape(-1)
    ok = mask.astype(bool)
    E_master = None
    errors = {}
    for prec, E in outputs.items():
        pr = round_params(params, prec)
        ref, _, _, x0 = O.query(oc, pr, pos, nrm, mask=mask, want_x0=True)
        if prec == "fp32":
            E_master = ref
        a, b = E[ok], ref[ok]
        sc = term_scale(O.split_params(oc, pr)[1:], x0[ok])
        del x0
        floor = 1e-3 * np.abs(b).max()
        errors[prec] = {
            "max_rel_err": float(np.max(np.abs(a - b) / np.maximum(np.abs(b), sc))),
            "max_rel_err_floored_1e-3": float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))),
            "rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
            "vs": "FP64 oracle on the same rounded parameters, every valid pixel",
        }
        log(f"[bench] room_1080p {prec} error vs oracle: {errors[prec]}")
    if E_master is None:
        E_master, _, _ = O.query(oc, params.astype(np.float64), pos, nrm, mask=mask)
    for prec, E in outputs.items():
        if prec != "fp32":
            errors[prec]["rel_l2_vs_fp32_master"] = float(
                np.linalg.norm(E[ok] - E_master[ok]) / np.linalg.norm(E_master[ok]))
    return errors


def host_cpu():
    """Model and topology of the host CPU (lscpu), for the CPU baseline."""
    import subprocess
    info = {}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in ("Model name", "Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "CPU(s)", "CPU max MHz"):
                info[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    info["os_cpu_count"] = os.cpu_count()
    return info


def cpu_baseline_1080p(w, g, params):
    import oracle as O
    oc = O.config_from_workload(w)
    pos, nrm, mask = g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3), g["mask"].reshape(-1)
    n_valid = int(mask.sum())
    p64 = params.astype(np.float64)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    O.set_threads(cores)
    log(f"[bench] CPU oracle: 3 full frames on {cores} threads, 1/16 frame on 1 thread")
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        O.query(oc, p64, pos, nrm, mask=mask)
        runs.append(time.perf_counter() - t0)
    med = float(np.median(runs))
    O.set_threads(1)
    k = len(pos) // 16
    t0 = time.perf_counter()
    O.query(oc, p64, pos[:k], nrm[:k], mask=mask[:k])
    one = (time.perf_counter() - t0) * 16
    O.set_threads(cores)
    return {"value": med * 1e3, "unit": "ms/frame", "cores": cores, "kind": "oracle",
            "host_cpu": host_cpu(),
            "sample": "three full 1920x1080 frames of room_1080p (FP64 forward, OpenMP over "
                      "pixels), median; plus 1/16 of the frame on one thread, scaled",
            "queries_per_s": n_valid / med, "one_thread_ms_per_frame": one * 1e3,
            "runs_s": runs}


def gradient_check(w, m, params, x, n, E, valid, dev):
    """The FP16 gradient of one full batch (2^18 samples: coarse grid bins
    split over several accumulating workgroups) against the FP64 oracle on
    the FP16-rounded parameters, per parameter block."""
    import torch
    import oracle as O
    from paper_2602_12949_amd import Trainer
    tr = Trainer(m, torch.from_numpy(params).to(dev), "fp16", max_batch=len(x))
    loss = float(tr.backward(x, n, E, valid=valid).item())
    g = tr.grads.cpu().numpy().astype(np.float64)
    oc = O.config_from_workload(w)
    p16 = params.astype(np.float16).astype(np.float64)
    t0 = time.perf_counter()
    l_ref, g_ref = O.loss_grad(oc, p16, x.cpu().numpy(), n.cpu().numpy(), E.cpu().numpy(),
                               valid=valid.cpu().numpy())
    cs = time.perf_counter() - t0
    out = {"batch": len(x), "precision": "fp16", "loss_rel_err": abs(loss - l_ref) / abs(l_ref),
           "oracle_s": cs, "blocks": {}}
    k = 0
    names = ["grid"] + [f"W{i}" for i in range(len(O.mat_shapes(oc)))]
    sizes = [O.n_grid_values(oc)] + [o * i for o, i in O.mat_shapes(oc)]
    for name, sz in zip(names, sizes):
        a, b = g[k:k + sz], g_ref[k:k + sz]
        k += sz
        out["blocks"][name] = {"rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                               "max_over_max": float(np.abs(a - b).max() / np.abs(b).max())}
    log("[bench] FP16 gradient at 2^18 vs oracle: " +
        ", ".join(f"{k}: rel-L2 {v['rel_l2']:.2e}" for k, v in out["blocks"].items()) +
        f" (loss rel err {out['loss_rel_err']:.1e})")
    return out


def bench_train(args, dev):
    import torch
    from niv_synth import get_workload, make_params, make_room
    from paper_2602_12949_amd import NIV, McScene, Trainer
    from paper_2602_12949_amd.bake import lr_at
    w = get_workload("room_train")
    m = NIV(w.model_dict())
    B = w.n_queries
    params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
    p = torch.from_numpy(params).to(dev)
    room = make_room(w.scene_seeds[0])
    scene = McScene(room["prims"])
    tr = Trainer(m, p, "fp16", max_batch=B)
    lo, hi = w.aabb_min, w.aabb_max
    n_surf = int(round(0.2 * B))
    x, n = scene.sample_points(lo, hi, B, n_surf, seed=1, device=dev)
    E = torch.empty((B, 3), dtype=torch.float32, device=dev)
    valid = torch.empty(B, dtype=torch.uint8, device=dev)
    scene.targets(x, n, 256, 3, seed=2, out=(E, valid))
    steps = max(3, args.steps // 10)
    tt, tp = time_steps(lambda: tr.step(x, n, E, 1e-3, valid=valid), steps * 4, 3)
    st, sp = time_steps(lambda: scene.sample_points(lo, hi, B, n_surf, seed=3, out=(x, n)),
                        steps, 2)
    mt, mp = time_steps(lambda: scene.targets(x, n, 256, 3, seed=4, out=(E, valid)), 3, 1)
    state = {"k": 0}

    def whole():
        state["k"] += 1
        s = state["k"]
        scene.sample_points(lo, hi, B, n_surf, seed=(7 << 20) + s, out=(x, n))
        scene.targets(x, n, 256, 3, seed=(7 << 20) + s + (1 << 19), out=(E, valid))
        tr.step(x, n, E, lr_at(s, 4000), valid=valid)

    et, ep = time_steps(whole, 3, 1)
    # gather rates of the texture path (niv_probe_gather): n x 128 four-byte
    # gathers per pass; the random pattern is the training forward's ceiling
    from paper_2602_12949_amd.niv import probe_gather
    table = torch.ones(1 << 21, dtype=torch.int32, device=dev)       # 8 MiB
    sink = torch.empty(2048 * 256, dtype=torch.int32, device=dev)
    gather = {}
    for mode, what in ((0, "random words over 8 MiB (64 lines per instruction)"),
                       (1, "consecutive words (2 lines per instruction, L1)"),
                       (2, "quads share a line (16 lines per instruction, L1)"),
                       (3, "a line per lane (64 lines per instruction, L1)")):
        # 2^21 x 128 gathers per launch (launch overhead negligible), reported per 2^18 x 128
        gt, gp = time_steps(lambda: probe_gather(mode, 1 << 21, table, sink), 10, 3)
        gather[what] = {"us_per_2^18x128": gt * 1e3 / 8, "G_gathers_per_s": (1 << 21) * 128 / (gt * 1e-3) / 1e9}
    log(f"[bench] gather rates (per 2^18 x 128 gathers): " +
        ", ".join(f"{k.split(' (')[0]}: {v['us_per_2^18x128']:.1f} us" for k, v in gather.items()))
    res = {
        "workload": "room_train: B=2^18 points/step (80 % volume, 20 % surface), targets at "
                    "256 spp, 3 bounces, NEE to 2 rect lights; model of room_1080p, FP16",
        "batch": B,
        "train_step": {**stats(tt, tp), "samples_per_s": B / (tt * 1e-3)},
        "sampler": {**stats(st, sp), "points_per_s": B / (st * 1e-3)},
        "mc_targets": {**stats(mt, mp), "points_per_s": B / (mt * 1e-3),
                       "spp": 256, "bounces": 3},
        "bake_step": {**stats(et, ep), "samples_per_s": B / (et * 1e-3)},
        "valid_fraction": float(valid.float().mean().item()),
        "gather_rates": gather,
    }
    if not args.no_cpu:
        # the estimator's oracle on a bounded sample: 512 points x 4096 spp
        import oracle as O
        xs, ns = x[:512].cpu().numpy(), n[:512].cpu().numpy()
        t0 = time.perf_counter()
        O.mc_irradiance(room["prims"], xs, ns, 4096, 3, O.MC_NEE, 5)
        cs = time.perf_counter() - t0
        res["mc_cpu_oracle"] = {"points_per_s_at_256spp": 512 * 16 / cs, "s": cs,
                                "threads": os.cpu_count(),
                                "sample": "512 points x 4096 spp, 3 bounces, NEE, FP64 on the "
                                          "host threads (points/s scaled to 256 spp)"}
        log(f"[bench] MC oracle: 512 x 4096 spp in {cs:.2f} s")
        res["gradient_vs_oracle"] = gradient_check(w, m, params, x, n, E, valid, dev)
    log(f"[bench] train: step {tt:.3f} ms ({B / (tt * 1e-3) / 1e6:.2f} M samples/s), "
        f"MC {mt:.1f} ms ({B / (mt * 1e-3) / 1e6:.3f} M points/s), bake step {et:.1f} ms")
    return res


def bench_trained(args, dev, steps=4000, batch=1 << 18, spp=256, checkpoints=(500, 1000, 2000)):
    """The on-GPU-trained model judged by the estimator: bake room_train for
    `steps` steps of `batch` points at `spp` samples (the workload's stated
    configuration), then held-out relative L2 against 4096-spp Monte Carlo on
    2^16 points (also at the checkpoints), next to Monte Carlo at 1 sample
    per point at a similar cost."""
    import torch
    from niv_synth import get_workload, make_params, make_room
    from paper_2602_12949_amd import NIV
    from paper_2602_12949_amd.bake import Baker, held_out_error
    w = get_workload("room_train")
    room = make_room(w.scene_seeds[0])
    m = NIV(w.model_dict())
    params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
    bk = Baker(m, torch.from_numpy(params).to(dev), room["prims"], room["lo"], room["hi"],
               prec="fp16", batch=batch, spp=spp, bounces=3, seed=11)
    hx, hn = bk.scene.sample_points(room["lo"], room["hi"], 1 << 16, int(0.2 * (1 << 16)),
                                    seed=3003)
    Eh, _, _, vh = bk.scene.irradiance(hx, hn, 4096, 3, 1, 199)
    Eh = Eh.float()
    err0 = held_out_error(m, bk.trainer.model, "fp16", hx, hn, Eh, vh)
    curve = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(1, steps + 1):
        bk.step(s, steps)
        if s in checkpoints:
            e = held_out_error(m, bk.trainer.model, "fp16", hx, hn, Eh, vh)
            curve.append({"step": s, "held_out_rel_l2": e[0]})
            log(f"[bench] bake step {s}: held-out rel-L2 {e[0]:.3f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    err1 = held_out_error(m, bk.trainer.model, "fp16", hx, hn, Eh, vh)
    curve.append({"step": steps, "held_out_rel_l2": err1[0]})
    qt, _ = time_steps(lambda: m.query(hx, hn, bk.trainer.model, "fp16"), 20, 3)
    mt, _ = time_steps(lambda: bk.scene.irradiance(hx, hn, 1, 3, 1, 777), 5, 1)
    E1, _, _, _ = bk.scene.irradiance(hx, hn, 1, 3, 1, 778)
    v = vh.bool()
    mc1 = float(torch.linalg.norm((E1.float() - Eh)[v]) / torch.linalg.norm(Eh[v]))
    log(f"[bench] trained model: {steps} steps x {batch} at {spp} spp in {dt:.1f} s; held-out "
        f"rel-L2 {err0[0]:.3f} -> {err1[0]:.3f}; query {qt:.3f} ms vs 1-spp MC {mt:.3f} ms "
        f"(rel-L2 {mc1:.3f})")
    return {"workload": f"room_train baked {steps} steps x {batch} points at {spp} spp, 3 bounces "
                        "(FP16), judged on 2^16 held-out points against 4096-spp Monte Carlo",
            "bake_s": dt, "samples_per_s": steps * batch / dt,
            "held_out_rel_l2_before": err0[0], "held_out_rel_l2": err1[0],
            "held_out_relmse": err1[1], "curve": curve,
            "valid_fraction": float(vh.float().mean().item()),
            "query_ms": qt, "mc_1spp_ms": mt, "mc_1spp_rel_l2": mc1}


def bench_batched(args, dev):
    import torch
    from niv_synth import get_workload, make_params, make_room_gbuffers
    from paper_2602_12949_amd import NIV, McScene, niv as N
    w = get_workload("batched_8_rooms")
    log(f"[bench] batched_8_rooms: building 8 G-buffers")
    rooms = make_room_gbuffers(w.scene_seeds, w.frames)
    m = NIV(w.model_dict())
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    prepared, frames, keep = [], [], []
    rng = np.random.default_rng(4200)
    n_px = n_valid = 0
    for k, (room, g) in enumerate(rooms):
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed + k, *w.grid_init)
        pm = m.prepare(t(params), "fp16")
        mask = g["mask"].reshape(-1)
        inf = np.zeros(len(mask), np.uint8)
        vi = np.nonzero(mask)[0]
        inf[rng.choice(vi, size=int(0.005 * len(vi)), replace=False)] = 1
        sc = McScene(room["prims"])
        d = dict(pos=t(g["pos"]), nrm=t(g["nrm"]), alb=t(g["albedo"]), mask=t(g["mask"]),
                 inf=t(inf))
        f, outs = m.frame(d["pos"], d["nrm"], pm, albedo=d["alb"], mask=d["mask"],
                          in_flags=d["inf"], scene=sc)
        frames.append(f)
        keep.append((pm, d, outs, sc))
        n_px += len(mask)
        n_valid += len(vi)
    tune = m.autotune(frames, "fp16")
    log(f"[bench] autotune: {tune}")
    graph = m.capture(frames, "fp16")
    qt, qp = time_steps(graph.launch, args.steps, args.warmup)
    fb = m.fallback(flag_mask=N.FLAG_OUTSIDE | N.FLAG_BAD_OUTPUT, spp=64, bounces=3,
                    mc_flags=N.MC_NEE, seed=11)
    ws = m.fallback_workspace(1 << 20, device=dev)
    gfb = m.capture(frames, "fp16", fb, ws)
    ft, fp = time_steps(gfb.launch, max(5, args.steps // 10), 2)
    torch.cuda.synchronize()
    flagged = int(ws[:4].view(torch.int32).item())
    taken = sum(int(((o[2] & 8) != 0).sum().item()) for _, _, o, _ in keep)
    res = {
        "workload": "batched_8_rooms: 8 G-buffers 1280x720 .. 2560x1440 (8 rooms, 8 models), "
                    "one persistent launch from a HIP graph, FP16",
        "pixels": n_px, "valid_pixels": n_valid,
        "query": {**stats(qt, qp), "Mpix_per_s": n_px / (qt * 1e-3) / 1e6,
                  "queries_per_s": n_valid / (qt * 1e-3)},
        "with_fallback": {**stats(ft, fp), "flagged": flagged, "estimated": taken,
                          "spp": 64, "bounces": 3,
                          "triggers": "caller flags on 0.5 % of valid pixels, outside the "
                                      "volume, non-finite E"},
        "autotune": {"block": tune["block"], "blocks_per_cu": tune["blocks_per_cu"],
                     "xcd_order": tune["xcd_order"], "candidates": tune["candidates"]},
        "alu_frac": ALU_OPS_PER_QUERY * n_valid / (qt * 1e-3) / 1e12 / ALU_PEAK_TOPS,
    }
    # sampled error of the query-only outputs against the oracle, frame by frame
    import oracle as O
    oc = O.config_from_workload(w)
    graph.launch()
    torch.cuda.synchronize()
    worst = 0.0
    for k, (room, g) in enumerate(rooms):
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed + k, *w.grid_init)
        pos, nrm, mask = g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3), g["mask"].reshape(-1)
        s = rng.choice(len(pos), 4096, replace=False)
        s = s[mask[s] > 0]
        ref, _, _ = O.query(oc, round_params(params, "fp16"), pos[s], nrm[s])
        E = keep[k][2][0].reshape(-1, 3).cpu().numpy().astype(np.float64)[s]
        worst = max(worst, float(np.linalg.norm(E - ref) / np.linalg.norm(ref)))
    res["sampled_rel_l2_max_over_frames"] = worst
    log(f"[bench] batched: {qt:.3f} ms/batch ({n_px / (qt * 1e-3) / 1e6:.0f} M px/s), "
        f"with fallback {ft:.3f} ms ({flagged} flagged), sampled rel-L2 {worst:.2e}")
    del graph, gfb
    return res


def bench_field_4k(args, dev):
    import torch
    from niv_synth import get_workload, make_params, make_workload_gbuffer
    from paper_2602_12949_amd import NIV
    w = get_workload("room_4k_6d")
    log(f"[bench] room_4k_6d: building the 3840x2160 G-buffer with meshes")
    room, g = make_workload_gbuffer(w)
    m = NIV(w.model_dict())
    cfg = w.model_dict()
    params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pm = m.prepare(t(params), "bf16")
    d = dict(pos=t(g["pos"]), nrm=t(g["nrm"]), alb=t(g["albedo"]), mask=t(g["mask"]))
    mask = g["mask"].reshape(-1)
    n_valid = int(mask.sum())
    per_t = {}
    import oracle as O
    oc = O.config_from_workload(w)
    rng = np.random.default_rng(5)
    s = rng.choice(len(mask), 8192, replace=False)
    s = s[mask[s] > 0]
    pos, nrm = g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3)
    f, outs = m.frame(d["pos"], d["nrm"], pm, albedo=d["alb"], mask=d["mask"], extra=(0.37,))
    tune = m.autotune([f], "bf16")
    log(f"[bench] room_4k_6d autotune: block {tune['block']} x {tune['blocks_per_cu']} per CU, "
        f"xcd order {tune['xcd_order']}: {tune['candidates']}")
    for tv in w.extra_values:
        f, outs = m.frame(d["pos"], d["nrm"], pm, albedo=d["alb"], mask=d["mask"], extra=(tv,))
        graph = m.capture([f], "bf16")
        tt, tp = time_steps(graph.launch, args.steps, args.warmup)
        torch.cuda.synchronize()
        E = outs[0].reshape(-1, 3).cpu().numpy().astype(np.float64)[s]
        ex = np.full((len(s), 1), tv, np.float32)
        ref, _, _ = O.query(oc, round_params(params, "bf16"), pos[s], nrm[s], extra=ex)
        err = float(np.linalg.norm(E - ref) / np.linalg.norm(ref))
        per_t[str(tv)] = {**stats(tt, tp), "sampled_rel_l2": err}
        log(f"[bench] room_4k_6d t={tv}: {tt:.4f} ms/frame, sampled rel-L2 {err:.2e}")
        del graph
    ms = float(np.mean([v["ms"] for v in per_t.values()]))
    fl = mlp_flops(cfg) * n_valid
    ao = bench_dynamic_ao(args, w, g, d, outs, s_near_seed=7)
    return {
        "workload": "room_4k_6d: 3840x2160 G-buffer, room + 2 displaced icospheres "
                    "(20,480 triangles each), 16 levels T=2^19, MLP 64-128^4-3, BF16",
        "pixels": len(mask), "valid_pixels": n_valid, "ms_per_frame": ms, "per_t": per_t,
        "mlp_tflops": fl / (ms * 1e-3) / 1e12,
        "mfma_frac": fl / (ms * 1e-3) / 1e12 / MFMA_PEAK_TFLOPS["bf16"],
        "dynamic_ao": ao,
    }


AO_RAYS, AO_RADIUS, AO_EPS = 16, 1.0, 1e-3


def bench_dynamic_ao(args, w, g, d, outs, s_near_seed):
    """Dynamic ambient occlusion (Sec. 4.4) over the frame's query output:
    the two meshes' 40,960 triangles, 16 rays per pixel within 1 m; sampled
    pixels near the meshes checked ray for ray against the oracle."""
    import torch
    import oracle as O
    from niv_synth import workload_meshes, mesh_triangles
    from paper_2602_12949_amd.niv import DynamicAO
    meshes = workload_meshes(w)
    tris = mesh_triangles(meshes)
    ao = DynamicAO(tris)
    pos, nrm, mask = d["pos"].reshape(-1, 3), d["nrm"].reshape(-1, 3), d["mask"].reshape(-1)
    E, L = outs[0].reshape(-1, 3).clone(), outs[1].reshape(-1, 3).clone()
    vis = ao.apply(pos, nrm, AO_RAYS, AO_RADIUS, AO_EPS, 23, mask=mask)
    tt, tp = time_steps(lambda: ao.apply(pos, nrm, AO_RAYS, AO_RADIUS, AO_EPS, 23, mask=mask, E=E, L=L,
                                         vis=vis), args.steps, args.warmup)
    v = vis.cpu().numpy()
    P, N, M = g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3), g["mask"].reshape(-1)
    near = np.zeros(len(P), bool)
    for m in meshes:
        near |= np.linalg.norm(P - m["center"][None, :], axis=1) <= m["radius"] + AO_RADIUS + 0.1
    near = np.flatnonzero(near & (M > 0))
    rng = np.random.default_rng(s_near_seed)
    sel = np.sort(rng.choice(near, min(256, len(near)), replace=False))
    ref = O.dynamic_ao(tris, P[sel], N[sel], AO_RAYS, AO_RADIUS, AO_EPS, 23, point_id=sel)
    dh = np.abs(np.rint((1 - v[sel].astype(np.float64)) * AO_RAYS) - np.rint((1 - ref) * AO_RAYS))
    nodes, depth = ao.info()
    log(f"[bench] dynamic AO room_4k_6d: {tt:.4f} ms/frame ({AO_RAYS} rays, radius {AO_RADIUS} m, "
        f"{len(near) / len(P):.3f} of the pixels within reach, {np.mean(v < 1):.3f} occluded; "
        f"sampled pixels differing from the oracle {np.mean(dh > 0):.4f}, max |dhits| {dh.max():.0f})")
    return {**stats(tt, tp), "rays": AO_RAYS, "radius_m": AO_RADIUS, "triangles": int(len(tris)),
            "bvh_nodes": nodes, "bvh_depth": depth, "pixels_within_reach": float(len(near) / len(P)),
            "occluded_fraction": float(np.mean(v < 1)), "sampled_pixels_differing": float(np.mean(dh > 0)),
            "sampled_max_hit_difference": int(dh.max())}


# Table 1 (RTX 4090, full HD, half precision): full and half ms per frame
# of each network, for context (other hardware).
TABLE1_PAPER_MS = {"pe16": (0.19, 0.029), "pe32": (0.20, 0.031), "pe64": (0.25, 0.069),
                   "g2": (0.31, 0.088), "g4": (0.67, 0.18), "g6": (1.06, 0.26), "g8": (1.35, 0.37)}


def bench_table1(args, dev):
    """The rows of Table 1 on the room_1080p G-buffer, FP16: the grid-free
    networks and the grid networks of 2 to 8 levels of four features."""
    import torch
    import oracle as O
    from niv_synth import get_workload, make_params, make_room_gbuffer
    from paper_2602_12949_amd import NIV
    w0 = get_workload("room_1080p_pe16")
    Wd, Ht = w0.frames[0]
    _, g = make_room_gbuffer(w0.scene_seeds[0], Wd, Ht)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    d = dict(pos=t(g["pos"]), nrm=t(g["nrm"]), alb=t(g["albedo"]), mask=t(g["mask"]))
    mask = g["mask"].reshape(-1)
    n_valid = int(mask.sum())
    rng = np.random.default_rng(6)
    s = rng.choice(len(mask), 8192, replace=False)
    s = s[mask[s] > 0]
    pos, nrm = g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3)
    rows = {}
    for key in TABLE1_PAPER_MS:
        w = get_workload(f"room_1080p_{key}")
        m = NIV(w.model_dict())
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
        pm = m.prepare(t(params), "fp16")
        f, outs = m.frame(d["pos"], d["nrm"], pm, albedo=d["alb"], mask=d["mask"])
        tune = m.autotune([f], "fp16")
        graph = m.capture([f], "fp16")
        tt, tp = time_steps(graph.launch, args.steps, args.warmup)
        torch.cuda.synchronize()
        E = outs[0].reshape(-1, 3).cpu().numpy().astype(np.float64)[s]
        oc = O.config_from_workload(w)
        ref, _, _ = O.query(oc, round_params(params, "fp16"), pos[s], nrm[s])
        err = float(np.linalg.norm(E - ref) / np.linalg.norm(ref))
        fl = mlp_flops(w.model_dict()) * n_valid
        rows[key] = {
            **stats(tt, tp), "ms_per_frame": tt, "queries_per_s": n_valid / (tt * 1e-3),
            "params_MB_fp16": 2 * m.n_params / 1e6, "sampled_rel_l2": err,
            "mlp_tflops": fl / (tt * 1e-3) / 1e12,
            "paper_rtx4090_ms": TABLE1_PAPER_MS[key][0],
            "autotune": {k: tune[k] for k in ("block", "blocks_per_cu", "xcd_order")}}
        log(f"[bench] room_1080p_{key} fp16: {tt:.4f} ms/frame, sampled rel-L2 {err:.2e}")
        del graph
    return {"workload": "room_1080p G-buffer, FP16: grid-free models (u + 8-band positional "
                        "code of x, SH-16, MLP 67-W-W-W-3, W = 16, 32, 64) and grid models "
                        "(2/4/6/8 levels of 4 features, T = 2^17, SH-16, MLP (4L+16)-64-64-64-3)",
            "valid_pixels": n_valid, "rows": rows}


# Compulsory HBM bytes per pixel of the upsampler: pos, nrm, albedo (3 x 12),
# mask 1, a quarter of the half-resolution E (12 / 4), E and L out (2 x 12),
# flags 1.
UPSAMPLE_BYTES_PER_PX = 12 * 3 + 1 + 3 + 12 * 2 + 1


def bench_half(args, dev):
    """Half-resolution rendering of the room_1080p G-buffer, FP16."""
    import torch
    from niv_synth import get_workload, make_params, make_room_gbuffer
    from paper_2602_12949_amd import NIV
    w0 = get_workload("room_1080p")
    Wd, Ht = w0.frames[0]
    _, g = make_room_gbuffer(w0.scene_seeds[0], Wd, Ht)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    d = dict(pos=t(g["pos"]), nrm=t(g["nrm"]), alb=t(g["albedo"]), mask=t(g["mask"]))
    rows = {}
    for name in ("room_1080p",) + tuple(f"room_1080p_{k}" for k in TABLE1_PAPER_MS):
        w = get_workload(name)
        m = NIV(w.model_dict())
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
        pm = m.prepare(t(params), "fp16")
        f, outs = m.half_frame(Wd, Ht, d["pos"], d["nrm"], model=pm, albedo=d["alb"], mask=d["mask"])
        up = m.upsample_params()
        tt, tp = time_steps(lambda: m.query_half(f, "fp16", up), args.steps, args.warmup)
        ut, upr = time_steps(lambda: m.upsample(f, up), args.steps, args.warmup)
        key = name[len("room_1080p_"):]
        ctx = {"paper_rtx4090_ms": TABLE1_PAPER_MS[key][1]} if key in TABLE1_PAPER_MS else {}
        rows[name] = {**stats(tt, tp), "ms_per_frame": tt, "upsample_ms": ut, **ctx,
                      "query_ms": tt - ut, "half_pixels": ((Wd + 1) // 2) * ((Ht + 1) // 2),
                      "upsample_hbm_GBs": UPSAMPLE_BYTES_PER_PX * Wd * Ht / (ut * 1e-3) / 1e9}
        log(f"[bench] half {name} fp16: {tt:.4f} ms/frame (upsampling {ut:.4f} ms, "
            f"{rows[name]['upsample_hbm_GBs']:.0f} GB/s compulsory)")
    return {"workload": "room_1080p G-buffer rendered at 960x540 samples + joint bilateral "
                        "upsampling (sigma 1 px, 0.1 m, normal power 8), full-resolution albedo, FP16",
            "rows": rows}


# ---------------------------------------------------------------- profiling cases
def profile_case(case, steps, tune=None):
    import torch
    dev = torch.device("cuda:0")
    if case == "copy":
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)   # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(steps):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"[profile] copy: {steps} x 1 GiB device-to-device")
        return
    if case.startswith("query_"):
        prec = case.split("_")[1]
        w, g, m, params, d = setup_1080p(dev)
        if tune:
            m.set_tune(prec, *tune)
        pm = m.prepare(d["params"], prec)
        f, _ = m.frame(d["pos"], d["nrm"], pm, albedo=d["alb"], mask=d["mask"])
        for _ in range(steps):   # warm-up: clocks and caches as in the timed loop of the bench
            m.query_frames([f], prec)
        torch.cuda.synchronize()
        # the traced launches, timed in this process with HIP events on the launch stream
        total, per = time_steps(lambda: m.query_frames([f], prec), steps, 0)
        log(f"[profile] {case}: {steps} launches, HIP events in this process: mean {total:.4f} ms, "
            f"p50 {np.median(per):.4f} ms per launch")
        # then the encoding stage alone at the same launch shape
        pf, _ = m.frame(d["pos"], d["nrm"], pm, albedo=d["alb"], mask=d["mask"])
        total, per = time_steps(lambda: m.probe_encode(pf, prec), steps, steps)
        log(f"[profile] {case}: encoding stage alone, HIP events: mean {total:.4f} ms per launch")
        torch.cuda.synchronize()
        return
    if case == "gather":
        from paper_2602_12949_amd.niv import probe_gather
        table = torch.ones(1 << 21, dtype=torch.int32, device=dev)
        sink = torch.empty(2048 * 256, dtype=torch.int32, device=dev)
        for mode in range(4):   # 2^21 x 128 gathers per pass, reported per 2^18 x 128
            total, _ = time_steps(lambda: probe_gather(mode, 1 << 21, table, sink), steps, steps)
            log(f"[profile] gather mode {mode}: HIP events {total * 1e3:.1f} us per pass, "
                f"{total * 1e3 / 8:.1f} us per 2^18 x 128 gathers")
        return
    if case in ("train_step", "mc"):
        from niv_synth import get_workload, make_params, make_room
        from paper_2602_12949_amd import NIV, McScene, Trainer
        w = get_workload("room_train")
        m = NIV(w.model_dict())
        B = w.n_queries
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
        scene = McScene(make_room(w.scene_seeds[0])["prims"])
        x, n = scene.sample_points(w.aabb_min, w.aabb_max, B, int(round(0.2 * B)), seed=1,
                                   device=dev)
        E = torch.empty((B, 3), dtype=torch.float32, device=dev)
        valid = torch.empty(B, dtype=torch.uint8, device=dev)
        if case == "mc":
            total, per = time_steps(lambda: scene.targets(x, n, 256, 3, seed=2, out=(E, valid)),
                                    max(1, steps // 10), 1)
            log(f"[profile] mc: HIP events in this process: mean {total:.3f} ms per launch")
            return
        scene.targets(x, n, 256, 3, seed=2, out=(E, valid))
        tr = Trainer(m, torch.from_numpy(params).to(dev), "fp16", max_batch=B)
        total, per = time_steps(lambda: tr.step(x, n, E, 1e-3, valid=valid), steps, steps)
        log(f"[profile] train_step: HIP events in this process: mean {total:.4f} ms, p50 "
            f"{np.median(per):.4f} ms per step")
        return
    if case in TABLE1_PAPER_MS:
        from niv_synth import get_workload, make_params, make_room_gbuffer
        from paper_2602_12949_amd import NIV
        w = get_workload(f"room_1080p_{case}")
        _, g = make_room_gbuffer(w.scene_seeds[0], *w.frames[0])
        m = NIV(w.model_dict())
        if tune:
            m.set_tune("fp16", *tune)
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        pm = m.prepare(t(params), "fp16")
        f, _ = m.frame(t(g["pos"]), t(g["nrm"]), pm, albedo=t(g["albedo"]), mask=t(g["mask"]))
        total, _ = time_steps(lambda: m.query_frames([f], "fp16"), steps, steps)
        log(f"[profile] {case}: HIP events in this process: mean {total:.4f} ms per launch")
        return
    if case == "half":
        from niv_synth import get_workload, make_params, make_room_gbuffer
        from paper_2602_12949_amd import NIV
        w = get_workload("room_1080p")
        Wd, Ht = w.frames[0]
        _, g = make_room_gbuffer(w.scene_seeds[0], Wd, Ht)
        m = NIV(w.model_dict())
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        pm = m.prepare(t(params), "fp16")
        f, _ = m.half_frame(Wd, Ht, t(g["pos"]), t(g["nrm"]), model=pm, albedo=t(g["albedo"]),
                            mask=t(g["mask"]))
        total, _ = time_steps(lambda: m.query_half(f, "fp16"), steps, steps)
        log(f"[profile] {case}: HIP events in this process: mean {total:.4f} ms per frame "
            f"(query and upsampling)")
        return
    if case == "field_4k":
        from niv_synth import get_workload, make_params, make_workload_gbuffer
        from paper_2602_12949_amd import NIV
        w = get_workload("room_4k_6d")
        _, g = make_workload_gbuffer(w)
        m = NIV(w.model_dict())
        if tune:
            m.set_tune("bf16", *tune)
        params = make_params(m.n_grid_values, m.mat_shapes(), w.param_seed, *w.grid_init)
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        pm = m.prepare(t(params), "bf16")
        d = [t(g["pos"]), t(g["nrm"]), t(g["albedo"]), t(g["mask"])]
        f, outs = m.frame(d[0], d[1], pm, albedo=d[2], mask=d[3], extra=(0.37,))
        total, _ = time_steps(lambda: m.query_frames([f], "bf16"), steps, steps)
        log(f"[profile] {case}: HIP events in this process: query mean {total:.4f} ms per launch")
        # then the dynamic ambient occlusion pass over the same frame
        from niv_synth import workload_meshes, mesh_triangles
        from paper_2602_12949_amd.niv import DynamicAO
        ao = DynamicAO(mesh_triangles(workload_meshes(w)))
        total, _ = time_steps(lambda: ao.apply(d[0], d[1], AO_RAYS, AO_RADIUS, AO_EPS, 23, mask=d[3],
                                               E=outs[0], L=outs[1]), steps, steps)
        log(f"[profile] {case}: HIP events in this process: occlusion pass mean {total:.4f} ms per launch")
        return
    raise SystemExit(f"unknown profile case {case}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precisions", default="fp16,fp32,bf16")
    ap.add_argument("--only", default="query,train,batched,field_4k,table1,half",
                    help="comma list of parts to run")
    ap.add_argument("--bake-steps", type=int, default=4000,
                    help="steps of the stated room_train bake (2^18 points x 256 spp each)")
    ap.add_argument("--profile", default=None, help="run one kernel case for rocprofv3")
    ap.add_argument("--tune", default=None,
                    help="launch shape block,blocks_per_cu,xcd_order: for --profile, and for the "
                         "headline query instead of the autotuner (trace runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the query shards per pixel with no exchange and is measured on one GPU)",
              file=sys.stderr)
        sys.exit(2)
    if args.profile:
        tune = [int(v) for v in args.tune.split(",")] if args.tune else None
        profile_case(args.profile, args.steps, tune)
        return

    import torch
    dev = torch.device("cuda:0")
    parts = set(args.only.split(","))
    precs = args.precisions.split(",")
    w, g, params, results, outputs, n_valid, Q = bench_1080p(args, dev, precs)
    head = "fp16" if "fp16" in results else precs[0]
    ms = results[head]["ms_per_frame"]
    cfg = w.model_dict()

    # rooflines of the query kernel; the tightest (highest fraction) is the bound
    alu = ALU_OPS_PER_QUERY * n_valid / (ms * 1e-3) / 1e12
    mfma = mlp_flops(cfg) * n_valid / (ms * 1e-3) / 1e12
    hbm = HBM_BYTES_PER_PX * Q / (ms * 1e-3) / 1e9
    bounds = {
        "alu": {"achieved": alu, "peak": ALU_PEAK_TOPS, "unit": "Tops/s",
                "per_query": ALU_OPS_PER_QUERY},
        "mfma": {"achieved": mfma, "peak": MFMA_PEAK_TFLOPS[head], "unit": "TFLOP/s",
                 "per_query": mlp_flops(cfg)},
        "hbm": {"achieved": hbm, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "per_query": HBM_BYTES_PER_PX},
    }
    for b in bounds.values():
        b["frac"] = b["achieved"] / b["peak"]
    enc = results[head]["encode_only"]["ms"]
    bounds["encode"] = {"achieved": n_valid / (ms * 1e-3) / 1e9, "peak": n_valid / (enc * 1e-3) / 1e9,
                        "unit": "G queries/s", "per_query": "128 latent gathers + blends",
                        "peak_kind": "measured: the query's encoding stage alone (niv_probe_encode), "
                                     "same frame and launch shape"}
    for b in bounds.values():
        b["frac"] = b["achieved"] / b["peak"]
    bound = max(bounds, key=lambda k: bounds[k]["frac"])
    traffic = measured_traffic(f"k_query {head} room_1080p")
    roof = {"bound": bound, "achieved": bounds[bound]["achieved"], "peak": bounds[bound]["peak"],
            "unit": bounds[bound]["unit"], "frac": bounds[bound]["frac"], "traffic": traffic,
            "kernel": f"k_query ({head}, room_1080p)", "all": bounds}

    cpu, errors = None, {}
    if not args.no_cpu:
        cpu = cpu_baseline_1080p(w, g, params)
        errors = errors_1080p(w, g, params, outputs)
    extra = {}
    if "train" in parts:
        extra["train"] = bench_train(args, dev)
        extra["trained_model"] = bench_trained(args, dev, steps=args.bake_steps)
        # a short bake of a quarter of the points at a quarter of the samples
        extra["trained_model_reduced"] = bench_trained(args, dev, steps=2000, batch=1 << 16, spp=64,
                                                       checkpoints=())
    if "batched" in parts:
        extra["batched"] = bench_batched(args, dev)
    if "field_4k" in parts:
        extra["field_4k"] = bench_field_4k(args, dev)
    if "table1" in parts:
        extra["table1"] = bench_table1(args, dev)
    if "half" in parts:
        extra["half"] = bench_half(args, dev)

    line = {
        "metric": "1080p NIV query ms/frame, FP16-MFMA vs FP32 at stated err; train samples/s",
        "value": ms,
        "unit": "ms/frame",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16",
        "data": "synthetic",
        "config": {"workload": "room_1080p: 1920x1080 G-buffer, 10x4x10 m room, 32 boxes; "
                               "16 levels T=2^17 F=2, SH-16, MLP 48-64-64-64-3",
                   "pixels": Q, "valid_pixels": n_valid},
        "queries_per_s": results[head]["queries_per_s"],
        "fp32_ms_per_frame": results.get("fp32", {}).get("ms_per_frame"),
        "train_samples_per_s": extra.get("train", {}).get("train_step", {}).get("samples_per_s"),
        "precisions": results,
        "errors_vs_oracle": errors,
        "roofline": roof,
        "cpu_baseline": cpu,
        **extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
