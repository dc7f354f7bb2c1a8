"""Benchmark of the Neural Irradiance Volume hot path on one MI355X.

Workload: one 1920x1080 G-buffer of a 10x4x10 m room with 32 boxes (seeded,
~4-5 % sky pixels masked), model of 16 hash-grid levels (T = 2^17, F = 2),
16 SH of the normal, MLP 48-64-64-64-3.  A step is one fused query of the
whole frame (G-buffer read, encoding, MLP, E and albedo * E / pi written),
inputs resident in HBM.  The headline is the FP16-MFMA path; FP32 and BF16
are timed on the same inputs and weights.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "fp32": 157.3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def mlp_flops(cfg):
    din = cfg["n_levels"] * cfg["n_features"] + cfg["sh_bands"] ** 2 + \
        cfg["n_extra"] * 2 * cfg["extra_bands"]
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


def time_kernel(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return start.elapsed_time(stop) / steps, wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--precisions", default="fp16,fp32,bf16")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: --gpus {args.gpus} is not supported "
              "(the query shards per pixel with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from niv_synth import get_workload, make_params, make_room_gbuffer
    from paper_2602_12949_amd import NIV

    w = get_workload("room_1080p")
    cfg = w.model_dict()
    Wd, Ht = w.frames[0]
    log(f"[bench] building G-buffer {Wd}x{Ht} seed {w.scene_seeds[0]}")
    _, g = make_room_gbuffer(w.scene_seeds[0], Wd, Ht)
    m = NIV(cfg)
    n_grid = m.n_grid_values
    din = cfg["n_levels"] * 2 + 16
    shapes = [(cfg["width"], din)] + [(cfg["width"], cfg["width"])] * (cfg["n_hidden"] - 1) + \
        [(cfg["n_out"], cfg["width"])]
    params = make_params(n_grid, shapes, w.param_seed, *w.grid_init)
    dev = torch.device("cuda:0")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    pos, nrm, alb = t(g["pos"]), t(g["nrm"]), t(g["albedo"])
    mask = t(g["mask"])
    p_d = t(params)
    Q = Wd * Ht
    n_valid = int(g["mask"].sum())

    results = {}
    outputs = {}
    for prec in args.precisions.split(","):
        prepared = m.prepare(p_d, prec)
        frame, outs = m.frame(pos, nrm, prepared, albedo=alb, mask=mask)
        fn = lambda: m.query_frames([frame], prec)
        ms, wall = time_kernel(fn, args.steps, args.warmup)
        torch.cuda.synchronize()
        outputs[prec] = outs[0].reshape(-1, 3).cpu().numpy().astype(np.float64)
        results[prec] = {"ms_per_frame": ms, "queries_per_s": n_valid / (ms * 1e-3),
                         "wall_s": wall}
        log(f"[bench] {prec}: {ms:.4f} ms/frame, {n_valid / (ms * 1e-3) / 1e9:.3f} G valid queries/s")

    head = "fp16" if "fp16" in results else list(results)[0]
    ms = results[head]["ms_per_frame"]
    bytes_per_px = 12 * 3 + 1 + 12 * 2 + 1  # pos, nrm, albedo, mask, E, L, flags
    flops = mlp_flops(cfg) * n_valid
    roof = {
        "bound": "mfma",
        "achieved": flops / (ms * 1e-3) / 1e12,
        "peak": MFMA_PEAK_TFLOPS[head],
        "unit": "TFLOP/s",
        "traffic": None,
    }
    roof["frac"] = roof["achieved"] / roof["peak"]
    hbm = bytes_per_px * Q / (ms * 1e-3) / 1e9

    cpu = None
    errors = {}
    if not args.no_cpu:
        import oracle as O
        oc = O.config_from_workload(w)
        cores = os.cpu_count()
        O.set_threads(cores)
        log(f"[bench] CPU oracle: full frame, {cores} threads")
        p64 = params.astype(np.float64)
        t0 = time.perf_counter()
        E_ref, _, _ = O.query(oc, p64, g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3),
                              mask=g["mask"].reshape(-1))
        cpu_s = time.perf_counter() - t0
        cpu = {"value": cpu_s * 1e3, "unit": "ms/frame", "cores": cores, "kind": "oracle",
               "sample": "one full 1920x1080 frame, FP64, OpenMP over pixels",
               "queries_per_s": n_valid / cpu_s}
        ok = g["mask"].reshape(-1).astype(bool)
        for prec, E in outputs.items():
            if prec == "fp16":
                pr = params.astype(np.float16).astype(np.float64)
            elif prec == "bf16":
                pr = torch.from_numpy(params).to(torch.bfloat16).to(torch.float64).numpy()
            else:
                pr = p64
            ref, _, _, x0 = O.query(oc, pr, g["pos"].reshape(-1, 3), g["nrm"].reshape(-1, 3),
                                    mask=g["mask"].reshape(-1), want_x0=True)
            a, b = E[ok], ref[ok]
            sc = term_scale(O.split_params(oc, pr)[1:], x0[ok])
            del x0
            floor = 1e-3 * np.abs(b).max()
            errors[prec] = {
                "max_rel_err": float(np.max(np.abs(a - b) / np.maximum(np.abs(b), sc))),
                "max_rel_err_floored_1e-3": float(np.max(np.abs(a - b) / np.maximum(np.abs(b), floor))),
                "rel_l2": float(np.linalg.norm(a - b) / np.linalg.norm(b)),
                "vs": "oracle on the same rounded parameters",
            }
            if prec != "fp32":
                errors[prec]["rel_l2_vs_fp32_master"] = float(
                    np.linalg.norm(a - E_ref[ok]) / np.linalg.norm(E_ref[ok]))
            log(f"[bench] {prec} error vs oracle: {errors[prec]}")

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
        "precisions": results,
        "errors_vs_oracle": errors,
        "hbm_compulsory_GBs": hbm,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
