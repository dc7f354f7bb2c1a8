"""Parity of the fused query for the grid-free models of Table 1 (no grid
levels, eight-band positional code of x, width 16, 32 or 64) with the FP64
oracle, through the C interface, on the GPU.  Same bars as the grid models:
FP32 max relative error <= 1e-5 (term scale), FP16/BF16 per-image relative
L2 <= 2e-3 against the oracle on the same rounded parameters; flags exact."""
import numpy as np
import pytest
import torch

import oracle as O
from niv_synth import get_workload, make_params, make_room_gbuffer
from niv_metrics import term_scale, max_rel_fp32, max_rel_floored, rel_l2, assert_flags, sign_margin

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
WIDTHS = (16, 32, 64)


def _round(p, prec):
    if prec == "fp32":
        return p.astype(np.float64)
    if prec == "fp16":
        return p.astype(np.float16).astype(np.float64)
    return torch.from_numpy(p).to(torch.bfloat16).to(torch.float64).numpy()


def _check(prec, E, E_ref, scale):
    if prec == "fp32":
        err = max_rel_fp32(E, E_ref, scale)
        assert err <= 1e-5, (err, max_rel_floored(E, E_ref))
    else:
        err = rel_l2(E, E_ref)
        assert err <= 2e-3, err
    return err


@pytest.fixture(scope="module")
def room_gbuffer():
    w = get_workload("room_1080p_pe64")
    W, H = w.frames[0]
    _, g = make_room_gbuffer(w.scene_seeds[0], W, H)
    return {k: g[k].reshape(-1, g[k].shape[-1]) if g[k].ndim == 3 else g[k].reshape(-1)
            for k in ("pos", "nrm", "albedo", "mask")}


def _model(width):
    from paper_2602_12949_amd import NIV
    w = get_workload(f"room_1080p_pe{width}")
    oc = O.config_from_workload(w)
    params = make_params(0, O.mat_shapes(oc), w.param_seed, *w.grid_init)
    return w, oc, NIV(w.model_dict()), params


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
@pytest.mark.parametrize("width", WIDTHS)
def test_pe_room_1080p_full_frame_parity(room_gbuffer, width, prec):
    """Every pixel of the 1920x1080 room G-buffer against the oracle."""
    g = room_gbuffer
    w, oc, m, params = _model(width)
    print(f"room_1080p_pe{width} {prec}", flush=True)
    prepared = m.prepare(_t(params), prec)
    E, L, fl = m.query(_t(g["pos"]), _t(g["nrm"]), prepared, prec, albedo=_t(g["albedo"]),
                       mask=_t(g["mask"]))
    torch.cuda.synchronize()
    E, L, fl = (E.cpu().numpy().astype(np.float64), L.cpu().numpy().astype(np.float64),
                fl.cpu().numpy())
    pr = _round(params, prec)
    E_ref, L_ref, fl_ref, x0 = O.query(oc, pr, g["pos"], g["nrm"], albedo=g["albedo"],
                                       mask=g["mask"], want_x0=True)
    sc = term_scale(O.split_params(oc, pr)[1:], x0)
    ok = g["mask"].astype(bool)
    err = _check(prec, E[ok], E_ref[ok], sc[ok])
    _check(prec, L[ok], L_ref[ok], (sc * g["albedo"] / np.pi)[ok])
    assert_flags(fl, fl_ref, E_ref, sign_margin(prec, E_ref, sc))
    assert (E[~ok] == 0).all()
    print(f"  err {err:.3e}", flush=True)


@pytest.mark.parametrize("prec", ["fp32", "fp16", "bf16"])
def test_pe_encoded_inputs(room_gbuffer, prec):
    """The positional code, SH and zero padding the kernel feeds the network,
    in the parameter order, against the oracle's input vector."""
    g = room_gbuffer
    w, oc, m, params = _model(32)
    rng = np.random.default_rng(21)
    idx = rng.choice(np.nonzero(g["mask"])[0], 5000, replace=False)
    pos, nrm = g["pos"][idx], g["nrm"][idx]
    # points straddling the box and exact dyadic positions
    pos[:4] = [[-0.5, 2.0, 5.0], [10.0, 4.0, 10.0], [0.0, 0.0, 0.0], [5.0, 1.0, 2.5]]
    prepared = m.prepare(_t(params), prec)
    _, _, fl, x_in = m.query(_t(pos), _t(nrm), prepared, prec, want_inputs=True)
    torch.cuda.synchronize()
    x_in = x_in.cpu().numpy().astype(np.float64)
    fl = fl.cpu().numpy()
    _, _, fl_ref, x0 = O.query(oc, _round(params, prec), pos, nrm, want_x0=True)
    assert x_in.shape == x0.shape == (5000, 67)
    # FP16 rounds to 11 significant bits; BF16 is split into hi + lo (16 bits)
    tol = {"fp32": 2e-6, "fp16": 2.0 ** -10, "bf16": 2.0 ** -15}[prec]
    err = np.abs(x_in - x0) / np.maximum(np.abs(x0), 1.0)
    assert err.max() <= tol, (err.max(), np.unravel_index(err.argmax(), err.shape))
    assert (fl[:4] & 1).tolist() == [1, 0, 0, 0] and ((fl_ref[:4] & 1) == (fl[:4] & 1)).all()


@pytest.mark.parametrize("n", [1, 63, 65, 4097])
def test_pe_ragged_counts(room_gbuffer, n):
    g = room_gbuffer
    w, oc, m, params = _model(16)
    pos, nrm = g["pos"][-n:], g["nrm"][-n:]
    mask = g["mask"][-n:]
    prepared = m.prepare(_t(params), "fp32")
    E, _, fl = m.query(_t(pos), _t(nrm), prepared, "fp32", mask=_t(mask))
    torch.cuda.synchronize()
    E = E.cpu().numpy().astype(np.float64)
    E_ref, _, fl_ref, x0 = O.query(oc, params.astype(np.float64), pos, nrm, mask=mask,
                                   want_x0=True)
    sc = term_scale(O.split_params(oc, params.astype(np.float64))[1:], x0)
    _check("fp32", E, E_ref, sc)
    assert_flags(fl.cpu().numpy(), fl_ref, E_ref, sign_margin("fp32", E_ref, sc))


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_pe_edge_inputs(room_gbuffer, prec):
    """Masked pixels, non-finite inputs, zero normals and points outside the
    box under the grid-free model."""
    g = room_gbuffer
    w, oc, m, params = _model(64)
    pos = g["pos"][:300].copy()
    nrm = g["nrm"][:300].copy()
    mask = np.ones(300, np.uint8)
    pos[0] = [np.nan, 1.0, 1.0]
    nrm[1] = [0.0, 0.0, 0.0]
    pos[2] = [11.0, -1.0, 4.0]
    nrm[3] = [np.inf, 0.0, 0.0]
    mask[5:9] = 0
    prepared = m.prepare(_t(params), prec)
    E, _, fl = m.query(_t(pos), _t(nrm), prepared, prec, mask=_t(mask))
    torch.cuda.synchronize()
    E, fl = E.cpu().numpy().astype(np.float64), fl.cpu().numpy()
    pr = _round(params, prec)
    E_ref, _, fl_ref, x0 = O.query(oc, pr, pos, nrm, mask=mask, want_x0=True)
    sc = term_scale(O.split_params(oc, pr)[1:], x0)
    assert_flags(fl, fl_ref, E_ref, sign_margin(prec, E_ref, sc))
    assert fl[0] & 2 and fl[1] & 2 and fl[3] & 2 and fl[2] & 1
    assert (E[[0, 1, 3]] == 0).all() and (E[5:9] == 0).all()
    ok = mask.astype(bool) & ((fl_ref & 2) == 0)
    _check(prec, E[ok], E_ref[ok], sc[ok])


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_wide_6d_fp32_fp16(prec):
    """The width-128 6-D field at FP32 (inputs staged, weights from memory)
    and FP16 (lane-sliced encoding) on room points, one scene variable."""
    from paper_2602_12949_amd import NIV
    w = get_workload("room_4k_6d")
    oc = O.config_from_workload(w)
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), w.param_seed, *w.grid_init)
    m = NIV(w.model_dict())
    rng = np.random.default_rng(31)
    n = 3000
    pos = (rng.random((n, 3)) * [10.0, 4.0, 10.0]).astype(np.float32)
    nrm = rng.normal(size=(n, 3)).astype(np.float32)
    prepared = m.prepare(_t(params), prec)
    E, _, fl = m.query(_t(pos), _t(nrm), prepared, prec, extra=(0.37,))
    torch.cuda.synchronize()
    E, fl = E.cpu().numpy().astype(np.float64), fl.cpu().numpy()
    pr = _round(params, prec)
    E_ref, _, fl_ref, x0 = O.query(oc, pr, pos, nrm, extra=np.full((n, 1), 0.37, np.float32),
                                   want_x0=True)
    sc = term_scale(O.split_params(oc, pr)[1:], x0)
    _check(prec, E, E_ref, sc)
    assert_flags(fl, fl_ref, E_ref, sign_margin(prec, E_ref, sc))


@pytest.mark.parametrize("prec", ["fp16", "bf16"])
@pytest.mark.parametrize("block", [256, 768])
def test_wide_6d_launch_shapes(prec, block):
    """The lane-sliced width-128 6-D field at the launch shapes besides the
    default 512 threads (768: three waves per SIMD), room points, one scene
    variable, against the oracle at the 16-bit bar."""
    from paper_2602_12949_amd import NIV
    w = get_workload("room_4k_6d")
    oc = O.config_from_workload(w)
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), w.param_seed, *w.grid_init)
    m = NIV(w.model_dict())
    m.set_tune(prec, block, 0, 1)
    rng = np.random.default_rng(33)
    n = 100000 + 37
    pos = (rng.random((n, 3)) * [10.0, 4.0, 10.0]).astype(np.float32)
    nrm = rng.normal(size=(n, 3)).astype(np.float32)
    prepared = m.prepare(_t(params), prec)
    E, _, fl = m.query(_t(pos), _t(nrm), prepared, prec, extra=(0.6,))
    torch.cuda.synchronize()
    E, fl = E.cpu().numpy().astype(np.float64), fl.cpu().numpy()
    pr = _round(params, prec)
    E_ref, _, fl_ref, x0 = O.query(oc, pr, pos, nrm, extra=np.full((n, 1), 0.6, np.float32),
                                   want_x0=True)
    sc = term_scale(O.split_params(oc, pr)[1:], x0)
    _check(prec, E, E_ref, sc)
    assert_flags(fl, fl_ref, E_ref, sign_margin(prec, E_ref, sc))
