"""Half-resolution rendering (Sec. 4.4) on the GPU against the FP64 oracle,
through the C interface: the joint bilateral upsampler alone on the same
half-resolution input (FP32 arithmetic: max relative error 1e-5, flags
exact), and the whole path (the query at the pixels (2x, 2y), then the
upsampler) at the bars of the query: FP32 1e-5 of the term scale carried
through the same weights, FP16/BF16 relative L2 2e-3."""
import numpy as np
import pytest
import torch

import oracle as O
from niv_synth import get_workload, make_params, make_room_gbuffer
from niv_metrics import term_scale, rel_l2

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
UP = dict(sigma_px=1.0, sigma_pos=0.1, normal_power=8)


def _t(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _round(p, prec):
    if prec == "fp32":
        return p.astype(np.float64)
    if prec == "fp16":
        return p.astype(np.float16).astype(np.float64)
    return torch.from_numpy(p).to(torch.bfloat16).to(torch.float64).numpy()


def _gbuffer(W, H, seed=2001, plant=True):
    _, g = make_room_gbuffer(seed, W, H)
    pos = g["pos"].reshape(-1, 3).copy()
    nrm = g["nrm"].reshape(-1, 3).copy()
    alb = g["albedo"].reshape(-1, 3).copy()
    mask = g["mask"].reshape(-1).copy()
    if plant:
        rng = np.random.default_rng(seed)
        valid = np.nonzero(mask)[0]
        k = rng.choice(valid, 40, replace=False)
        pos[k[:8], 0] = np.nan                 # non-finite inputs
        nrm[k[8:16]] = 0.0                     # zero normals
        pos[k[16:24]] += [0.0, 50.0, 0.0]      # outside the box
        nrm[k[24:40]] *= -1.0                  # pixels facing away from their neighbours
    return pos, nrm, alb, mask


def _model(wname):
    from paper_2602_12949_amd import NIV
    w = get_workload(wname)
    oc = O.config_from_workload(w)
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), w.param_seed, *w.grid_init)
    return w, oc, NIV(w.model_dict()), params


@pytest.mark.parametrize("W,H", [(480, 270), (333, 187), (1920, 1080)])
def test_upsampler_parity(W, H):
    """Same half-resolution irradiance into both upsamplers."""
    w, oc, m, params = _model("room_1080p")
    pos, nrm, alb, mask = _gbuffer(W, H)
    hw, hh = (W + 1) // 2, (H + 1) // 2
    rng = np.random.default_rng(W)
    hE = rng.uniform(0.05, 3.0, size=(hh * hw, 3)).astype(np.float32)
    print(f"upsampler {W}x{H}", flush=True)
    f, out = m.half_frame(W, H, _t(pos), _t(nrm), albedo=_t(alb), mask=_t(mask), half_E=_t(hE))
    m.upsample(f, m.upsample_params(**UP))
    torch.cuda.synchronize()
    E, L, fl = (out["E"].cpu().numpy().astype(np.float64), out["L"].cpu().numpy().astype(np.float64),
                out["flags"].cpu().numpy())
    E_ref, L_ref, fl_ref = O.upsample(oc, W, H, pos, nrm, hE.astype(np.float64), mask=mask,
                                      albedo=alb, **UP)
    np.testing.assert_array_equal(fl, fl_ref)
    err = np.abs(E - E_ref).max() / np.abs(E_ref).max()
    errL = np.abs(L - L_ref).max() / np.abs(L_ref).max()
    print(f"  max err / max |E| {err:.2e} (L {errL:.2e}); flags "
          f"{ {b: int(((fl_ref & b) != 0).sum()) for b in (1, 2, 32, 64)} }", flush=True)
    assert err <= 1e-5 and errL <= 1e-5
    assert ((fl_ref & 32) != 0).any() and ((fl_ref & 2) != 0).any()


@pytest.mark.parametrize("wname,prec", [("room_1080p", "fp32"), ("room_1080p", "fp16"),
                                        ("room_1080p", "bf16"), ("room_1080p_pe64", "fp16"),
                                        ("room_1080p_g8", "fp16"), ("room_1080p_g8", "fp32")])
def test_query_half_parity(wname, prec):
    """The whole half-resolution path on the 1920x1080 room G-buffer."""
    w, oc, m, params = _model(wname)
    W, H = w.frames[0]
    pos, nrm, alb, mask = _gbuffer(W, H)
    print(f"query_half {wname} {prec}", flush=True)
    prepared = m.prepare(_t(params), prec)
    f, out = m.half_frame(W, H, _t(pos), _t(nrm), model=prepared, albedo=_t(alb), mask=_t(mask))
    m.query_half(f, prec, m.upsample_params(**UP))
    torch.cuda.synchronize()
    E = out["E"].cpu().numpy().astype(np.float64)
    hE = out["half_E"].cpu().numpy().astype(np.float64)
    hfl = out["half_flags"].cpu().numpy()
    fl = out["flags"].cpu().numpy()
    # oracle: the query at the samples (2x, 2y), then the upsampler
    hpos, hnrm, hmask = O.half_samples(W, H, pos, nrm, mask)
    pr = _round(params, prec)
    hE_ref, _, hfl_ref, x0 = O.query(oc, pr, hpos, hnrm, mask=hmask, want_x0=True)
    np.testing.assert_array_equal(hfl & 0xEF, hfl_ref & 0xEF)
    E_ref, _, fl_ref = O.upsample(oc, W, H, pos, nrm, hE_ref, mask=mask, **UP)
    np.testing.assert_array_equal(fl, fl_ref)
    ok = mask.astype(bool) & ((fl_ref & 66) == 0)
    if prec == "fp32":
        # errors of the samples are at most 1e-5 of their term scale; the
        # upsampler's convex weights carry that bound to every pixel
        sc = term_scale(O.split_params(oc, pr)[1:], x0)
        bound, _, _ = O.upsample(oc, W, H, pos, nrm, np.maximum(sc, np.abs(hE_ref)), mask=mask, **UP)
        err = float(np.max(np.abs(E - E_ref)[ok] / np.maximum(bound[ok], 1e-30)))
        herr = float(np.max(np.abs(hE - hE_ref) / np.maximum(np.maximum(sc, np.abs(hE_ref)), 1e-30)))
        print(f"  max err {err:.2e} of the carried term scale (samples {herr:.2e})", flush=True)
        assert err <= 1e-5 and herr <= 1e-5
    else:
        err = rel_l2(E[ok], E_ref[ok])
        hok = hmask.astype(bool) & ((hfl_ref & 2) == 0)
        herr = rel_l2(hE[hok], hE_ref[hok])
        print(f"  rel-L2 {err:.2e} (samples {herr:.2e})", flush=True)
        assert err <= 2e-3 and herr <= 2e-3


def test_query_half_ragged_and_args():
    """Odd sizes down to a single pixel, and argument checks."""
    from paper_2602_12949_amd import niv as N
    w, oc, m, params = _model("room_1080p")
    prepared = m.prepare(_t(params), "fp32")
    for (W, H) in [(1, 1), (1, 7), (9, 1), (65, 33)]:
        pos, nrm, alb, mask = _gbuffer(W, H, plant=False)
        f, out = m.half_frame(W, H, _t(pos), _t(nrm), model=prepared, albedo=_t(alb), mask=_t(mask))
        m.query_half(f, "fp32", m.upsample_params(**UP))
        torch.cuda.synchronize()
        hpos, hnrm, hmask = O.half_samples(W, H, pos, nrm, mask)
        hE_ref, _, _ = O.query(oc, params.astype(np.float64), hpos, hnrm, mask=hmask)
        E_ref, _, fl_ref = O.upsample(oc, W, H, pos, nrm, hE_ref, mask=mask, **UP)
        np.testing.assert_array_equal(out["flags"].cpu().numpy(), fl_ref)
        np.testing.assert_allclose(out["E"].cpu().numpy(), E_ref, rtol=1e-4, atol=1e-4 * np.abs(E_ref).max() + 1e-12)
    pos, nrm, alb, mask = _gbuffer(8, 8, plant=False)
    f, _ = m.half_frame(8, 8, _t(pos), _t(nrm), model=prepared)
    for bad in (m.upsample_params(sigma_px=0.0), m.upsample_params(sigma_pos=-1.0),
                m.upsample_params(normal_power=65)):
        with pytest.raises(N.NivError) as e:
            m.query_half(f, "fp32", bad)
        assert e.value.status == N.NIV_ERR_INVALID_ARG
    f.width = 0
    with pytest.raises(N.NivError):
        m.upsample(f)
