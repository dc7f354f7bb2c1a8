"""On-GPU training through the C interface against the FP64 oracle: Eq. 3
loss, the gradient of every parameter (MLP weights and hash-grid latents),
Adam, and convergence on a target the model can represent.

Gradient bars: FP32 path relative L2 <= 1e-4 over each parameter block and
max error <= 1e-3 of the block's largest gradient (FP32 sums over chunks and
waves; the grid sums in 64-bit fixed point); FP16 path relative L2 <= 2e-2 (activations and gradients
are FP16 operands with unit roundoff 2^-11, summed over 64-sample chunks)
against the oracle on the FP16-rounded parameters, and 3e-2 for the grid
block: a hashed grid entry holds the contribution of about one sample, a
64-term FP16 contraction W_0^T delta_1 whose terms cancel, so its error is
not averaged over samples as the weight blocks' errors are."""
import numpy as np
import pytest
import torch

import oracle as O
from niv_synth import get_workload, make_params, unit_cube_queries
from niv_metrics import relu_margin

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _setup(wname, n, seed=3, grid=(-0.5, 0.5)):
    w = get_workload(wname)
    oc = O.config_from_workload(w)
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), seed, *grid)
    rng = np.random.default_rng(seed + 1)
    lo, hi = np.array(w.aabb_min), np.array(w.aabb_max)
    x = rng.uniform(lo, hi, size=(n, 3)).astype(np.float32)
    v = rng.standard_normal((n, 3))
    nrm = (v / np.linalg.norm(v, axis=1, keepdims=True)).astype(np.float32)
    tgt = rng.uniform(0.05, 2.0, size=(n, 3)).astype(np.float32)
    return w, oc, params, x, nrm, tgt


def _gpu_grad(w, params, x, nrm, tgt, prec, valid=None, extra=None):
    from paper_2602_12949_amd import NIV, Trainer
    m = NIV(w.model_dict())
    p = torch.from_numpy(params).to(DEV)
    tr = Trainer(m, p, prec, max_batch=len(x))
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    loss = tr.backward(t(x), t(nrm), t(tgt), valid=None if valid is None else t(valid),
                       extra=None if extra is None else t(extra))
    torch.cuda.synchronize()
    return float(loss.item()), tr.grads.cpu().numpy().astype(np.float64)


def _clear_of_ties(oc, params, x, nrm, extra=None, margin=1e-5):
    """valid flags leaving out the samples with a hidden pre-activation within
    `margin` of zero relative to its terms (FP64 pass): there the FP32 and FP64
    ReLU decisions may differ and both gradients are right to the precision."""
    _, _, _, x0 = O.query(oc, params, x, nrm, extra=extra, want_x0=True)
    ok = relu_margin(O.split_params(oc, params)[1:], x0) > margin
    print(f"  {int((~ok).sum())} of {len(ok)} samples within {margin} of a ReLU tie left out",
          flush=True)
    return ok.astype(np.uint8)


def _blocks(oc, g):
    n_grid = O.n_grid_values(oc)
    out = {"grid": g[:n_grid]}
    k = n_grid
    for i, (o, inn) in enumerate(O.mat_shapes(oc)):
        out[f"W{i}"] = g[k:k + o * inn]
        k += o * inn
    return out


def _compare(oc, g, g_ref, rel_l2_bar, max_bar=None, grid_bar=None):
    gb, rb = _blocks(oc, g), _blocks(oc, g_ref)
    res = {}
    for name in gb:
        a, b = gb[name], rb[name]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        mx = np.abs(a - b).max() / np.abs(b).max()
        print(f"  {name}: rel-L2 {rel:.2e}, max/max {mx:.2e}", flush=True)
        res[name] = (rel, mx)
    for name, (rel, mx) in res.items():
        assert rel <= (grid_bar if (name == "grid" and grid_bar) else rel_l2_bar), (name, rel)
        if max_bar is not None:
            assert mx <= max_bar, (name, mx)


@pytest.mark.parametrize("wname,n", [("unit_cube_16k", 1000), ("room_1080p", 4096)])
def test_fp32_gradient_matches_oracle(wname, n):
    w, oc, params, x, nrm, tgt = _setup(wname, n)
    print(f"{wname} fp32 n={n}", flush=True)
    vd = _clear_of_ties(oc, params.astype(np.float64), x, nrm)
    loss, g = _gpu_grad(w, params, x, nrm, tgt, "fp32", valid=vd)
    l_ref, g_ref = O.loss_grad(oc, params.astype(np.float64), x, nrm, tgt, valid=vd)
    assert loss == pytest.approx(l_ref, rel=1e-5)
    _compare(oc, g, g_ref, 1e-4, 1e-3)


@pytest.mark.parametrize("wname,n", [("unit_cube_16k", 1000), ("room_1080p", 4096)])
def test_fp16_gradient_matches_oracle(wname, n):
    w, oc, params, x, nrm, tgt = _setup(wname, n)
    print(f"{wname} fp16 n={n}", flush=True)
    loss, g = _gpu_grad(w, params, x, nrm, tgt, "fp16")
    p16 = params.astype(np.float16).astype(np.float64)
    l_ref, g_ref = O.loss_grad(oc, p16, x, nrm, tgt)
    assert loss == pytest.approx(l_ref, rel=5e-3)
    _compare(oc, g, g_ref, 2e-2, grid_bar=3e-2)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_split_bin_gradient_matches_oracle(prec):
    """2^16 samples on the room model: level 0 (17^3 = 4913 dense entries)
    puts ~2^16 x 8 x 4096 / 4913 = 437k contributions into its first grid bin
    of 4096 entries, more than one accumulating workgroup takes (98,304), so
    that bin (and those of levels 1-2) is summed in parts whose integer
    partial sums are merged; every block is compared with the FP64 oracle at
    the bars of the small-batch tests."""
    n = 1 << 16
    assert n * 8 * 4096 / 4913 > 98304
    w, oc, params, x, nrm, tgt = _setup("room_1080p", n, seed=21)
    print(f"room_1080p {prec} n={n}", flush=True)
    pr = params.astype(np.float64) if prec == "fp32" else params.astype(np.float16).astype(np.float64)
    vd = _clear_of_ties(oc, pr, x, nrm) if prec == "fp32" else None
    loss, g = _gpu_grad(w, params, x, nrm, tgt, prec, valid=vd)
    l_ref, g_ref = O.loss_grad(oc, pr, x, nrm, tgt, valid=vd)
    if prec == "fp32":
        assert loss == pytest.approx(l_ref, rel=1e-5)
        _compare(oc, g, g_ref, 1e-4, 1e-3)
    else:
        assert loss == pytest.approx(l_ref, rel=5e-3)
        _compare(oc, g, g_ref, 2e-2, grid_bar=3e-2)


def test_full_batch_gradient_is_bit_reproducible():
    """At the benchmark's batch (2^18 samples, FP16) every gradient value is
    a sum in a fixed order or in integers: two calls on the same batch give
    the same bits, although the contributions reach their bins in a
    different order each time."""
    n = 1 << 18
    w, oc, params, x, nrm, tgt = _setup("room_1080p", n, seed=23)
    from paper_2602_12949_amd import NIV, Trainer
    m = NIV(w.model_dict())
    tr = Trainer(m, torch.from_numpy(params).to(DEV), "fp16", max_batch=n)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    xd, nd, td = t(x), t(nrm), t(tgt)
    tr.backward(xd, nd, td)
    g1 = tr.grads.clone()
    tr.backward(xd, nd, td)
    torch.cuda.synchronize()
    same = torch.equal(g1, tr.grads)
    print(f"  equal bits: {same}; differing values {int((g1 != tr.grads).sum())}", flush=True)
    assert same


def test_two_streams_at_once_match_one_at_a_time():
    """Two training states on two streams with their calls interleaved (the
    count passes of both go to the library's second stream, each call with
    its own fork and join events): each gradient equals the same call made
    alone, bit for bit, on every one of three rounds."""
    n = 1 << 16
    from paper_2602_12949_amd import NIV, Trainer
    w, oc, params, x, nrm, tgt = _setup("room_1080p", n, seed=31)
    _, _, _, x2, nrm2, tgt2 = _setup("room_1080p", n, seed=32)
    m = NIV(w.model_dict())
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    pa, pb = t(params), t(params)
    in_a, in_b = (t(x), t(nrm), t(tgt)), (t(x2), t(nrm2), t(tgt2))
    ta = Trainer(m, pa, "fp16", max_batch=n)
    tb = Trainer(m, pb, "fp16", max_batch=n)
    ta.backward(*in_a)
    tb.backward(*in_b)
    torch.cuda.synchronize()
    ga, gb = ta.grads.clone(), tb.grads.clone()
    assert not torch.equal(ga, gb)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    cur = torch.cuda.current_stream()
    for r in range(3):
        ta.grads.zero_()
        tb.grads.zero_()
        s1.wait_stream(cur)
        s2.wait_stream(cur)
        with torch.cuda.stream(s1):
            ta.backward(*in_a)
        with torch.cuda.stream(s2):
            tb.backward(*in_b)
        cur.wait_stream(s1)
        cur.wait_stream(s2)
        torch.cuda.synchronize()
        print(f"  round {r}: equal {torch.equal(ga, ta.grads)} {torch.equal(gb, tb.grads)}", flush=True)
        assert torch.equal(ga, ta.grads) and torch.equal(gb, tb.grads)


def test_gradient_pass_replays_from_a_graph():
    """niv_backward captured in a HIP graph (its count pass on the library's
    second stream becomes a fork and join inside the graph) and replayed
    three times, with eager calls and synchronisations between the replays:
    every replay and every eager call gives the first eager gradient bit for
    bit, and its loss (a sum of per-wave float additions, whose order
    varies) to 1e-6."""
    n = 1 << 14
    from paper_2602_12949_amd import NIV, Trainer
    w, oc, params, x, nrm, tgt = _setup("room_1080p", n, seed=41)
    m = NIV(w.model_dict())
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    tr = Trainer(m, t(params), "fp16", max_batch=n)
    inp = (t(x), t(nrm), t(tgt))
    loss = tr.backward(*inp)
    torch.cuda.synchronize()
    g_ref, l_ref = tr.grads.clone(), loss.clone()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        tr.backward(*inp)
    for r in range(3):
        tr.grads.zero_()
        tr.loss.zero_()
        graph.replay()
        torch.cuda.synchronize()
        close = lambda: abs(float(tr.loss) - float(l_ref)) <= 1e-6 * abs(float(l_ref))
        rep_ok = torch.equal(tr.grads, g_ref) and close()
        tr.backward(*inp)
        torch.cuda.synchronize()
        eager_ok = torch.equal(tr.grads, g_ref) and close()
        print(f"  replay {r}: {rep_ok}, eager after it: {eager_ok}", flush=True)
        assert rep_ok and eager_ok


def test_largest_batch_gradient_matches_oracle():
    """The largest batch niv_backward takes, 2^24 samples (2^31 contribution
    records on the 16-level room model; level 0's first bin alone gets ~1.1e8
    records, summed in ~1,100 parts): FP16 gradient of every block against
    the FP64 oracle at the bars of the small batches."""
    n = 1 << 24
    w, oc, params, x, nrm, tgt = _setup("room_1080p", n, seed=24)
    print(f"room_1080p fp16 n={n}", flush=True)
    loss, g = _gpu_grad(w, params, x, nrm, tgt, "fp16")
    p16 = params.astype(np.float16).astype(np.float64)
    l_ref, g_ref = O.loss_grad(oc, p16, x, nrm, tgt)
    assert loss == pytest.approx(l_ref, rel=5e-3)
    _compare(oc, g, g_ref, 2e-2, grid_bar=3e-2)


def test_nonfinite_step_is_reported_and_skipped():
    """A non-finite target makes the step's loss non-finite: niv_train_step
    leaves parameters and moments as they were and niv_train_status reports
    it; the non-finite sample puts nothing into the grid gradient.  The next
    finite step updates again."""
    from paper_2602_12949_amd import NIV, Trainer
    w, oc, params, x, nrm, tgt = _setup("unit_cube_16k", 2048, seed=25)
    m = NIV(w.model_dict())
    tr = Trainer(m, torch.from_numpy(params).to(DEV), "fp32", max_batch=2048)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    xd, nd = t(x), t(nrm)
    tr.step(xd, nd, t(tgt), lr=1e-2)
    assert tr.status()
    p0, m0, v0 = tr.params.clone(), tr.m.clone(), tr.v.clone()
    bad = tgt.copy()
    bad[77, 1] = np.inf
    loss = tr.step(xd, nd, t(bad), lr=1e-2)
    ok = tr.status()
    print(f"  loss {float(loss.item())}, status ok {ok}", flush=True)
    assert not ok and not np.isfinite(float(loss.item()))
    assert torch.equal(tr.params, p0) and torch.equal(tr.m, m0) and torch.equal(tr.v, v0)
    g = tr.grads[:m.n_grid_values].clone()
    assert bool(torch.isfinite(g).all())
    # the finite samples' grid gradient equals that of the batch without the bad one
    keep = np.ones(2048, np.uint8)
    keep[77] = 0
    tr.backward(xd, nd, t(bad), valid=t(keep))
    assert tr.status()
    torch.cuda.synchronize()
    assert torch.equal(g, tr.grads[:m.n_grid_values])
    tr.step(xd, nd, t(tgt), lr=1e-2)
    assert tr.status() and not torch.equal(tr.params, p0)


@pytest.mark.parametrize("wname", ["unit_cube_16k", "room_1080p", "room_train_6d"])
def test_init_params_match_oracle(wname):
    """niv_init_params equals the oracle's seeded initialisation bit for bit
    (the same generator stream per parameter, one rounding to FP32)."""
    from paper_2602_12949_amd import NIV
    w = get_workload(wname)
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    lo, hi = np.float32(-1e-4), np.float32(1e-4)
    got = m.init_params(97, float(lo), float(hi)).cpu().numpy()
    want = O.init_params(oc, 97, float(lo), float(hi))
    print(f"  {wname}: {got.size} parameters, {int((got != want).sum())} differ", flush=True)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_scene_variable_gradient_matches_oracle(prec):
    """The field with one scene variable (Sec. 6): each sample carries its own
    t, frequency-encoded into the input; gradients of every block."""
    w, oc, params, x, nrm, tgt = _setup("room_train_6d", 4096)
    tv = np.random.default_rng(9).uniform(0, 1, size=(4096, 1)).astype(np.float32)
    print(f"room_train_6d {prec}", flush=True)
    loss, g = _gpu_grad(w, params, x, nrm, tgt, prec, extra=tv)
    pr = params.astype(np.float64) if prec == "fp32" else params.astype(np.float16).astype(np.float64)
    l_ref, g_ref = O.loss_grad(oc, pr, x, nrm, tgt, extra=tv)
    if prec == "fp32":
        assert loss == pytest.approx(l_ref, rel=1e-5)
        _compare(oc, g, g_ref, 1e-4, 1e-3)
    else:
        assert loss == pytest.approx(l_ref, rel=5e-3)
        _compare(oc, g, g_ref, 2e-2, grid_bar=3e-2)
    # the variable reaches the network: another t gives another loss
    l2, _ = _gpu_grad(w, params, x, nrm, tgt, prec, extra=1.0 - tv)
    assert abs(l2 - loss) > 1e-6 * abs(loss)


def test_invalid_samples_and_ragged_batch():
    w, oc, params, x, nrm, tgt = _setup("unit_cube_16k", 777)
    valid = (np.arange(777) % 5 != 0).astype(np.uint8)
    x[3] = [np.nan, 0.2, 0.2]  # a non-finite sample must not reach the grid
    valid[3] = 1
    loss, g = _gpu_grad(w, params, x, nrm, tgt, "fp32", valid=valid)
    v2 = valid.copy()
    v2[3] = 0  # the oracle skips it: a non-finite input has no gradient
    l_ref, g_ref = O.loss_grad(oc, params.astype(np.float64), x, nrm, tgt, valid=v2)
    assert np.isfinite(g).all()
    assert loss == pytest.approx(l_ref, rel=1e-5)
    _compare(oc, g, g_ref, 1e-4, 1e-3)


def test_adam_matches_oracle():
    from paper_2602_12949_amd import NIV, Trainer
    w, oc, params, x, nrm, tgt = _setup("unit_cube_16k", 256)
    m = NIV(w.model_dict())
    p = torch.from_numpy(params.copy()).to(DEV)
    tr = Trainer(m, p, "fp32", max_batch=256)
    rng = np.random.default_rng(9)
    p64 = params.astype(np.float64)
    m64 = np.zeros_like(p64)
    v64 = np.zeros_like(p64)
    for step in range(1, 4):
        g = rng.standard_normal(params.size).astype(np.float32)
        tr.grads.copy_(torch.from_numpy(g))
        tr.adam(lr=1e-2, step=step)
        O.adam(p64, g.astype(np.float64), m64, v64, lr=1e-2, step=step)
    torch.cuda.synchronize()
    got = p.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, p64, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_training_fits_representable_target(prec):
    """E(x, n) = a + b x_0 is smooth and positive: Adam on Eq. 3 drives the
    relative loss from O(1) to below 1e-3 in a few hundred steps."""
    from paper_2602_12949_amd import NIV, Trainer
    w = get_workload("unit_cube_16k")
    oc = O.config_from_workload(w)
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), 5, -1e-4, 1e-4)
    m = NIV(w.model_dict())
    p = torch.from_numpy(params).to(DEV)
    tr = Trainer(m, p, prec, max_batch=4096)
    gen = torch.Generator(device="cpu").manual_seed(0)
    a = torch.tensor([0.5, 1.0, 0.3])
    b = torch.tensor([1.0, -0.4, 0.6])
    first = last = None
    for step in range(400):
        xs = torch.rand((4096, 3), generator=gen)
        ns = torch.nn.functional.normalize(torch.randn((4096, 3), generator=gen), dim=1)
        ys = a + b * xs[:, :1]
        loss = tr.step(xs.to(DEV), ns.to(DEV), ys.to(DEV), lr=1e-2)
        if step == 0:
            first = float(loss.item())
    torch.cuda.synchronize()
    last = float(loss.item())
    print(f"  {prec}: loss {first:.3e} -> {last:.3e}", flush=True)
    assert last < 1e-3 and last < first / 100


def test_full_batch_gradient_is_the_sum_of_its_halves():
    """At the benchmark's batch (2^18 samples), where the oracle's gradient
    is out of reach: the loss is a mean over samples, so the batch gradient
    equals the sample-weighted mean of the gradients of its two halves.  This
    checks the grid-gradient bins (including bins split over workgroups) and
    the weight-gradient row sums at full size; the halves share the batch's
    64-sample chunks, so only summation order and grouping differ."""
    n = 1 << 18
    w, oc, params, x, nrm, tgt = _setup("room_1080p", n)
    h = n // 2
    loss, g = _gpu_grad(w, params, x, nrm, tgt, "fp16")
    la, ga = _gpu_grad(w, params, x[:h], nrm[:h], tgt[:h], "fp16")
    lb, gb = _gpu_grad(w, params, x[h:], nrm[h:], tgt[h:], "fp16")
    assert loss == pytest.approx((la + lb) / 2, rel=1e-5)
    comb = (ga + gb) / 2
    for name, a in _blocks(oc, g).items():
        b = _blocks(oc, comb)[name]
        rel = np.linalg.norm(a - b) / np.linalg.norm(a)
        mx = np.abs(a - b).max() / np.abs(a).max()
        print(f"  {name}: rel-L2 {rel:.2e}, max/max {mx:.2e}", flush=True)
        assert rel <= 1e-5 and mx <= 1e-4, (name, rel, mx)
