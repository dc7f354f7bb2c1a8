"""The measurement entry points on the GPU: niv_probe_encode runs the
query's encoding stage alone and writes, per pixel, the XOR of the encoded
input vector as the network would receive it (FP16 pairs), which must equal
the same XOR of the encoded inputs the query itself reports (out_inputs);
niv_probe_gather reads every word of its pattern exactly once per sample and
level corner, so over a table of ones its sums count the gathers."""
import numpy as np
import pytest
import torch

import oracle as O
from niv_synth import get_workload, make_params

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_probe_encode_equals_the_query_encoding():
    from paper_2602_12949_amd import NIV
    w = get_workload("room_1080p")
    oc = O.config_from_workload(w)
    m = NIV(w.model_dict())
    params = make_params(O.n_grid_values(oc), O.mat_shapes(oc), w.param_seed, *w.grid_init)
    pm = m.prepare(torch.from_numpy(params).to(DEV), "fp16")
    rng = np.random.default_rng(8)
    n = 5000 + 37
    pos = rng.uniform([0, 0, 0], [10, 4, 10], size=(n, 3)).astype(np.float32)
    nrm = rng.standard_normal((n, 3)).astype(np.float32)
    mask = (rng.uniform(size=n) > 0.1).astype(np.uint8)
    pos[:5] = [[np.nan, 1, 1]] * 5                       # no work: zero inputs
    pd, nd, md = (torch.from_numpy(a).to(DEV) for a in (pos, nrm, mask))
    E, _, _, inputs = m.query(pd, nd, pm, "fp16", mask=md, want_inputs=True)
    f, outs = m.frame(pd, nd, pm, mask=md)
    outs[0].fill_(float("nan"))
    m.probe_encode(f, "fp16")
    torch.cuda.synchronize()
    got = outs[0].cpu().numpy().reshape(-1, 3)[:, 0].view(np.uint32)
    x = inputs.cpu().numpy().astype(np.float16).view(np.uint16).astype(np.uint32)
    pairs = x[:, 0::2] | (x[:, 1::2] << 16)
    want = np.bitwise_xor.reduce(pairs, axis=1)
    on = mask != 0
    np.testing.assert_array_equal(got[on], want[on])
    assert (want[:5] == 0).all()


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_probe_gather_counts(mode):
    from paper_2602_12949_amd.niv import probe_gather
    table = torch.ones(1 << 21, dtype=torch.int32, device=DEV)
    out = torch.zeros(2048 * 256, dtype=torch.int32, device=DEV)
    n = (1 << 18) + 5
    probe_gather(mode, n, table, out)
    torch.cuda.synchronize()
    assert int(out.sum().item()) == n * 128
