"""The STREAM-triad bandwidth probe (hx_stream_triad) that bench.py uses to state the sustained HBM
rate: a = b + s c, element by element against numpy (the probe is plain FP64 arithmetic, one fused
multiply-add per element, so the two agree to one rounding), odd and even lengths, and its
argument checks."""
import numpy as np
import pytest

import paper_2408_12479_amd as hx

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 7, 512, 513, 100_003])
def test_triad_matches_numpy(device, n):
    import torch
    rng = np.random.default_rng(n)
    b, c = rng.standard_normal(n), rng.standard_normal(n)
    bd, cd = torch.tensor(b, device=device), torch.tensor(c, device=device)
    a = torch.full((n,), np.nan, dtype=torch.float64, device=device)
    hx.stream_triad(a, bd, cd, 0.75)
    ref = b + 0.75 * c
    got = a.cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-15 * (np.abs(b) + np.abs(0.75 * c)))


def test_triad_argument_checks(device):
    import torch
    x = torch.zeros(17, dtype=torch.float64, device=device)
    y = torch.ones(17, dtype=torch.float64, device=device)
    hx.stream_triad(x[:0], y[:0], y[:0], 2.0)  # empty: nothing to do
    with pytest.raises(hx.HxError) as err:
        hx.stream_triad(x[1:], y[1:], y[1:], 2.0)  # 8-byte offset: not 16-byte aligned
    assert err.value.name == "HX_E_ARG"
    assert torch.all(x == 0)
    assert hx.STATUS[hx.lib.hx_stream_triad(-1, None, None, None, 1.0, None)] == "HX_E_ARG"
    assert hx.STATUS[hx.lib.hx_stream_triad(4, None, None, None, 1.0, None)] == "HX_E_ARG"


def test_fp64_pipe_probe_results(device):
    """The FP64 issue-rate probe (hx_fp64_pipe_probe) computes what it states: every vector chain
    is the recurrence x <- x y + z from x0 = 1e-3 c (closed form y^n x0 + z (1 - y^n) / (1 - y)),
    and the matrix chains of each wave sum to iters x 0.129024 whatever the lane layout of the
    matrix instruction; both together give the sum of the two."""
    import torch
    iters = 5
    outs = []
    for kind in range(3):
        out = torch.full((hx.PIPE_PROBE_THREADS,), np.nan, dtype=torch.float64, device=device)
        flops = hx.fp64_pipe_probe(kind, iters, out)
        assert flops == 2048 * 4 * iters * (16384 if kind == 2 else 8192)
        outs.append(out.cpu().numpy())
    y, z, n = 0.999999, 1e-6, 8 * iters
    vec = sum(y ** n * 1e-3 * c + z * (1 - y ** n) / (1 - y) for c in range(8))
    assert np.allclose(outs[0], vec, rtol=1e-13, atol=0)
    waves = outs[1].reshape(-1, 64).sum(axis=1)
    assert np.allclose(waves, iters * 0.129024, rtol=1e-12, atol=0)
    np.testing.assert_allclose(outs[2], outs[0] + outs[1], rtol=1e-12, atol=1e-15)


def test_fp64_pipe_probe_argument_checks(device):
    import torch
    out = torch.zeros(hx.PIPE_PROBE_THREADS, dtype=torch.float64, device=device)
    for kind, iters in ((3, 1), (-1, 1), (0, 0), (1, 1_000_001)):
        assert hx.STATUS[hx.lib.hx_fp64_pipe_probe(kind, iters, out.data_ptr(), None)] == "HX_E_ARG"
    assert hx.STATUS[hx.lib.hx_fp64_pipe_probe(0, 1, None, None)] == "HX_E_ARG"
    assert torch.all(out == 0)
