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
