"""GPU q-point functions against the 80-digit reference (forward-stability study, Section 7.1).

hx_qpoint_eval runs the stable forms that the operator kernels use (form "stable") or the
standard forms of Section 3 (form "standard"), in FP64 or FP32. Checked per sample (relative
Frobenius error):
* stable FP64 reproduces P and P' to 1e-12 at every strain scale from 1e-8 to 0.3;
* standard FP64 loses accuracy in the small-strain limit (the effect the stable forms remove);
* stable FP32 stays near FP32 rounding at every scale, while standard FP32 degrades as the
  strain shrinks;
* Algorithm 2 for J^-2/3 (3 steps, FP32) is accurate near J = 1.
"""
import numpy as np
import pytest
import torch

import paper_2408_12479_amd as hx
import workloads
from oracle import stability
from tests.helpers import make_material

pytestmark = pytest.mark.gpu

LAWS = ["cnh", "inh", "fiber"]


def _matkw(mat):
    return dict(mu=mat.mu, lam=mat.lam, kappa=mat.kappa, k1=mat.k1, k2=mat.k2, H4=mat.H4, H6=mat.H6,
                M4=mat.M4, M6=mat.M6)


def _errors(law, scale, form, precision, n=12, jpow=0, seed=5):
    mat = make_material(law)
    H, G = workloads.stability_samples(scale, n, seed=seed)
    Hd = torch.tensor(H, dtype=torch.float64, device="cuda")
    Gd = torch.tensor(G, dtype=torch.float64, device="cuda")
    P, dP = hx.qpoint_eval(Hd, Gd, law, form=form, precision=precision, jpow_newton_iters=jpow, **_matkw(mat))
    P, dP = P.cpu().numpy(), dP.cpu().numpy()
    eP, edP = 0.0, 0.0
    for s in range(n):
        h, g = H[s], G[s]
        if precision == "fp32":   # the reference sees the inputs as the FP32 evaluation does
            h, g = h.astype(np.float32).astype(np.float64), g.astype(np.float32).astype(np.float64)
        rP, rdP = (np.array(x) for x in stability.stress_and_derivative(h, g, mat))
        eP = max(eP, np.linalg.norm(P[s] - rP) / np.linalg.norm(rP))
        edP = max(edP, np.linalg.norm(dP[s] - rdP) / np.linalg.norm(rdP))
    return eP, edP


@pytest.mark.parametrize("law", LAWS)
def test_stable_fp64_accurate_at_all_scales(device, law):
    for scale in [1e-8, 1e-5, 1e-2, 0.3]:
        eP, edP = _errors(law, scale, "stable", "fp64")
        assert eP < 1e-12 and edP < 1e-12, (scale, eP, edP)


@pytest.mark.parametrize("law", LAWS)
def test_standard_fp64_unstable_at_small_strain(device, law):
    eP, _ = _errors(law, 1e-8, "standard", "fp64")
    eS, _ = _errors(law, 1e-8, "stable", "fp64")
    assert eP > 1e-10 and eP > 100 * eS, (eP, eS)
    # and it agrees with the reference at moderate strain
    eP, edP = _errors(law, 0.1, "standard", "fp64")
    assert eP < 1e-12 and edP < 1e-11


@pytest.mark.parametrize("law", LAWS)
def test_fp32_stable_vs_standard(device, law):
    for scale in [1e-7, 1e-4, 1e-2]:
        eP, edP = _errors(law, scale, "stable", "fp32")
        assert eP < 2e-5 and edP < 2e-5, (scale, eP, edP)
    eP_std, _ = _errors(law, 1e-4, "standard", "fp32")
    eP_st, _ = _errors(law, 1e-4, "stable", "fp32")
    assert eP_std > 10 * eP_st, (eP_std, eP_st)


def test_fp32_algorithm2_near_incompressible(device):
    for scale in [1e-6, 1e-3, 1e-2]:
        eP, edP = _errors("inh", scale, "stable", "fp32", jpow=3)
        assert eP < 2e-5 and edP < 2e-5, (scale, eP, edP)
