"""Pins of the 80-digit stress reference of the forward-stability study.

* at moderate strain it equals the FP64 oracle (material.first_pk, pinned by complex-step
  derivatives of Psi) and its directional derivative equals the first elasticity tensor applied to
  G (material.first_elasticity);
* at small strain (1e-8) it equals linear elasticity (isotropic, plus the linearised law of the
  fibre families in tension) to first order;
* the sample generator keeps every entry inside [scale/10, scale] in magnitude and det(I + H) > 0.
"""
import numpy as np
import pytest

import workloads
from oracle import material, stability
from tests.helpers import make_material

LAWS = ["cnh", "inh", "fiber"]


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.mark.parametrize("law", LAWS)
@pytest.mark.parametrize("scale", [1e-3, 1e-1, 0.4])
def test_matches_fp64_oracle_at_moderate_strain(law, scale):
    mat = make_material(law)
    H, G = workloads.stability_samples(scale, 4, seed=1)
    for h, g in zip(H, G):
        P, dP = stability.stress_and_derivative(h, g, mat)
        F = np.eye(3) + h
        assert _rel(P, material.first_pk(F[None], mat)[0]) < 1e-12
        A = material.first_elasticity(F[None], mat)[0]
        assert _rel(dP, np.einsum("iJkL,kL->iJ", A, g)) < 1e-10


@pytest.mark.parametrize("law", LAWS)
def test_small_strain_is_linear_elasticity(law):
    mat = make_material(law)
    lam_lin, mu = (2.0 * mat.lam, mat.mu) if law == "cnh" else (mat.kappa - 2.0 * mat.mu / 3.0, mat.mu)
    H, G = workloads.stability_samples(1e-8, 3, seed=2)
    for h, g in zip(H, G):
        P, dP = stability.stress_and_derivative(h, g, mat)
        eps, deps = 0.5 * (h + h.T), 0.5 * (g + g.T)
        sig = lam_lin * np.trace(eps) * np.eye(3) + 2 * mu * eps
        lin = lam_lin * np.trace(deps) * np.eye(3) + 2 * mu * deps
        for Hf, M in mat.families():
            # active families (M.eps.M > 0) add the linear fibre law 2 k1 (2 H:eps) H
            if M @ eps @ M > 0:
                sig = sig + 2 * mat.k1 * 2 * np.sum(Hf * eps) * Hf
                lin = lin + 2 * mat.k1 * 2 * np.sum(Hf * deps) * Hf
        assert _rel(P, sig) < 1e-6          # O(strain) relative deviation
        assert _rel(dP, lin) < 1e-6


def test_samples():
    for scale in [1e-8, 1e-2, 10.0]:
        H, G = workloads.stability_samples(scale, 50, seed=3)
        assert H.shape == (50, 3, 3) and G.shape == (50, 3, 3)
        assert np.all(np.abs(H) >= scale / 10 * (1 - 1e-12)) and np.all(np.abs(H) <= scale * (1 + 1e-12))
        assert np.all(np.linalg.det(np.eye(3) + H) > 0)
