"""Pins of the oracle's constitutive functions against derivatives of the strain energy.

The strain energies are the paper's definitions (Section 3). Stresses and moduli are checked
against complex-step derivatives of those energies, so a dropped term, a wrong sign or a
transposed index in the closed forms fails here.
"""
import numpy as np
import pytest

from oracle import material
from tests.helpers import fiber_material, make_material, random_F

H = 1e-30  # complex step


def _complex_step_S(F, mat):
    """S_AB = 2 dPsi/dC_AB by the complex step on Psi(C) (C treated as a general matrix)."""
    C = np.einsum("ki,kj->ij", F, F)
    S = np.zeros((3, 3))
    for a in range(3):
        for b in range(3):
            dC = np.zeros((3, 3), dtype=complex)
            dC[a, b] = 1j * H
            S[a, b] = 2.0 * material.psi(C + dC, mat).imag / H
    return S


def _complex_step_A(F, mat):
    A = np.zeros((3, 3, 3, 3))
    for k in range(3):
        for L in range(3):
            dF = np.zeros((3, 3), dtype=complex)
            dF[k, L] = 1j * H
            A[:, :, k, L] = material.first_pk((F + dF)[None], mat)[0].imag / H
    return A


MATS = {
    "cnh": make_material("cnh", mu=1.0, lam=10.0),
    "inh": make_material("inh", mu=2.0, kappa=1e3),
    "fiber": fiber_material(),
    "fiber_nodisp": fiber_material(dispersion=None),
}


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("scale", [1e-3, 0.1, 0.3])
def test_stress_is_energy_derivative(name, scale):
    mat = MATS[name]
    rng = np.random.default_rng(7)
    for F in random_F(rng, 6, scale):
        S = material.second_pk(F[None], mat)[0]
        Sref = _complex_step_S(F, mat)
        assert np.max(np.abs(S - Sref)) <= 1e-11 * max(1.0, np.max(np.abs(Sref)))
        assert np.max(np.abs(S - S.T)) < 1e-12 * max(1.0, np.max(np.abs(S)))


@pytest.mark.parametrize("name", list(MATS))
@pytest.mark.parametrize("scale", [1e-3, 0.1, 0.3])
def test_first_elasticity_is_derivative_of_P(name, scale):
    mat = MATS[name]
    rng = np.random.default_rng(11)
    for F in random_F(rng, 6, scale):
        A = material.first_elasticity(F[None], mat)[0]
        Aref = _complex_step_A(F, mat)
        assert np.max(np.abs(A - Aref)) <= 1e-11 * np.max(np.abs(Aref))
        # major symmetry of a hyperelastic tangent: A_iJkL = A_kLiJ
        assert np.max(np.abs(A - A.transpose(2, 3, 0, 1))) <= 1e-11 * np.max(np.abs(A))


def test_fiber_switch_active_and_inactive_states_are_both_sampled():
    mat = MATS["fiber"]
    rng = np.random.default_rng(11)
    F = random_F(rng, 200, 0.3)
    C = np.einsum("nki,nkj->nij", F, F)
    I4 = np.einsum("i,nij,j->n", mat.M4, C, mat.M4)
    assert np.any(I4 > 1) and np.any(I4 < 1)


@pytest.mark.parametrize("name", list(MATS))
def test_stress_free_reference_state(name):
    S = material.second_pk(np.eye(3)[None], MATS[name])[0]
    assert np.max(np.abs(S)) < 1e-13


@pytest.mark.parametrize("name", ["cnh", "inh", "fiber"])
def test_linearisation_at_identity_is_isotropic_elasticity(name):
    mat = MATS[name]
    mu = mat.mu
    lam_lin = 2.0 * mat.lam if mat.law == "cnh" else mat.kappa - 2.0 * mu / 3.0
    d = np.eye(3)
    Alin = (lam_lin * np.einsum("ij,kl->ijkl", d, d)
            + mu * (np.einsum("ik,jl->ijkl", d, d) + np.einsum("il,jk->ijkl", d, d)))
    A = material.first_elasticity(np.eye(3)[None], mat)[0]
    assert np.max(np.abs(A - Alin)) < 1e-10 * np.max(np.abs(Alin))


@pytest.mark.parametrize("name", ["cnh", "inh"])
def test_objectivity(name):
    mat = MATS[name]
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    for F in random_F(rng, 5, 0.3):
        S1 = material.second_pk(F[None], mat)[0]
        S2 = material.second_pk((Q @ F)[None], mat)[0]
        assert np.max(np.abs(S1 - S2)) < 1e-12 * np.max(np.abs(S1))
