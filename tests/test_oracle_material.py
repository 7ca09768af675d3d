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


@pytest.mark.parametrize("law", ["cnh", "inh", "fiber"])
def test_spatial_linearisation_is_material_one(law):
    # (grad du) tau + J c : sym(grad du) = (A : Grad du) F^T with grad du = Grad du F^-1, and
    # tau = P F^T: the spatial integrand equals the material one (Section 2 derivation)
    from tests.helpers import make_material
    mat = make_material(law)
    rng = np.random.default_rng(17)
    F = np.eye(3)[None] + 0.2 * rng.uniform(-1, 1, size=(6, 3, 3))
    G = rng.standard_normal((6, 3, 3))
    tau = material.kirchhoff_stress(F, mat)
    np.testing.assert_allclose(tau, np.einsum("nij,nkj->nik", material.first_pk(F, mat), F), atol=1e-12)
    c = material.spatial_moduli(F, mat)
    g = np.einsum("nij,njk->nik", G, np.linalg.inv(F))
    eps = 0.5 * (g + np.swapaxes(g, 1, 2))
    lhs = np.einsum("nik,nkj->nij", g, tau) + np.einsum("nijkl,nkl->nij", c, eps)
    A = material.first_elasticity(F, mat)
    rhs = np.einsum("niJ,nkJ->nik", np.einsum("niJkL,nkL->niJ", A, G), F)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-11, atol=1e-11 * np.abs(rhs).max())


def test_spatial_inh_push_forward_uses_b():
    # the iNH volumetric-deviatoric cross term of J c is -2mu/3 J^-2/3 [b tr(e) + (b:e) I] (the
    # push-forward of the symmetrised second derivative), not a term with C
    from tests.helpers import make_material
    mat = make_material("inh")
    rng = np.random.default_rng(3)
    F = np.eye(3) + 0.3 * rng.uniform(-1, 1, size=(3, 3))
    J = np.linalg.det(F)
    b = F @ F.T
    C = F.T @ F
    Jp = J ** (-2.0 / 3.0)
    I1 = np.trace(b)
    c1 = 0.5 * mat.kappa * (J * J - 1) - mat.mu / 3 * Jp * I1
    c2 = 2 * mat.mu / 9 * Jp * I1 + mat.kappa * J * J
    e = rng.standard_normal((3, 3))
    e = 0.5 * (e + e.T)
    ref = np.einsum("ijkl,kl->ij", material.spatial_moduli(F[None], mat)[0], e)
    ours = -2 * mat.mu / 3 * Jp * (b * np.trace(e) + np.sum(b * e) * np.eye(3)) - 2 * c1 * e + c2 * np.trace(e) * np.eye(3)
    np.testing.assert_allclose(ours, ref, atol=1e-10 * np.abs(ref).max())
    printed = -4 * mat.mu / 3 * Jp * np.trace(e) * C - 2 * c1 * e + c2 * np.trace(e) * np.eye(3)
    assert np.abs(printed - ref).max() > 1e-3 * np.abs(ref).max()
