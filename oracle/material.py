"""Strain energies, stresses and tangent moduli of the three laws (Section 3 and the appendix).

All functions take batched tensors ``[..., 3, 3]`` (float64 or complex128, so that tests can
differentiate them by the complex step) and return plain closed forms, without the stable
rewritings of Section 4; those rewritings are exact in real arithmetic and belong to the GPU
path, whose results the oracle defines.

Laws (Section 3):

* cNH:   Psi = mu/2 (I1 - 3 - 2 ln J) + lambda ln^2 J           (lambda enters as printed)
* iNH:   Psi = mu/2 (J^(-2/3) I1 - 3) + kappa/4 (J^2 - 1 - 2 ln J)
* fibre: Psi = Psi_iNH + sum_{i=4,6} k1/(2 k2) [exp(k2 E_i^2) - 1]  if I*_i > 1 (else 0),
         E_i = H_i : (C - I),  I*_i = (M_i (x) M_i) : C, each family with its own mean direction.

Second Piola-Kirchhoff stress S = 2 dPsi/dC (Section 3, standard forms), fourth-order moduli
CC = 4 d^2Psi/dCdC (appendix) and the first elasticity tensor A_iJkL = dP_iJ/dF_kL with P = F S.

The structure tensors H_i [..., 3, 3] and directions M_i [..., 3] may carry leading dimensions that
broadcast against those of F (fibre frames that vary from cell to cell).

Reading of the appendix: the iNH second derivative is printed with the single term
-mu/3 J^(-2/3) I (x) C^-1, which lacks major symmetry and disagrees with the directional
derivative of Section 5 that the same appendix derives; differentiating Psi gives the symmetric
pair -mu/6 J^(-2/3) (I (x) C^-1 + C^-1 (x) I) (times 4 here). The main-text iNH directional
derivative also carries a sign error on its c1 term (the appendix form with D C^-1 = -2 [..]^S
is the consistent one). The oracle is built from Psi, and the tests pin S and A against
complex-step derivatives of Psi, so neither printed slip can enter.

Test infrastructure only. Pinned in tests/test_oracle_material.py.
"""
from dataclasses import dataclass, field

import numpy as np

LAWS = ("cnh", "inh", "fiber")


@dataclass
class Material:
    law: str
    mu: float
    lam: float = 0.0
    kappa: float = 0.0
    k1: float = 0.0
    k2: float = 0.0
    H4: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))
    H6: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))
    M4: np.ndarray = field(default_factory=lambda: np.zeros(3))
    M6: np.ndarray = field(default_factory=lambda: np.zeros(3))

    def __post_init__(self):
        if self.law not in LAWS:
            raise ValueError(f"unknown law {self.law}")

    def families(self):
        if self.law != "fiber":
            return []
        return [(np.asarray(self.H4, float), np.asarray(self.M4, float)),
                (np.asarray(self.H6, float), np.asarray(self.M6, float))]


def _eye(shape, dtype):
    out = np.zeros(shape + (3, 3), dtype=dtype)
    out[..., 0, 0] = out[..., 1, 1] = out[..., 2, 2] = 1.0
    return out


def _ddot(A, B):
    return np.einsum("...ij,...ij->...", A, B)


def psi(C, mat):
    """Strain-energy density per unit reference volume as a function of C (Section 3)."""
    C = np.asarray(C)
    detC = np.linalg.det(C)
    lnJ = 0.5 * np.log(detC)
    I1 = np.trace(C, axis1=-2, axis2=-1)
    if mat.law == "cnh":
        return 0.5 * mat.mu * (I1 - 3.0 - 2.0 * lnJ) + mat.lam * lnJ ** 2
    Jm23 = np.exp(-2.0 / 3.0 * lnJ)
    J2 = detC
    out = 0.5 * mat.mu * (Jm23 * I1 - 3.0) + 0.25 * mat.kappa * (J2 - 1.0 - 2.0 * lnJ)
    for H, M in mat.families():
        Ei = _ddot(np.broadcast_to(H, C.shape), C) - np.trace(H, axis1=-2, axis2=-1)
        Istar = np.einsum("...i,...ij,...j->...", M, C, M)
        term = mat.k1 / (2.0 * mat.k2) * (np.exp(mat.k2 * Ei ** 2) - 1.0)
        out = out + np.where(np.real(Istar) > 1.0, term, 0.0)
    return out


def kinematics(F):
    """C = F^T F, C^-1, J = det F, ln J, I1 = tr C (plain definitions)."""
    C = np.einsum("...ki,...kj->...ij", F, F)
    Ci = np.linalg.inv(C)
    J = np.linalg.det(F)
    return C, Ci, J, np.log(J), np.trace(C, axis1=-2, axis2=-1)


def second_pk(F, mat):
    """S(F) in the standard (printed) forms of Section 3."""
    C, Ci, J, lnJ, I1 = kinematics(F)
    I = _eye(F.shape[:-2], F.dtype)
    if mat.law == "cnh":
        return mat.mu * I - (mat.mu - 2.0 * mat.lam * lnJ)[..., None, None] * Ci
    Jp = np.exp(-2.0 / 3.0 * lnJ)
    c1 = 0.5 * mat.kappa * (J ** 2 - 1.0) - mat.mu / 3.0 * Jp * I1
    S = mat.mu * Jp[..., None, None] * I + c1[..., None, None] * Ci
    for H, M in mat.families():
        Ei = _ddot(np.broadcast_to(H, C.shape), C) - np.trace(H, axis1=-2, axis2=-1)
        Istar = np.einsum("...i,...ij,...j->...", M, C, M)
        c3 = np.where(np.real(Istar) > 1.0, 2.0 * mat.k1 * np.exp(mat.k2 * Ei ** 2), 0.0)
        S = S + (c3 * Ei)[..., None, None] * H
    return S


def moduli(F, mat):
    """CC_ABCD = 4 d^2 Psi / dC_AB dC_CD (appendix, with the symmetric iNH term)."""
    C, Ci, J, lnJ, I1 = kinematics(F)
    I = _eye(F.shape[:-2], F.dtype)
    CiCi_sym = 0.5 * (np.einsum("...ac,...bd->...abcd", Ci, Ci) + np.einsum("...ad,...bc->...abcd", Ci, Ci))
    CixCi = np.einsum("...ab,...cd->...abcd", Ci, Ci)

    def s(x):
        return x[..., None, None, None, None]

    if mat.law == "cnh":
        return 2.0 * s(mat.mu - 2.0 * mat.lam * lnJ) * CiCi_sym + 2.0 * mat.lam * CixCi
    Jp = np.exp(-2.0 / 3.0 * lnJ)
    IxCi = np.einsum("...ab,...cd->...abcd", I, Ci)
    CixI = np.einsum("...ab,...cd->...abcd", Ci, I)
    CC = (-2.0 * mat.mu / 3.0) * s(Jp) * (IxCi + CixI) \
        + s(2.0 * mat.mu / 3.0 * Jp * I1 - mat.kappa * (J ** 2 - 1.0)) * CiCi_sym \
        + s(2.0 * mat.mu / 9.0 * Jp * I1 + mat.kappa * J ** 2) * CixCi
    for H, M in mat.families():
        Ei = _ddot(np.broadcast_to(H, C.shape), C) - np.trace(H, axis1=-2, axis2=-1)
        Istar = np.einsum("...i,...ij,...j->...", M, C, M)
        coef = np.where(np.real(Istar) > 1.0,
                        4.0 * mat.k1 * np.exp(mat.k2 * Ei ** 2) * (2.0 * mat.k2 * Ei ** 2 + 1.0), 0.0)
        CC = CC + s(coef) * np.einsum("...ab,...cd->...abcd", H, H)
    return CC


def first_pk(F, mat):
    """P = F S."""
    return np.einsum("...ia,...aj->...ij", F, second_pk(F, mat))


def kirchhoff_stress(F, mat):
    """tau = F S F^T (Section 2, spatial residual)."""
    return np.einsum("...ia,...ab,...jb->...ij", F, second_pk(F, mat), F)


def spatial_moduli(F, mat):
    """J c_ijkl = F_iA F_jB CC_ABCD F_kC F_lD: the push-forward of the material moduli (Section 2,
    spatial linearisation), taken from CC by its definition rather than from printed forms."""
    return np.einsum("...ia,...jb,...abcd,...kc,...ld->...ijkl", F, F, moduli(F, mat), F, F)


def first_elasticity(F, mat):
    """A_iJkL = delta_ik S_JL + F_iA CC_AJCL F_kC  (= dP_iJ / dF_kL)."""
    S = second_pk(F, mat)
    CC = moduli(F, mat)
    I3 = np.eye(3)
    geo = np.einsum("ik,...jl->...ijkl", I3, S)
    mat_part = np.einsum("...ia,...ajcl,...kc->...ijkl", F, CC, F)
    return geo + mat_part
