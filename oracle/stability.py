"""High-precision reference for the forward-stability study of the q-point functions (Section 7.1).

For a displacement gradient H and a direction G: the first Piola-Kirchhoff stress P = F S(C) of
each law (the standard forms of Section 3, evaluated in 80-digit arithmetic, where the cancellations
that make them unstable in floating point cost nothing) and its directional derivative
P'(H)[G] = d/dt P(H + t G) at t = 0 by a central difference with step 1e-25 (truncation ~1e-50).

Pure-Python mpmath loops: for a few hundred samples only. Test infrastructure only. Pinned in
tests/test_oracle_stability.py against the FP64 oracle (material.first_pk and
material.first_elasticity) at moderate strain, and against isotropic linear elasticity at small
strain.
"""
import mpmath as mp

DPS = 80
STEP = mp.mpf("1e-25")


def _mat(A):
    return mp.matrix([[A[i][j] for j in range(3)] for i in range(3)])


def _stress(H, mat):
    """P(I + H) as an mpmath 3x3 matrix (H: mpmath matrix)."""
    F = mp.eye(3) + H
    C = F.T * F
    J = mp.det(F)
    Ci = C ** -1
    lnJ = mp.log(J)
    I = mp.eye(3)
    if mat.law == "cnh":
        S = mat.mu * (I - Ci) + 2 * mat.lam * lnJ * Ci
    else:
        Jp = J ** (mp.mpf(-2) / 3)
        I1 = C[0, 0] + C[1, 1] + C[2, 2]
        c1 = mp.mpf(mat.kappa) / 2 * (J * J - 1) - mp.mpf(mat.mu) / 3 * Jp * I1
        S = mat.mu * Jp * I + c1 * Ci
        for Hf, M in mat.families():
            Hm = _mat(Hf)
            Ei = sum(Hm[i, j] * C[i, j] for i in range(3) for j in range(3)) - (Hm[0, 0] + Hm[1, 1] + Hm[2, 2])
            Istar = sum(M[i] * C[i, j] * M[j] for i in range(3) for j in range(3))
            if Istar > 1:
                S = S + 2 * mat.k1 * mp.exp(mat.k2 * Ei ** 2) * Ei * Hm
    return F * S


def stress_and_derivative(H, G, mat):
    """(P, P') as nested float lists [3][3], from H, G given as 3x3 nested sequences of floats."""
    with mp.workdps(DPS):
        Hm, Gm = _mat([[mp.mpf(float(H[i][j])) for j in range(3)] for i in range(3)]), \
            _mat([[mp.mpf(float(G[i][j])) for j in range(3)] for i in range(3)])
        P = _stress(Hm, mat)
        dP = (_stress(Hm + STEP * Gm, mat) - _stress(Hm - STEP * Gm, mat)) / (2 * STEP)
        return ([[float(P[i, j]) for j in range(3)] for i in range(3)],
                [[float(dP[i, j]) for j in range(3)] for i in range(3)])
