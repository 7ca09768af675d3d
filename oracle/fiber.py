"""Fibre frame and generalised structure tensors of the dispersed two-fibre model (Section 3).

* H11, H22, H33 from the dispersion parameters (a, b): H33 from b through the error function,
  H11/H22 split the remaining 1 - H33 with the ratio of modified Bessel functions I1(a)/I0(a).
* Directions of family i: the mean fibre direction M1 lies in the E1-E2 plane at the mean
  in-plane angle Phi, M2 is the in-plane normal to it, M3 = E3 (out-of-plane angle Theta = 0).
  The printed formulas for M1 and M2 are garbled (each repeats one basis vector); the reading
  used here is M1 = cos(Phi) E1 + sin(Phi) E2, M2 = -sin(Phi) E1 + cos(Phi) E2, which gives an
  orthonormal right-handed frame. The second family uses -Phi (the symmetric helix).
* H_i = H11 M1 (x) M1 + H22 M2 (x) M2 + H33 M3 (x) M3.

Test infrastructure only. Pinned in tests/test_oracle_fiber.py by the worked example of the
fibre-parameter table (a = 3.62, b = 34.3 -> 0.9168, 0.0759, 0.0073; tests/golden/), by
H11 + H22 + H33 = 1, and by orthonormality of the frame.
"""
import numpy as np
from scipy import special


def dispersion_coefficients(a, b):
    """(H11, H22, H33) of the bivariate von Mises fibre density (Section 3)."""
    H33 = 1.0 / (4.0 * b) - np.exp(-2.0 * b) / (np.sqrt(2.0 * np.pi * b) * special.erf(np.sqrt(2.0 * b)))
    ratio = special.i1(a) / special.i0(a)
    H11 = 0.5 * (1.0 - H33) * (1.0 + ratio)
    H22 = 0.5 * (1.0 - H33) * (1.0 - ratio)
    return H11, H22, H33


def family_frames(E1, E2, E3, phi):
    """[(M1, M2, M3) for family 4 (angle +phi), (M1, M2, M3) for family 6 (angle -phi)]."""
    E1, E2, E3 = (np.asarray(v, dtype=np.float64) for v in (E1, E2, E3))
    out = []
    for ang in (phi, -phi):
        c, s = np.cos(ang), np.sin(ang)
        out.append((c * E1 + s * E2, -s * E1 + c * E2, E3.copy()))
    return out


def structure_tensors(E1, E2, E3, phi, H11, H22, H33):
    """(H_4, H_6, M_4, M_6): structure tensors and mean fibre directions of both families."""
    Hs, Ms = [], []
    for M1, M2, M3 in family_frames(E1, E2, E3, phi):
        Hs.append(H11 * np.outer(M1, M1) + H22 * np.outer(M2, M2) + H33 * np.outer(M3, M3))
        Ms.append(M1)
    return Hs[0], Hs[1], Ms[0], Ms[1]


def cell_structure_tensors(frames, phi, H11, H22, H33):
    """Per-cell (H4 [E,3,3], H6, M4 [E,3], M6) from local frames [E, 3, 3] (rows E1, E2, E3)."""
    frames = np.asarray(frames, dtype=np.float64)
    out = [np.zeros((len(frames), 3, 3)), np.zeros((len(frames), 3, 3)),
           np.zeros((len(frames), 3)), np.zeros((len(frames), 3))]
    for e, (E1, E2, E3) in enumerate(frames):
        for k, t in enumerate(structure_tensors(E1, E2, E3, phi, H11, H22, H33)):
            out[k][e] = t
    return tuple(out)
