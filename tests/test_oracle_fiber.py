"""Pins of the fibre structure tensors: the paper's worked example and frame geometry."""
import os

import numpy as np

from oracle import fiber

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fiber_parameters_table.txt")


def test_dispersion_table_worked_example():
    rows = np.loadtxt(GOLDEN, ndmin=2)
    for a, b, h11, h22, h33 in rows:
        H11, H22, H33 = fiber.dispersion_coefficients(a, b)
        # printed to four digits
        assert abs(H11 - h11) < 5e-5 and abs(H22 - h22) < 5e-5 and abs(H33 - h33) < 5e-5
        assert abs(H11 + H22 + H33 - 1.0) < 1e-15


def test_dispersion_limits():
    # a, b -> infinity: all density along the mean fibre (H11 -> 1); a -> 0: isotropic in-plane
    H11, H22, H33 = fiber.dispersion_coefficients(400.0, 1e4)
    assert H11 > 0.998 and H22 < 2e-3 and H33 < 1e-4
    H11, H22, _ = fiber.dispersion_coefficients(1e-8, 34.3)
    assert abs(H11 - H22) < 1e-8


def test_frames_orthonormal_and_angles():
    E1, E2, E3 = np.eye(3)
    phi = np.deg2rad(27.47)
    for sign, (M1, M2, M3) in zip((1, -1), fiber.family_frames(E1, E2, E3, phi)):
        R = np.stack([M1, M2, M3])
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-15)
        assert abs(np.linalg.det(R) - 1.0) < 1e-15
        assert abs(np.dot(M1, E1) - np.cos(phi)) < 1e-15
        assert abs(np.dot(M1, E2) - sign * np.sin(phi)) < 1e-15
        assert abs(np.dot(M1, E3)) < 1e-15
    H4, H6, M4, M6 = fiber.structure_tensors(E1, E2, E3, phi, 0.9, 0.07, 0.03)
    assert abs(np.trace(H4) - 1.0) < 1e-15 and abs(np.trace(H6) - 1.0) < 1e-15
    np.testing.assert_allclose(H4 @ M4, 0.9 * M4, atol=1e-15)
