"""Seeded synthetic inputs for the operator configurations (shared by the tests and the benchmark).

This module holds NONE of the method's arithmetic: no basis functions, quadrature, kinematics or
material laws. It produces lattice vertex positions, analytic displacement fields sampled at
given node coordinates, random directions, and the topological Dirichlet mask of a lattice.
Node coordinates are an input (each side computes its own: the oracle in numpy, the library in
its C++ host code), so nothing here depends on either implementation.

Workload recipes (stand-ins for the paper's unspecified "deformed cube", Section 7.2):

* ``cube_small``  4^3 cells on [0,1]^3, Q2, cNH mu=1 lambda=10; u = 0.05 sin(pi x) sin(pi y)
  sin(pi z) in each component + U(-1e-3, 1e-3) noise (seed 0, drawn over [3][n_nodes]);
  du ~ N(0,1) (seed 1); homogeneous Dirichlet on x = 0 (constrained entries zeroed).
* ``cube_sweep``  32^3 cells on [0,1]^3, interior vertices perturbed by U(-0.2h, 0.2h) per
  coordinate (seed 2), Q_p p = 2, 3, 4, 6; cNH mu=1 lambda=100; u = alpha s(x) (1,1,1) with
  s = sin(pi x) sin(pi y) sin(pi z) and alpha such that the largest principal stretch of the
  continuous field over the cube is 1.3; du ~ N(0,1) (seed 3); Dirichlet on x = 0.
* ``fiber_box``   64x32x32 cells on [0,2]x[0,1]^2, Q3; iNH mu=2 (c10=1) kappa=1e3 plus two fibre
  families at +-45 deg in the x-y plane, k1=1, k2=10; u = alpha grad(psi),
  psi = sin(pi x) sin(pi y) sin(pi z) / pi, alpha such that max |J - 1| = 0.05 for the
  continuous field; du ~ N(0,1) (seed 4); no constraints.
"""
import functools

import numpy as np

FACE_MINUS_X, FACE_PLUS_X, FACE_MINUS_Y, FACE_PLUS_Y, FACE_MINUS_Z, FACE_PLUS_Z = range(6)


def box_vertices(nx, ny, nz, lengths=(1.0, 1.0, 1.0), perturb=0.0, seed=None):
    """Vertices of an nx x ny x nz lattice on [0,Lx]x[0,Ly]x[0,Lz], x fastest: [(nx+1)(ny+1)(nz+1), 3].

    With ``perturb`` > 0 every *interior* vertex coordinate is moved by U(-perturb*h_d, perturb*h_d),
    h_d = L_d / n_d, drawn from numpy.random.default_rng(seed) as one [n_vertices, 3] array
    (boundary vertices keep their position, so the faces stay planar and the volume is exact).
    """
    xs = [np.linspace(0.0, L, m + 1) for L, m in zip(lengths, (nx, ny, nz))]
    Z, Y, X = np.meshgrid(xs[2], xs[1], xs[0], indexing="ij")
    V = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if perturb > 0.0:
        rng = np.random.default_rng(seed)
        h = np.array([L / m for L, m in zip(lengths, (nx, ny, nz))])
        noise = rng.uniform(-1.0, 1.0, size=V.shape) * perturb * h[None, :]
        vi = np.arange(V.shape[0])
        ix, iy, iz = vi % (nx + 1), (vi // (nx + 1)) % (ny + 1), vi // ((nx + 1) * (ny + 1))
        interior = (ix > 0) & (ix < nx) & (iy > 0) & (iy < ny) & (iz > 0) & (iz < nz)
        V[interior] += noise[interior]
    return V


def lattice_dirichlet_mask(ndims, faces, periodic=(False, False, False)):
    """Boolean [n_nodes] mask of lattice nodes lying on the given boundary faces (0..5)."""
    Nx, Ny, Nz = ndims
    node = np.arange(Nx * Ny * Nz)
    lat = (node % Nx, (node // Nx) % Ny, node // (Nx * Ny))
    mask = np.zeros(node.shape, dtype=bool)
    for f in faces:
        d, side = f // 2, f % 2
        if periodic[d]:
            continue
        mask |= lat[d] == (0 if side == 0 else ndims[d] - 1)
    return mask


def sine_bump(coords):
    x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def _sine_bump_grad(x, y, z):
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx, cy, cz = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    return np.pi * np.stack([cx * sy * sz, sx * cy * sz, sx * sy * cz], axis=-1)


def small_cube_fields(coords, mask, amplitude=0.05, noise=1e-3):
    """(u, du) of the 4^3 Q2 workload: seeds 0 (noise) and 1 (direction), [3, n_nodes] each."""
    n = coords.shape[0]
    u = np.tile(amplitude * sine_bump(coords), (3, 1))
    u += np.random.default_rng(0).uniform(-noise, noise, size=(3, n))
    du = np.random.default_rng(1).standard_normal((3, n))
    u[:, mask] = 0.0
    du[:, mask] = 0.0
    return u, du


def _max_stretch_of_bump(alpha, samples=41):
    t = np.linspace(0.0, 1.0, samples)
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    g = _sine_bump_grad(X.ravel(), Y.ravel(), Z.ravel())          # [M, 3]
    H = alpha * np.ones(3)[None, :, None] * g[:, None, :]           # H_cJ = alpha * g_J
    F = np.eye(3)[None] + H
    C = np.einsum("mki,mkj->mij", F, F)
    return np.sqrt(np.max(np.linalg.eigvalsh(C)[:, -1])), np.min(np.linalg.det(F))


@functools.lru_cache(maxsize=None)
def bump_amplitude_for_stretch(target=1.3):
    """alpha with max principal stretch of u = alpha s(x)(1,1,1) equal to ``target`` (bisection)."""
    lo, hi = 0.0, 1.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if _max_stretch_of_bump(mid)[0] < target:
            lo = mid
        else:
            hi = mid
    alpha = 0.5 * (lo + hi)
    if _max_stretch_of_bump(alpha)[1] <= 0.0:
        raise ValueError("field inverts the cube")
    return alpha


def sweep_fields(coords, mask, seed_du=3, stretch=1.3):
    """(u, du) of the 32^3 operator-sweep workload."""
    alpha = bump_amplitude_for_stretch(stretch)
    u = np.tile(alpha * sine_bump(coords), (3, 1))
    du = np.random.default_rng(seed_du).standard_normal((3, coords.shape[0]))
    u[:, mask] = 0.0
    du[:, mask] = 0.0
    return u, du


def _grad_psi(coords):
    # psi = sin(pi x) sin(pi y) sin(pi z) / pi  ->  grad psi = grad(s) / pi
    return _sine_bump_grad(coords[:, 0], coords[:, 1], coords[:, 2]) / np.pi


def _max_dev_J(alpha, lengths=(2.0, 1.0, 1.0), samples=(61, 31, 31)):
    ax = [np.linspace(0.0, L, m) for L, m in zip(lengths, samples)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    x, y, z = X.ravel(), Y.ravel(), Z.ravel()
    sx, sy, sz = np.sin(np.pi * x), np.sin(np.pi * y), np.sin(np.pi * z)
    cx, cy, cz = np.cos(np.pi * x), np.cos(np.pi * y), np.cos(np.pi * z)
    # Hessian of psi = pi * [[-s s s, c c s, c s c], ...]
    Hs = np.pi * np.stack([
        np.stack([-sx * sy * sz, cx * cy * sz, cx * sy * cz], -1),
        np.stack([cx * cy * sz, -sx * sy * sz, sx * cy * cz], -1),
        np.stack([cx * sy * cz, sx * cy * cz, -sx * sy * sz], -1)], -2)
    J = np.linalg.det(np.eye(3)[None] + alpha * Hs)
    return np.max(np.abs(J - 1.0))


@functools.lru_cache(maxsize=None)
def gradient_field_amplitude(target=0.05):
    lo, hi = 0.0, 1.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if _max_dev_J(mid) < target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def fiber_fields(coords, seed_du=4, target=0.05):
    """(u, du) of the anisotropic 64x32x32 workload (u = alpha grad psi, no constraints)."""
    alpha = gradient_field_amplitude(target)
    u = np.ascontiguousarray((alpha * _grad_psi(coords)).T)
    du = np.random.default_rng(seed_du).standard_normal((3, coords.shape[0]))
    return u, du


def tube_vertices(n_theta, n_wall, n_axial, r_in=1.0, wall=0.2, length=10.0, bend=1.0):
    """Vertices of a curved tube, periodic in the first lattice direction: [n_wall+1][n_theta]... x fastest.

    Lattice index 1 runs around the circumference (periodic, so n_theta vertices), index 2
    through the wall from r_in to r_in + wall, index 3 along the centreline
    x_c(s) = (bend sin(pi s / length), 0, s), s in [0, length]; each cross-section lies in the
    x-y plane. The angle decreases with the first index so that the lattice frame
    (circumferential, radial, axial) is right-handed.
    """
    th = -2.0 * np.pi * np.arange(n_theta) / n_theta
    r = r_in + wall * np.arange(n_wall + 1) / n_wall
    s = length * np.arange(n_axial + 1) / n_axial
    S, Rr, Th = np.meshgrid(s, r, th, indexing="ij")
    X = bend * np.sin(np.pi * S / length) + Rr * np.cos(Th)
    Y = Rr * np.sin(Th)
    return np.stack([X.ravel(), Y.ravel(), S.ravel()], axis=1)


def tube_frames(n_theta, n_wall, n_axial, length=10.0, bend=1.0):
    """Local fibre frames of the tube cells [cells, 3, 3] (rows E1, E2, E3, cells x fastest).

    At each cell centre (angle and centreline parameter of the cell's middle): E2 is the unit
    tangent of the centreline, E1 the circumferential direction of increasing angle made
    orthogonal to E2, E3 = E1 x E2 (the outward radial direction for a straight tube).
    """
    th = -2.0 * np.pi * (np.arange(n_theta) + 0.5) / n_theta
    s = length * (np.arange(n_axial) + 0.5) / n_axial
    S, _, Th = np.meshgrid(s, np.arange(n_wall), th, indexing="ij")
    S, Th = S.ravel(), Th.ravel()
    t = np.stack([bend * np.pi / length * np.cos(np.pi * S / length), np.zeros_like(S), np.ones_like(S)], axis=1)
    t /= np.linalg.norm(t, axis=1, keepdims=True)
    e1 = np.stack([-np.sin(Th), np.cos(Th), np.zeros_like(Th)], axis=1)
    e1 -= np.sum(e1 * t, axis=1, keepdims=True) * t
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e3 = np.cross(e1, t)
    return np.stack([e1, t, e3], axis=1)


def stability_samples(scale, n, seed):
    """Displacement gradients for the forward-stability study: every entry uniform in
    [scale/10, scale] with a random sign (the band below scale/10 left out so the sample has the
    intended order of magnitude); samples with det(I + H) <= 0 are drawn again. Also a direction
    G with entries uniform in [-1, 1]. Returns (H [n, 3, 3], G [n, 3, 3])."""
    rng = np.random.default_rng(seed)
    out = np.zeros((0, 3, 3))
    while len(out) < n:
        mag = rng.uniform(scale / 10.0, scale, size=(2 * n, 3, 3))
        sign = np.where(rng.random((2 * n, 3, 3)) < 0.5, -1.0, 1.0)
        H = mag * sign
        ok = np.linalg.det(np.eye(3) + H) > 0.0
        out = np.concatenate([out, H[ok]])
    G = rng.uniform(-1.0, 1.0, size=(n, 3, 3))
    return out[:n], G


def random_direction(n_nodes, seed, mask=None):
    du = np.random.default_rng(seed).standard_normal((3, n_nodes))
    if mask is not None:
        du[:, mask] = 0.0
    return du
