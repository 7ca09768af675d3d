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

General meshes (connectivity input): ``lattice_as_hex`` writes a lattice as vertex list, cell
corner lists and face boundary ids, optionally with renumbered vertices, shuffled cells and each
cell's local orientation turned by one of the 24 rotations of the cube (seeded); ``ogrid_cylinder``
is a genuinely unstructured mesh (an O-grid of a disk, corner vertices of valence 3, extruded
along z) with curved cells on the outer circle. Curved cells are described by their map sampled at
the (g+1)^3 equispaced points (i/g, j/g, k/g) of the reference cell (``*_geometry_nodes``).
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


# ----------------------------------------------------------------------------------------------
# General (connectivity) meshes and curved cells
# ----------------------------------------------------------------------------------------------
def _cube_rotations():
    """The 24 rotations of the reference cube as signed permutation matrices (det +1)."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            R = np.zeros((3, 3), dtype=np.int64)
            for r in range(3):
                R[r, perm[r]] = signs[r]
            if round(np.linalg.det(R)) == 1:
                out.append(R)
    return out


def _rotated_index(R, m):
    """For a cell whose local points form an (m+1)^3 lattice (x fastest), new_of_old[old index] =
    index of the same point after turning the local frame by R (centred integer coordinates
    u = 2 i - m are mapped by R)."""
    idx = np.arange((m + 1) ** 3)
    i, j, k = idx % (m + 1), (idx // (m + 1)) % (m + 1), idx // (m + 1) ** 2
    u = np.stack([2 * i - m, 2 * j - m, 2 * k - m])
    v = R @ u
    ni, nj, nk = (v + m) // 2
    return ni + (m + 1) * (nj + (m + 1) * nk)


def _rotated_faces(R):
    """new_face_of_old[f]: local face f = (d, side) has outward normal (2 side - 1) e_d."""
    out = np.zeros(6, dtype=np.int64)
    for f in range(6):
        nrm = np.zeros(3, dtype=np.int64)
        nrm[f // 2] = 2 * (f % 2) - 1
        v = R @ nrm
        d = int(np.nonzero(v)[0][0])
        out[f] = 2 * d + (1 if v[d] > 0 else 0)
    return out


def scramble_hex(vertices, cells, face_bid, geom_nodes=None, geom_degree=1, seed=0, frames=None):
    """The same mesh with renumbered vertices, cells in a random order and each cell's local frame
    turned by a random rotation of the cube (seeded). Returns (vertices, cells, face_bid,
    geom_nodes, frames, cell_order) with cell_order[new cell] = old cell."""
    rng = np.random.default_rng(seed)
    vertices = np.asarray(vertices, dtype=np.float64)
    cells = np.asarray(cells, dtype=np.int64)
    face_bid = np.asarray(face_bid, dtype=np.int64)
    nv, ne = len(vertices), len(cells)
    vperm = rng.permutation(nv)          # new id of old vertex v: vperm[v]
    Vn = np.zeros_like(vertices)
    Vn[vperm] = vertices
    order = rng.permutation(ne)
    rots = _cube_rotations()
    Cn = np.zeros_like(cells)
    Fn = np.zeros_like(face_bid)
    Gn = None if geom_nodes is None else np.zeros_like(np.asarray(geom_nodes, dtype=np.float64))
    for new, old in enumerate(order):
        R = rots[rng.integers(len(rots))]
        nidx = _rotated_index(R, 1)
        Cn[new, nidx] = vperm[cells[old]]
        Fn[new, _rotated_faces(R)] = face_bid[old]
        if Gn is not None:
            Gn[new, _rotated_index(R, geom_degree)] = geom_nodes[old]
    Fr = None if frames is None else np.asarray(frames)[order]
    return Vn, Cn, Fn, Gn, Fr, order


def lattice_as_hex(nx, ny, nz, V, periodic=(False, False, False), faces=()):
    """A lattice (vertices V as for the lattice meshes) as connectivity: (vertices, cells [E, 8],
    face_bid [E, 6]) with cells in lattice order, corner a + 2b + 4c at lattice offset (a, b, c),
    and boundary id f + 1 on the cell faces that lie on lattice boundary face f (0..5, x fastest),
    for the faces listed (all six boundary faces when ``faces`` is None)."""
    per = tuple(bool(x) for x in periodic)
    Vx, Vy, Vz = (n + (0 if q else 1) for n, q in zip((nx, ny, nz), per))
    E = nx * ny * nz
    e = np.arange(E)
    ex, ey, ez = e % nx, (e // nx) % ny, e // (nx * ny)
    cells = np.zeros((E, 8), dtype=np.int64)
    for c in range(2):
        for b in range(2):
            for a in range(2):
                cells[:, a + 2 * b + 4 * c] = ((ex + a) % Vx) + Vx * (((ey + b) % Vy) + Vy * ((ez + c) % Vz))
    fb = np.zeros((E, 6), dtype=np.int64)
    pos = (ex, ey, ez)
    ncell = (nx, ny, nz)
    for f in (range(6) if faces is None else faces):
        d, side = f // 2, f % 2
        if per[d]:
            continue
        on = pos[d] == (ncell[d] - 1 if side else 0)
        fb[on, f] = f + 1
    return np.asarray(V, dtype=np.float64).reshape(-1, 3), cells, fb


def tube_geometry_nodes(n_theta, n_wall, n_axial, g, r_in=1.0, wall=0.2, length=10.0, bend=1.0):
    """The curved tube's map sampled at the (g+1)^3 equispaced points of every lattice cell:
    [cells, (g+1)^3, 3], cells x fastest, local point i + (g+1)(j + (g+1) k) at (i/g, j/g, k/g).

    Cell (ei, ej, ek) at local point (s, t, r) sits at lattice coordinates (ei + s, ej + t, ek + r):
    angle -2 pi (ei + s) / n_theta, radius r_in + wall (ej + t) / n_wall, centreline parameter
    length (ek + r) / n_axial (the same map as ``tube_vertices`` at the lattice vertices).
    """
    t1 = np.arange(g + 1) / g
    k3, j3, i3 = np.meshgrid(t1, t1, t1, indexing="ij")
    loc = np.stack([i3.ravel(), j3.ravel(), k3.ravel()], axis=1)       # [(g+1)^3, 3]
    E = n_theta * n_wall * n_axial
    e = np.arange(E)
    ex, ey, ez = e % n_theta, (e // n_theta) % n_wall, e // (n_theta * n_wall)
    th = -2.0 * np.pi * (ex[:, None] + loc[None, :, 0]) / n_theta
    rr = r_in + wall * (ey[:, None] + loc[None, :, 1]) / n_wall
    sa = length * (ez[:, None] + loc[None, :, 2]) / n_axial
    X = bend * np.sin(np.pi * sa / length) + rr * np.cos(th)
    Y = rr * np.sin(th)
    return np.stack([X, Y, sa], axis=-1)


def ogrid_cylinder(m, nz, radius=1.0, inner=0.4, height=1.0, g=1, bottom_bid=1, side_bid=2, top_bid=3):
    """An O-grid of the disk of the given radius extruded over [0, height]: a central square
    [-inner, inner]^2 of m x m cells and four blocks of m x m cells between its sides and the circle
    (radial lines blended linearly from the square's side to the arc), nz layers along z. The
    square's corners are vertices of valence 3 in each layer, so the mesh is not a lattice.

    Returns (vertices, cells [E, 8], face_bid [E, 6], geom_nodes [E, (g+1)^3, 3]): every cell
    right-handed, corner a + 2b + 4c at its local (a, b, c); boundary ids on the bottom (z = 0),
    the curved side and the top; the map of each cell sampled at its equispaced points of degree g
    (the blocks' arcs are then curved for g > 1; g = 1 gives the vertices).
    """
    a = inner

    def block_map(b, u, v):
        # (u, v) in [0,1]^2 of block b -> (x, y); b = 0 square, 1..4 the blocks east, north, west, south
        if b == 0:
            return -a + 2 * a * u, -a + 2 * a * v
        th0 = -0.25 * np.pi + 0.5 * np.pi * (b - 1)
        th = th0 + 0.5 * np.pi * v
        # inner side of the square under the arc, running counter-clockwise
        c, s_ = np.cos(th0 + 0.25 * np.pi), np.sin(th0 + 0.25 * np.pi)   # outward normal of the side
        tx, ty = -s_, c                                                   # counter-clockwise tangent
        px = a * c + a * (2 * v - 1) * tx
        py = a * s_ + a * (2 * v - 1) * ty
        qx, qy = radius * np.cos(th), radius * np.sin(th)
        return (1 - u) * px + u * qx, (1 - u) * py + u * qy

    t1 = np.arange(g + 1) / g
    kk, jj, ii = np.meshgrid(t1, t1, t1, indexing="ij")
    loc = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    corner = np.array([[a_, b_, c_] for c_ in (0, 1) for b_ in (0, 1) for a_ in (0, 1)], dtype=np.float64)
    geo, corners, fbs = [], [], []
    for kz in range(nz):
        for b in range(5):
            for j in range(m):
                for i in range(m):
                    def pts(L):
                        u = (i + L[:, 0]) / m
                        v = (j + L[:, 1]) / m
                        x, y = block_map(b, u, v)
                        z = height * (kz + L[:, 2]) / nz
                        return np.stack([x, y, z], axis=1)
                    geo.append(pts(loc))
                    corners.append(pts(corner))
                    fb = np.zeros(6, dtype=np.int64)
                    if kz == 0:
                        fb[4] = bottom_bid
                    if kz == nz - 1:
                        fb[5] = top_bid
                    if b > 0 and i == m - 1:
                        fb[1] = side_bid
                    fbs.append(fb)
    C = np.array(corners)                                                 # [E, 8, 3]
    # vertices: corner positions merged where they coincide (to 1e-9)
    key = np.round(C.reshape(-1, 3) / (1e-9 * max(radius, height)))
    _, first, inv = np.unique(key, axis=0, return_index=True, return_inverse=True)
    verts = C.reshape(-1, 3)[first]
    cells = inv.reshape(-1, 8)
    return verts, cells, np.array(fbs), np.array(geo)
