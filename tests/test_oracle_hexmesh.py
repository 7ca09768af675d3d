"""Pins of the oracle's general (connectivity) meshes and curved cells, without a GPU.

* A lattice written as connectivity, with renumbered vertices, shuffled cells and every cell's
  local frame turned by one of the 24 rotations of the cube, reproduces the lattice oracle's
  residual, tangent action and constrained set (which the lattice pins already tie to the paper's
  definitions), node for node under the coordinate matching.
* Node counts equal V + E (p-1) + F (p-1)^2 + C (p-1)^3 on the O-grid (vertices, distinct edges,
  faces and cells counted from the connectivity by brute force).
* Geometry of degree g sampled from a trilinear map reproduces the trilinear results; the volume
  of a body curved by a polynomial map equals its exact value; the discrete divergence theorem
  (the pressure load on a closed curved surface against the volume) holds.
* Rigid rotation gives a zero residual on curved cells; residual and tangent are the complex-step
  derivatives of the energy and the residual on the curved O-grid.
"""
import itertools

import numpy as np
import pytest

import workloads
from oracle import basis, fem, material, mesh
from tests.helpers import make_material


def _match(coords_a, coords_b):
    """perm with coords_b[perm] == coords_a (to 1e-10), by sorting rounded coordinates."""
    ka = np.round(coords_a * 1e9).astype(np.int64)
    kb = np.round(coords_b * 1e9).astype(np.int64)
    oa = np.lexsort(ka.T[::-1])
    ob = np.lexsort(kb.T[::-1])
    perm = np.empty(len(coords_a), dtype=np.int64)
    perm[oa] = ob
    assert np.allclose(coords_b[perm], coords_a, atol=1e-10)
    return perm


def _field(X, scale=0.03):
    return scale * np.stack([np.sin(X[:, 0] + 2 * X[:, 1]), np.cos(X[:, 2] - X[:, 0]), np.sin(3 * X[:, 1] * X[:, 2])])


@pytest.mark.parametrize("p,periodic", [(1, False), (2, False), (3, False), (2, True)])
def test_scrambled_lattice_reproduces_the_lattice_operator(p, periodic):
    nx, ny, nz = (4, 2, 2) if periodic else (3, 2, 2)
    per = (periodic, False, False)
    if periodic:
        V = workloads.tube_vertices(nx, ny, nz, length=1.0, bend=0.3)
    else:
        V = workloads.box_vertices(nx, ny, nz, perturb=0.2, seed=4)
    faces = (2, 5) if periodic else (0, 3)
    lat = mesh.BoxMesh(nx, ny, nz, V, p, dirichlet_faces=faces, periodic=per)
    Vh, C, F = workloads.lattice_as_hex(nx, ny, nz, V, periodic=per, faces=faces)
    Vh, C, F, _, _, _ = workloads.scramble_hex(Vh, C, F, seed=7)
    hexm = mesh.HexMesh(Vh, C, p, face_bid=F, dirichlet_bids=[f + 1 for f in faces])
    assert hexm.n_nodes == lat.n_nodes
    perm = _match(lat.node_coords, hexm.node_coords)       # hex node perm[i] is lattice node i
    np.testing.assert_array_equal(hexm.constrained[perm], lat.constrained)
    mat = make_material("inh", mu=2.0, kappa=50.0)
    pl, ph = fem.Problem(lat, mat), fem.Problem(hexm, mat)
    u = _field(lat.node_coords, 0.005)   # small: zeroing u on the thin wall's faces steepens it
    u[:, lat.constrained] = 0.0
    du = workloads.random_direction(lat.n_nodes, 3, lat.constrained)
    uh = np.zeros_like(u)
    duh = np.zeros_like(du)
    uh[:, perm], duh[:, perm] = u, du
    rl, rh = pl.residual(u), ph.residual(uh)[:, perm]
    yl, yh = pl.apply_tangent(u, du), ph.apply_tangent(uh, duh)[:, perm]
    assert np.linalg.norm(rh - rl) <= 1e-13 * np.linalg.norm(rl)
    assert np.linalg.norm(yh - yl) <= 1e-13 * np.linalg.norm(yl)


def _entity_counts(C):
    edges, faces = set(), set()
    for cell in C:
        for d in range(3):
            for a, b in itertools.product((0, 1), repeat=2):
                ends = []
                for t in (0, 1):
                    c = [0, 0, 0]
                    c[d] = t
                    c[(d + 1) % 3], c[(d + 2) % 3] = a, b
                    ends.append(int(cell[c[0] + 2 * c[1] + 4 * c[2]]))
                edges.add(tuple(sorted(ends)))
            for side in (0, 1):
                vs = []
                for a, b in itertools.product((0, 1), repeat=2):
                    c = [0, 0, 0]
                    c[d] = side
                    c[(d + 1) % 3], c[(d + 2) % 3] = a, b
                    vs.append(int(cell[c[0] + 2 * c[1] + 4 * c[2]]))
                faces.add(tuple(sorted(vs)))
    return len(np.unique(C)), len(edges), len(faces), len(C)


@pytest.mark.parametrize("p", [1, 2, 4])
def test_node_count_by_entity_on_the_ogrid(p):
    V, C, F, G = workloads.ogrid_cylinder(2, 2, g=2)
    V, C, F, G, _, _ = workloads.scramble_hex(V, C, F, G, geom_degree=2, seed=3)
    m = mesh.HexMesh(V, C, p, face_bid=F, geom_degree=2, geom_nodes=G)
    nv, ne, nf, nc = _entity_counts(C)
    assert m.n_nodes == nv + ne * (p - 1) + nf * (p - 1) ** 2 + nc * (p - 1) ** 3
    # every node is met first as some cell's local node, and cell_nodes covers all of them
    assert set(np.unique(m.cell_nodes)) == set(range(m.n_nodes))


def test_geometry_tables_of_degree_one_are_the_trilinear_ones():
    tab = fem.ElementTables(3)
    xe = np.linspace(0.0, 1.0, 2)
    del xe
    tab._geo.pop(1)                  # force the generic construction for g = 1
    np.testing.assert_allclose(tab.geometry_derivatives(1), tab.TN, atol=1e-15)


@pytest.mark.parametrize("g", [2, 3])
def test_degree_g_geometry_reproduces_the_trilinear_map(g):
    nx, ny, nz, p = 2, 2, 3, 2
    V = workloads.box_vertices(nx, ny, nz, perturb=0.25, seed=9)
    lat = mesh.BoxMesh(nx, ny, nz, V, p, dirichlet_faces=(0,))
    t = np.arange(g + 1) / g
    kk, jj, ii = np.meshgrid(t, t, t, indexing="ij")
    G = mesh.trilinear_point(lat.cell_vertex_xyz[:, None], ii.ravel()[None], jj.ravel()[None], kk.ravel()[None])
    cur = mesh.BoxMesh(nx, ny, nz, V, p, dirichlet_faces=(0,), geom_degree=g, geom_nodes=G)
    np.testing.assert_allclose(cur.node_coords, lat.node_coords, atol=1e-14)
    mat = make_material("cnh", mu=1.0, lam=10.0)
    pl, pc = fem.Problem(lat, mat), fem.Problem(cur, mat)
    cells = np.arange(lat.n_cells)
    Kl, wl = pl.geometry(cells)
    Kc, wc = pc.geometry(cells)
    np.testing.assert_allclose(Kc, Kl, rtol=0, atol=1e-12)
    np.testing.assert_allclose(wc, wl, rtol=1e-13)
    u = _field(lat.node_coords)
    u[:, lat.constrained] = 0.0
    du = workloads.random_direction(lat.n_nodes, 5, lat.constrained)
    assert np.linalg.norm(pc.apply_tangent(u, du) - pl.apply_tangent(u, du)) <= 1e-13 * np.linalg.norm(pl.apply_tangent(u, du))


def _curved_unit_cube(n, g, p, amp=0.1):
    """n^3 cells of [0,1]^3 under Phi(x) = x + amp (x1^2 x2, x2^2 x3, x3^2 x1): each cell's map is
    of degree 2 per direction, represented exactly with g >= 2 points per direction."""
    V = workloads.box_vertices(n, n, n)
    t = np.arange(g + 1) / g
    kk, jj, ii = np.meshgrid(t, t, t, indexing="ij")
    e = np.arange(n ** 3)
    ex, ey, ez = e % n, (e // n) % n, e // (n * n)
    x1 = (ex[:, None] + ii.ravel()[None]) / n
    x2 = (ey[:, None] + jj.ravel()[None]) / n
    x3 = (ez[:, None] + kk.ravel()[None]) / n
    G = np.stack([x1 + amp * x1 ** 2 * x2, x2 + amp * x2 ** 2 * x3, x3 + amp * x3 ** 2 * x1], axis=-1)
    return mesh.BoxMesh(n, n, n, V, p, geom_degree=g, geom_nodes=G)


def _exact_volume(amp=0.1, k=8):
    # det of the Jacobian of Phi integrated over [0,1]^3 with a k-point Gauss rule (exact: the
    # integrand has degree <= 2 in each variable)
    x, w = basis.gauss_rule(k)
    X3, X2, X1 = np.meshgrid(x, x, x, indexing="ij")
    W = np.einsum("i,j,k->ijk", w, w, w)
    J = np.zeros(X1.shape + (3, 3))
    J[..., 0, 0] = 1 + 2 * amp * X1 * X2
    J[..., 0, 1] = amp * X1 ** 2
    J[..., 1, 1] = 1 + 2 * amp * X2 * X3
    J[..., 1, 2] = amp * X2 ** 2
    J[..., 2, 2] = 1 + 2 * amp * X3 * X1
    J[..., 2, 0] = amp * X3 ** 2
    return float(np.sum(W * np.linalg.det(J)))


@pytest.mark.parametrize("g,p", [(2, 1), (2, 2), (3, 3)])
def test_volume_of_a_polynomially_curved_body(g, p):
    m = _curved_unit_cube(2, g, p)
    pb = fem.Problem(m, make_material("cnh"))
    _, wdet = pb.geometry(np.arange(m.n_cells))
    vol = _exact_volume()
    assert vol != pytest.approx(1.0, abs=1e-3)
    assert abs(wdet.sum() - vol) < 1e-13


def test_divergence_theorem_on_the_curved_cylinder():
    """For a closed surface, sum_a f_a . X_a = -p int X . N dA = -3 p Vol, and sum_a f_a = 0
    (isoparametric cells, quadrature exact for these polynomials at p = 3, g = 2)."""
    V, C, F, G = workloads.ogrid_cylinder(2, 2, g=2)
    V, C, F, G, _, _ = workloads.scramble_hex(V, C, F, G, geom_degree=2, seed=11)
    m = mesh.HexMesh(V, C, 3, face_bid=F, geom_degree=2, geom_nodes=G)
    pb = fem.Problem(m, make_material("cnh"))
    _, wdet = pb.geometry(np.arange(m.n_cells))
    vol = wdet.sum()
    assert abs(vol - np.pi) < 2e-2 * np.pi    # unit radius and height; degree-2 arcs approximate the circle
    pr = 0.7
    f = sum(fem.surface_load_bid(pb, b, pr) for b in (1, 2, 3))
    np.testing.assert_allclose(f.sum(axis=1), 0.0, atol=1e-13)
    assert abs(np.sum(f * m.node_coords.T) + 3 * pr * vol) < 1e-12
    # the lateral surface alone: horizontal normals, resultant zero by the four-fold symmetry
    fs = fem.surface_load_bid(pb, 2, pr)
    np.testing.assert_allclose(fs.sum(axis=1), 0.0, atol=1e-13)


@pytest.mark.parametrize("p", [2, 3])
def test_rigid_rotation_on_curved_cells(p):
    V, C, F, G = workloads.ogrid_cylinder(2, 1, g=2)
    V, C, F, G, _, _ = workloads.scramble_hex(V, C, F, G, geom_degree=2, seed=5)
    m = mesh.HexMesh(V, C, p, face_bid=F, geom_degree=2, geom_nodes=G)
    th = 0.4
    Q = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    ax = np.array([1.0, 2.0, 2.0]) / 3.0
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    Q = Q @ (np.eye(3) + np.sin(0.3) * K + (1 - np.cos(0.3)) * K @ K)
    X = m.node_coords
    u = (X @ Q.T - X).T
    for law in ("cnh", "inh", "fiber"):
        pb = fem.Problem(m, make_material(law))
        r = pb.residual(u, constrain=False)
        assert np.max(np.abs(r)) < 1e-12, law


def test_complex_step_on_the_curved_ogrid():
    V, C, F, G = workloads.ogrid_cylinder(1, 1, g=2)
    V, C, F, G, _, _ = workloads.scramble_hex(V, C, F, G, geom_degree=2, seed=2)
    m = mesh.HexMesh(V, C, 2, face_bid=F, dirichlet_bids=(1,), geom_degree=2, geom_nodes=G)
    pb = fem.Problem(m, make_material("fiber", dispersion=None))
    u = _field(m.node_coords, 0.05)
    u[:, m.constrained] = 0.0
    h = 1e-30
    rng = np.random.default_rng(4)
    # residual = gradient of the energy (free DoFs), by the complex step along random directions
    r = pb.residual(u)
    for _ in range(3):
        v = rng.standard_normal(u.shape)
        v[:, m.constrained] = 0.0
        d = np.imag(pb.energy(u + 1j * h * v)) / h
        assert abs(d - np.sum(r * v)) <= 1e-10 * abs(d)
    # tangent = derivative of the residual (free rows; constrained rows are identity rows)
    du = workloads.random_direction(m.n_nodes, 6, m.constrained)
    y = pb.apply_tangent(u, du)
    d = np.imag(pb.residual(u + 1j * h * du)) / h
    free = ~m.constrained
    assert np.linalg.norm(y[:, free] - d[:, free]) <= 1e-11 * np.linalg.norm(d[:, free])
