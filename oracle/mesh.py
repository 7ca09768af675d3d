"""Structured hexahedral lattices with continuous Q_p Lagrange nodes, written out plainly.

A mesh is an nx x ny x nz lattice of hexahedra whose vertex positions are given (so interior
vertices can be perturbed, making the trilinear element maps non-affine: the "deformed cube" of
Section 7.2). Any lattice direction may be periodic (the last vertex plane is then identified
with the first), which closes a tube in the circumferential direction.

Numbering conventions (the library documents the same contract in its public header; the two
implementations are independent):

* cells:    e = ex + nx * (ey + ny * ez)                              (x fastest)
* vertices: v = vx + Vx * (vy + Vy * vz),  Vd = nd (+1 if not periodic)
* nodes:    the (N_x, N_y, N_z) lattice of GLL points, N_d = nd*p (+1 if not periodic),
            node = I + N_x * (J + N_y * K)
* element-local node (i, j, k) in [0, p]^3, a = i + n*(j + n*k), n = p + 1
* vectors:  structure-of-arrays [3][n_nodes], DoF index c * n_nodes + node

Boundary faces are numbered 0..5 = -x, +x, -y, +y, -z, +z. A node is constrained (homogeneous
Dirichlet data, the test space H^1_0 of Problems 2.1/2.2 in Section 2) when it lies on a face in
``dirichlet_faces``.

Geometry of a cell: by default the trilinear map of its 8 vertices; optionally a polynomial map
of degree g given by its values at the (g+1)^3 equispaced points of the reference cell
(``geom_degree``, ``geom_nodes`` [n_cells, (g+1)^3, 3], local index i + (g+1)(j + (g+1) k) for
the point (i/g, j/g, k/g)), as high-order mesh files describe curved cells. With g = 1 the
equispaced points are the vertices and the map is the trilinear one.

``HexMesh`` is a general conforming mesh of hexahedra given by connectivity (vertex ids of each
cell's corners), with boundary ids on cell faces. Its Q_p nodes are numbered in first-touch
order: cells in order, each cell's local nodes in lexicographic order (x fastest), a node getting
the next free number where it is first met. Which local nodes of different cells are the same
node is decided from the vertex ids alone: local node (i, j, k) of a cell is identified by the
multiset of (vertex id, w) over the cell's corners with nonzero trilinear weight numerator
w = (i or p - i)(j or p - j)(k or p - k); a node on a shared vertex, edge or face has weights on
that vertex, edge or face's corners only, and the same weights seen from every cell that shares
it, whatever the cells' local orientations. (Meshes in which two distinct edges join the same two
vertices, or two distinct faces the same four, are outside this contract.)

Test infrastructure only. Pinned in tests/test_oracle_mesh.py (vertex reproduction, volume of
the perturbed unit cube, periodic identification, node counts) and tests/test_oracle_hexmesh.py
(a lattice given as connectivity with renumbered vertices, shuffled cells and rotated local
orientations reproduces the lattice operator; node counts by entity; geometry of degree g that
reproduces a trilinear map; the exact volume of a polynomially curved body).
"""
import numpy as np

from . import basis


def equispaced_points(g):
    """The g+1 geometry interpolation points i/g of the reference interval [0, 1]."""
    return np.linspace(0.0, 1.0, g + 1)


def geometry_map(Xg, g, s, t, r):
    """Map of a cell of degree g (values Xg [..., (g+1)^3, 3] at the equispaced points) at the
    reference points (s, t, r), broadcast against the leading dimensions of Xg."""
    xe = equispaced_points(g)
    s, t, r = (np.atleast_1d(np.asarray(v, dtype=np.float64)) for v in (s, t, r))
    Ls, Lt, Lr = (basis.lagrange_values(xe, v.ravel()) for v in (s, t, r))
    n = g + 1
    # weight of geometry point a = i + n (j + n k): l_i(s) l_j(t) l_k(r)
    W = (Lr[:, :, None, None] * Lt[:, None, :, None] * Ls[:, None, None, :]).reshape(len(s), n ** 3)
    return np.einsum("...ac,ma->...mc", Xg, W).reshape(np.shape(Xg)[:-2] + (len(s), 3))


def _trilinear_as_geometry(X8):
    """The 8 vertices [E, 8, 3] as degree-1 geometry points (the same order a + 2b + 4c)."""
    return np.asarray(X8, dtype=np.float64)


class BoxMesh:
    def __init__(self, nx, ny, nz, vertices, p, dirichlet_faces=(), periodic=(False, False, False),
                 geom_degree=1, geom_nodes=None):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.p = int(p)
        self.n = self.p + 1
        self.periodic = tuple(bool(x) for x in periodic)
        cells = (self.nx, self.ny, self.nz)
        self.vdims = tuple(c + (0 if per else 1) for c, per in zip(cells, self.periodic))
        self.ndims = tuple(c * self.p + (0 if per else 1) for c, per in zip(cells, self.periodic))
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        if self.vertices.shape[0] != self.vdims[0] * self.vdims[1] * self.vdims[2]:
            raise ValueError("vertex array does not match the lattice")
        self.n_cells = self.nx * self.ny * self.nz
        self.n_nodes = self.ndims[0] * self.ndims[1] * self.ndims[2]
        self.dirichlet_faces = tuple(sorted(set(dirichlet_faces)))
        self.geom_degree = int(geom_degree)
        self._geom_nodes = None if geom_nodes is None else np.asarray(geom_nodes, dtype=np.float64)
        self._build()

    # -- connectivity -------------------------------------------------------------------------
    def _build(self):
        n, p = self.n, self.p
        Vx, Vy, Vz = self.vdims
        Nx, Ny, Nz = self.ndims
        E = self.n_cells
        e = np.arange(E)
        ex, ey, ez = e % self.nx, (e // self.nx) % self.ny, e // (self.nx * self.ny)
        self.cell_vertices = np.zeros((E, 8), dtype=np.int64)
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    self.cell_vertices[:, a + 2 * b + 4 * c] = \
                        ((ex + a) % Vx) + Vx * (((ey + b) % Vy) + Vy * ((ez + c) % Vz))
        self.cell_nodes = np.zeros((E, n ** 3), dtype=np.int64)
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    I = (ex * p + i) % Nx
                    J = (ey * p + j) % Ny
                    K = (ez * p + k) % Nz
                    self.cell_nodes[:, i + n * (j + n * k)] = I + Nx * (J + Ny * K)
        self.cell_vertex_xyz = self.vertices[self.cell_vertices]  # [E, 8, 3]
        self.cell_geom_xyz = _cell_geometry(self.cell_vertex_xyz, self.geom_degree, self._geom_nodes)

        # node coordinates: the map of the owning cell, which for lattice index I is
        # cell min(I // p, n_cells_d - 1) (the last cell owns the closing boundary plane)
        xi = basis.gll_points(p)
        node = np.arange(self.n_nodes)
        lat = (node % Nx, (node // Nx) % Ny, node // (Nx * Ny))
        cell, loc = [], []
        for d, nd in enumerate((self.nx, self.ny, self.nz)):
            cd = np.minimum(lat[d] // p, nd - 1)
            cell.append(cd)
            loc.append(xi[lat[d] - cd * p])
        owner = cell[0] + self.nx * (cell[1] + self.ny * cell[2])
        if self.geom_degree == 1 and self._geom_nodes is None:
            self.node_coords = trilinear_point(self.cell_vertex_xyz[owner], loc[0], loc[1], loc[2])
        else:
            self.node_coords = _map_points(self.cell_geom_xyz, self.geom_degree, owner, loc)

        # constrained nodes
        mask = np.zeros(self.n_nodes, dtype=bool)
        for f in self.dirichlet_faces:
            d, side = f // 2, f % 2
            if self.periodic[d]:
                continue
            mask |= lat[d] == (0 if side == 0 else self.ndims[d] - 1)
        self.constrained = mask


def trilinear_point(X8, s, t, r):
    """Trilinear map of reference points (s, t, r) in [0,1]^3; X8[..., a+2b+4c, :] is vertex (a,b,c).

    Batched: X8 is [..., 8, 3] and s, t, r broadcast against its leading dimensions.
    """
    X8 = np.asarray(X8, dtype=np.float64)
    s, t, r = (np.asarray(v, dtype=np.float64)[..., None] for v in (s, t, r))
    out = np.zeros(X8.shape[:-2] + (3,))
    for c in range(2):
        for b in range(2):
            for a in range(2):
                wgt = (s if a else 1 - s) * (t if b else 1 - t) * (r if c else 1 - r)
                out = out + wgt * X8[..., a + 2 * b + 4 * c, :]
    return out


def _cell_geometry(X8, g, geom_nodes):
    """Geometry points [E, (g+1)^3, 3] of every cell: the given ones, or the 8 vertices (g = 1)."""
    E = X8.shape[0]
    if geom_nodes is None:
        if g != 1:
            raise ValueError("geometry of degree > 1 needs its points")
        return _trilinear_as_geometry(X8)
    G = np.asarray(geom_nodes, dtype=np.float64)
    if G.shape != (E, (g + 1) ** 3, 3):
        raise ValueError(f"geom_nodes must have shape [{E}, {(g + 1) ** 3}, 3]")
    return G


def _map_points(cell_geom, g, cells, loc, chunk=20000):
    """Map of each listed cell at its own reference point (loc = three arrays of coordinates)."""
    xe = equispaced_points(g)
    n = g + 1
    cells = np.asarray(cells)
    out = np.zeros((len(cells), 3))
    for s0 in range(0, len(cells), chunk):
        sl = slice(s0, s0 + chunk)
        Ls, Lt, Lr = (basis.lagrange_values(xe, np.asarray(v)[sl]) for v in loc)
        W = (Lr[:, :, None, None] * Lt[:, None, :, None] * Ls[:, None, None, :]).reshape(-1, n ** 3)
        out[sl] = np.einsum("mac,ma->mc", cell_geom[cells[sl]], W)
    return out


# local vertex a + 2b + 4c of each of the six faces (-x, +x, -y, +y, -z, +z) and local node test
def face_local_nodes(p, f):
    """Local node indices (i + n (j + n k)) on local face f of a cell of degree p."""
    n = p + 1
    d, side = f // 2, f % 2
    out = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                if (i, j, k)[d] == (p if side else 0):
                    out.append(i + n * (j + n * k))
    return np.array(out, dtype=np.int64)


class HexMesh:
    """A conforming mesh of hexahedra given by connectivity, with Q_p nodes in first-touch order.

    vertices [V, 3]; cells [E, 8] vertex ids, local corner a + 2b + 4c at reference corner (a, b, c);
    face_bid [E, 6] boundary id of each local face (-x, +x, -y, +y, -z, +z), 0 for none; nodes on
    the faces whose id is in ``dirichlet_bids`` are constrained (homogeneous data); geometry as in
    the module docstring. Provides the attributes fem.Problem uses (n_nodes, n_cells, p, n,
    cell_nodes, constrained, node_coords, cell_geom_xyz, geom_degree).
    """

    def __init__(self, vertices, cells, p, face_bid=None, dirichlet_bids=(), geom_degree=1, geom_nodes=None):
        self.vertices = np.asarray(vertices, dtype=np.float64).reshape(-1, 3)
        self.cells = np.asarray(cells, dtype=np.int64).reshape(-1, 8)
        self.p = int(p)
        self.n = self.p + 1
        self.n_cells = self.cells.shape[0]
        if np.any(self.cells < 0) or np.any(self.cells >= len(self.vertices)):
            raise ValueError("vertex id out of range")
        for e in range(self.n_cells):
            if len(set(self.cells[e].tolist())) != 8:
                raise ValueError("a cell repeats a vertex")
        self.face_bid = (np.zeros((self.n_cells, 6), dtype=np.int64) if face_bid is None
                         else np.asarray(face_bid, dtype=np.int64).reshape(-1, 6))
        self.dirichlet_bids = tuple(sorted(set(int(b) for b in dirichlet_bids)))
        self.geom_degree = int(geom_degree)
        self.cell_vertex_xyz = self.vertices[self.cells]
        self.cell_geom_xyz = _cell_geometry(self.cell_vertex_xyz, self.geom_degree, geom_nodes)
        self._number_nodes()

    def node_key(self, e, i, j, k):
        """Identity of local node (i, j, k) of cell e: its nonzero trilinear weight numerators by
        vertex id (see the module docstring)."""
        p = self.p
        key = []
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    w = (i if a else p - i) * (j if b else p - j) * (k if c else p - k)
                    if w:
                        key.append((int(self.cells[e, a + 2 * b + 4 * c]), w))
        return tuple(sorted(key))

    def _number_nodes(self):
        n, p = self.n, self.p
        ids = {}
        self.cell_nodes = np.zeros((self.n_cells, n ** 3), dtype=np.int64)
        owner = []
        for e in range(self.n_cells):
            for k in range(n):
                for j in range(n):
                    for i in range(n):
                        key = self.node_key(e, i, j, k)
                        if key not in ids:
                            ids[key] = len(ids)
                            owner.append((e, i, j, k))
                        self.cell_nodes[e, i + n * (j + n * k)] = ids[key]
        self.n_nodes = len(ids)
        mask = np.zeros(self.n_nodes, dtype=bool)
        for e in range(self.n_cells):
            for f in range(6):
                if self.face_bid[e, f] in self.dirichlet_bids and self.face_bid[e, f] != 0:
                    mask[self.cell_nodes[e, face_local_nodes(p, f)]] = True
        self.constrained = mask
        xi = basis.gll_points(p)
        own = np.array(owner, dtype=np.int64)
        self.node_owner = own
        self.node_coords = _map_points(self.cell_geom_xyz, self.geom_degree, own[:, 0],
                                       (xi[own[:, 1]], xi[own[:, 2]], xi[own[:, 3]]))
