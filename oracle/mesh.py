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

Test infrastructure only. Pinned in tests/test_oracle_mesh.py (vertex reproduction, volume of
the perturbed unit cube, periodic identification, node counts).
"""
import numpy as np

from . import basis


class BoxMesh:
    def __init__(self, nx, ny, nz, vertices, p, dirichlet_faces=(), periodic=(False, False, False)):
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

        # node coordinates: trilinear map of the owning cell, which for lattice index I is
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
        self.node_coords = trilinear_point(self.cell_vertex_xyz[owner], loc[0], loc[1], loc[2])

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
