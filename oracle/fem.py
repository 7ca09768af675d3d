"""Galerkin residual, linearised operator and energy, from dense element tables (no sum factorisation).

Definitions (Section 2, material configuration, no body force or traction in the operator
configurations):

* residual     r_(c,a) = sum_q w_q detJ0 sum_J P_cJ(F_q) (Grad phi_a)_J                (Eq. of r_Omega0)
* linearised   (K du)_(c,a) = sum_q w_q detJ0 sum_J,k,L (Grad phi_a)_J A_cJkL (Grad du)_kL
               with A = dP/dF, i.e. the directional derivative of the residual (Problem 2.2)
* energy       Pi(u) = sum_q w_q detJ0 Psi(C_q)  (whose gradient is the residual)

Geometry: the map of each hexahedron, trilinear from its 8 vertices or of degree g from its values
at the equispaced points of the reference cell (curved cells), J0 = dX/dxi at every Gauss point,
Grad phi = J0^-T grad_xi phi, weights w_q det J0 (Gauss weights are tensor products on [0,1]^3).

Constraints (the test space H^1_0 with homogeneous data, Problems 2.1-2.2; the operator reading
is identity rows and columns on constrained DoFs): r~ = P_f r,  K~ du = P_f K P_f du + P_c du.

All functions accept complex displacement vectors so that tests can take complex-step derivatives.
Work proceeds over chunks of cells; arrays are the plain [cells, q-points, ...] tensors.

Also: the dead-load surface vector of a pressure on a boundary face, and the dense transfer
matrices between two degrees on one lattice (prolongation = coarse basis at the fine nodes;
interpolation of a fine field onto the coarse nodes), and between two degree-1 lattices, one
with half the cells in some directions (the same in lattice reference coordinates).

Test infrastructure only. Pinned in tests/test_oracle_fem.py and tests/test_oracle_transfer.py
(patch test, rigid rotation, translation invariance, residual = complex-step gradient of the
energy, tangent = complex-step derivative of the residual, symmetry, linear elasticity at u = 0
against an independent Voigt-notation stiffness; face resultant of a pressure on a planar face,
zero resultant on a closed surface; exact reproduction of polynomials by the transfers and
J P = I; the Galerkin identity P^T K_fine P = K_coarse for nested lattices of an affine body).
"""
import dataclasses

import numpy as np

from . import basis, material


class ElementTables:
    """Dense 3D tables of the Q_p basis at the (p+1)^3 Gauss points.

    N[q, a] = l_i(x_qx) l_j(x_qy) l_k(x_qz),  dN[q, a, d] its reference derivatives,
    W[q] = product Gauss weight;  q = qx + n (qy + n qz),  a = i + n (j + n k).
    TN[q, v, d]: reference derivatives of the 8 trilinear vertex functions (geometry).
    """

    def __init__(self, p):
        n = p + 1
        self.p, self.n = p, n
        xg = basis.gll_points(p)
        xq, wq = basis.gauss_rule(n)
        L = basis.lagrange_values(xg, xq)
        dL = basis.lagrange_derivatives(xg, xq)
        n3 = n ** 3

        def t3(A, B, C):
            return np.einsum("xi,yj,zk->zyxkji", A, B, C).reshape(n3, n3)

        self.N = t3(L, L, L)
        self.dN = np.stack([t3(dL, L, L), t3(L, dL, L), t3(L, L, dL)], axis=-1)
        self.W = np.einsum("x,y,z->zyx", wq, wq, wq).reshape(n3)
        self.xq = xq
        # trilinear vertex functions phi_0(s) = 1 - s, phi_1(s) = s
        qz, qy, qx = np.meshgrid(xq, xq, xq, indexing="ij")
        s, t, r = qx.ravel(), qy.ravel(), qz.ravel()
        TN = np.zeros((n3, 8, 3))
        for c in range(2):
            for b in range(2):
                for a in range(2):
                    fa, fb, fc = (s if a else 1 - s), (t if b else 1 - t), (r if c else 1 - r)
                    da, db, dc = (1.0 if a else -1.0), (1.0 if b else -1.0), (1.0 if c else -1.0)
                    v = a + 2 * b + 4 * c
                    TN[:, v, 0] = da * fb * fc
                    TN[:, v, 1] = fa * db * fc
                    TN[:, v, 2] = fa * fb * dc
        self.TN = TN
        self._geo = {1: TN}

    def geometry_derivatives(self, g):
        """dG[q, a, d]: reference derivatives of the degree-g geometry basis (Lagrange on the g+1
        equispaced points per direction, a = i + (g+1)(j + (g+1) k)) at the Gauss points. For
        g = 1 these are the trilinear vertex functions' derivatives (TN)."""
        if g not in self._geo:
            n = self.n
            xe = np.linspace(0.0, 1.0, g + 1)
            L = basis.lagrange_values(xe, self.xq)
            dL = basis.lagrange_derivatives(xe, self.xq)
            m3 = (g + 1) ** 3

            def t3(A, B, C):
                # [qz, qy, qx, k, j, i] -> [q, a]
                return np.einsum("xi,yj,zk->zyxkji", A, B, C).reshape(n ** 3, m3)

            self._geo[g] = np.stack([t3(dL, L, L), t3(L, dL, L), t3(L, L, dL)], axis=-1)
        return self._geo[g]


class Problem:
    """A mesh, a material and the element tables; the operator evaluations act on (3, n_nodes).

    cell_fibers: optional (H4 [E, 3, 3], H6, M4 [E, 3], M6) per cell (fibre law with fibre frames
    that vary over the mesh); they replace the material's uniform tensors cell by cell.
    """

    def __init__(self, mesh, mat, chunk=256, cell_fibers=None):
        self.mesh = mesh
        self.mat = mat
        self.tab = ElementTables(mesh.p)
        self.chunk = chunk
        self.cell_fibers = None
        if cell_fibers is not None:
            H4, H6, M4, M6 = (np.asarray(a, dtype=np.float64) for a in cell_fibers)
            if H4.shape != (mesh.n_cells, 3, 3) or M4.shape != (mesh.n_cells, 3):
                raise ValueError("cell_fibers must be ([E,3,3], [E,3,3], [E,3], [E,3])")
            self.cell_fibers = (H4, H6, M4, M6)

    def material_of(self, cells):
        """The material seen by the q-points of ``cells`` (tensors shaped [E, 1, ...])."""
        if self.cell_fibers is None:
            return self.mat
        H4, H6, M4, M6 = self.cell_fibers
        return dataclasses.replace(self.mat, H4=H4[cells][:, None], H6=H6[cells][:, None],
                                   M4=M4[cells][:, None], M6=M6[cells][:, None])

    # -- geometry -----------------------------------------------------------------------------
    def geometry(self, cells):
        """(invJ0 [E, Q, 3(d), 3(J)], wdet [E, Q]) for the given cells; asserts det J0 > 0."""
        g = getattr(self.mesh, "geom_degree", 1)
        Xg = self.mesh.cell_geom_xyz[cells]                         # [E, (g+1)^3, 3]
        J0 = np.einsum("evc,qvd->eqcd", Xg, self.tab.geometry_derivatives(g))   # dX_c / dxi_d
        det = np.linalg.det(J0)
        if np.any(det <= 0.0):
            raise ValueError("inverted or degenerate cell: det J0 <= 0")
        return np.linalg.inv(J0), det * self.tab.W[None, :]

    def physical_gradients(self, cells):
        """Grad phi_a at every q-point: [E, Q, n^3, 3] = sum_d dN[q,a,d] invJ0[d,J]."""
        invJ0, wdet = self.geometry(cells)
        return np.einsum("qad,eqdJ->eqaJ", self.tab.dN, invJ0), wdet

    def _cell_values(self, vec, cells):
        """Element-local values [E, 3, n^3] of a (3, n_nodes) vector."""
        return np.transpose(vec[:, self.mesh.cell_nodes[cells]], (1, 0, 2))

    def _chunks(self, cells=None):
        cells = np.arange(self.mesh.n_cells) if cells is None else np.asarray(cells)
        for s in range(0, len(cells), self.chunk):
            yield cells[s:s + self.chunk]

    def _scatter(self, out, cells, contrib):
        nodes = self.mesh.cell_nodes[cells]
        for c in range(3):
            np.add.at(out[c], nodes.ravel(), contrib[:, c, :].ravel())

    def deformation_gradient(self, u, cells):
        Gphi, wdet = self.physical_gradients(cells)
        ue = self._cell_values(u, cells)
        H = np.einsum("eca,eqaJ->eqcJ", ue, Gphi)
        F = np.eye(3) + H
        if np.any(np.real(np.linalg.det(F)) <= 0.0):
            raise ValueError("deformation inverts a q-point: J <= 0")
        return F, Gphi, wdet

    # -- operator evaluations -----------------------------------------------------------------
    def energy(self, u):
        total = 0.0
        for cells in self._chunks():
            F, _, wdet = self.deformation_gradient(u, cells)
            C = np.einsum("...ki,...kj->...ij", F, F)
            total = total + np.sum(wdet * material.psi(C, self.material_of(cells)))
        return total

    def residual(self, u, cells=None, constrain=True):
        """r~(u) with constrained rows set to zero; ``cells`` restricts the sum (for sampling)."""
        u = np.asarray(u)
        out = np.zeros((3, self.mesh.n_nodes), dtype=np.result_type(u.dtype, np.float64))
        for ch in self._chunks(cells):
            F, Gphi, wdet = self.deformation_gradient(u, ch)
            P = material.first_pk(F, self.material_of(ch))
            contrib = np.einsum("eq,eqcJ,eqaJ->eca", wdet, P, Gphi)
            self._scatter(out, ch, contrib)
        if constrain:
            out[:, self.mesh.constrained] = 0.0
        return out

    def apply_tangent(self, u, du, cells=None, constrain=True):
        """K~(u) du = P_f K P_f du + P_c du, cell by cell (no global matrix)."""
        u = np.asarray(u)
        du = np.array(du, dtype=np.result_type(du, np.float64), copy=True)
        mask = self.mesh.constrained if constrain else np.zeros(self.mesh.n_nodes, dtype=bool)
        du_f = du.copy()
        du_f[:, mask] = 0.0
        out = np.zeros((3, self.mesh.n_nodes), dtype=np.result_type(u.dtype, du.dtype, np.float64))
        for ch in self._chunks(cells):
            F, Gphi, wdet = self.deformation_gradient(u, ch)
            A = material.first_elasticity(F, self.material_of(ch))
            G = np.einsum("eka,eqaL->eqkL", self._cell_values(du_f, ch), Gphi)
            Pdot = np.einsum("eqiJkL,eqkL->eqiJ", A, G)
            contrib = np.einsum("eq,eqcJ,eqaJ->eca", wdet, Pdot, Gphi)
            self._scatter(out, ch, contrib)
        out[:, mask] = du[:, mask]
        return out

    def cells_touching(self, nodes):
        """Cells whose node lists contain any of ``nodes`` (for sampled rows)."""
        hit = np.isin(self.mesh.cell_nodes, np.asarray(nodes)).any(axis=1)
        return np.nonzero(hit)[0]

    def tangent_matrix(self, u, constrain=True):
        """Assembled K~ (dense, DoF order c * n_nodes + node); for small meshes only."""
        nn = self.mesh.n_nodes
        K = np.zeros((3 * nn, 3 * nn))
        for ch in self._chunks():
            F, Gphi, wdet = self.deformation_gradient(u, ch)
            A = material.first_elasticity(F, self.material_of(ch))
            Ke = np.einsum("eq,eqaJ,eqiJkL,eqbL->eiakb", wdet, Gphi, A, Gphi)
            nodes = self.mesh.cell_nodes[ch]
            for e in range(len(ch)):
                dof = (np.arange(3)[:, None] * nn + nodes[e][None, :]).ravel()
                K[np.ix_(dof, dof)] += Ke[e].reshape(3 * nodes.shape[1], 3 * nodes.shape[1])
        if constrain:
            cdofs = np.nonzero(np.tile(self.mesh.constrained, 3))[0]
            K[cdofs, :] = 0.0
            K[:, cdofs] = 0.0
            K[cdofs, cdofs] = 1.0
        return K


def surface_load_faces(problem, faces, pressure):
    """Dead-load pressure vector f_(c,a) = -p sum over the listed cell faces of int phi_a N_c dA.

    Section 2 residual, Neumann term: h_N = -p N with N the outward unit normal of the reference
    body, integrated with (p+1)^2 Gauss points on each listed (cell, local face) of the cell's map
    (trilinear or of degree g). The outward normal area element of local face f = (d, side) is
    sign * (dX/dxi_a x dX/dxi_b), (a, b) = (d + 1, d + 2) mod 3, sign +1 on the side xi_d = 1.
    """
    m = problem.mesh
    p, n = m.p, m.n
    g = getattr(m, "geom_degree", 1)
    xg = basis.gll_points(p)
    xq, wq = basis.gauss_rule(n)
    xe = np.linspace(0.0, 1.0, g + 1)
    L = basis.lagrange_values(xg, xq)             # L[q, i], the Q_p basis on the face
    f = np.zeros((3, m.n_nodes))
    for e, face in faces:
        d, side = face // 2, face % 2
        da, db = (d + 1) % 3, (d + 2) % 3
        Xg = m.cell_geom_xyz[e]                   # [(g+1)^3, 3]
        for q2 in range(n):
            for q1 in range(n):
                xi = [0.0, 0.0, 0.0]
                xi[d], xi[da], xi[db] = (1.0 if side else 0.0), xq[q1], xq[q2]
                val = [basis.lagrange_values(xe, [xi[k]])[0] for k in range(3)]
                der = [basis.lagrange_derivatives(xe, [xi[k]])[0] for k in range(3)]

                def grad(dir_):
                    f3 = [der[k] if k == dir_ else val[k] for k in range(3)]
                    w3 = np.einsum("k,j,i->kji", f3[2], f3[1], f3[0]).ravel()
                    return w3 @ Xg

                ta, tb = grad(da), grad(db)
                NdA = np.cross(ta, tb) * (1.0 if side else -1.0)
                w = wq[q1] * wq[q2]
                for j2 in range(n):
                    for j1 in range(n):
                        loc = [0, 0, 0]
                        loc[d], loc[da], loc[db] = (n - 1 if side else 0), j1, j2
                        node = m.cell_nodes[e, loc[0] + n * (loc[1] + n * loc[2])]
                        f[:, node] += -pressure * NdA * w * L[q1, j1] * L[q2, j2]
    return f


def surface_load(problem, face, pressure):
    """Dead-load pressure vector on lattice boundary face ``face`` (0..5) of a BoxMesh."""
    m = problem.mesh
    d, side = face // 2, face % 2
    if m.periodic[d]:
        raise ValueError("face of a periodic direction")
    da, db = (d + 1) % 3, (d + 2) % 3
    ncells = (m.nx, m.ny, m.nz)
    cd = ncells[d] - 1 if side else 0
    faces = []
    for c2 in range(ncells[db]):
        for c1 in range(ncells[da]):
            cell = [0, 0, 0]
            cell[d], cell[da], cell[db] = cd, c1, c2
            faces.append((cell[0] + m.nx * (cell[1] + m.ny * cell[2]), face))
    return surface_load_faces(problem, faces, pressure)


def surface_load_bid(problem, bid, pressure):
    """Dead-load pressure vector on every cell face of a HexMesh whose boundary id is ``bid``."""
    m = problem.mesh
    faces = [(e, f) for e in range(m.n_cells) for f in range(6) if m.face_bid[e, f] == bid]
    return surface_load_faces(problem, faces, pressure)


def _owner_local(mesh, node):
    """(cell, local lattice index (i, j, k)) of the owning cell of a node (node-coordinate rule)."""
    Nx, Ny, _ = mesh.ndims
    lat = (node % Nx, (node // Nx) % Ny, node // (Nx * Ny))
    cell, loc = [], []
    for dd, nd in enumerate((mesh.nx, mesh.ny, mesh.nz)):
        c = min(lat[dd] // mesh.p, nd - 1)
        cell.append(c)
        loc.append(lat[dd] - c * mesh.p)
    return cell[0] + mesh.nx * (cell[1] + mesh.ny * cell[2]), loc


def prolongation_matrix(mesh_f, mesh_c):
    """Dense P [fine nodes, coarse nodes]: the coarse nodal basis evaluated at each fine node,
    through the reference coordinates of the node in an owning cell (scalar field; the vector
    operator applies it to each component)."""
    xf = basis.gll_points(mesh_f.p)
    xc = basis.gll_points(mesh_c.p)
    P = np.zeros((mesh_f.n_nodes, mesh_c.n_nodes))
    nc = mesh_c.n
    for node in range(mesh_f.n_nodes):
        e, loc = _owner_local(mesh_f, node)
        vals = [basis.lagrange_values(xc, [xf[loc[dd]]])[0] for dd in range(3)]
        for k in range(nc):
            for j in range(nc):
                for i in range(nc):
                    P[node, mesh_c.cell_nodes[e, i + nc * (j + nc * k)]] = vals[0][i] * vals[1][j] * vals[2][k]
    return P


def interpolation_matrix(mesh_f, mesh_c):
    """Dense J [coarse nodes, fine nodes]: the fine nodal basis evaluated at each coarse node."""
    xf = basis.gll_points(mesh_f.p)
    xc = basis.gll_points(mesh_c.p)
    J = np.zeros((mesh_c.n_nodes, mesh_f.n_nodes))
    nf = mesh_f.n
    for node in range(mesh_c.n_nodes):
        e, loc = _owner_local(mesh_c, node)
        vals = [basis.lagrange_values(xf, [xc[loc[dd]]])[0] for dd in range(3)]
        for k in range(nf):
            for j in range(nf):
                for i in range(nf):
                    J[node, mesh_f.cell_nodes[e, i + nf * (j + nf * k)]] = vals[0][i] * vals[1][j] * vals[2][k]
    return J


def _lattice_factors(mesh_f, mesh_c):
    if mesh_f.p != 1 or mesh_c.p != 1:
        raise ValueError("lattice transfers act between degree-1 meshes")
    fac = []
    for nf, nc in zip((mesh_f.nx, mesh_f.ny, mesh_f.nz), (mesh_c.nx, mesh_c.ny, mesh_c.nz)):
        if nf not in (nc, 2 * nc):
            raise ValueError("each direction must keep or halve its cells")
        fac.append(nf // nc)
    return fac


def _q1_row(mesh, pos):
    """{node: weight} of the trilinear basis of ``mesh`` at lattice coordinates ``pos`` (cell units)."""
    ncs = (mesh.nx, mesh.ny, mesh.nz)
    cell, xi = [], []
    for d in range(3):
        c = min(int(np.floor(pos[d])), ncs[d] - 1)
        cell.append(c)
        xi.append(pos[d] - c)
    e = cell[0] + mesh.nx * (cell[1] + mesh.ny * cell[2])
    row = {}
    for k in range(2):
        for j in range(2):
            for i in range(2):
                w = (xi[0] if i else 1 - xi[0]) * (xi[1] if j else 1 - xi[1]) * (xi[2] if k else 1 - xi[2])
                node = mesh.cell_nodes[e, i + 2 * (j + 2 * k)]
                row[node] = row.get(node, 0.0) + w
    return row


def lattice_prolongation_matrix(mesh_f, mesh_c):
    """Dense P [fine nodes, coarse nodes] between degree-1 meshes whose coarse lattice has half the
    cells in some directions: the coarse trilinear basis evaluated at every fine node, the fine
    node with lattice index I sitting at coarse lattice coordinate I / f (f = 1 or 2)."""
    fac = _lattice_factors(mesh_f, mesh_c)
    Nx, Ny, _ = mesh_f.ndims
    P = np.zeros((mesh_f.n_nodes, mesh_c.n_nodes))
    for node in range(mesh_f.n_nodes):
        lat = (node % Nx, (node // Nx) % Ny, node // (Nx * Ny))
        for cn, w in _q1_row(mesh_c, [lat[d] / fac[d] for d in range(3)]).items():
            P[node, cn] += w
    return P


def lattice_interpolation_matrix(mesh_f, mesh_c):
    """Dense J [coarse nodes, fine nodes]: the fine trilinear basis at every coarse node (coarse
    lattice index I sits at fine lattice coordinate f I)."""
    fac = _lattice_factors(mesh_f, mesh_c)
    Nx, Ny, _ = mesh_c.ndims
    J = np.zeros((mesh_c.n_nodes, mesh_f.n_nodes))
    for node in range(mesh_c.n_nodes):
        lat = (node % Nx, (node // Nx) % Ny, node // (Nx * Ny))
        for fn, w in _q1_row(mesh_f, [lat[d] * fac[d] for d in range(3)]).items():
            J[node, fn] += w
    return J
