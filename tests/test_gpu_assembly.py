"""Assembly of the element vectors (the node kernel that sums the cells' bricks) on lattices that
are periodic in the second or the third direction and on the smallest lattices, against the
oracle: residual and the applies of every storage mode, FP64 <= 1e-12 and FP32 <= 1e-5; and the
largest lattice the 32-bit indexing admits.

The periodic cases place the tube's circumferential index on lattice direction y or z by an even
(cyclic) permutation of the lattice axes, which keeps every cell right-handed; the clamped faces
are the two axial ends.
"""
import numpy as np
import pytest

import paper_2408_12479_amd as hx
import workloads
from oracle import fem, mesh as omesh
from tests.gpu_helpers import rel, to_dev, to_host
from tests.helpers import make_material

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
TUBE = dict(r_in=1.0, wall=0.2, length=1.0, bend=0.3)


def _permuted_tube(n_theta, n_wall, n_axial, periodic_dir):
    """Vertices [V][3] and (cells, periodic, axial lattice direction) with the circumferential
    index on lattice direction periodic_dir (1: y, 2: z)."""
    V = workloads.tube_vertices(n_theta, n_wall, n_axial, **TUBE).reshape(n_axial + 1, n_wall + 1, n_theta, 3)
    if periodic_dir == 1:   # x = axial, y = circumferential, z = wall: array [wall][theta][axial]
        return V.transpose(1, 2, 0, 3).reshape(-1, 3), (n_axial, n_theta, n_wall), (False, True, False), 0
    # x = wall, y = axial, z = circumferential: array [theta][axial][wall]
    return V.transpose(2, 0, 1, 3).reshape(-1, 3), (n_wall, n_axial, n_theta), (False, False, True), 1


def _pair(V, cells, p, law, faces, periodic):
    m = omesh.BoxMesh(*cells, V, p, dirichlet_faces=faces, periodic=periodic)
    mat = make_material(law)
    pb = fem.Problem(m, mat)
    op = hx.Operator(*cells, V, p, law=law, mu=mat.mu, lam=mat.lam, kappa=mat.kappa, k1=mat.k1, k2=mat.k2,
                     H4=mat.H4, H6=mat.H6, M4=mat.M4, M6=mat.M6, dirichlet_faces=faces, periodic=periodic)
    return op, pb


def _fields(pb, seed):
    X = pb.mesh.node_coords
    z = X[:, 2] / TUBE["length"]
    rng = np.random.default_rng(seed)
    u = 0.03 * z * (1.0 - z) * np.stack([np.sin(2.0 * X[:, 0] + X[:, 1]), np.cos(1.5 * X[:, 2] - X[:, 0]),
                                         np.sin(X[:, 1] - X[:, 2])])
    u[:, pb.mesh.constrained] = 0.0
    du = rng.standard_normal(u.shape)
    return u, du


def _check_all(op, pb, u, du):
    ud, dud, du32 = to_dev(u), to_dev(du), to_dev(du, "float32")
    assert rel(to_host(op.residual(ud), op.num_nodes), pb.residual(u)) < TOL64
    ref = pb.apply_tangent(u, du)
    ref32 = pb.apply_tangent(u, du.astype(np.float32).astype(np.float64))
    for mode in ["none", "finv_j", "tangent", "spatial"]:
        op.update_linearization(ud, mode=mode, precision="fp64")
        assert rel(to_host(op.apply_tangent(dud), op.num_nodes), ref) < TOL64, mode
        op.update_linearization(ud, mode=mode, precision="fp32")
        y = to_host(op.apply_tangent(du32, precision="fp32"), op.num_nodes)
        assert rel(y, ref32) < TOL32, (mode, rel(y, ref32))


@pytest.mark.parametrize("periodic_dir,p,law", [(1, 2, "cnh"), (1, 3, "inh"), (2, 2, "inh"), (2, 4, "cnh")])
def test_periodic_y_and_z(device, periodic_dir, p, law):
    V, cells, periodic, axial = _permuted_tube(6, 2, 3, periodic_dir)
    op, pb = _pair(V, cells, p, law, (2 * axial, 2 * axial + 1), periodic)
    u, du = _fields(pb, seed=5 + p)
    _check_all(op, pb, u, du)
    op.close()


@pytest.mark.parametrize("cells,p", [((1, 1, 1), 1), ((1, 1, 1), 4), ((1, 1, 1), 6), ((2, 1, 3), 1),
                                     ((3, 1, 1), 3), ((1, 2, 1), 2)])
def test_smallest_lattices(device, cells, p):
    V = workloads.box_vertices(*cells, perturb=0.0)
    op, pb = _pair(V, cells, p, "cnh", (0,), (False, False, False))
    X = pb.mesh.node_coords
    rng = np.random.default_rng(3)
    u = 0.02 * X[:, 0] * np.stack([np.sin(X[:, 1] + 1.0), np.cos(X[:, 2]), X[:, 0] * X[:, 1]])
    u[:, pb.mesh.constrained] = 0.0
    du = rng.standard_normal(u.shape)
    _check_all(op, pb, u, du)
    op.close()


def test_repeated_applies_bit_identical(device):
    """The node kernel sums the bricks in a fixed order: repeated applies agree to the bit."""
    V, cells, periodic, axial = _permuted_tube(8, 2, 4, 2)
    op, pb = _pair(V, cells, 3, "inh", (2 * axial, 2 * axial + 1), periodic)
    u, du = _fields(pb, seed=9)
    ud, dud = to_dev(u), to_dev(du)
    op.update_linearization(ud, mode="spatial")
    y0 = op.apply_tangent(dud).cpu().numpy()
    for _ in range(5):
        assert np.array_equal(op.apply_tangent(dud).cpu().numpy(), y0)
    op.close()


def test_lattice_beyond_the_index_range_is_refused(device):
    """The kernels index Gauss points and nodes in 32 bits: hx_setup refuses a lattice with
    cells * (p+1)^3 >= 2^31 (here 200 x 200 x 157 cells at Q6, 2.16e9 Gauss points) before it
    allocates or checks anything else."""
    nx, ny, nz = 200, 200, 157
    assert nx * ny * nz * 343 > 2 ** 31 - 1
    V = np.zeros(((nz + 1) * (ny + 1) * (nx + 1), 3))
    with pytest.raises(hx.HxError) as err:
        hx.Operator(nx, ny, nz, V, 6, law="cnh", mu=1.0, lam=1.0)
    assert err.value.name == "HX_E_ARG"
    assert "too large" in str(err.value)
