"""GPU parity: the HIP path through the C ABI against the FP64 oracle, element by element.

Tolerances (relative 2-norm over the whole output vector): 1e-12 for FP64, 1e-5 for FP32 with
FP32 data. BF16 and FP16 stored data have no accuracy target; their error is bounded loosely here
(it is reported by the benchmark) so that a broken path still fails.
"""
import numpy as np
import pytest

import paper_2408_12479_amd as hx
import workloads
from tests.gpu_helpers import make_pair, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL64, TOL32 = 1e-12, 1e-5
LAWS = ["cnh", "inh", "fiber"]


def _inputs(op, pb, scale=0.03, seed=11):
    # smooth field plus nodal noise scaled by 1/p^2 so the q-point gradients stay O(scale)
    m = pb.mesh
    rng = np.random.default_rng(seed)
    X = m.node_coords
    # damp the field linearly to zero on every constrained face (distance to the face plane)
    damp = np.ones(m.n_nodes)
    lo, hi = X.min(axis=0), X.max(axis=0)
    for f in m.dirichlet_faces:
        d = f // 2
        if not m.periodic[d]:
            damp *= (X[:, d] - lo[d]) if f % 2 == 0 else (hi[d] - X[:, d])
    u = scale * damp * np.stack([np.sin(2.0 * X[:, 0] + X[:, 1]), np.cos(1.5 * X[:, 2] - X[:, 0]),
                                 np.sin(X[:, 0] * X[:, 1] + 2 * X[:, 2])])
    u = u + 0.05 * scale / m.p ** 2 * rng.uniform(-1, 1, u.shape)
    u[:, m.constrained] = 0.0
    du = rng.standard_normal((3, m.n_nodes))
    return u, du


def test_node_coords_and_mask(device):
    op, pb = make_pair((3, 2, 2), 3, "cnh", faces=(0, 3, 5))
    np.testing.assert_allclose(op.node_coords(), pb.mesh.node_coords, rtol=0, atol=1e-14)
    np.testing.assert_array_equal(op.constrained_mask(), pb.mesh.constrained)
    op.close()


def test_config1_small_cube(device):
    """4^3 cells, Q2, cNH mu=1 lambda=10, Dirichlet x=0: one residual and one tangent apply."""
    op, pb = make_pair((4, 4, 4), 2, "cnh", perturb=0.0, mu=1.0, lam=10.0)
    u, du = workloads.small_cube_fields(pb.mesh.node_coords, pb.mesh.constrained)
    r_ref = pb.residual(u)
    Kdu_ref = pb.apply_tangent(u, du)
    ud, dud = to_dev(u), to_dev(du)
    r = to_host(op.residual(ud), op.num_nodes)
    assert rel(r, r_ref) < TOL64
    assert rel(to_host(op.residual(ud, form="spatial"), op.num_nodes), r_ref) < TOL64
    for mode in hx.STORAGE_MODES:
        op.update_linearization(ud, mode=mode, precision="fp64")
        y = to_host(op.apply_tangent(dud, precision="fp64"), op.num_nodes)
        assert rel(y, Kdu_ref) < TOL64, mode
    op.close()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("law", LAWS)
def test_fp64_all_modes(device, p, law):
    # 3x2x2 cells: a ragged last workgroup for every blocking, perturbed geometry
    op, pb = make_pair((3, 2, 2), p, law, faces=(0, 5))
    u, du = _inputs(op, pb)
    ud, dud = to_dev(u), to_dev(du)
    r_ref = pb.residual(u)
    r = to_host(op.residual(ud), op.num_nodes)
    assert rel(r, r_ref) < TOL64
    # the residual over the spatial configuration equals the material one (Section 2)
    assert rel(to_host(op.residual(ud, form="spatial"), op.num_nodes), r_ref) < TOL64
    Kdu_ref = pb.apply_tangent(u, du)
    for mode in hx.STORAGE_MODES:
        op.update_linearization(ud, mode=mode, precision="fp64")
        y = to_host(op.apply_tangent(dud, precision="fp64"), op.num_nodes)
        assert rel(y, Kdu_ref) < TOL64, mode
    op.close()


@pytest.mark.parametrize("p", [2, 3, 4, 6])
@pytest.mark.parametrize("law", LAWS)
def test_fp32_and_16bit_data(device, p, law):
    op, pb = make_pair((3, 2, 2), p, law, faces=(0,))
    u, du = _inputs(op, pb)
    ud, du32 = to_dev(u), to_dev(du, "float32")
    Kdu_ref = pb.apply_tangent(u, du.astype(np.float32).astype(np.float64))
    bounds = {"fp32": TOL32, "fp32_bf16": 2e-2, "fp32_fp16": 3e-3}
    for mode, precs in [("none", ["fp32"]), ("finv_j", ["fp32", "fp32_bf16"]), ("spatial", ["fp32", "fp32_bf16"]),
                        ("spatial_recompute", ["fp32"]), ("tangent", ["fp32", "fp32_bf16", "fp32_fp16"]),
                        ("scalars", ["fp32"]), ("tensors", ["fp32"]),
                        ("spatial_scalars", ["fp32"])]:
        for prec in precs:
            op.update_linearization(ud, mode=mode, precision=prec)
            y = to_host(op.apply_tangent(du32, precision=prec), op.num_nodes)
            assert rel(y, Kdu_ref) < bounds[prec], (mode, prec, rel(y, Kdu_ref))
    op.close()


def test_periodic_direction(device):
    # a closed ring (periodic circumferential index), clamped at one end
    op, pb = make_pair((8, 2, 3), 2, "inh", faces=(4,), periodic=(True, False, False),
                       tube=dict(r_in=1.0, wall=0.2, length=1.0, bend=0.3))
    u, du = _inputs(op, pb)
    ud, dud = to_dev(u), to_dev(du)
    assert rel(to_host(op.residual(ud), op.num_nodes), pb.residual(u)) < TOL64
    for mode in ["tangent", "spatial"]:
        op.update_linearization(ud, mode=mode)
        assert rel(to_host(op.apply_tangent(dud), op.num_nodes), pb.apply_tangent(u, du)) < TOL64, mode
    op.close()


def _random_frames(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        Q, R = np.linalg.qr(rng.standard_normal((3, 3)))
        Q = Q * np.sign(np.diag(R))
        if np.linalg.det(Q) < 0:
            Q[:, 0] = -Q[:, 0]
        out.append(Q)
    return np.stack(out)


@pytest.mark.parametrize("p", [2, 3])
def test_cell_frames_tube(device, p):
    """Fibre law with one local frame per cell (circumferential, axial, radial) on a ring."""
    cells = (8, 2, 3)
    tube = dict(r_in=1.0, wall=0.2, length=1.0, bend=0.3)
    frames = workloads.tube_frames(*cells, length=1.0, bend=0.3)
    op, pb = make_pair(cells, p, "fiber", faces=(4, 5), periodic=(True, False, False), tube=tube,
                       frames=frames)
    u, du = _inputs(op, pb)
    X = pb.mesh.node_coords
    z = X[:, 2]
    u += 0.04 * z * (1.0 - z) * np.stack([X[:, 0], X[:, 1], np.zeros_like(z)])   # inflation: fibres in tension
    u[:, pb.mesh.constrained] = 0.0
    ud, dud, du32 = to_dev(u), to_dev(du), to_dev(du, "float32")
    assert rel(to_host(op.residual(ud), op.num_nodes), pb.residual(u)) < TOL64
    assert rel(to_host(op.residual(ud, form="spatial"), op.num_nodes), pb.residual(u)) < TOL64
    ref = pb.apply_tangent(u, du)
    ref32 = pb.apply_tangent(u, du.astype(np.float32).astype(np.float64))
    for mode in hx.STORAGE_MODES:
        op.update_linearization(ud, mode=mode, precision="fp64")
        assert rel(to_host(op.apply_tangent(dud), op.num_nodes), ref) < TOL64, mode
        op.update_linearization(ud, mode=mode, precision="fp32")
        y = to_host(op.apply_tangent(du32, precision="fp32"), op.num_nodes)
        assert rel(y, ref32) < TOL32, (mode, rel(y, ref32))
    op.close()


def test_cell_frames_random_box(device):
    """Random frames per cell at p = 4 (two cells per workgroup: frames differ inside a block)."""
    op, pb = make_pair((3, 2, 2), 4, "fiber", faces=(0,), frames=_random_frames(12, 7))
    u, du = _inputs(op, pb, scale=0.05)
    ud, dud = to_dev(u), to_dev(du)
    assert rel(to_host(op.residual(ud), op.num_nodes), pb.residual(u)) < TOL64
    ref = pb.apply_tangent(u, du)
    for mode in ["none", "finv_j", "tangent", "spatial", "scalars", "tensors", "spatial_scalars"]:
        op.update_linearization(ud, mode=mode, precision="fp64")
        assert rel(to_host(op.apply_tangent(dud), op.num_nodes), ref) < TOL64, mode
    op.close()


def test_fp32_newton_jpow_near_incompressible(device):
    """Algorithm 2 (3 Newton steps for J^-2/3) in its regime J in [0.95, 1.05]."""
    op, pb = make_pair((4, 2, 2), 3, "fiber", perturb=0.0, faces=(), lengths=(2.0, 1.0, 1.0),
                       jpow_newton_iters=3, kappa=1e3)
    u, du = workloads.fiber_fields(pb.mesh.node_coords)
    F, _, _ = pb.deformation_gradient(u, np.arange(pb.mesh.n_cells))
    J = np.linalg.det(F)
    assert J.min() > 0.94 and J.max() < 1.06
    ref = pb.apply_tangent(u, du.astype(np.float32).astype(np.float64))
    ud, du32 = to_dev(u), to_dev(du, "float32")
    for mode in ["none", "finv_j"]:
        op.update_linearization(ud, mode=mode, precision="fp32")
        y = to_host(op.apply_tangent(du32, precision="fp32"), op.num_nodes)
        assert rel(y, ref) < TOL32, (mode, rel(y, ref))
    op.close()


def test_identity_state_and_fp64_fp32_slots_coexist(device):
    op, pb = make_pair((2, 3, 2), 3, "fiber", faces=(0,))
    u = np.zeros((3, pb.mesh.n_nodes))
    _, du = _inputs(op, pb)
    ref = pb.apply_tangent(u, du)
    ud = to_dev(u)
    op.update_linearization(ud, mode="tangent", precision="fp64")
    op.update_linearization(ud, mode="finv_j", precision="fp32")
    y64 = to_host(op.apply_tangent(to_dev(du)), op.num_nodes)
    y32 = to_host(op.apply_tangent(to_dev(du, "float32"), precision="fp32"), op.num_nodes)
    assert rel(y64, ref) < TOL64 and rel(y32, ref) < TOL32
    op.close()


def test_determinism_of_repeated_apply(device):
    op, pb = make_pair((3, 3, 3), 2, "cnh")
    u, du = _inputs(op, pb)
    op.update_linearization(to_dev(u), mode="finv_j")
    a = to_host(op.apply_tangent(to_dev(du)), op.num_nodes)
    b = to_host(op.apply_tangent(to_dev(du)), op.num_nodes)
    # the element vectors are summed per node in a fixed order: repeats are bit-identical
    assert np.array_equal(a, b)
    op.close()


def test_error_paths(device):
    import paper_2408_12479_amd as hx
    import torch
    op, pb = make_pair((2, 2, 2), 2, "cnh")
    du = torch.zeros(op.num_dofs, dtype=torch.float64, device="cuda:0")
    with pytest.raises(hx.HxError) as ei:
        op.apply_tangent(du)
    assert ei.value.name == "HX_E_STATE"
    # a displacement that inverts the q-points: u = -2 X
    u = -2.0 * pb.mesh.node_coords.T
    with pytest.raises(hx.HxError) as ei:
        op.update_linearization(to_dev(u), mode="tangent")
    assert ei.value.name == "HX_E_INVERTED"
    # a NaN in the displacement makes J - 1 NaN at the q-points of the cells around that node: the
    # test J > 0 fails there in every storage mode, the recompute one included
    u = np.zeros_like(u)
    u[1, 62] = np.nan   # the centre node of the 2 x 2 x 2 lattice of Q2 cells
    for mode in hx.STORAGE_MODES:
        with pytest.raises(hx.HxError) as ei:
            op.update_linearization(to_dev(u), mode=mode)
        assert ei.value.name == "HX_E_INVERTED", mode
    u[1, 62] = 0.0
    # binary16 data exists for the stored tangent only (its words share one magnitude per cell)
    for mode in ("finv_j", "spatial"):
        with pytest.raises(hx.HxError) as ei:
            op.update_linearization(to_dev(np.zeros_like(u)), mode=mode, precision="fp32_fp16")
        assert ei.value.name == "HX_E_UNSUPPORTED"
    # the scalar and tensor stages store FP64 or FP32 words only
    for mode in ("scalars", "tensors", "spatial_scalars"):
        for prec in ("fp32_bf16", "fp32_fp16"):
            with pytest.raises(hx.HxError) as ei:
                op.update_linearization(to_dev(np.zeros_like(u)), mode=mode, precision=prec)
            assert ei.value.name == "HX_E_UNSUPPORTED"
    op.close()
    V = workloads.box_vertices(1, 1, 1)
    V[7] = [-1.0, -1.0, -1.0]
    with pytest.raises(hx.HxError) as ei:
        hx.Operator(1, 1, 1, V, 2)
    assert ei.value.name == "HX_E_INVERTED"
    with pytest.raises(hx.HxError) as ei:
        hx.Operator(1, 1, 1, workloads.box_vertices(1, 1, 1), 7)
    assert ei.value.name == "HX_E_UNSUPPORTED"
    V = workloads.box_vertices(1, 1, 1)
    V[3, 1] = np.inf
    with pytest.raises(hx.HxError) as ei:
        hx.Operator(1, 1, 1, V, 2)
    assert ei.value.name == "HX_E_ARG"
    # cell frames must be orthonormal and right-handed
    for bad in (2.0 * np.eye(3), np.diag([1.0, 1.0, -1.0])):
        with pytest.raises(hx.HxError) as ei:
            hx.Operator(1, 1, 1, workloads.box_vertices(1, 1, 1), 2, law="fiber", mu=1.0, kappa=10.0,
                        frames=bad[None])
        assert ei.value.name == "HX_E_ARG"


def test_single_cell_all_degrees(device):
    for p in range(1, 7):
        op, pb = make_pair((1, 1, 1), p, "fiber", perturb=0.0, faces=())
        u, du = _inputs(op, pb, scale=0.1)
        ud = to_dev(u)
        op.update_linearization(ud, mode="none")
        assert rel(to_host(op.apply_tangent(to_dev(du)), op.num_nodes), pb.apply_tangent(u, du)) < TOL64
        op.close()
