"""GPU checks of the configuration autotuner (hx_autotune, hx_set_tuning) through the C ABI.

* Every cells-per-workgroup variant of every degree, storage mode and precision matches the FP64
  oracle (1e-12 FP64, 1e-5 FP32): the alternative variant lays the stored data out in its own
  blocks of cells, and the update and apply of that variant must agree on it.
* The autotuner times 16 configurations on a lattice of trilinear cells (8 on a general mesh),
  reports the fastest, records the choice per mode and leaves the slot in it; the multigrid keeps
  its default configuration on a tuned context.
* The stored table (JSON keyed by degree, law, precision, mode, mesh kind) is written by a tuning
  run and read back without timing.
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_2408_12479_amd as hx
import workloads
from tests.gpu_helpers import make_pair, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


def _fields(pb, seed=2):
    m = pb.mesh
    u, _ = workloads.small_cube_fields(m.node_coords, m.constrained)
    du = workloads.random_direction(m.n_nodes, seed, m.constrained)
    return u, du


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_alternative_variant_matches_oracle(device, p):
    cells = (5, 3, 4) if p <= 3 else (3, 2, 3)   # ragged last workgroups for both variants
    op, pb = make_pair(cells, p, "fiber")
    u, du = _fields(pb)
    ref = pb.apply_tangent(u, du)
    ud = to_dev(u)
    assert hx.cells_per_workgroup(p, 1) > 0 and hx.cells_per_workgroup(p, 1) != hx.cells_per_workgroup(p, 0)
    for prec in ("fp64", "fp32"):
        dt = "float64" if prec == "fp64" else "float32"
        for mode in hx.STORAGE_MODES:
            for nt in (0, 1):
                op.set_tuning(mode, prec, variant=1, nontemporal=nt)
                op.update_linearization(ud, mode=mode, precision=prec)
                y = to_host(op.apply_tangent(to_dev(du, dt), precision=prec), pb.mesh.n_nodes)
                err = rel(y, ref)
                assert err < (1e-12 if prec == "fp64" else 1e-5), (prec, mode, nt, err)
    op.close()


def test_autotune_picks_the_fastest_and_keeps_it(device):
    op, pb = make_pair((8, 8, 8), 3, "cnh", lam=100.0)
    u, du = _fields(pb)
    best, entries = op.autotune(to_dev(u), "fp64", reps=5)
    assert len(entries) == 28
    assert {e["mode"] for e in entries} == {"none", "finv_j", "tangent", "spatial", "spatial_recompute", "scalars",
                                            "tensors", "spatial_scalars"}
    assert {e["variant"] for e in entries} == {0, 1}
    assert best["ms"] == min(e["ms"] for e in entries)
    # the slot is left in the best configuration: the apply reproduces the oracle
    y = to_host(op.apply_tangent(to_dev(du)), pb.mesh.n_nodes)
    assert rel(y, pb.apply_tangent(u, du)) < 1e-12
    # later updates of a mode use its recorded configuration; the multigrid keeps the default
    # (linearised at u = 0, where the tangent is positive definite: at this u, with lambda = 100,
    # the stresses make it indefinite and the dense coarse Cholesky fails)
    mg = hx.Multigrid([op, make_pair((8, 8, 8), 1, "cnh", lam=100.0)[0]], precision="fp64")
    mg.update(to_dev(0.0 * u))
    z = mg.vcycle(to_dev(du))
    assert torch.isfinite(z).all()
    mg.close()
    op.close()


def test_autotune_on_a_general_mesh(device):
    V, C, F, G = workloads.ogrid_cylinder(2, 2, g=2)
    op = hx.HexOperator(V, C, 2, face_bid=F, dirichlet_bids=(1,), geom_degree=2, geom_nodes=G, law="cnh", mu=1.0,
                        lam=10.0)
    X = op.node_coords()
    u = 0.01 * np.stack([X[:, 2] * X[:, 0], X[:, 2] * X[:, 1], X[:, 2] ** 2])
    best, entries = op.autotune(to_dev(u), "fp32", reps=3)
    assert len(entries) == 14 and {e["variant"] for e in entries} == {0}
    with pytest.raises(hx.HxError):
        op.set_tuning("tangent", "fp64", variant=1)
    op.close()


def test_stored_table_round_trip(device, tmp_path):
    path = str(tmp_path / "tuning.json")
    op, pb = make_pair((6, 6, 6), 2, "inh")
    u, du = _fields(pb)
    ud = to_dev(u)
    best, used = hx.autotune_with_table(op, ud, "inh", "fp64", reps=3, path=path)
    table = json.load(open(path))
    assert len(table) == 8 and all(k.startswith("p2/inh/fp64/") for k in table)
    op.close()
    op, pb = make_pair((6, 6, 6), 2, "inh")
    best2, used2 = hx.autotune_with_table(op, ud, "inh", "fp64", reps=3, path=path)
    assert best2 == best and used2 == used
    y = to_host(op.apply_tangent(to_dev(du)), pb.mesh.n_nodes)
    assert rel(y, pb.apply_tangent(u, du)) < 1e-12
    op.close()
