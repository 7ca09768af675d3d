"""Host logic of bench.py (no GPU): the single-GPU guard, the algorithmic bytes per DoF against the
per-degree table of the measurement plan, and the reader of the committed counter traffic, which
must drop a figure taken on another kernel source."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

CUBE = {2: (32768, 823875), 3: (32768, 2738019), 4: (32768, 6440067), 6: (32768, 21567171)}


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


# bytes per DoF of the 32^3 cube (FP64, cNH) as tabulated in the measurement plan: vectors du and
# dst (and u_k in recompute mode) plus the stored words of every q-point; the plan's entries of the
# two modes that form the geometry from the vertices also count up to 1 B/DoF of vertex reads,
# which the bench leaves out
PLAN_BYTES_PER_DOF = {
    2: {"none": 25.1, "finv_j": 102.9, "tangent": 402.6},
    3: {"none": 24.3, "finv_j": 77.6, "tangent": 291.7},
    4: {"none": 24.1, "finv_j": 67.0, "tangent": 245.0},
    6: {"none": 24.0, "finv_j": 57.7, "tangent": 203.6},
}


@pytest.mark.parametrize("p", [2, 3, 4, 6])
def test_algorithmic_bytes_match_the_plan(p):
    cells, dofs = CUBE[p]
    for mode, ref in PLAN_BYTES_PER_DOF[p].items():
        b, f = bench.algorithmic(p, mode, cells, dofs)
        slack = 1.1 if mode in ("none", "finv_j") else 0.06
        assert ref - slack <= b / dofs <= ref + 0.06, (p, mode, b / dofs, ref)
        assert f > 0


def test_spatial_bytes_of_the_headline():
    b, _ = bench.algorithmic(4, "spatial", 32768, 6440067)
    # 16 words per q-point, 125 q-points per cell, plus du and dst
    assert b == pytest.approx(627.3e6, rel=1e-3)


def test_traffic_reader_checks_the_kernel_source(tmp_path, monkeypatch):
    src_dir = tmp_path / "paper_2408_12479_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    kernel = src_dir / "hx_kernels.hpp"
    kernel.write_text("// kernel A\n")
    sha = hashlib.sha256(kernel.read_bytes()).hexdigest()
    (tmp_path / "profiles" / "apply_hbm_traffic_cube32.txt").write_text(
        "header line\n"
        f"traffic p=4 mode=spatial hbm_bytes_per_apply=8.5e+08 kernel_src_sha256={sha}\n"
        f"traffic p=4 mode=tangent hbm_bytes_per_apply=1.9e+09 kernel_src_sha256={'0' * 64}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(4, "spatial") == pytest.approx(8.5e8)
    assert bench.measured_traffic(4, "tangent") is None      # taken on another source
    assert bench.measured_traffic(6, "spatial") is None      # not measured
    kernel.write_text("// kernel B\n")
    assert bench.measured_traffic(4, "spatial") is None      # source changed since


def test_sweep_parity_on_a_small_cube():
    """The oracle leg's sampled-row check: rows equal to the oracle's full apply give zero error, a
    relative perturbation of 1e-9 gives 1e-9."""
    import numpy as np

    import workloads
    from oracle import fem, material, mesh
    p, cells = 2, 4
    V = workloads.box_vertices(cells, cells, cells, perturb=0.2, seed=2)
    m = mesh.BoxMesh(cells, cells, cells, V, p, dirichlet_faces=(0,))
    pb = fem.Problem(m, material.Material("cnh", mu=1.0, lam=100.0))
    u, du = workloads.sweep_fields(m.node_coords, m.constrained)
    nodes = bench.sample_nodes(m.n_nodes, p)
    assert nodes[0] == 0 and nodes[-1] == m.n_nodes - 1
    full = pb.apply_tangent(u, du).reshape(3, m.n_nodes)[:, nodes]
    out = bench.sweep_parity({p: (nodes, {"same": full, "scaled": full * (1 + 1e-9)})}, cells)
    assert out["p2"]["same"] == 0.0
    assert out["p2"]["scaled"] == pytest.approx(1e-9, rel=1e-3)
    assert out["p2"]["rows"] == 3 * len(nodes)


def test_line_flops_follow_the_even_odd_form():
    """Flops of one 1D contraction as executed: plain n^2 multiply-adds up to n = 4; from n = 5 on
    the even-odd form (n = 5: 13 multiply-adds and 8 additions for the interpolation matrix, n = 7:
    25 and 12), always below the plain count."""
    assert bench.line_flops(3, 1) == 18 and bench.line_flops(4, -1) == 32
    assert bench.line_flops(5, 1) == 2 * 13 + 8
    assert bench.line_flops(7, 1) == 2 * 25 + 12
    for n in (5, 6, 7):
        assert bench.line_flops(n, 1) < 2 * n * n and bench.line_flops(n, -1) < 2 * n * n


def test_oracle_leg_runs_in_a_worker_pool():
    """The cpu_baseline leg on a tiny cube: every cell is timed, all rows compared give zero error
    against the oracle's own full apply, and the cores and host model are stated."""
    import numpy as np

    import workloads
    from oracle import fem, material, mesh
    p, cells = 2, 3
    V = workloads.box_vertices(cells, cells, cells, perturb=0.2, seed=2)
    m = mesh.BoxMesh(cells, cells, cells, V, p, dirichlet_faces=(0,))
    pb = fem.Problem(m, material.Material("cnh", mu=1.0, lam=100.0))
    u, du = workloads.sweep_fields(m.node_coords, m.constrained)
    full = pb.apply_tangent(u, du).reshape(-1)
    pool = bench.start_oracle_pool(2)
    out = bench.cpu_baseline(pool, 2, p, cells, budget_s=30.0, gpu_dst=full)
    assert out["cores"] == 2 and out["host"]["nproc"] >= 1 and out["host"]["model"]
    assert f"{m.n_cells} of {m.n_cells} cells" in out["sample"]
    assert out["rel_err_vs_oracle"] < 1e-14
    assert out["rows_compared"] > 0
    assert np.isfinite(out["value"]) and out["value"] > 0
