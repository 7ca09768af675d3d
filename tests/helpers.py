"""Shared construction of oracle problems for the tests (test-side only)."""
import numpy as np

import workloads
from oracle import fem, fiber, material, mesh


def fiber_material(mu=2.0, kappa=1e3, k1=1.0, k2=10.0, phi_deg=45.0, dispersion=(3.62, 34.3)):
    if dispersion is None:
        H11, H22, H33 = 1.0, 0.0, 0.0
    else:
        H11, H22, H33 = fiber.dispersion_coefficients(*dispersion)
    E1, E2, E3 = np.eye(3)
    H4, H6, M4, M6 = fiber.structure_tensors(E1, E2, E3, np.deg2rad(phi_deg), H11, H22, H33)
    return material.Material("fiber", mu=mu, kappa=kappa, k1=k1, k2=k2, H4=H4, H6=H6, M4=M4, M6=M6)


def make_material(law, **kw):
    if law == "cnh":
        return material.Material("cnh", mu=kw.get("mu", 1.0), lam=kw.get("lam", 10.0))
    if law == "inh":
        return material.Material("inh", mu=kw.get("mu", 2.0), kappa=kw.get("kappa", 50.0))
    return fiber_material(mu=kw.get("mu", 2.0), kappa=kw.get("kappa", 50.0), k1=kw.get("k1", 1.0),
                          k2=kw.get("k2", 10.0), dispersion=kw.get("dispersion", (3.62, 34.3)))


def box_problem(nc, p, law="cnh", perturb=0.2, seed=2, faces=(0,), lengths=(1.0, 1.0, 1.0), **kw):
    nx, ny, nz = (nc, nc, nc) if np.isscalar(nc) else nc
    V = workloads.box_vertices(nx, ny, nz, lengths=lengths, perturb=perturb, seed=seed)
    m = mesh.BoxMesh(nx, ny, nz, V, p, dirichlet_faces=faces)
    return fem.Problem(m, make_material(law, **kw))


def random_F(rng, n, scale):
    return np.eye(3)[None] + scale * rng.uniform(-1, 1, size=(n, 3, 3))
