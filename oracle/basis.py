"""1D rules of the discretisation: Gauss-Lobatto-Legendre (GLL) nodes, Gauss-Legendre quadrature
and the Lagrange basis, all on the reference interval [0, 1].

The paper discretises with continuous Lagrange elements of degree p and integrates by sum
factorisation with tensor-product quadrature (Section 6, matrix-free evaluation; Section 7.2).
The node set and the rule are fixed by the operator configurations: nodes at the p+1 GLL
points, Gauss quadrature with p+1 points per direction.

Test infrastructure only (see the package docstring). Pinned in tests/test_oracle_basis.py by:
textbook closed forms of the GLL points for p <= 4, exactness of the Gauss rule on monomials,
Kronecker property / partition of unity of the basis, and exact differentiation of polynomials.
"""
import numpy as np


def legendre(n, x):
    """Legendre polynomial P_n and its derivative at x in [-1, 1] (three-term recurrence)."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for k in range(2, n + 1):
        p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
    # derivative from (1 - x^2) P_n' = n (P_{n-1} - x P_n)
    dp = n * (p0 - x * p1) / (1.0 - x * x)
    return p1, dp


def gll_points(p):
    """The p+1 Gauss-Lobatto-Legendre points on [0, 1], ascending.

    Interior points are the roots of P_p'; they are found with numpy's polynomial root finder and
    polished by Newton steps on P_p' (its derivative from the Legendre ODE).
    """
    if p < 1:
        raise ValueError("degree must be >= 1")
    if p == 1:
        return np.array([0.0, 1.0])
    dP = np.polynomial.legendre.Legendre.basis(p).deriv()
    r = np.sort(np.real(dP.roots()))
    for _ in range(4):
        pn, dpn = legendre(p, r)
        # P_p'' from (1 - x^2) P'' = 2 x P' - p(p+1) P
        d2 = (2 * r * dpn - p * (p + 1) * pn) / (1.0 - r * r)
        r = r - dpn / d2
    x = np.concatenate(([-1.0], r, [1.0]))
    return 0.5 * (x + 1.0)


def gauss_rule(n):
    """n-point Gauss-Legendre rule on [0, 1]: (points ascending, weights summing to 1)."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def lagrange_values(nodes, x):
    """L[k, i] = l_i(x_k) for the Lagrange polynomials l_i on ``nodes`` (product formula)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    L = np.ones((len(x), n))
    for i in range(n):
        for m in range(n):
            if m != i:
                L[:, i] *= (x - nodes[m]) / (nodes[i] - nodes[m])
    return L


def lagrange_derivatives(nodes, x):
    """dL[k, i] = l_i'(x_k): derivative of the product formula, term by term."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    dL = np.zeros((len(x), n))
    for i in range(n):
        for m in range(n):
            if m == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[m]))
            for l in range(n):
                if l != i and l != m:
                    term *= (x - nodes[l]) / (nodes[i] - nodes[l])
            dL[:, i] += term
    return dL
