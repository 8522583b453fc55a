"""Brute-force quadrature used by the tests to pin the oracle's exact formulas.

Collapsed (Duffy) tensor Gauss-Legendre rules on the unit simplex; exact for
polynomials of degree <= 2 n - 1 - (dim - 1).  Independent of the Bernstein
moment formula the oracle uses."""
import numpy as np


def simplex_rule(dim, n):
    """Points (barycentric, (N, dim+1)) and weights (sum = 1) on a dim-simplex."""
    g, w = np.polynomial.legendre.leggauss(n)
    g = 0.5 * (g + 1.0)
    w = 0.5 * w
    if dim == 1:
        x = g
        lam = np.stack([1 - x, x], axis=1)
        return lam, w
    if dim == 2:
        U, V = np.meshgrid(g, g, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        x = U
        y = V * (1 - U)
        wt = WU * WV * (1 - U)
        lam = np.stack([1 - x - y, x, y], axis=-1).reshape(-1, 3)
        return lam, 2.0 * wt.ravel()
    if dim == 3:
        U, V, Z = np.meshgrid(g, g, g, indexing="ij")
        WU, WV, WZ = np.meshgrid(w, w, w, indexing="ij")
        x = U
        y = V * (1 - U)
        z = Z * (1 - U) * (1 - V)
        wt = WU * WV * WZ * (1 - U) ** 2 * (1 - V)
        lam = np.stack([1 - x - y - z, x, y, z], axis=-1).reshape(-1, 4)
        return lam, 6.0 * wt.ravel()
    raise ValueError(dim)


def element_rule(X, n):
    """Physical points (N, d), barycentrics (N, d+1) and weights on simplex X."""
    d = X.shape[1]
    lam, w = simplex_rule(d, n)
    J = (X[1:] - X[0]).T
    vol = abs(np.linalg.det(J)) / np.prod(np.arange(1, d + 1))
    return lam @ X, lam, w * vol


def facet_rule(P, n):
    """Points (N, d) and weights on the (d-1)-simplex with vertices P (d, d)."""
    d = P.shape[1]
    lam, w = simplex_rule(d - 1, n)
    if d == 2:
        meas = np.linalg.norm(P[1] - P[0])
    else:
        meas = 0.5 * np.linalg.norm(np.cross(P[1] - P[0], P[2] - P[0]))
    return lam @ P, lam, w * meas
