"""Barycentric (Bernstein-monomial) polynomial algebra on simplices -- oracle.

A polynomial of degree p on a d-simplex T is stored by its coefficients in the
homogeneous barycentric monomials lambda^alpha, |alpha| = p, alpha in N^{d+1}
(every polynomial of degree <= p has exactly one such representation, since
sum_i lambda_i = 1).  Integrals use the exact simplex formula

    int_T lambda^alpha dx = |T| d! alpha! / (|alpha| + d)!,

and on a facet F (a (d-1)-simplex; alpha supported on its vertices)

    int_F lambda^alpha ds = |F| (d-1)! alpha! / (|alpha| + d - 1)!.

No quadrature is used anywhere in the oracle.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def multi_indices(n_vars: int, degree: int):
    """All alpha in N^{n_vars} with |alpha| = degree, lexicographically descending."""
    if n_vars == 1:
        return ((degree,),)
    out = []
    for a in range(degree, -1, -1):
        for rest in multi_indices(n_vars - 1, degree - a):
            out.append((a,) + rest)
    return tuple(out)


@lru_cache(maxsize=None)
def index_map(n_vars: int, degree: int):
    return {a: i for i, a in enumerate(multi_indices(n_vars, degree))}


def _mfact(alpha):
    r = 1
    for a in alpha:
        r *= math.factorial(a)
    return r


@lru_cache(maxsize=None)
def simplex_moment(alpha: tuple) -> float:
    """int over the simplex of dimension len(alpha)-1 of lambda^alpha, divided by its measure."""
    dim = len(alpha) - 1
    return math.factorial(dim) * _mfact(alpha) / math.factorial(sum(alpha) + dim)


@lru_cache(maxsize=None)
def product_moments(n_vars: int, p: int, q: int) -> np.ndarray:
    """G[i, j] = (1/|T|) int_T lambda^{alpha_i + beta_j}, alpha in I_p, beta in I_q."""
    Ip = multi_indices(n_vars, p)
    Iq = multi_indices(n_vars, q)
    G = np.empty((len(Ip), len(Iq)))
    for i, a in enumerate(Ip):
        for j, b in enumerate(Iq):
            G[i, j] = simplex_moment(tuple(x + y for x, y in zip(a, b)))
    return G


@lru_cache(maxsize=None)
def facet_product_moments(n_vars: int, p: int, q: int, facet: int) -> np.ndarray:
    """G[i, j] = (1/|F|) int_F lambda^{alpha_i + beta_j} over the facet opposite
    vertex `facet`; zero whenever alpha or beta involves lambda_facet."""
    Ip = multi_indices(n_vars, p)
    Iq = multi_indices(n_vars, q)
    G = np.zeros((len(Ip), len(Iq)))
    for i, a in enumerate(Ip):
        if a[facet]:
            continue
        for j, b in enumerate(Iq):
            if b[facet]:
                continue
            s = tuple(x + y for k, (x, y) in enumerate(zip(a, b)) if k != facet)
            G[i, j] = simplex_moment(s)
    return G


@lru_cache(maxsize=None)
def derivative_tables(n_vars: int, p: int):
    """T[v] (|I_{p-1}| x |I_p|): d/d lambda_v applied to coefficient vectors."""
    Ip = multi_indices(n_vars, p)
    im = index_map(n_vars, p - 1)
    T = np.zeros((n_vars, len(im), len(Ip)))
    for j, a in enumerate(Ip):
        for v in range(n_vars):
            if a[v] > 0:
                b = list(a)
                b[v] -= 1
                T[v, im[tuple(b)], j] += a[v]
    return T


def gradient_matrices(n_vars: int, p: int, grad_lambda: np.ndarray) -> np.ndarray:
    """D[s] (|I_{p-1}| x |I_p|): d/dx_s on coefficient vectors (chain rule through
    the constant gradients of the barycentric coordinates)."""
    T = derivative_tables(n_vars, p)
    return np.einsum("vab,vs->sab", T, grad_lambda)


@lru_cache(maxsize=None)
def elevation(n_vars: int, p: int) -> np.ndarray:
    """E (|I_{p+1}| x |I_p|): degree elevation lambda^a = sum_v lambda^{a+e_v}."""
    Ip = multi_indices(n_vars, p)
    im = index_map(n_vars, p + 1)
    E = np.zeros((len(im), len(Ip)))
    for j, a in enumerate(Ip):
        for v in range(n_vars):
            b = list(a)
            b[v] += 1
            E[im[tuple(b)], j] += 1.0
    return E


def elevate_to(c: np.ndarray, n_vars: int, p: int, q: int) -> np.ndarray:
    """Re-express coefficient array c (leading axis over I_p) in degree q >= p."""
    out = c
    for r in range(p, q):
        out = np.tensordot(elevation(n_vars, r), out, axes=(1, 0))
    return out


def evaluate(c: np.ndarray, n_vars: int, p: int, lam: np.ndarray) -> np.ndarray:
    """Evaluate coefficient array c (leading axis over I_p) at barycentric points
    lam (n_pts, n_vars).  Returns (n_pts, *c.shape[1:])."""
    Ip = np.asarray(multi_indices(n_vars, p))
    V = np.prod(lam[:, None, :] ** Ip[None, :, :], axis=2)
    return np.tensordot(V, c, axes=(1, 0))
