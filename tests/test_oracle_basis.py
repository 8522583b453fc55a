"""Pins of the oracle's polynomial machinery, spaces and element matrices
against brute-force quadrature, closed forms and the identities of Sec. 4."""
import json
import math
import os

import numpy as np
import pytest

from oracle.poly import multi_indices, simplex_moment, product_moments, evaluate
from oracle.element import (element_geometry, element_system, expected_dims,
                            sigma_space, trace_free_basis)
from oracle.topology import Topology
import workloads as W
from tests.quadrature import element_rule, facet_rule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_simplex(d, seed):
    rng = np.random.default_rng(seed)
    X = np.vstack([np.zeros(d), np.eye(d)]) + 0.15 * rng.standard_normal((d + 1, d))
    return X


@pytest.mark.parametrize("d", [2, 3])
def test_bernstein_moment_formula_vs_quadrature(d):
    """int_T lambda^alpha = |T| d! alpha!/(|alpha|+d)!  (closed form) against a
    collapsed Gauss-Legendre rule on a random simplex."""
    X = _rand_simplex(d, 1)
    x, lam, w = element_rule(X, 8)
    vol = w.sum()
    for p in range(0, 7):
        for a in multi_indices(d + 1, p):
            q = np.sum(w * np.prod(lam ** np.asarray(a), axis=1))
            assert abs(q - vol * simplex_moment(a)) < 1e-13 * max(1.0, abs(q))


def test_local_dimensions_golden():
    """Local space dimensions (eqs. fes_V .. fes_Q) against the table in
    tests/golden/local_dims.json, and Sigma_h(T) against an independent rank
    count of the top-degree nt-trace constraints."""
    with open(os.path.join(GOLDEN, "local_dims.json")) as fh:
        gold = json.load(fh)
    for row in gold["rows"]:
        d, k = row["d"], row["k"]
        dims = expected_dims(d, k)
        for key in ("n_u", "n_bub", "n_F", "n_hat", "n_sig", "n_om", "n_p", "n_A", "n_d"):
            assert dims[key] == row[key], (d, k, key)
        if k <= 4 or d == 2:
            ed = element_geometry(_rand_simplex(d, 3), k)
            Z, _ = sigma_space(ed)
            assert Z.shape[1] == row["n_sig"]


@pytest.mark.parametrize("d,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_bdm_basis_spans_Pk(d, k):
    """The BDM basis (bubbles + facet functions) is a basis of P^k(T, R^d)."""
    ed = element_geometry(_rand_simplex(d, 5), k)
    M = ed.Phi.reshape(ed.Phi.shape[0], -1)
    assert np.linalg.matrix_rank(M) == d * math.comb(k + d, d) == M.shape[0]


@pytest.mark.parametrize("d,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_normal_traces(d, k):
    """Facet function (i, beta) has normal trace lambda^beta/|F_i| w.r.t. the
    global facet normal on F_i and zero on the other facets; bubbles have zero
    normal trace everywhere (Sec. 4.2, split of BDM into bubbles and facet
    functions).  Checked at quadrature points."""
    X = _rand_simplex(d, 7)
    ed = element_geometry(X, k)
    nb = ed.dims["n_bub"]
    nF = ed.dims["n_F"]
    for i in range(d + 1):
        fv = [j for j in range(d + 1) if j != i]
        pts, lamf, w = facet_rule(X[fv], 5)
        lam = np.zeros((len(pts), d + 1))
        lam[:, fv] = lamf
        vals = evaluate(np.moveaxis(ed.Phi, 0, 1), d + 1, k, lam)   # (N, n_u, d)
        nn = vals @ ed.normals_geo[i]
        assert np.abs(nn[:, :nb]).max() < 1e-10
        for jf in range(d + 1):
            blk = nn[:, nb + jf * nF: nb + (jf + 1) * nF]
            if jf != i:
                assert np.abs(blk).max() < 1e-10
            else:
                betas = multi_indices(d, k)
                expect = np.stack([np.prod(lamf ** np.asarray(b), axis=1) for b in betas], 1)
                assert np.allclose(blk, expect / ed.areas[i], atol=1e-10)


@pytest.mark.parametrize("d,k", [(2, 2), (3, 2), (3, 3)])
def test_global_normal_and_tangential_continuity(d, k):
    """Both neighbours of every interior facet produce the same normal trace of
    each facet basis function and the same tangential basis (H(div)
    conformity of V_h and single-valued hat V_h)."""
    mesh = W.unit_square_mesh(2) if d == 2 else W.unit_cube_mesh(1)
    topo = Topology(mesh.vertices, mesh.elements)
    nb = expected_dims(d, k)["n_bub"]
    nF = expected_dims(d, k)["n_F"]
    eds = [element_geometry(topo.element_coords(e), k) for e in range(len(topo.elements))]
    for f in topo.free_facets:
        (t1, i1), (t2, i2) = topo.facet_neighbors[f]
        P = topo.vertices[topo.facet_vertices[f]]
        pts, lamf, w = facet_rule(P, 4)
        tr = []
        tang = []
        for t, i in ((t1, i1), (t2, i2)):
            ed = eds[t]
            fv = [j for j in range(d + 1) if j != i]
            lam = np.zeros((len(pts), d + 1))
            lam[:, fv] = lamf
            vals = evaluate(np.moveaxis(ed.Phi, 0, 1), d + 1, k, lam)
            tr.append(vals[:, nb + i * nF: nb + (i + 1) * nF] @ ed.normals_geo[i])
            tv = evaluate(np.moveaxis(ed.Vhat[i], 0, 1), d + 1, k - 1, lam)
            tang.append(tv)
        assert np.allclose(tr[0], tr[1], atol=1e-10)
        assert np.allclose(tang[0], tang[1], atol=1e-12)


def _rigid_modes(d):
    modes = [lambda x, c=c: np.eye(d)[c] * np.ones((len(x), 1)) for c in range(d)]
    if d == 2:
        modes.append(lambda x: np.stack([-x[:, 1], x[:, 0]], 1))
    else:
        for a in range(3):
            e = np.eye(3)[a]
            modes.append(lambda x, e=e: np.cross(e, x))
    return modes


def _coefficients_of(ed, k, ufun, lam_fn=None):
    """(BDM coefficients of u, and per facet the coefficients of the L2(F)
    projection of u_t onto hat V_h(F)), computed with quadrature only."""
    d = ed.d
    X = ed.X
    # Bernstein coefficients of u by interpolation on many points
    x, lam, w = element_rule(X, k + 3)
    Ik = np.asarray(multi_indices(d + 1, k))
    Vb = np.prod(lam[:, None, :] ** Ik[None], axis=2)
    U = ufun(x)
    cb, *_ = np.linalg.lstsq(Vb, U, rcond=None)
    M = ed.Phi.reshape(ed.Phi.shape[0], -1).T
    cu, *_ = np.linalg.lstsq(M, cb.ravel(), rcond=None)
    ch = []
    for i in range(d + 1):
        fv = [j for j in range(d + 1) if j != i]
        pts, lamf, wf = facet_rule(X[fv], k + 3)
        lamv = np.zeros((len(pts), d + 1))
        lamv[:, fv] = lamf
        n = ed.normals_out[i]
        ut = ufun(pts)
        ut = ut - np.outer(ut @ n, n)
        Vh = evaluate(np.moveaxis(ed.Vhat[i], 0, 1), d + 1, k - 1, lamv)    # (N, n_hat, d)
        Mh = np.einsum("q,qar,qbr->ab", wf, Vh, Vh)
        rh = np.einsum("q,qar,qr->a", wf, Vh, ut)
        ch.append(np.linalg.solve(Mh, rh))
    return np.concatenate([cu, np.concatenate(ch)])


@pytest.mark.parametrize("d,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_condensed_block_psd_with_rigid_kernel(d, k):
    """A_T is symmetric PSD; its kernel has dimension d(d+1)/2 and contains the
    rigid motions embedded as (v, v_t) (derived from eq. schurnormmat)."""
    X = np.vstack([np.zeros(d), np.eye(d)]) + 0.05 * np.arange((d + 1) * d).reshape(d + 1, d) / d
    ed = element_geometry(X, k)
    es = element_system(ed, 1.3, k)
    A = es["A"]
    assert np.allclose(A, A.T, atol=1e-12 * np.abs(A).max())
    w = np.linalg.eigvalsh(A)
    tol = 1e-10 * w.max()
    assert w.min() > -tol
    assert np.sum(w < tol) == d * (d + 1) // 2
    for mode in _rigid_modes(d):
        x = _coefficients_of(ed, k, mode)
        assert np.linalg.norm(A @ x) < 1e-9 * np.linalg.norm(A) * np.linalg.norm(x)


@pytest.mark.parametrize("d,k", [(2, 2), (2, 3), (3, 2), (3, 3)])
def test_conforming_energy_identity(d, k):
    """eq. schur_SPD_cont, element-wise: for v in P^k(T, R^d) and hat u the
    L2(F) projection of v_t onto P^{k-1}, x^T A_T x = nu ||eps(v)||^2_T.
    The right side is evaluated by quadrature of an explicit polynomial."""
    rng = np.random.default_rng(11 + d + k)
    X = _rand_simplex(d, 13)
    nu = 0.7
    ed = element_geometry(X, k)
    es = element_system(ed, nu, k)
    # random v with monomial coefficients in x
    exps = [e for e in np.ndindex(*(k + 1,) * d) if sum(e) <= k]
    C = rng.standard_normal((len(exps), d))

    def v(x):
        Mx = np.stack([np.prod(x ** np.asarray(e), axis=1) for e in exps], 1)
        return Mx @ C

    def grad_v(x):
        G = np.zeros((len(x), d, d))
        for j in range(d):
            cols = []
            for e in exps:
                e2 = list(e)
                if e2[j] == 0:
                    cols.append(np.zeros(len(x)))
                    continue
                c0 = e2[j]
                e2[j] -= 1
                cols.append(c0 * np.prod(x ** np.asarray(e2), axis=1))
            G[:, :, j] = np.stack(cols, 1) @ C
        return G

    xc = _coefficients_of(ed, k, v)
    lhs = xc @ es["A"] @ xc
    x, lam, w = element_rule(X, k + 2)
    G = grad_v(x)
    eps = 0.5 * (G + np.transpose(G, (0, 2, 1)))
    rhs = nu * np.sum(w[:, None, None] * eps * eps)
    assert abs(lhs - rhs) < 1e-10 * abs(rhs)


@pytest.mark.parametrize("d,k", [(2, 2), (3, 2)])
def test_element_matrices_against_quadrature(d, k):
    """A^div, B (pressure coupling) and M_p against quadrature of the basis."""
    X = _rand_simplex(d, 17)
    nu = 1.9
    ed = element_geometry(X, k)
    es = element_system(ed, nu, k)
    x, lam, w = element_rule(X, k + 2)
    from oracle.poly import gradient_matrices
    Dk = gradient_matrices(d + 1, k, ed.grad_lambda)
    divc = np.einsum("sab,ibs->ia", Dk, ed.Phi)
    div_vals = evaluate(divc.T, d + 1, k - 1, lam)            # (N, n_u)
    Ig = np.asarray(multi_indices(d + 1, k - 1))
    P = np.prod(lam[:, None, :] ** Ig[None], axis=2)           # (N, n_p)
    Adiv = nu / d * np.einsum("q,qi,qj->ij", w, div_vals, div_vals)
    B = -np.einsum("q,qp,qi->pi", w, P, div_vals)
    Mp = np.einsum("q,qa,qb->ab", w, P, P) / nu
    assert np.allclose(es["Adiv"], Adiv, atol=1e-11 * np.abs(Adiv).max())
    assert np.allclose(es["B"], B, atol=1e-11 * np.abs(B).max())
    assert np.allclose(es["Mp"], Mp, atol=1e-12 * np.abs(Mp).max())


def test_colouring_valid():
    mesh = W.unit_cube_mesh(3)
    topo = Topology(mesh.vertices, mesh.elements)
    for e in range(len(topo.elements)):
        cs = [topo.colour[topo.free_facet_of[f]] for f in topo.elem_facets[e]
              if topo.free_facet_of[f] >= 0]
        assert len(cs) == len(set(cs))
