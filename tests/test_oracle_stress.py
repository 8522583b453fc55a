"""Pins of the oracle's stress/vorticity recovery (Sec. 4.2, eq. projection).

* Lemma SPD (end of its proof): for conforming velocity data -- u a
  polynomial of degree k and uhat_F the L2 projection of its tangential
  trace onto P^{k-1}(F), so that the facet jump terms vanish -- the local
  problems give sigma_h = -nu dev eps(u) and omega_h = kappa(curl u), with
  kappa the skew embedding of the curl (Sec. 2 notation).
* Lemma SPD: the A-energy of any (u, uhat) equals
  nu^{-1} ||sigma_h||^2 + nu d^{-1} ||div u||^2 on the element.
"""
import numpy as np
import pytest

from oracle.element import element_geometry, element_system, recover_stress
from oracle.poly import evaluate, facet_product_moments, gradient_matrices, product_moments


def _simplex(d, seed):
    rng = np.random.default_rng(seed)
    while True:
        X = rng.uniform(-1.0, 1.0, size=(d + 1, d))
        det = np.linalg.det((X[1:] - X[0]).T)
        if abs(det) > 0.2:
            return X


def _conforming_local(ed, k, field):
    """Local (u, uhat) coefficients ([Phi | Vhat] order) of the polynomial
    velocity `field` (coefficients (|I_k|, d) over lambda^alpha), with uhat on
    every facet the L2 projection of the tangential trace."""
    nv = ed.d + 1
    n_u = ed.Phi.shape[0]
    cu = np.linalg.solve(ed.Phi.reshape(n_u, -1).T, field.ravel())
    ch = []
    for i in range(nv):
        Gf = facet_product_moments(nv, k, k - 1, i) * ed.areas[i]
        Gff = facet_product_moments(nv, k - 1, k - 1, i) * ed.areas[i]
        V = ed.Vhat[i]
        Mf = np.einsum("jgr,gh,lhr->jl", V, Gff, V)
        rf = np.einsum("ar,ag,jgr->j", field, Gf, V)
        ch.append(np.linalg.solve(Mf, rf))
    return np.concatenate([cu] + ch)


def _kappa(curl, d):
    n = curl.shape[0]
    K = np.zeros((n, d, d))
    if d == 2:
        K[:, 0, 1] = -curl / 2
        K[:, 1, 0] = curl / 2
    else:
        K[:, 0, 1], K[:, 0, 2] = -curl[:, 2] / 2, curl[:, 1] / 2
        K[:, 1, 0], K[:, 1, 2] = curl[:, 2] / 2, -curl[:, 0] / 2
        K[:, 2, 0], K[:, 2, 1] = -curl[:, 1] / 2, curl[:, 0] / 2
    return K


@pytest.mark.parametrize("d,k,nu", [(2, 2, 1.0), (2, 3, 0.3), (3, 2, 1.0), (3, 3, 2.5)])
def test_conforming_velocity_gives_deviatoric_strain_and_rotation(d, k, nu):
    ed = element_geometry(_simplex(d, 10 * d + k), k)
    nv = d + 1
    rng = np.random.default_rng(d + 7 * k)
    field = rng.standard_normal((len(ed.Phi[0]), d))
    S, W = recover_stress(ed, nu, k, _conforming_local(ed, k, field))
    lam = rng.dirichlet(np.ones(nv), size=6)
    Dk = gradient_matrices(nv, k, ed.grad_lambda)
    dudx = np.stack([evaluate(Dk[s] @ field, nv, k - 1, lam) for s in range(d)], axis=1)  # [n, s, r] = d_s u_r
    eps = 0.5 * (dudx + dudx.transpose(0, 2, 1))
    dev = eps - np.einsum("nii->n", eps)[:, None, None] * np.eye(d) / d
    if d == 2:
        curl = dudx[:, 0, 1] - dudx[:, 1, 0]
    else:
        curl = np.stack([dudx[:, 1, 2] - dudx[:, 2, 1], dudx[:, 2, 0] - dudx[:, 0, 2],
                         dudx[:, 0, 1] - dudx[:, 1, 0]], axis=1)
    sig = evaluate(S, nv, k, lam)
    om = evaluate(W, nv, k - 1, lam)
    scale = np.abs(dudx).max()
    assert np.abs(sig - (-nu * dev)).max() <= 1e-10 * nu * scale
    assert np.abs(om - _kappa(curl, d)).max() <= 1e-10 * scale


@pytest.mark.parametrize("d,k", [(2, 2), (2, 4), (3, 2), (3, 3)])
def test_energy_identity(d, k):
    """(u, uhat)^T A (u, uhat) = nu^{-1} int sigma : sigma + nu/d int (div u)^2
    for arbitrary element coefficients (no conformity needed)."""
    nu = 0.7
    ed = element_geometry(_simplex(d, 3 * d + k), k)
    es = element_system(ed, nu, k)
    rng = np.random.default_rng(5)
    ul = rng.standard_normal(es["A"].shape[0])
    S, W = recover_stress(ed, nu, k, ul)
    G = product_moments(d + 1, k, k) * ed.vol
    ss = np.einsum("ars,ab,brs->", S, G, S)
    cu = ul[: es["Adiv"].shape[0]]
    lhs = ul @ es["A"] @ ul
    rhs = ss / nu + cu @ es["Adiv"] @ cu
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)
    # sigma is trace free pointwise and weakly symmetric: orthogonal to every
    # skew lambda^gamma K, |gamma| = k-1
    lam = rng.dirichlet(np.ones(d + 1), size=4)
    assert np.abs(np.einsum("nii->n", evaluate(S, d + 1, k, lam))).max() <= 1e-11 * np.abs(S).max()
    Gm = product_moments(d + 1, k, k - 1) * ed.vol
    skew = S - S.transpose(0, 2, 1)
    assert np.abs(np.einsum("ars,ag->grs", skew, Gm)).max() <= 1e-11 * np.abs(S).max() * ed.vol
