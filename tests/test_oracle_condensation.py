"""Pins of the oracle's condensation of the bubbles and of A-hat_ext against
what the mathematics fixes, computed by routes that share nothing with the
element-by-element code they check.

* Condensation II (Sec. 4.2, eq. doubleschurinf): A^d is the Schur complement
  of the globally assembled velocity block A over its bubble dofs, and
  x^T A^d x is the minimum over the bubble values of the A-energy of (u_o, x).
* The bubble extension (eq. Hcoeffs): A_oo H = A_od element by element, so the
  globally assembled extension (-H x, x) leaves no residual in the bubble rows
  and has A-energy x^T A^d x.
* A-hat_ext (eq. factorSsigma, Sec. 6.1): with the exact A^d^{-1} in place of
  the auxiliary-space preconditioner the factorisation is exact, so
  A-hat_ext^{-1} = A^{-1} on the velocity block.
* K-hat^{-1} (eq. mhatinvfactor): with the exact A-hat = A, K-hat and K agree
  on every vector with zero pressure part, so K-hat^{-1} K (u, 0) = (u, 0).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.precond import Preconditioner
from tests.test_oracle_system import problem

CASES = [(2, 2, 2), (2, 2, 3), (3, 1, 2)]


def _velocity_block(gs):
    K = gs.assemble_K().tocsr()
    return K[:gs.off_p][:, :gs.off_p].toarray()


def _assembled_Ad(gs):
    idx = np.arange(gs.off_f, gs.off_p)
    Ad = np.zeros((len(idx), len(idx)))
    for e, es in enumerate(gs.elems):
        ld = gs.local_dofs(e)[gs.nb:] - gs.off_f
        m = ld >= 0
        Ad[np.ix_(ld[m], ld[m])] += es["Ad"][np.ix_(m, m)]
    return Ad


@pytest.mark.parametrize("d,n,k", CASES)
def test_Ad_is_global_schur_complement(d, n, k):
    """eq. doubleschurinf: the sum of the element A^d_T equals the Schur
    complement of the assembled A over all bubble dofs (a dense global
    solve; A_oo is block diagonal, so the two must agree)."""
    _, gs, _ = problem(d, n, k)
    A = _velocity_block(gs)
    o = slice(0, gs.off_f)
    f = slice(gs.off_f, gs.off_p)
    S = A[f, f] - A[f, o] @ np.linalg.solve(A[o, o], A[o, f])
    Ad = _assembled_Ad(gs)
    assert np.abs(Ad - S).max() <= 1e-11 * np.abs(S).max()
    # and it is not the uncondensed facet block
    assert np.abs(A[f, f] - S).max() > 1e-3 * np.abs(S).max()


@pytest.mark.parametrize("d,n,k", CASES)
def test_Ad_energy_is_minimum_over_bubbles(d, n, k):
    """x^T A^d x = min over u_o of the A-energy of (u_o, x): random bubble
    values never go below it, and conjugate gradients on the bubble block
    (a library solver) reach it."""
    _, gs, _ = problem(d, n, k)
    A = _velocity_block(gs)
    Ad = _assembled_Ad(gs)
    rng = np.random.default_rng(11)
    nb, nf = gs.off_f, gs.off_p - gs.off_f
    for _ in range(3):
        x = rng.standard_normal(nf)
        emin = x @ Ad @ x

        def energy(uo):
            v = np.concatenate([uo, x])
            return v @ A @ v

        uo, info = spla.cg(A[:nb, :nb], -A[:nb, nb:] @ x, rtol=1e-14, atol=0.0, maxiter=10 * nb)
        assert info == 0
        assert abs(energy(uo) - emin) <= 1e-10 * abs(emin)
        for _ in range(20):
            assert energy(uo + 0.1 * rng.standard_normal(nb)) >= emin * (1 - 1e-12)


@pytest.mark.parametrize("d,n,k", CASES)
def test_bubble_extension_is_discrete_harmonic(d, n, k):
    """eq. Hcoeffs: A_oo H = A_od per element, and the assembled extension
    (-H_T x_T per element, x) has zero residual in every bubble row of A and
    A-energy x^T A^d x."""
    _, gs, _ = problem(d, n, k)
    for es in gs.elems:
        assert np.abs(es["Aoo"] @ es["H"] - es["Aod"]).max() <= 1e-11 * np.abs(es["Aod"]).max()
    A = _velocity_block(gs)
    Ad = _assembled_Ad(gs)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(gs.off_p - gs.off_f)
    xg = np.zeros(gs.n_dof)
    xg[gs.off_f:gs.off_p] = x
    v = np.zeros(gs.off_p)
    v[gs.off_f:] = x
    for e, es in enumerate(gs.elems):
        ld = gs.local_dofs(e)[gs.nb:]
        xl = np.where(ld >= 0, xg[np.maximum(ld, 0)], 0.0)
        v[e * gs.nb:(e + 1) * gs.nb] = -es["H"] @ xl
    r = A @ v
    assert np.abs(r[:gs.off_f]).max() <= 1e-11 * np.abs(r).max()
    assert abs(v @ r - x @ Ad @ x) <= 1e-11 * abs(x @ Ad @ x)


@pytest.mark.parametrize("d,n,k", CASES)
def test_A_ext_with_exact_Ad_is_A_inverse(d, n, k):
    """eq. factorSsigma: A-hat_ext^{-1} with A^d^{-1} in place of
    A-hat^d_m^{-1} is A^{-1} (velocity block), for random right-hand sides."""
    mesh, gs, _ = problem(d, n, k)
    pc = Preconditioner(gs, mesh.lattice)
    Ad = _assembled_Ad(gs)
    f = slice(gs.off_f, gs.off_p)

    def exact_Ad_inv(s):
        t = np.zeros_like(s)
        t[f] = np.linalg.solve(Ad, s[f])
        return t

    pc.Ad_inv = exact_Ad_inv
    A = _velocity_block(gs)
    rng = np.random.default_rng(13)
    for _ in range(3):
        r = np.zeros(gs.n_dof)
        r[:gs.off_p] = rng.standard_normal(gs.off_p)
        y = pc.A_ext_inv(r)
        ye = np.linalg.solve(A, r[:gs.off_p])
        assert np.linalg.norm(y[:gs.off_p] - ye) <= 1e-10 * np.linalg.norm(ye)
        assert not np.any(y[gs.off_p:])


@pytest.mark.parametrize("d,n,k", CASES[:2])
def test_khat_with_exact_A_fixes_velocity_vectors(d, n, k):
    """eq. mhatinvfactor with A-hat = A: K-hat = [[A, B^T], [B, M_p + B A^{-1}
    B^T]], so K-hat (u, 0) = K (u, 0) and K-hat^{-1} K (u, 0) = (u, 0)."""
    mesh, gs, _ = problem(d, n, k)
    pc = Preconditioner(gs, mesh.lattice)
    A = _velocity_block(gs)

    def exact_A_inv(r):
        y = np.zeros_like(r)
        y[:gs.off_p] = np.linalg.solve(A, r[:gs.off_p])
        return y

    pc.A_hat_inv = exact_A_inv
    K = gs.assemble_K().tocsr()
    rng = np.random.default_rng(14)
    u = np.zeros(gs.n_dof)
    u[:gs.off_p] = rng.standard_normal(gs.off_p)
    z = pc.apply(K @ u)
    assert np.linalg.norm(z - u) <= 1e-10 * np.linalg.norm(u)
    # and K-hat (0, p) = (B^T p, M_p p + B A^{-1} B^T p) is mapped back to (0, p)
    p = np.zeros(gs.n_dof)
    p[gs.off_p:] = rng.standard_normal(gs.n_dof - gs.off_p)
    Btp = (K @ p)[:gs.off_p]
    Mp = np.zeros(gs.n_dof - gs.off_p)
    for e, es in enumerate(gs.elems):
        sl = gs.pressure_dofs(e) - gs.off_p
        Mp[sl] = es["Mp"] @ p[gs.off_p:][sl]
    Khat_p = np.concatenate([Btp, Mp + (K @ np.concatenate([np.linalg.solve(A, Btp),
                                                            np.zeros(gs.n_dof - gs.off_p)]))[gs.off_p:]])
    z = pc.apply(Khat_p)
    assert np.linalg.norm(z - p) <= 1e-10 * np.linalg.norm(p)


@pytest.mark.parametrize("d,k", [(2, 2), (2, 4), (3, 2), (3, 3), (3, 4), (3, 5)])
def test_condensed_operator_independent_of_sigma_basis(d, k):
    """sigma and omega are condensed element by element (Sec. 4.2), so the
    condensed velocity block A_T, and with it A_oo, H and A^d, do not depend
    on the basis of Sigma_h(T): computed in a randomly rotated orthonormal
    basis they agree with the natural one to rounding (1e-10 relative; H, the
    most sensitive, moves by ~2e-11 at k = 5), while the rotated stress mass
    matrix itself differs at O(1)."""
    from oracle.element import element_geometry, element_system
    rng = np.random.default_rng(5 + 10 * d + k)
    X = np.vstack([np.zeros(d), np.eye(d)]) + 0.2 * rng.standard_normal((d + 1, d))
    ed = element_geometry(X, k)
    a = element_system(ed, 0.7, k, keep_blocks=True)
    b = element_system(ed, 0.7, k, keep_blocks=True, sigma_rotation_seed=3)
    assert np.abs(a["Mss"] - b["Mss"]).max() > 1e-3 * np.abs(a["Mss"]).max()
    for key in ("A", "Aoo", "H", "Ad"):
        sc = max(np.abs(a[key]).max(), 1e-300)
        assert np.abs(a[key] - b[key]).max() <= 1e-10 * sc, key
