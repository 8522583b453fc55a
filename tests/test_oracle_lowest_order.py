"""Pins of the oracle's lowest-order method, k = 1 in 3D (Sec. 7, the lowest
order case): W_h the lowest-order Raviart-Thomas space (one flux per facet,
coupled across facets), kappa(omega) in place of omega, the stabilisation
nu h_T^2 (div omega, div eta)_T with h_T = |T|^(1/3), only sigma condensed,
facet blocks of 3 + 2 + 1 dofs, and E u = (u, Pi^0 u_t, curl u).

The pins are the facts that fix the method independently of how the oracle
writes it: the dimension count of Sec. 7, the rigid motions (the reason for
the extra dof: a rotation must cost no energy), a linear Stokes flow
reproduced exactly (patch test, with the pressure projected onto P^0), the
energy identity of E (Corollary embed), divergence-free velocities, the
condensed operator's independence of the stress basis, the robustness of the
preconditioner in h, and MINRES against the direct solve."""
import math

import numpy as np
import pytest

import workloads as W
from oracle.element import element_geometry, element_system, expected_dims
from oracle.minres import minres
from oracle.precond import Preconditioner, assemble_p1, embedding
from oracle.system import GlobalSystem
from tests.quadrature import element_rule

_cache = {}


def problem(n, nu=1.0):
    key = (n, nu)
    if key not in _cache:
        mesh = W.unit_cube_mesh(n)
        sol = W.CurlModes3D(seed=2, nu=nu)
        f = sol.f(W.lattice_points(mesh, 2))
        _cache[key] = (mesh, GlobalSystem(mesh.vertices, mesh.elements, nu, 1, f), sol)
    return _cache[key]


def test_dofs_per_facet():
    """Sec. 7: with k = 1 a facet has three coupling dofs in V_h (BDM^1), two
    in hat V_h, and the flux of omega in W_h makes six; there are no velocity
    bubbles, Sigma_h(T) has 16 dimensions and the pressure is P^0.  The
    two-dimensional method is not defined there."""
    dm = expected_dims(3, 1)
    assert (dm["n_F"], dm["n_hat"], dm["n_w"], dm["n_fb"]) == (3, 2, 1, 6)
    assert (dm["n_bub"], dm["n_sig"], dm["n_p"], dm["n_om"]) == (0, 16, 1, 4)
    assert dm["n_d"] == 24 and dm["n_A"] == 24
    assert expected_dims(3, 2)["n_w"] == 0
    with pytest.raises(ValueError):
        expected_dims(2, 1)


def _element():
    rng = np.random.default_rng(11)
    X = np.array([[0, 0, 0], [1, 0.1, 0], [0.2, 1, 0.1], [0.1, 0.3, 1.2]]) + 0.1 * rng.standard_normal((4, 3))
    return X, element_geometry(X, 1)


def _linear_field_dofs(X, ed, G, c, omega):
    """Local dofs (order of the element matrix 'A': BDM^1, hat V, omega) of
    the linear field u(x) = G x + c with the given omega: the BDM^1
    coefficients from the field's vertex values, the facet means of u_t in the
    tangent basis, the fluxes of omega through the facets w.r.t. n_F."""
    vals = X @ G.T + c                                   # lambda_j coefficients of u
    M = ed.Phi.reshape(ed.Phi.shape[0], -1).T
    cu = np.linalg.lstsq(M, vals.ravel(), rcond=None)[0]
    assert np.allclose(M @ cu, vals.ravel())
    ch = []
    for i in range(4):
        mean = np.delete(vals, i, axis=0).mean(axis=0)
        n = ed.normals_out[i]
        tgt = mean - n * (n @ mean)
        T = ed.Vhat[i][:, 0, :].T                        # the tangents t_b
        ch.append(np.linalg.lstsq(T, tgt, rcond=None)[0])
    om = [ed.areas[i] * omega @ ed.normals_geo[i] for i in range(4)]
    return np.concatenate([cu, np.concatenate(ch), om])


def test_rigid_motions_cost_no_energy():
    """The six rigid motions u = a + b x x (curl u = 2b) with omega = curl u
    lie in the kernel of the element's condensed operator: this is what the
    sixth facet dof is for (Sec. 7).  With omega = -curl u, or for a pure
    strain, the energy is not zero."""
    X, ed = _element()
    A = element_system(ed, 1.3, 1)["A"]
    nA = np.linalg.norm(A, 2)
    rng = np.random.default_rng(2)
    for _ in range(3):
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        Rb = np.array([[0, -b[2], b[1]], [b[2], 0, -b[0]], [-b[1], b[0], 0]])
        v = _linear_field_dofs(X, ed, Rb, a, 2 * b)
        assert np.linalg.norm(A @ v) <= 1e-12 * nA * np.linalg.norm(v)
        w = _linear_field_dofs(X, ed, Rb, a, -2 * b)
        assert np.linalg.norm(A @ w) >= 1e-3 * nA * np.linalg.norm(w)
    S = np.diag([1.0, -1.0, 0.0])
    v = _linear_field_dofs(X, ed, S, np.zeros(3), np.zeros(3))
    assert v @ A @ v >= 1e-3 * nA * (v @ v)


def test_linear_stokes_flow_reproduced():
    """Patch test: a linear divergence-free velocity with its Dirichlet data
    (the tangential means and the flux of curl g on the boundary facets) and
    f = grad p for a linear p: u_h = u exactly, and p_h is the element mean of
    p (Q_h = P^0), since div V_h = Q_h and f = grad p only tests div v."""
    G = np.array([[1.0, -1.0, 2.0], [3.0, 1.0, -1.0], [1.0, -2.0, -2.0]])
    c0 = np.array([0.3, -0.2, 0.5])
    mesh = W.unit_cube_mesh(2)
    pts = W.lattice_points(mesh, 2)
    gp = np.array([0.5, -1.0, 2.0])
    gs = GlobalSystem(mesh.vertices, mesh.elements, 0.8, 1, np.broadcast_to(gp, pts.shape).copy(),
                      g_lattice=pts @ G.T + c0)
    x = gs.normalize_pressure(gs.direct_solve())
    vol = 1.0 / (6 * 8)
    pm = []
    for e in range(gs.n_e):
        Xe = gs.topo.element_coords(e)
        xq, lam, w = element_rule(Xe, 3)
        u, p = gs.eval_element(x, e, lam)
        assert np.abs(u - (xq @ G.T + c0)).max() < 1e-11
        pm.append((p[0], Xe.mean(axis=0) @ gp))
    pm = np.asarray(pm)
    pm -= pm.mean(axis=0)                     # mean-free (equal volumes)
    assert np.abs(pm[:, 0] - pm[:, 1]).max() < 1e-10
    assert vol > 0


def test_embedding_energy_identity():
    """Corollary embed for the lowest order: ||E u||_A = ||u||_{A-bar} for
    continuous P1 u, with the curl component of E and the facet means of
    u_t."""
    mesh, gs, _ = problem(2)
    A = gs.assemble_K()[:gs.off_p, :gs.off_p].toarray()
    E = embedding(gs).toarray()[:gs.off_p]
    Abar = assemble_p1(gs).toarray()
    assert np.allclose(E.T @ A @ E, Abar, atol=1e-10 * np.abs(Abar).max())


def test_exactly_divergence_free():
    """div BDM^1 = P^0 = Q_h: div u_h = 0 pointwise to round-off."""
    from oracle.poly import gradient_matrices
    mesh, gs, _ = problem(2)
    x = gs.direct_solve()
    unorm = np.abs(x[:gs.off_p]).max()
    for e in range(gs.n_e):
        es = gs.elems[e]
        ed = es["ed"]
        ld = gs.local_dofs(e)
        coef = np.where(ld >= 0, x[np.maximum(ld, 0)], 0.0)
        orig = np.zeros(len(coef))
        orig[es["perm"]] = coef
        Dk = gradient_matrices(4, 1, ed.grad_lambda)
        divc = np.einsum("sab,ibs->ia", Dk, ed.Phi).T @ orig[:gs.dims["n_u"]]
        assert np.abs(divc).max() < 1e-9 * unorm / ed.vol ** (1.0 / 3)


def test_condensed_operator_independent_of_sigma_basis():
    """Only sigma is condensed; its basis does not enter the result."""
    X, ed = _element()
    a = element_system(ed, 0.7, 1, keep_blocks=True)
    b = element_system(ed, 0.7, 1, keep_blocks=True, sigma_rotation_seed=3)
    assert np.abs(a["Mss"] - b["Mss"]).max() > 1e-3 * np.abs(a["Mss"]).max()
    assert np.abs(a["A"] - b["A"]).max() <= 1e-11 * np.abs(a["A"]).max()


def _kappa(n, steps=40):
    """Extreme eigenvalues of A-hat^d^{-1} A^d by Lanczos in the A^d inner
    product (the operator is self-adjoint there), with full
    reorthogonalisation (two passes) and a stop once the Krylov space is
    invariant to rounding (the multiplicative preconditioner has a large
    eigenvalue cluster at exactly 1); 40 steps resolve both ends for
    condition numbers near 10 (n = 2: 0.10764 / 1.0 against 0.10764 / 1.0
    from the dense spectrum)."""
    mesh, gs, _ = problem(n)
    pc = Preconditioner(gs, mesh.lattice)
    idx = np.arange(gs.off_f, gs.off_p)
    Ad = pc.Ad.tocsr()[idx][:, idx]

    def T(v):
        z = np.zeros(gs.n_dof)
        z[idx] = Ad @ v
        return pc.Ad_inv(z)[idx]

    rng = np.random.default_rng(1)
    q = rng.standard_normal(len(idx))
    q /= math.sqrt(q @ (Ad @ q))
    Q, al, be = [q], [], []
    for j in range(steps):
        w = T(Q[-1])
        a = w @ (Ad @ Q[-1])
        for _ in range(2):
            for qq in Q:
                w = w - (w @ (Ad @ qq)) * qq
        al.append(a)
        b = math.sqrt(max(w @ (Ad @ w), 0.0))
        if b < 1e-8 * abs(a):
            break
        be.append(b)
        Q.append(w / b)
    m = len(al)
    Tm = np.diag(al) + np.diag(be[:m - 1], 1) + np.diag(be[:m - 1], -1)
    lam = np.linalg.eigvalsh(Tm)
    return lam.min(), lam.max()


def test_preconditioner_robust_in_h():
    """The multiplicative auxiliary-space preconditioner with the facet blocks
    of six dofs and E u = (u, Pi^0 u_t, curl u): its eigenvalues on A^d lie in
    (0, 1] and the condition number moves by less than 25 % from n = 2 to 3
    (measured 9.3 -> 10.7; with the unweighted stabilisation nu (div omega,
    div eta) it is 77 -> 222)."""
    lo2, hi2 = _kappa(2)
    lo3, hi3 = _kappa(3)
    assert lo2 > 0 and lo3 > 0 and hi2 <= 1 + 1e-9 and hi3 <= 1 + 1e-9
    k2, k3 = hi2 / lo2, hi3 / lo3
    assert k2 < 15 and k3 < 1.25 * k2, (k2, k3)


def test_preconditioned_minres_matches_direct():
    mesh, gs, _ = problem(2)
    pc = Preconditioner(gs, mesh.lattice)
    K = gs.assemble_K()
    b = gs.assemble_rhs()
    x, info = minres(lambda v: K @ v, pc.apply, b, tol=1e-10, max_it=1000)
    xd = gs.direct_solve(b)
    x, xd = gs.normalize_pressure(x), gs.normalize_pressure(xd)
    assert info["converged"]
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)


def test_velocity_converges_in_h():
    """Manufactured flow, n = 2, 3, 4: the error falls at an order near the
    lowest-order method's first order in h (the paper prints no rates for
    Sec. 7, so a lower bound on the observed order is asserted; measured
    errors 0.95, 0.61, 0.40, orders 1.1 and 1.5)."""
    errs = []
    for n in (2, 3, 4):
        mesh, gs, sol = problem(n)
        x = gs.normalize_pressure(gs.direct_solve())
        eu = nu_ = 0.0
        for e in range(gs.n_e):
            Xe = gs.topo.element_coords(e)
            xq, lam, w = element_rule(Xe, 4)
            u, _ = gs.eval_element(x, e, lam)
            ue = sol.u(xq)
            eu += np.sum(w[:, None] * (u - ue) ** 2)
            nu_ += np.sum(w[:, None] * ue ** 2)
        errs.append(math.sqrt(eu / nu_))
    r1 = math.log(errs[0] / errs[1]) / math.log(1.5)
    r2 = math.log(errs[1] / errs[2]) / math.log(4 / 3)
    assert errs[2] < errs[1] < errs[0] and r1 > 0.9 and r2 > 1.2, (errs, r1, r2)


def test_stress_of_a_linear_flow():
    """Recovery at k = 1: for a linear velocity with its facet means as uhat
    and omega = curl u (conforming data), sigma_h = -nu dev eps(u) and
    kappa(omega_h) = kappa(curl u), the skew part of grad u."""
    from oracle.element import recover_stress
    from oracle.poly import evaluate
    X, ed = _element()
    rng = np.random.default_rng(8)
    G = rng.standard_normal((3, 3))
    curl = np.array([G[2, 1] - G[1, 2], G[0, 2] - G[2, 0], G[1, 0] - G[0, 1]])
    ul = _linear_field_dofs(X, ed, G, rng.standard_normal(3), curl)
    nu = 0.6
    S, W = recover_stress(ed, nu, 1, ul)
    lam = rng.dirichlet(np.ones(4), size=5)
    eps = 0.5 * (G + G.T)
    dev = eps - np.trace(eps) / 3 * np.eye(3)
    assert np.abs(evaluate(S, 4, 1, lam) - (-nu * dev)).max() <= 1e-10 * np.abs(G).max()
    assert np.abs(evaluate(W, 4, 1, lam) - 0.5 * (G - G.T)).max() <= 1e-10 * np.abs(G).max()


def test_stress_energy_identity():
    """For arbitrary element coefficients (u, uhat, omega): the condensed
    energy is nu^-1 ||sigma_h||^2 + nu/3 ||div u||^2 plus the stabilisation
    nu |T|^(2/3) ||div omega||^2."""
    from oracle.element import recover_stress, rt0_basis
    from oracle.poly import product_moments
    X, ed = _element()
    nu = 0.7
    es = element_system(ed, nu, 1)
    rng = np.random.default_rng(5)
    ul = rng.standard_normal(es["A"].shape[0])
    S, _ = recover_stress(ed, nu, 1, ul)
    Gm = product_moments(4, 1, 1) * ed.vol
    ss = np.einsum("ars,ab,brs->", S, Gm, S)
    cu = ul[: es["Adiv"].shape[0]]
    _, divrt = rt0_basis(ed)
    w = ul[-4:]
    stab = nu * ed.vol ** (2.0 / 3.0) * ed.vol * (divrt @ w) ** 2
    lhs = ul @ es["A"] @ ul
    assert abs(lhs - (ss / nu + cu @ es["Adiv"] @ cu + stab)) <= 1e-11 * abs(lhs)


def _outlet_flow(cells=(3, 2, 2), L=1.5, nu=0.9):
    """u = (c0 + c1 y + c2 z, a (x - L), b (x - L)), p = 0, f = 0: divergence
    free, u_t = 0 on x = L and eps(u)_nn = du_x/dx = 0 there, so the outlet
    condition of eq. stokes_NT holds with p = 0; Dirichlet data on the other
    five faces."""
    c0, c1, c2, a, b = 0.4, -0.7, 1.1, 0.6, -0.3

    def u(X):
        X = np.asarray(X, dtype=np.float64)
        return np.stack([c0 + c1 * X[..., 1] + c2 * X[..., 2], a * (X[..., 0] - L), b * (X[..., 0] - L)], axis=-1)

    mesh = W.box_mesh(cells, (L, 1.0, 1.0))
    pts = W.lattice_points(mesh, 2)
    fbc = [0, 1, 0, 0, 0, 0]
    gs = GlobalSystem(mesh.vertices, mesh.elements, nu, 1, np.zeros(pts.shape), face_bc=fbc, g_lattice=u(pts))
    return mesh, gs, u, fbc


def test_linear_flow_with_outlet_reproduced():
    """Patch test with an outlet (eq. stokes_NT): the outlet's tangential dofs
    are fixed to zero, its normal dofs and the omega flux are free (W_h
    vanishes on Gamma_D only, Sec. 7).  The linear flow and p = 0 are
    reproduced exactly; the omega flux through the outlet is that of curl u
    (zero: curl u = (0, c2 - b, a - c1) is tangential to x = L)."""
    mesh, gs, u, _ = _outlet_flow()
    assert gs.topo.has_outlet and gs.topo.facet_outlet.sum() == 2 * 2 * 2
    x = gs.direct_solve()
    lam = np.random.default_rng(4).dirichlet(np.ones(4), size=6)
    for e in range(gs.n_e):
        Xe = gs.topo.element_coords(e)
        ue, pe = gs.eval_element(x, e, lam)
        assert np.abs(ue - u(lam @ Xe)).max() < 1e-11
        assert np.abs(pe).max() < 1e-11
    for g in np.nonzero(gs.topo.free_outlet)[0]:
        dofs = gs.facet_dofs(g)
        assert np.all(x[dofs[gs.nF:gs.nF + gs.nh]] == 0)
        assert abs(x[dofs[gs.nF + gs.nh]]) < 1e-11


def test_outlet_omega_flux_is_free():
    """The omega flux of an outlet facet is an unknown of the system: its row
    of K couples to other dofs, while the tangential rows of the outlet are
    identity rows.  (An exact flow with u_t = 0 on x = L has curl u . n = 0
    there, so the patch test alone cannot tell a free flux from a fixed one.)"""
    mesh, gs, _, _ = _outlet_flow(cells=(2, 2, 2), L=1.0)
    K = gs.assemble_K().tocsr()
    for g in np.nonzero(gs.topo.free_outlet)[0]:
        dofs = gs.facet_dofs(g)
        w = dofs[gs.nF + gs.nh]
        row = K[w].toarray().ravel()
        row[w] = 0.0
        assert np.abs(row).max() > 0
        for q in dofs[gs.nF:gs.nF + gs.nh]:
            r = K[q].toarray().ravel()
            assert r[q] == 1.0 and np.count_nonzero(r) == 1


def test_outlet_preconditioned_minres_matches_direct():
    """Lemma outflow for the lowest order: with the tangential penalty in
    A-bar and pi_0 in E (the curl row kept on outlets), E^T A E is bounded by
    A-bar, and the preconditioned MINRES reaches the direct solution."""
    mesh, gs, _, _ = _outlet_flow(cells=(2, 2, 2), L=1.0, nu=1.0)
    sol = W.CurlModes3D(seed=5, nu=1.0)
    f = sol.f(W.lattice_points(mesh, 2))
    gs = GlobalSystem(mesh.vertices, mesh.elements, 1.0, 1, f, face_bc=[0, 1, 0, 0, 0, 0])
    pc = Preconditioner(gs, mesh.lattice)
    idx = np.arange(gs.off_f, gs.off_p)
    Ad = pc.Ad.toarray()[np.ix_(idx, idx)]
    E = pc.E.toarray()[idx]
    lam = np.linalg.eigvals(np.linalg.solve(pc.Abar.toarray(), E.T @ Ad @ E)).real
    assert lam.max() <= 1.02
    K = gs.assemble_K()
    b = gs.assemble_rhs()
    x, info = minres(lambda v: K @ v, pc.apply, b, tol=1e-10, max_it=1000)
    xd = gs.direct_solve(b)
    assert info["converged"]
    assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
