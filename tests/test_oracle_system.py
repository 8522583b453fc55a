"""Pins of the oracle's global system, preconditioner and MINRES against the
identities, bounds and special cases of Secs. 4-6, brute force and closed forms."""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle.element import expected_dims
from oracle.minres import minres
from oracle.poly import evaluate
from oracle.precond import Preconditioner, embedding, assemble_p1, P1Multigrid
from oracle.system import GlobalSystem
from tests.quadrature import element_rule

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
_cache = {}


def problem(d, n, k, nu=1.0, force=None, coarse_max=512):
    key = (d, n, k, nu, force, coarse_max)
    if key in _cache:
        return _cache[key]
    mesh = W.unit_square_mesh(n) if d == 2 else W.unit_cube_mesh(n)
    m = k + 1
    pts = W.lattice_points(mesh, m)
    if force == "grad":
        f = np.zeros_like(pts)
        f[..., 0] = 1.0                       # f = grad(x - 1/2)
        sol = None
    else:
        sol = W.Manufactured2D(nu) if d == 2 else W.CurlModes3D(seed=2, nu=nu)
        f = sol.f(pts)
    gs = GlobalSystem(mesh.vertices, mesh.elements, nu, k, f)
    out = (mesh, gs, sol)
    _cache[key] = out
    return out


def test_paper_dofs_per_tet():
    """#D/|T| printed in tab::ST_ws / tab::plane approaches 2 n_fb + n_bub + n_p."""
    with open(os.path.join(GOLDEN, "paper_dofs_per_tet.json")) as fh:
        rows = json.load(fh)["rows"]
    for r in rows:
        dims = expected_dims(3, r["k"])
        per_tet = 2 * dims["n_fb"] + dims["n_bub"] + dims["n_p"]
        assert abs(r["D"] / r["tets"] - per_tet) / per_tet < 0.01


def _monolithic(gs):
    """Assemble the full (sigma, omega, u, uhat, p) system of eq. bigfemSPmat."""
    import scipy.sparse as sp
    blocks = []
    n_s = gs.elems[0]["Z"].shape[1]
    n_w = gs.elems[0]["Bws"].shape[0]
    nloc = n_s + n_w
    off = gs.n_dof
    N = off + gs.n_e * nloc
    rows, cols, vals = [], [], []

    def add(R, C, M):
        R = np.asarray(R); C = np.asarray(C)
        mr, mc = R >= 0, C >= 0
        RR, CC = np.meshgrid(R[mr], C[mc], indexing="ij")
        rows.append(RR.ravel()); cols.append(CC.ravel()); vals.append(M[np.ix_(mr, mc)].ravel())

    for e, es in enumerate(gs.elems):
        sw = np.arange(off + e * nloc, off + (e + 1) * nloc)
        Mloc = np.block([[-es["Mss"], es["Bws"].T], [es["Bws"], np.zeros((n_w, n_w))]])
        add(sw, sw, Mloc)
        ld = gs.local_dofs(e)
        perm = es["perm"]
        Bs = es["Bsig"][perm]                                    # reordered velocity rows
        Bs_full = np.hstack([Bs, np.zeros((Bs.shape[0], n_w))])
        add(ld, sw, Bs_full)
        add(sw, ld, Bs_full.T)
        Adx = np.zeros((len(ld), len(ld)))
        inv = gs.u_to_reordered(e)
        Adx[np.ix_(inv, inv)] = es["Adiv"]
        add(ld, ld, Adx)
        pd = gs.pressure_dofs(e)
        Bl = np.zeros((gs.np_, len(ld)))
        Bl[:, inv] = es["B"]
        add(pd, ld, Bl)
        add(ld, pd, Bl.T)
    Kfull = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(N, N))
    return Kfull, N


@pytest.mark.parametrize("d,n,k", [(2, 2, 2), (2, 2, 3), (3, 1, 2)])
def test_monolithic_equals_condensed(d, n, k):
    """Static condensation is exact (Sec. 4.2): the dense solve of the full
    (sigma, omega, u, uhat, p) system equals the condensed solve."""
    mesh = W.unit_square_mesh(n) if d == 2 else W.unit_cube_mesh(n)
    sol = W.Manufactured2D() if d == 2 else W.CurlModes3D(seed=2)
    f = sol.f(W.lattice_points(mesh, k + 1))
    gs = GlobalSystem(mesh.vertices, mesh.elements, 1.0, k, f)
    # rebuild elements keeping the sigma blocks
    from oracle.element import element_system
    lat = np.asarray(W.lattice_indices(d, k + 1))
    for e in range(gs.n_e):
        gs.elems[e] = element_system(gs.elems[e]["ed"], 1.0, k, f[e], lat[:, gs.topo.perm[e]],
                                     k + 1, keep_blocks=True)
    xc = gs.direct_solve()
    Kfull, N = _monolithic(gs)
    b = np.zeros(N)
    b[:gs.n_dof] = gs.assemble_rhs()
    c = np.zeros(N)
    c[:gs.n_dof] = gs.pressure_mean_functional()
    Kd = np.block([[Kfull.toarray(), c[:, None]], [c[None, :], np.zeros((1, 1))]])
    xf = np.linalg.solve(Kd, np.concatenate([b, [0.0]]))[:gs.n_dof]
    assert np.linalg.norm(xf - xc) < 1e-11 * np.linalg.norm(xc)


def _l2_errors(gs, x, sol):
    eu = nu_ = ep = npn = 0.0
    for e in range(gs.n_e):
        X = gs.topo.element_coords(e)
        xq, lam, w = element_rule(X, gs.k + 3)
        u, p = gs.eval_element(x, e, lam)
        ue = sol.u(xq)
        pe = sol.p(xq)
        eu += np.sum(w[:, None] * (u - ue) ** 2)
        nu_ += np.sum(w[:, None] * ue ** 2)
        ep += np.sum(w * (p - pe) ** 2)
        npn += np.sum(w * pe ** 2)
    return math.sqrt(eu / nu_), math.sqrt(ep / npn)


@pytest.mark.parametrize("k", [2, 3])
def test_convergence_rates_2d(k):
    """Manufactured-solution convergence in h: the orders of the method for
    smooth data (the paper prints no rates; conservative lower bounds below
    the expected orders are asserted)."""
    errs = []
    for n in (2, 4, 8):
        mesh, gs, sol = problem(2, n, k)
        x = gs.normalize_pressure(gs.direct_solve())
        errs.append(_l2_errors(gs, x, sol))
    errs = np.asarray(errs)
    ru = np.log2(errs[:-1, 0] / errs[1:, 0])
    rp = np.log2(errs[:-1, 1] / errs[1:, 1])
    assert ru[-1] >= k - 0.2, (errs, ru)
    assert rp[-1] >= k - 0.6, (errs, rp)


def test_convergence_rates_3d():
    """3D manufactured flow (a sum of curl modes, p linear), k = 2 on n = 2,
    3, 4 (the paper prints no rates; measured
    velocity orders 2.06, 2.25 and pressure orders 1.82, 2.38, still rising
    towards the asymptotic ones, so the 2D bounds are asserted on the last
    pair), and the error falls from k = 2 to k = 3 at n = 2 (0.69 -> 0.37)."""
    errs = []
    for n in (2, 3, 4):
        mesh, gs, sol = problem(3, n, 2)
        errs.append(_l2_errors(gs, gs.normalize_pressure(gs.direct_solve()), sol))
    errs = np.asarray(errs)
    h = 1.0 / np.array([2.0, 3.0, 4.0])
    ru = np.log(errs[:-1, 0] / errs[1:, 0]) / np.log(h[:-1] / h[1:])
    rp = np.log(errs[:-1, 1] / errs[1:, 1]) / np.log(h[:-1] / h[1:])
    assert ru[-1] >= 2 - 0.2 and ru[-1] > ru[0], (errs, ru)
    assert rp[-1] >= 2 - 0.6, (errs, rp)
    mesh, gs3, sol = problem(3, 2, 3)
    e3 = _l2_errors(gs3, gs3.normalize_pressure(gs3.direct_solve()), sol)[0]
    assert e3 < 0.7 * errs[0, 0], (e3, errs[0, 0])


def test_convergence_in_k_2d():
    """Error decreases monotonically in k for smooth data (n = 4)."""
    e = [_l2_errors(problem(2, 4, k)[1], problem(2, 4, k)[1].normalize_pressure(
        problem(2, 4, k)[1].direct_solve()), problem(2, 4, k)[2])[0] for k in (2, 3, 4)]
    assert e[0] > e[1] > e[2]


@pytest.mark.parametrize("d,n,k", [(2, 4, 2), (2, 2, 3), (3, 1, 3)])
def test_exactly_divergence_free(d, n, k):
    """div V_h = Q_h (Sec. 4.1): B u = 0 and div u_h = 0 pointwise to round-off."""
    mesh, gs, sol = problem(d, n, k)
    x = gs.direct_solve()
    from oracle.poly import gradient_matrices
    unorm = np.abs(x[:gs.off_p]).max()
    for e in range(gs.n_e):
        es = gs.elems[e]
        ed = es["ed"]
        ld = gs.local_dofs(e)
        coef = np.where(ld >= 0, x[np.maximum(ld, 0)], 0.0)
        orig = np.zeros(len(coef))
        orig[es["perm"]] = coef
        cu = orig[:gs.dims["n_u"]]
        Dk = gradient_matrices(d + 1, k, ed.grad_lambda)
        divc = np.einsum("sab,ibs->ia", Dk, ed.Phi).T @ cu
        assert np.abs(divc).max() < 1e-9 * unorm / ed.vol ** (1.0 / d)


@pytest.mark.parametrize("d,n,k", [(2, 4, 2), (3, 1, 2)])
def test_pressure_robustness(d, n, k):
    """f = grad(phi), phi = x - 1/2 in Q_h: u_h = 0 and p_h = phi exactly
    (pressure robustness, Sec. 1 and Sec. 4.1)."""
    mesh, gs, _ = problem(d, n, k, force="grad")
    x = gs.normalize_pressure(gs.direct_solve())
    assert np.abs(x[:gs.off_p]).max() < 1e-11
    for e in range(gs.n_e):
        X = gs.topo.element_coords(e)
        xq, lam, w = element_rule(X, 3)
        _, p = gs.eval_element(x, e, lam)
        assert np.allclose(p, xq[:, 0] - 0.5, atol=1e-11)


def test_nu_scaling_invariance():
    """Constant nu -> c nu: u_h -> u_h / c, p_h unchanged, identical MINRES
    iteration counts (the preconditioner scales with nu)."""
    mesh = W.unit_square_mesh(4)
    f = W.Manufactured2D().f(W.lattice_points(mesh, 3))
    res = []
    for nu in (1.0, 1e-3):
        gs = GlobalSystem(mesh.vertices, mesh.elements, nu, 2, f)
        pc = Preconditioner(gs, mesh.lattice)
        K = gs.assemble_K()
        b = gs.assemble_rhs()
        x, info = minres(lambda v: K @ v, pc.apply, b, tol=1e-10, max_it=300)
        res.append((gs, gs.normalize_pressure(x), info["iterations"]))
    (g1, x1, i1), (g2, x2, i2) = res
    assert abs(i1 - i2) <= 1
    assert np.allclose(x2[:g2.off_p] * 1e-3, x1[:g1.off_p], rtol=1e-6, atol=1e-9 * np.abs(x1).max())
    assert np.allclose(x2[g2.off_p:], x1[g1.off_p:], atol=1e-7 * np.abs(x1[g1.off_p:]).max())


@pytest.mark.parametrize("d,n,k", [(2, 2, 2), (2, 2, 3), (3, 2, 2)])
def test_embedding_energy_identity(d, n, k):
    """Corollary embed: ||E u||_A = ||u||_{A-bar} for continuous P1 u, i.e.
    E^T A E = A-bar with A-bar = nu int eps : eps (settles the nu vs nu^{-1}
    reading of eq. defAhat); and Corollary embed_schur: E^d^T A^d E^d <= A-bar."""
    mesh, gs, _ = problem(d, n, k)
    K = gs.assemble_K()
    A = K[:gs.off_p, :gs.off_p].toarray()
    E = embedding(gs, full=True).toarray()[:gs.off_p]
    Abar = assemble_p1(gs).toarray()
    assert np.allclose(E.T @ A @ E, Abar, atol=1e-10 * np.abs(Abar).max())
    pc = Preconditioner(gs, mesh.lattice)
    Ed = pc.E.toarray()[gs.off_f:gs.off_p]
    Ad = pc.Ad.toarray()[gs.off_f:gs.off_p, gs.off_f:gs.off_p]
    w = np.linalg.eigvalsh(Abar - Ed.T @ Ad @ Ed)
    assert w.min() > -1e-10 * np.abs(Abar).max()


def test_embedding_rows_agree_between_neighbours():
    """The facet rows of E^d do not depend on which neighbour computes them."""
    from oracle.precond import p1_in_element_basis
    mesh, gs, _ = problem(3, 1, 2)
    topo = gs.topo
    nb, nF, nh = gs.nb, gs.nF, gs.nh
    for f in topo.free_facets:
        rows = []
        for (t, i) in topo.facet_neighbors[f]:
            es = gs.elems[t]
            R = []
            for v in topo.facet_vertices[f]:
                vl = int(np.nonzero(topo.elements[t] == v)[0][0])
                for c in range(3):
                    cu, ch = p1_in_element_basis(es, vl, c)
                    R.append(np.concatenate([cu[nb + i * nF: nb + (i + 1) * nF], ch[i]]))
            rows.append(np.asarray(R))
        assert np.allclose(rows[0], rows[1], atol=1e-10)


def test_multigrid_is_spd_and_dominates():
    """The V(1,1) cycle C is symmetric and A-bar <= C (eigenvalues of
    C^{-1} A-bar in (0, 1]), as Corollary aux_pc_mult requires."""
    mesh = W.unit_cube_mesh(4)
    gs = GlobalSystem(mesh.vertices, mesh.elements, W.lognormal_nu(mesh.n_elements, 4), 2)
    Abar = assemble_p1(gs)
    mg = P1Multigrid(Abar, mesh.lattice, 3, coarse_max=10)
    assert len(mg.levels) >= 2
    n = Abar.shape[0]
    Cinv = np.stack([mg.vcycle(np.eye(n)[j]) for j in range(n)], 1)
    assert np.allclose(Cinv, Cinv.T, atol=1e-12 * np.abs(Cinv).max())
    lam = sla.eigh(Abar.toarray(), np.linalg.inv(Cinv), eigvals_only=True)
    assert lam.min() > 0 and lam.max() <= 1 + 1e-10


def _dense_op(fun, n, idx):
    M = np.zeros((len(idx), len(idx)))
    for j, g in enumerate(idx):
        v = np.zeros(n)
        v[g] = 1.0
        M[:, j] = fun(v)[idx]
    return M


@pytest.mark.parametrize("d,n,k,cm", [(2, 4, 2, 20), (3, 2, 2, 512)])
def test_aux_space_preconditioner_bounds(d, n, k, cm):
    """Corollary aux_pc_mult: A^d <= A-hat^d_m, i.e. the eigenvalues of
    A-hat^d_m^{-1} A^d lie in (0, 1]; A-hat^d_m^{-1} is symmetric."""
    mesh, gs, _ = problem(d, n, k)
    pc = Preconditioner(gs, mesh.lattice, coarse_max=cm)
    idx = np.arange(gs.off_f, gs.off_p)
    P = _dense_op(pc.Ad_mult_inv, gs.n_dof, idx)
    assert np.allclose(P, P.T, atol=1e-10 * np.abs(P).max())
    Ad = pc.Ad.toarray()[np.ix_(idx, idx)]
    lam = np.linalg.eigvals(P @ Ad).real
    assert lam.min() > 1e-8 and lam.max() <= 1 + 1e-9
    # the block-GS part alone also never over-corrects
    assert np.linalg.cond(P @ Ad) < 1e4


def test_khat_is_spd():
    mesh, gs, _ = problem(2, 2, 2)
    pc = Preconditioner(gs, mesh.lattice)
    idx = np.arange(gs.n_dof)
    P = _dense_op(pc.apply, gs.n_dof, idx)
    assert np.allclose(P, P.T, atol=1e-10 * np.abs(P).max())
    assert np.linalg.eigvalsh(0.5 * (P + P.T)).min() > 0


def test_exact_blocks_give_three_iterations():
    """Special case of eq. Kfactor: with A-hat = A and S-hat = S_p (regular on
    the complement of constants), K-hat^{-1} K has eigenvalues +-1 and MINRES
    converges in at most 3 iterations."""
    mesh, gs, _ = problem(2, 2, 2)
    K = gs.assemble_K().toarray()
    b = gs.assemble_rhs()
    A = K[:gs.off_p, :gs.off_p]
    B = K[gs.off_p:, :gs.off_p]
    Ainv = np.linalg.inv(A)
    S = B @ Ainv @ B.T
    c1 = gs.constant_pressure()[gs.off_p:]
    Sreg = S + np.outer(c1, c1) / (c1 @ c1)
    Sinv = np.linalg.inv(Sreg)

    def Minv(r):
        a = Ainv @ r[:gs.off_p]
        yp = Sinv @ (r[gs.off_p:] - B @ a)
        yu = a - Ainv @ (B.T @ yp)
        return np.concatenate([yu, yp])

    x, info = minres(lambda v: K @ v, Minv, b, tol=1e-12, max_it=20)
    assert info["iterations"] <= 3
    xd = gs.direct_solve()
    assert np.linalg.norm(gs.normalize_pressure(x) - xd) < 1e-9 * np.linalg.norm(xd)


def test_minres_textbook():
    """MINRES on a random symmetric indefinite system with an SPD
    preconditioner matches a dense solve."""
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.concatenate([rng.uniform(1, 10, 40), -rng.uniform(1, 10, 20)])
    K = Q @ np.diag(lam) @ Q.T
    D = np.diag(rng.uniform(0.5, 2.0, 60))
    b = rng.standard_normal(60)
    x, info = minres(lambda v: K @ v, lambda r: np.linalg.solve(D, r), b, tol=1e-12, max_it=200)
    assert info["converged"]
    assert np.allclose(x, np.linalg.solve(K, b), rtol=1e-9, atol=1e-10)
    # monotone decrease of the preconditioned residual estimate
    h = np.asarray(info["history"])
    assert np.all(np.diff(h) <= 1e-14)


@pytest.mark.parametrize("d,n,k", [(2, 4, 2), (3, 1, 2)])
def test_preconditioned_minres_matches_direct(d, n, k):
    mesh, gs, _ = problem(d, n, k)
    pc = Preconditioner(gs, mesh.lattice)
    K = gs.assemble_K()
    b = gs.assemble_rhs()
    x, info = minres(lambda v: K @ v, pc.apply, b, tol=1e-12, max_it=500)
    assert info["converged"]
    xd = gs.direct_solve()
    assert np.linalg.norm(gs.normalize_pressure(x) - xd) < 1e-9 * np.linalg.norm(xd)


@pytest.mark.parametrize("d,n,k,cm", [(2, 4, 2, 20), (3, 2, 2, 512)])
def test_additive_asp_bounds(d, n, k, cm):
    """Additive variant (Sec. 5.2, Theorem aux_pc_schur) with the facet block
    Jacobi D.  Facets of one colour share no element, so A^d restricted to a
    colour is block diagonal and Cauchy-Schwarz over the colours gives
    A^d <= n_colours D: the eigenvalues of D^{-1} A^d lie in (0, n_colours] and
    those of (D^{-1} + E^d C^{-1} E^d^T) A^d in (0, n_colours + 1] (the coarse
    term adds at most 1 since E^d^T A^d E^d <= A-bar <= C).  The diagonal blocks
    of D^{-1} A^d are identities."""
    mesh, gs, _ = problem(d, n, k)
    pc = Preconditioner(gs, mesh.lattice, coarse_max=cm, variant="additive")
    nc = gs.topo.n_colours
    idx = np.arange(gs.off_f, gs.off_p)
    Ad = pc.Ad.toarray()[np.ix_(idx, idx)]
    Dinv = _dense_op(pc.block_jacobi, gs.n_dof, idx)
    DA = Dinv @ Ad
    for g in range(gs.topo.n_free_facets):
        fd = gs.facet_dofs(g) - gs.off_f
        assert np.allclose(DA[np.ix_(fd, fd)], np.eye(len(fd)), atol=1e-9)
    lam_s = np.linalg.eigvals(DA).real
    assert lam_s.min() > 0 and lam_s.max() <= nc + 1e-9
    P = _dense_op(pc.Ad_add_inv, gs.n_dof, idx)
    assert np.allclose(P, P.T, atol=1e-10 * np.abs(P).max())
    lam = np.linalg.eigvals(P @ Ad).real
    assert lam.min() > 1e-8 and lam.max() <= nc + 1 + 1e-9


def test_additive_asp_mesh_independent():
    """Theorem aux_pc_schur bounds the condition number of the additive
    preconditioner independently of h: halving h (2D, k=2, n = 4 -> 8) leaves
    the spectral condition number of A-hat^d_a^{-1} A^d within 25%."""
    kap = []
    for n in (4, 8):
        mesh, gs, _ = problem(2, n, 2)
        pc = Preconditioner(gs, mesh.lattice, variant="additive")
        idx = np.arange(gs.off_f, gs.off_p)
        Ad = pc.Ad.toarray()[np.ix_(idx, idx)]
        lam = np.sort(np.linalg.eigvals(_dense_op(pc.Ad_add_inv, gs.n_dof, idx) @ Ad).real)
        kap.append(lam[-1] / lam[0])
    assert kap[1] <= 1.25 * kap[0], kap


def test_additive_needs_more_iterations_than_multiplicative():
    """The paper's smoothing comparison (Table ST_smoothing): the multiplicative
    auxiliary-space preconditioner needs fewer MINRES iterations than the
    additive one with an l1 block smoother; both reach the direct solution."""
    mesh, gs, _ = problem(3, 2, 2)
    K = gs.assemble_K()
    b = gs.assemble_rhs()
    xd = gs.direct_solve()
    its = {}
    for variant in ("multiplicative", "additive"):
        pc = Preconditioner(gs, mesh.lattice, variant=variant)
        x, info = minres(lambda v: K @ v, pc.apply, b, tol=1e-10, max_it=2000)
        x = gs.normalize_pressure(x)
        assert np.linalg.norm(x - xd) <= 1e-7 * np.linalg.norm(xd)
        its[variant] = info["iterations"]
    assert its["multiplicative"] < its["additive"], its


@pytest.mark.parametrize("d,n,k,cm", [(2, 4, 2, 20), (3, 2, 2, 512)])
def test_full_system_asp_bounds(d, n, k, cm):
    """Full-system variant (Theorem aux_pc with the Gauss-Seidel smoother of
    Corollary aux_pc_mult): blocks of one colour share no element, so their
    coupling in A vanishes and a colour phase is exact; the symmetric
    multiplicative preconditioner satisfies A <= A-hat (eigenvalues of
    A-hat^{-1} A in (0, 1], using E^T A E = A-bar <= C with the full
    embedding)."""
    mesh, gs, _ = problem(d, n, k)
    pc = Preconditioner(gs, mesh.lattice, coarse_max=cm, variant="full")
    A = pc.Afull.toarray()
    for lst in pc.full_colour_lists:
        for i, f in enumerate(lst):
            for g in lst[i + 1:]:
                assert not np.any(A[np.ix_(pc.blocks[f], pc.blocks[g])]), (f, g)
    # every velocity dof lies in some block (bubbles in d+1 overlapping ones)
    cover = np.zeros(gs.off_p, dtype=int)
    for B in pc.blocks:
        cover[B] += 1
    assert cover[:gs.off_f].min() == d + 1 and cover[gs.off_f:].min() == 1
    idx = np.arange(gs.off_p)
    P = pc.A_full_inv(np.eye(gs.n_dof)[:, idx])[idx]
    assert np.allclose(P, P.T, atol=1e-10 * np.abs(P).max())
    lam = np.linalg.eigvals(P @ A).real
    assert lam.min() > 1e-8 and lam.max() <= 1 + 1e-9


def test_full_system_asp_columns_match_vectors():
    """The matrix form of A_full_inv (several right-hand sides at once, used
    to form dense operators) equals column-by-column application."""
    mesh, gs, _ = problem(2, 4, 2)
    pc = Preconditioner(gs, mesh.lattice, variant="full")
    R = np.random.default_rng(1).standard_normal((gs.n_dof, 3))
    Y = pc.A_full_inv(R)
    for j in range(3):
        assert np.allclose(Y[:, j], pc.A_full_inv(R[:, j].copy()), rtol=1e-12, atol=1e-12 * np.abs(Y).max())


def test_full_system_asp_mesh_independent():
    """Theorem aux_pc: the condition number of the full-system preconditioner
    does not grow with 1/h (2D, k = 2, n = 4 -> 8: within 25%)."""
    kap = []
    for n in (4, 8):
        mesh, gs, _ = problem(2, n, 2)
        pc = Preconditioner(gs, mesh.lattice, variant="full")
        idx = np.arange(gs.off_p)
        P = pc.A_full_inv(np.eye(gs.n_dof)[:, idx])[idx]
        lam = np.sort(np.linalg.eigvals(P @ pc.Afull.toarray()).real)
        kap.append(lam[-1] / lam[0])
    assert kap[1] <= 1.25 * kap[0], kap


def test_full_system_asp_solves():
    """MINRES with the full-system variant reaches the direct solution."""
    mesh, gs, _ = problem(3, 2, 2)
    K = gs.assemble_K()
    pc = Preconditioner(gs, mesh.lattice, variant="full")
    x, info = minres(lambda v: K @ v, pc.apply, gs.assemble_rhs(), tol=1e-10, max_it=2000)
    xd = gs.direct_solve()
    assert np.linalg.norm(gs.normalize_pressure(x) - xd) <= 1e-7 * np.linalg.norm(xd)
    assert info["iterations"] < 200
