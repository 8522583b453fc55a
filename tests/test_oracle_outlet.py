"""Pins of the outlet boundary condition Gamma_NT and of inhomogeneous
Dirichlet data (eq. stokes_D, stokes_NT; Lemma outflow) in the oracle.

* Plane channel flow u = (4y(1-y), 0[, 0]), p = 4 nu (L - x) solves the Stokes
  problem with the profile as Dirichlet data on the inlet (and on z = 0, 1),
  no-slip plates and an outlet at x = L where u_t = 0 and the normal stress
  (sigma + p I) n . n = p vanishes.  u is quadratic and p linear, so they lie
  in the discrete spaces for k >= 2 and the discrete solution equals them.
* Outlet tangential dofs are kept in the vector layout with identity rows:
  the solution equals that of the system with those dofs removed.
* Lemma outflow: with the tangential penalty in A-bar and pi_0 in E, the
  auxiliary-space pieces stay bounded; the preconditioned MINRES converges.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
import oracle.precond as OP
from oracle.minres import minres
from oracle.system import GlobalSystem


def channel(d, cells, k, nu=0.7, L=1.0):
    mesh = W.box_mesh(cells, (L,) + (1.0,) * (d - 1))
    ch = W.PlaneChannel(d, nu=nu, L=L)
    pts = W.lattice_points(mesh, k + 1)
    gs = GlobalSystem(mesh.vertices, mesh.elements, nu, k, ch.f(pts), face_bc=ch.face_bc(), g_lattice=ch.u(pts))
    return mesh, ch, gs


@pytest.mark.parametrize("d,cells,k,L", [(2, (4, 2), 2, 2.0), (2, (3, 3), 3, 1.0), (3, (2, 2, 2), 2, 1.0)])
def test_plane_channel_is_reproduced_exactly(d, cells, k, L):
    mesh, ch, gs = channel(d, cells, k, L=L)
    assert gs.topo.has_outlet and gs.topo.facet_outlet.sum() == (2 if d == 3 else 1) * np.prod(cells[1:])
    x = gs.direct_solve()
    lam = np.random.default_rng(0).dirichlet(np.ones(d + 1), size=5)
    for e in range(gs.n_e):
        u, p = gs.eval_element(x, e, lam)
        X = lam @ gs.elems[e]["ed"].X
        assert np.abs(u - ch.u(X)).max() <= 1e-11
        assert np.abs(p - ch.p(X)).max() <= 1e-11 * 4 * ch.nu * L


def test_outlet_tangential_dofs_decouple():
    """Identity rows for the fixed tangential outlet dofs give the solution of
    the system without them (and zero in those slots)."""
    mesh, ch, gs = channel(2, (3, 2), 2)
    K = gs.assemble_K().tocsr()
    b = gs.assemble_rhs()
    pinned = []
    for g in np.nonzero(gs.topo.free_outlet)[0]:
        pinned += list(gs.facet_dofs(g)[gs.nF:])
    keep = np.setdiff1d(np.arange(gs.n_dof), pinned)
    assert np.all(b[pinned] == 0)
    xr = spla.splu(K[keep][:, keep].tocsc()).solve(b[keep])
    x = gs.direct_solve()
    assert np.all(np.abs(x[pinned]) <= 1e-14)
    assert np.allclose(x[keep], xr, rtol=0, atol=1e-12 * np.abs(xr).max())


@pytest.mark.parametrize("d,cells,k,dense", [(2, (4, 4), 2, True), (3, (2, 2, 2), 2, False)])
def test_outlet_auxiliary_space_bounds(d, cells, k, dense):
    """Lemma outflow: E^d^T A^d E^d is bounded by A-bar with the penalty; with
    the chosen constant the bound holds to within 2 % (the excess decays like
    1/C), the multiplicative preconditioner stays symmetric with eigenvalues
    of A-hat^d_m^{-1} A^d in (0, 1.05], and MINRES reaches the direct solution."""
    mesh, ch, gs = channel(d, cells, k, nu=1.0)
    pc = OP.Preconditioner(gs, mesh.lattice)
    idx = np.arange(gs.off_f, gs.off_p)
    Ad = pc.Ad.toarray()[np.ix_(idx, idx)]
    E = pc.E.toarray()[idx]
    lam = np.linalg.eigvals(np.linalg.solve(pc.Abar.toarray(), E.T @ Ad @ E)).real
    assert 0.99 <= lam.max() <= 1.02
    if dense:
        P = np.zeros((len(idx), len(idx)))
        for j, g in enumerate(idx):
            v = np.zeros(gs.n_dof)
            v[g] = 1.0
            P[:, j] = pc.Ad_mult_inv(v)[idx]
        assert np.allclose(P, P.T, atol=1e-10 * np.abs(P).max())
        mu = np.linalg.eigvals(P @ Ad).real
        assert mu.min() > 1e-8 and mu.max() <= 1.05
    K = gs.assemble_K()
    x, info = minres(lambda v: K @ v, pc.apply, gs.assemble_rhs(), tol=1e-10, max_it=2000)
    xd = gs.direct_solve()
    assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_outlet_penalty_excess_decays():
    """The excess of E^d^T A^d E^d over A-bar decays as the penalty grows."""
    mesh, ch, gs = channel(2, (4, 4), 2, nu=1.0)
    idx = np.arange(gs.off_f, gs.off_p)
    ex = []
    C0 = OP.OUTLET_PENALTY
    try:
        for C in (2.0, 8.0):
            OP.OUTLET_PENALTY = C
            pc = OP.Preconditioner(gs, mesh.lattice)
            Ad = pc.Ad.toarray()[np.ix_(idx, idx)]
            E = pc.E.toarray()[idx]
            ex.append(np.linalg.eigvals(np.linalg.solve(pc.Abar.toarray(), E.T @ Ad @ E)).real.max() - 1.0)
    finally:
        OP.OUTLET_PENALTY = C0
    assert ex[1] < 0.5 * ex[0], ex
