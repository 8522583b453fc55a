"""GPU parity of the lowest-order method, k = 1 in 3D (Sec. 7): the HIP path
through the C ABI against the FP64 oracle (tests/test_oracle_lowest_order.py
pins the oracle).

Element operators (omega's facet fluxes in the condensed block A^d, the
stabilisation, no bubbles) to 1e-10 relative; every operator of mcs_apply and
mcs_precond_apply to 1e-12 (1e-11 with the V-cycle); FP64 MINRES iterations
within +-1 of the oracle's at tol 1e-10 and, after two thirds of the
oracle's iteration count on both sides, the equal-iteration bar of
tests/minres_parity.py; the mixed-precision solve to 1e-8 of the direct solve.
Cases: n = 1, 2 (one multigrid level), and n = 4 with coarse_max 20 (two
levels)."""
import numpy as np
import pytest

import workloads as W
from tests.minres_parity import check_equal_iterations, check_iterations, oracle_twin
from tests.test_gpu_parity import _l2_rel, _rel, setup_case

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n,nu_kind", [(1, "one"), (2, "one"), (2, "lognormal")])
def test_lowest_order_element_operators(n, nu_kind):
    c = setup_case(3, n, 1, nu_kind)
    pb, gs = c["pb"], c["gs"]
    nd = gs.dims["n_d"]
    assert pb.info.n_bub == 0 and pb.info.n_fb == 6
    Ad = pb.get_array("Ad").cpu().numpy().reshape(-1, nd, nd)
    for e, es in enumerate(gs.elems):
        assert np.abs(Ad[e] - es["Ad"]).max() < 1e-10 * np.abs(es["Ad"]).max(), e


@pytest.mark.parametrize("n,nu_kind", [(2, "one"), (2, "lognormal")])
def test_lowest_order_load_and_applies(n, nu_kind):
    # (on one cube, n = 1, the curl modes' load is rounding noise, ~1e-14)
    c = setup_case(3, n, 1, nu_kind)
    pb, gs, K = c["pb"], c["gs"], c["K"]
    b = pb.load(torch.as_tensor(c["f"], device="cuda:0")).cpu().numpy()
    assert _rel(b, gs.assemble_rhs()) < 1e-12
    x = np.random.default_rng(7).standard_normal(gs.n_dof)
    xt = torch.as_tensor(x, device="cuda:0")
    assert _rel(pb.apply("K", xt).cpu().numpy(), K @ x) < 1e-12
    u = x.copy()
    u[gs.off_p:] = 0
    yA = pb.apply("A", xt).cpu().numpy()
    assert _rel(yA[:gs.off_p], (K @ u)[:gs.off_p]) < 1e-12
    yAd = pb.apply("ADELTA", xt).cpu().numpy()
    assert _rel(yAd[gs.off_f:gs.off_p], (c["pc"].Ad @ x)[gs.off_f:gs.off_p]) < 1e-12
    yB = pb.apply("B", xt).cpu().numpy()
    assert _rel(yB[gs.off_p:], (K @ u)[gs.off_p:]) < 1e-12
    p = np.zeros_like(x)
    p[gs.off_p:] = x[gs.off_p:]
    assert _rel(pb.apply("BT", xt).cpu().numpy()[:gs.off_p], (K @ p)[:gs.off_p]) < 1e-12
    assert _rel(pb.apply("K", xt.float()).double().cpu().numpy(), K @ x) < 1e-5


@pytest.mark.parametrize("n,cm,levels", [(2, 512, 1), (4, 20, 2)])
def test_lowest_order_preconditioner_pieces(n, cm, levels):
    """Sweeps over facet blocks of six dofs, E^d with its curl rows and the
    facet means of u_t, the V-cycle, A-hat^d, A-hat_ext (= A-hat^d: no
    bubbles) and K-hat."""
    c = setup_case(3, n, 1, coarse_max=cm)
    pb, gs, pc = c["pb"], c["gs"], c["pc"]
    assert pb.info.n_mg_levels == levels == len(pc.mg.levels)
    rng = np.random.default_rng(11)
    r = rng.standard_normal(gs.n_dof)
    rt = torch.as_tensor(r, device="cuda:0")
    fd = slice(gs.off_f, gs.off_p)
    xf = np.zeros(gs.n_dof)
    for _ in range(pc.steps):
        xf = pc.forward_sweep(xf, r)
    assert _rel(pb.precond_apply("SMOOTH_FWD", rt).cpu().numpy()[fd], xf[fd]) < 1e-12
    xb = np.zeros(gs.n_dof)
    for _ in range(pc.steps):
        xb = pc.backward_sweep(xb, r)
    assert _rel(pb.precond_apply("SMOOTH_BWD", rt).cpu().numpy()[fd], xb[fd]) < 1e-12
    rr = r.copy()
    rr[:gs.off_f] = 0
    rr[gs.off_p:] = 0
    q = rng.standard_normal(pb.info.n_p1_dofs)
    qt = torch.as_tensor(q, device="cuda:0")
    assert _rel(pb.precond_apply("EDELTA", qt).cpu().numpy()[fd], (pc.E @ q)[fd]) < 1e-12
    assert _rel(pb.precond_apply("EDELTA_T", rt).cpu().numpy(), pc.E.T @ rr) < 1e-12
    assert _rel(pb.precond_apply("MG", qt).cpu().numpy(), pc.mg.vcycle(q)) < 1e-11
    assert _rel(pb.precond_apply("AUX", rt).cpu().numpy()[fd], pc.aux_correction(rr)[fd]) < 1e-11
    assert _rel(pb.precond_apply("ADELTA_MULT", rt).cpu().numpy()[fd], pc.Ad_mult_inv(rr)[fd]) < 1e-11
    ru = r.copy()
    ru[gs.off_p:] = 0
    assert _rel(pb.precond_apply("AEXT", rt).cpu().numpy()[:gs.off_p], pc.A_ext_inv(ru)[:gs.off_p]) < 1e-11
    ref = pc.apply(r.copy())
    assert _rel(pb.precond_apply("KHAT", rt).cpu().numpy(), ref) < 1e-11
    assert _rel(pb.precond_apply("KHAT", rt.float()).double().cpu().numpy(), ref) < 1e-4


def _oracle_minres(c, tol=1e-10):
    if "minres" not in c:
        from oracle.minres import minres
        gs = c["gs"]
        xo, info = minres(lambda v: c["K"] @ v, c["pc"].apply, gs.assemble_rhs(), tol=tol, max_it=3000)
        c["minres"] = (gs.normalize_pressure(xo), info["iterations"])
    return c["minres"]


@pytest.mark.parametrize("n,nu_kind,cm", [(2, "one", 512), (2, "lognormal", 512), (4, "one", 20)])
def test_lowest_order_solve_fp64(n, nu_kind, cm):
    """FP64 MINRES: iterations within +-1 of the oracle's (or of its twins'
    range) at tol 1e-10, and the solution within 1e-8 of the oracle's direct
    solve; after two thirds of the oracle's iteration count (before the
    Krylov space of these small systems is exhausted: at n = 2 the next
    Lanczos norm comes out negative at the oracle's last iteration, and both
    MINRES stop there) the GPU iterate meets the equal-iteration bar against
    the oracle's iterate after as many iterations."""
    from paper_2207_08481_amd import Problem
    c = setup_case(3, n, 1, nu_kind, coarse_max=cm)
    gs, m = c["gs"], c["mesh"]
    xo, ito = _oracle_minres(c)
    f = torch.as_tensor(c["f"], device="cuda:0")
    nut = torch.as_tensor(c["nu"], device="cuda:0")
    twin = oracle_twin(m, c["nu"], 1, c["f"], coarse_max=cm)
    pb = Problem(m.vertices, m.elements, m.lattice, 1, coarse_max=cm, tol=1e-10, max_it=3000).bind("cuda:0")
    pb.condense(nut)
    x, si = pb.solve(f)
    assert si["status"] == 0, si
    print(f"  iterations gpu {si['iterations']} oracle {ito}", flush=True)
    check_iterations(gs, si["iterations"], ito, twin)
    eu, ep = _l2_rel(gs, x.cpu().numpy(), gs.normalize_pressure(gs.direct_solve()))
    assert eu < 1e-8 and ep < 1e-8, (eu, ep)
    from oracle.minres import minres
    neq = (2 * ito) // 3
    xe, _ = minres(lambda v: c["K"] @ v, c["pc"].apply, gs.assemble_rhs(), tol=0.0, max_it=neq)
    pbn = Problem(m.vertices, m.elements, m.lattice, 1, coarse_max=cm, tol=0.0, max_it=neq).bind("cuda:0")
    pbn.condense(nut)
    xn, sin = pbn.solve(f, allow_max_it=True)
    assert sin["iterations"] == neq
    check_equal_iterations(gs, xn.cpu().numpy(), gs.normalize_pressure(xe), neq, twin)


def test_lowest_order_mixed_precision():
    """FP32 inner MINRES with FP64 refinement: 1e-8 against the direct solve."""
    from paper_2207_08481_amd import Problem
    c = setup_case(3, 2, 1, "lognormal")
    gs, m = c["gs"], c["mesh"]
    pb = Problem(m.vertices, m.elements, m.lattice, 1, precision=1, tol=1e-10, inner_tol=1e-5).bind("cuda:0")
    pb.condense(torch.as_tensor(c["nu"], device="cuda:0"))
    x, si = pb.solve(torch.as_tensor(c["f"], device="cuda:0"))
    assert si["status"] == 0, si
    eu, ep = _l2_rel(gs, x.cpu().numpy(), gs.normalize_pressure(gs.direct_solve()))
    assert eu < 1e-8 and ep < 1e-8, (eu, ep)


@pytest.mark.parametrize("smoother,variant", [(1, "additive"), (3, "l1")])
def test_lowest_order_variants(smoother, variant):
    """The additive (facet block Jacobi) and the l1 variants at k = 1: FP64
    MINRES iterations against the oracle's variant, then the equal-iteration
    bar."""
    from oracle.minres import minres
    from oracle.precond import Preconditioner
    from paper_2207_08481_amd import Problem
    c = setup_case(3, 2, 1)
    gs, m, K = c["gs"], c["mesh"], c["K"]
    pc = Preconditioner(gs, m.lattice, variant=variant)
    xo, info = minres(lambda v: K @ v, pc.apply, gs.assemble_rhs(), tol=1e-10, max_it=3000)
    xo, ito = gs.normalize_pressure(xo), info["iterations"]
    f = torch.as_tensor(c["f"], device="cuda:0")
    nut = torch.as_tensor(c["nu"], device="cuda:0")
    twin = oracle_twin(m, c["nu"], 1, c["f"], variant=variant)
    pb = Problem(m.vertices, m.elements, m.lattice, 1, smoother=smoother, tol=1e-10, max_it=3000).bind("cuda:0")
    pb.condense(nut)
    x, si = pb.solve(f)
    assert si["status"] == 0, si
    print(f"  {variant}: iterations gpu {si['iterations']} oracle {ito}", flush=True)
    check_iterations(gs, si["iterations"], ito, twin)
    neq = (2 * ito) // 3
    xe, _ = minres(lambda v: K @ v, pc.apply, gs.assemble_rhs(), tol=0.0, max_it=neq)
    pb.set_solve_options(0.0, neq)
    xn, sin = pb.solve(f, allow_max_it=True)
    assert sin["iterations"] == neq
    check_equal_iterations(gs, xn.cpu().numpy(), gs.normalize_pressure(xe), neq, twin)


def test_lowest_order_linear_flow_with_dirichlet_data():
    """Inhomogeneous Dirichlet data at k = 1: on a Dirichlet facet the lift
    holds the normal moments and tangential means of g and the flux of curl g
    (omega's dof).  A linear divergence-free flow with its boundary values and
    f = grad p for a linear p (the oracle's patch test) is reproduced at
    points of every element, the pressure as its element means, and the load
    vector with the lift equals the oracle's."""
    from oracle.system import GlobalSystem
    from paper_2207_08481_amd import Problem
    Gm = np.array([[1.0, -1.0, 2.0], [3.0, 1.0, -1.0], [1.0, -2.0, -2.0]])
    c0 = np.array([0.3, -0.2, 0.5])
    gp = np.array([0.5, -1.0, 2.0])
    mesh = W.unit_cube_mesh(2)
    pts = W.lattice_points(mesh, 2)
    f = np.broadcast_to(gp, pts.shape).copy()
    g = pts @ Gm.T + c0
    gs = GlobalSystem(mesh.vertices, mesh.elements, 0.8, 1, f, g_lattice=g)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 1, tol=1e-12, max_it=3000).bind("cuda:0")
    pb.condense(torch.full((mesh.n_elements,), 0.8, dtype=torch.float64, device="cuda:0"))
    pb.set_dirichlet(g)
    ft = torch.as_tensor(f, device="cuda:0")
    assert _rel(pb.load(ft).cpu().numpy(), gs.assemble_rhs()) < 1e-12
    x, si = pb.solve(ft)
    assert si["status"] == 0, si
    lam = np.random.default_rng(4).dirichlet(np.ones(4), size=5)
    u, p = pb.eval(x, lam)
    X = np.einsum("pj,ejr->epr", lam, mesh.vertices[mesh.elements])
    assert np.abs(u.cpu().numpy() - (X @ Gm.T + c0)).max() < 1e-8
    pm = mesh.vertices[mesh.elements].mean(axis=1) @ gp       # element means of p (equal volumes)
    ph = p.cpu().numpy()
    assert np.abs(ph - ph[:, :1]).max() < 1e-10               # P^0 pressure
    assert np.abs((ph[:, 0] - ph[:, 0].mean()) - (pm - pm.mean())).max() < 1e-8


@pytest.mark.parametrize("forced", [False, True])
def test_lowest_order_with_outlet(forced):
    """k = 1 with an outlet at x = L (eq. stokes_NT): the outlet's tangential
    dofs are identity rows, its normal dofs and omega flux are unknowns.
    forced = False: the oracle's outlet patch test (a linear flow with
    Dirichlet data on the other faces, p = 0), whose load, operators and
    K-hat^{-1} equal the oracle's and whose solution is the flow itself.
    forced = True: homogeneous data and a smooth load; FP64 MINRES iterations
    against the oracle's (or its twins'), then the equal-iteration bar."""
    from oracle.minres import minres
    from oracle.precond import Preconditioner
    from oracle.system import GlobalSystem
    from paper_2207_08481_amd import Problem
    from tests.test_oracle_lowest_order import _outlet_flow
    mesh, gs, u, fbc = _outlet_flow()
    nu = 0.9
    pts = W.lattice_points(mesh, 2)
    g = u(pts)
    f = np.zeros(pts.shape)
    if forced:
        f = W.CurlModes3D(seed=5, nu=nu).f(pts)
        g = None
        gs = GlobalSystem(mesh.vertices, mesh.elements, nu, 1, f, face_bc=fbc)
    print(f"[k1 outlet] forced={forced} n_e={mesh.n_elements}", flush=True)
    pc = Preconditioner(gs, mesh.lattice)
    K = gs.assemble_K()
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 1, face_bc=fbc, tol=1e-10,
                 max_it=3000).bind("cuda:0")
    pb.condense(torch.full((mesh.n_elements,), nu, dtype=torch.float64, device="cuda:0"))
    if g is not None:
        pb.set_dirichlet(g)
    ft = torch.as_tensor(f, device="cuda:0")
    x = np.random.default_rng(3).standard_normal(gs.n_dof)
    xt = torch.as_tensor(x, device="cuda:0")
    assert _rel(pb.apply("K", xt).cpu().numpy(), K @ x) < 1e-12
    yAd = pb.apply("ADELTA", xt).cpu().numpy()
    assert _rel(yAd[gs.off_f:gs.off_p], (pc.Ad @ x)[gs.off_f:gs.off_p]) < 1e-12
    assert _rel(pb.load(ft).cpu().numpy(), gs.assemble_rhs()) < 1e-12
    assert _rel(pb.precond_apply("KHAT", xt).cpu().numpy(), pc.apply(x.copy())) < 1e-11
    xs, si = pb.solve(ft)
    assert si["status"] == 0, si
    xn = xs.cpu().numpy()
    assert _rel(xn, gs.direct_solve()) < 1e-8
    if not forced:
        lam = np.random.default_rng(4).dirichlet(np.ones(4), size=5)
        uh, ph = pb.eval(xs, lam)
        X = np.einsum("pj,ejr->epr", lam, mesh.vertices[mesh.elements])
        assert np.abs(uh.cpu().numpy() - u(X)).max() < 1e-8
        assert np.abs(ph.cpu().numpy()).max() < 1e-8
        return
    xo, info = minres(lambda v: K @ v, pc.apply, gs.assemble_rhs(), tol=1e-10, max_it=3000)
    ito = info["iterations"]
    twin = oracle_twin(mesh, nu, 1, f, face_bc=fbc)
    print(f"  iterations gpu {si['iterations']} oracle {ito}", flush=True)
    check_iterations(gs, si["iterations"], ito, twin)
    neq = (2 * ito) // 3
    xe, _ = minres(lambda v: K @ v, pc.apply, gs.assemble_rhs(), tol=0.0, max_it=neq)
    pb.set_solve_options(0.0, neq)
    xq, sq = pb.solve(ft, allow_max_it=True)
    assert sq["iterations"] == neq
    check_equal_iterations(gs, xq.cpu().numpy(), xe, neq, twin)


@pytest.mark.parametrize("smoother,variant,precision", [(1, "additive", 0), (3, "l1", 0), (0, "multiplicative", 1)])
def test_lowest_order_outlet_variants(smoother, variant, precision):
    """k = 1 with an outlet under the additive and the l1 variants (K-hat^{-1}
    against the oracle's variant to 1e-11, the FP64 solve to 1e-8 of the
    direct solve) and in mixed precision (1e-8 of the direct solve)."""
    from oracle.precond import Preconditioner
    from oracle.system import GlobalSystem
    from paper_2207_08481_amd import Problem
    from tests.test_oracle_lowest_order import _outlet_flow
    mesh, _, _, fbc = _outlet_flow()
    nu = 0.9
    f = W.CurlModes3D(seed=5, nu=nu).f(W.lattice_points(mesh, 2))
    gs = GlobalSystem(mesh.vertices, mesh.elements, nu, 1, f, face_bc=fbc)
    print(f"[k1 outlet variant] {variant} precision={precision}", flush=True)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, 1, face_bc=fbc, smoother=smoother, precision=precision,
                 tol=1e-10, max_it=3000).bind("cuda:0")
    pb.condense(torch.full((mesh.n_elements,), nu, dtype=torch.float64, device="cuda:0"))
    if precision == 0:
        pc = Preconditioner(gs, mesh.lattice, variant=variant)
        x = np.random.default_rng(6).standard_normal(gs.n_dof)
        z = pb.precond_apply("KHAT", torch.as_tensor(x, device="cuda:0")).cpu().numpy()
        assert _rel(z, pc.apply(x.copy())) < 1e-11
    xs, si = pb.solve(torch.as_tensor(f, device="cuda:0"))
    assert si["status"] == 0, si
    eu, ep = _l2_rel(gs, xs.cpu().numpy(), gs.direct_solve())
    assert eu < 1e-8 and ep < 1e-8, (eu, ep, si)
