"""GPU parity of the outlet boundary Gamma_NT and inhomogeneous Dirichlet data
(eq. stokes_D, stokes_NT; Lemma outflow) against the oracle, and the exact
reproduction of plane channel flow (u = (4y(1-y), 0[, 0]), p = 4 nu (L - x),
which lies in the discrete spaces for k >= 2)."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [(2, (4, 2), 2, 2.0), (2, (3, 3), 3, 1.0), (3, (2, 2, 2), 2, 1.0), (3, (3, 2, 2), 3, 1.5)]


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


_cache = {}


def channel_case(d, cells, k, L, smoother=0):
    key = (d, cells, k, L, smoother)
    if key in _cache:
        return _cache[key]
    _need_gpu()
    from paper_2207_08481_amd import Problem
    from oracle.system import GlobalSystem
    from oracle.precond import Preconditioner
    mesh = W.box_mesh(cells, (L,) + (1.0,) * (d - 1))
    ch = W.PlaneChannel(d, nu=0.7, L=L)
    pts = W.lattice_points(mesh, k + 1)
    f, g = ch.f(pts), ch.u(pts)
    print(f"[outlet case] d={d} cells={cells} k={k} smoother={smoother}", flush=True)
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, k, face_bc=ch.face_bc(), smoother=smoother,
                 tol=1e-12, max_it=3000).bind("cuda:0")
    pb.condense(torch.full((mesh.n_elements,), ch.nu, dtype=torch.float64, device="cuda:0"))
    pb.set_dirichlet(g)
    gs = GlobalSystem(mesh.vertices, mesh.elements, ch.nu, k, f, face_bc=ch.face_bc(), g_lattice=g)
    variant = {0: "multiplicative", 1: "additive", 2: "full"}[smoother]
    pc = Preconditioner(gs, mesh.lattice, variant=variant)
    out = dict(mesh=mesh, ch=ch, f=f, pb=pb, gs=gs, pc=pc, K=gs.assemble_K())
    _cache[key] = out
    return out


@pytest.mark.parametrize("d,cells,k,L", CASES)
def test_outlet_operators_and_load(d, cells, k, L):
    """K (with the identity rows of the fixed outlet tangential dofs), A^d,
    the lifted load b = F - K x_D, and K-hat^{-1} against the oracle."""
    c = channel_case(d, cells, k, L)
    pb, gs, K, pc = c["pb"], c["gs"], c["K"], c["pc"]
    x = np.random.default_rng(3).standard_normal(gs.n_dof)
    xt = torch.as_tensor(x, device="cuda:0")
    assert _rel(pb.apply("K", xt).cpu().numpy(), K @ x) < 1e-12
    yAd = pb.apply("ADELTA", xt).cpu().numpy()
    assert _rel(yAd[gs.off_f:gs.off_p], (pc.Ad @ x)[gs.off_f:gs.off_p]) < 1e-12
    b = pb.load(c["f"]).cpu().numpy()
    assert _rel(b, gs.assemble_rhs()) < 1e-12
    z = pb.precond_apply("KHAT", xt).cpu().numpy()
    assert _rel(z, pc.apply(x.copy())) < 1e-11


@pytest.mark.parametrize("d,cells,k,L", CASES)
def test_plane_channel_solve(d, cells, k, L):
    """MINRES on the GPU: iterations within +-1 of the oracle's, the solution
    equals the oracle's direct solution, and u_h, p_h (with the lifted
    Dirichlet data) equal the exact channel flow at points of every element."""
    from oracle.minres import minres
    c = channel_case(d, cells, k, L)
    pb, gs, K, pc, ch, mesh = c["pb"], c["gs"], c["K"], c["pc"], c["ch"], c["mesh"]
    x, si = pb.solve(torch.as_tensor(c["f"], device="cuda:0"))
    assert si["status"] == 0
    b = gs.assemble_rhs()
    xo, info = minres(lambda v: K @ v, pc.apply, b, tol=1e-12, max_it=3000)
    assert abs(si["iterations"] - info["iterations"]) <= 1, (si["iterations"], info["iterations"])
    xd = gs.direct_solve()
    xn = x.cpu().numpy()
    assert _rel(xn, xd) < 1e-9
    pts = np.random.default_rng(4).dirichlet(np.ones(d + 1), size=4)
    u, p = pb.eval(x, pts)
    u, p = u.cpu().numpy(), p.cpu().numpy()
    X = np.einsum("pj,ejr->epr", pts, mesh.vertices[mesh.elements])
    assert np.abs(u - ch.u(X)).max() <= 1e-9
    assert np.abs(p - ch.p(X)).max() <= 1e-9 * 4 * ch.nu * L


@pytest.mark.parametrize("smoother", [1, 2])
def test_outlet_other_variants(smoother):
    """The additive and the full-system variants with an outlet and lifted
    Dirichlet data: K-hat^{-1} against the oracle's variant and an exact solve."""
    d, cells, k, L = 3, (2, 2, 2), 2, 1.0
    c = channel_case(d, cells, k, L, smoother=smoother)
    pb, gs, pc, ch, mesh = c["pb"], c["gs"], c["pc"], c["ch"], c["mesh"]
    x = np.random.default_rng(5).standard_normal(gs.n_dof)
    z = pb.precond_apply("KHAT", torch.as_tensor(x, device="cuda:0")).cpu().numpy()
    assert _rel(z, pc.apply(x.copy())) < 1e-11
    xs, si = pb.solve(torch.as_tensor(c["f"], device="cuda:0"))
    assert si["status"] == 0
    assert _rel(xs.cpu().numpy(), gs.direct_solve()) < 1e-9
