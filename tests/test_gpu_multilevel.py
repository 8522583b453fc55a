"""GPU parity of the lattice multigrid with two and three levels.

The benchmark meshes run the P1 V(1,1) cycle on 3 (16^3) and 4 (32^3) lattice
levels.  These cases use a small coarsest-level size (coarse_max) so that
meshes the oracle handles in seconds also coarsen:

* 2D n = 9, coarse_max 20: intervals 9 -> 5 -> 3 (odd n, three levels);
* 2D n = 7: 7 -> 4 (the last coarse interval has length one);
* 3D n = 4, coarse_max 20: 4 -> 2 (two levels);
* 3D n = 5, coarse_max 50: 5 -> 3 (odd n, two levels).

Compared with the oracle (one V-cycle of the multigrid, the embedding, the
multiplicative auxiliary space preconditioner, A-hat_ext^{-1}, K-hat^{-1}):
single applies to 1e-12 (sweeps, embedding) and 1e-11 (anything with the
V-cycle), FP32 K-hat^{-1} to 1e-4.  Solves: FP64 MINRES iterations within +-1
of the oracle's MINRES at tol 1e-10, and after the same number of iterations
the GPU iterate equals the oracle's to 1e-12 relative L2 in the velocity and
in the mean-free pressure (or ten times the oracle's distance to itself under
another dof numbering, where that is larger).
"""
import numpy as np
import pytest

import workloads as W
from tests.minres_parity import check_equal_iterations, oracle_twin

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


_cache = {}


def case(d, n, k, cm, nu_kind="one"):
    key = (d, n, k, cm, nu_kind)
    if key in _cache:
        return _cache[key]
    _need_gpu()
    from oracle.system import GlobalSystem
    from oracle.precond import Preconditioner
    mesh = W.unit_square_mesh(n) if d == 2 else W.unit_cube_mesh(n)
    nu = np.ones(mesh.n_elements) if nu_kind == "one" else W.lognormal_nu(mesh.n_elements, seed=4)
    sol = W.Manufactured2D() if d == 2 else W.CurlModes3D(seed=2)
    f = sol.f(W.lattice_points(mesh, k + 1))
    gs = GlobalSystem(mesh.vertices, mesh.elements, nu, k, f)
    pc = Preconditioner(gs, mesh.lattice, coarse_max=cm)
    out = dict(mesh=mesh, nu=nu, f=f, gs=gs, pc=pc, k=k, cm=cm)
    _cache[key] = out
    return out


def gpu_problem(c, **kw):
    from paper_2207_08481_amd import Problem
    m = c["mesh"]
    pb = Problem(m.vertices, m.elements, m.lattice, c["k"], coarse_max=c["cm"], **kw).bind("cuda:0")
    pb.condense(torch.as_tensor(c["nu"], device="cuda:0"))
    return pb


def oracle_minres(c, tol=1e-10):
    """The oracle's MINRES solution (mean-free pressure) and iteration count."""
    if "minres" not in c:
        from oracle.minres import minres
        gs = c["gs"]
        K = gs.assemble_K()
        xo, info = minres(lambda v: K @ v, c["pc"].apply, gs.assemble_rhs(), tol=tol, max_it=3000)
        c["minres"] = (gs.normalize_pressure(xo), info["iterations"])
    return c["minres"]


def twin(c):
    return oracle_twin(c["mesh"], c["nu"], c["k"], c["f"], coarse_max=c["cm"])


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


PIECES = [(2, 9, 2, 20, "one", 3), (2, 9, 3, 20, "lognormal", 3), (2, 7, 2, 20, "one", 2),
          (3, 4, 2, 20, "one", 2), (3, 5, 2, 50, "lognormal", 2)]


@pytest.mark.parametrize("d,n,k,cm,nu_kind,levels", PIECES)
def test_multilevel_preconditioner_pieces(d, n, k, cm, nu_kind, levels):
    c = case(d, n, k, cm, nu_kind)
    gs, pc = c["gs"], c["pc"]
    print(f"[case] multilevel pieces d={d} n={n} k={k} cm={cm} nu={nu_kind}", flush=True)
    pb = gpu_problem(c)
    assert len(pc.mg.levels) == levels
    assert pb.info.n_mg_levels == levels
    rng = np.random.default_rng(17)
    r = rng.standard_normal(gs.n_dof)
    rt = torch.as_tensor(r, device="cuda:0")
    fd = slice(gs.off_f, gs.off_p)
    rr = r.copy()
    rr[:gs.off_f] = 0
    rr[gs.off_p:] = 0
    n1 = pb.info.n_p1_dofs
    assert n1 == pc.mg.levels[0]["A"].shape[0]
    q = rng.standard_normal(n1)
    qt = torch.as_tensor(q, device="cuda:0")
    # one V(1,1) cycle on the P1 lattice hierarchy
    z = pb.precond_apply("MG", qt).cpu().numpy()
    assert _rel(z, pc.mg.vcycle(q)) < 1e-11
    z = pb.precond_apply("EDELTA", qt).cpu().numpy()
    assert _rel(z[fd], (pc.E @ q)[fd]) < 1e-12
    z = pb.precond_apply("EDELTA_T", rt).cpu().numpy()
    assert _rel(z, pc.E.T @ rr) < 1e-12
    z = pb.precond_apply("AUX", rt).cpu().numpy()
    assert _rel(z[fd], pc.aux_correction(rr)[fd]) < 1e-11
    z = pb.precond_apply("ADELTA_MULT", rt).cpu().numpy()
    assert _rel(z[fd], pc.Ad_mult_inv(rr)[fd]) < 1e-11
    ru = r.copy()
    ru[gs.off_p:] = 0
    z = pb.precond_apply("AEXT", rt).cpu().numpy()
    assert _rel(z[:gs.off_p], pc.A_ext_inv(ru)[:gs.off_p]) < 1e-11
    ref = pc.apply(r.copy())
    z = pb.precond_apply("KHAT", rt).cpu().numpy()
    assert _rel(z, ref) < 1e-11
    z32 = pb.precond_apply("KHAT", rt.float()).double().cpu().numpy()
    assert _rel(z32, ref) < 1e-4


SOLVES = [(2, 9, 2, 20, "one"), (2, 9, 3, 20, "lognormal"), (3, 4, 2, 20, "one")]


@pytest.mark.parametrize("d,n,k,cm,nu_kind", SOLVES)
def test_multilevel_solve_matches_oracle_minres(d, n, k, cm, nu_kind):
    """FP64 MINRES with the multilevel V-cycle: iterations within +-1 of the
    oracle's at tol 1e-10; run for exactly the oracle's iteration count, the
    GPU iterate equals the oracle's iterate to the equal-iteration bar."""
    c = case(d, n, k, cm, nu_kind)
    gs = c["gs"]
    print(f"[case] multilevel solve d={d} n={n} k={k} cm={cm} nu={nu_kind}", flush=True)
    xo, ito = oracle_minres(c)
    f = torch.as_tensor(c["f"], device="cuda:0")
    pb = gpu_problem(c, tol=1e-10, max_it=3000)
    assert pb.info.n_mg_levels >= 2
    x, si = pb.solve(f)
    assert si["status"] == 0
    print(f"  iterations gpu {si['iterations']} oracle {ito}", flush=True)
    assert abs(si["iterations"] - ito) <= 1, (si, ito)
    pbn = gpu_problem(c, tol=0.0, max_it=ito)
    xn, sin = pbn.solve(f, allow_max_it=True)
    assert sin["iterations"] == ito
    check_equal_iterations(gs, xn.cpu().numpy(), xo, ito, twin(c))


def test_batch_members_of_different_depths():
    """One batch whose members stop at different multigrid depths (2D n = 9:
    three levels; n = 7: two; n = 4: one; 3D n = 4: two): each member within
    +-1 iteration of its oracle MINRES; where the counts are equal, the
    iterates meet the equal-iteration bar (else 1e-8 relative, the distance of
    two tolerance-1e-10 iterates)."""
    _need_gpu()
    from paper_2207_08481_amd import Batch
    keys = [(2, 9, 2, 20, "one"), (2, 7, 2, 20, "one"), (2, 4, 2, 20, "one"), (3, 4, 2, 20, "one")]
    cs = [case(*kk) for kk in keys]
    print("[batch] multilevel members", keys, flush=True)
    b = Batch([(c["mesh"].vertices, c["mesh"].elements, c["mesh"].lattice) for c in cs], [c["k"] for c in cs],
              precision=0, tol=1e-10, max_it=3000, coarse_max=20).bind("cuda:0")
    b.condense([torch.as_tensor(c["nu"], device="cuda:0") for c in cs])
    depths = [len(c["pc"].mg.levels) for c in cs]
    assert depths == [3, 2, 1, 2]
    for m, dep in zip(b.members, depths):
        assert m.n_mg_levels == dep
    xs, infos = b.solve([torch.as_tensor(c["f"], device="cuda:0") for c in cs])
    for kk, x, c, inf in zip(keys, xs, cs, infos):
        assert inf["status"] == 0, inf
        xo, ito = oracle_minres(c)
        its = inf["iterations"]
        print(f"  member {kk}: iterations gpu {its} oracle {ito}", flush=True)
        assert abs(its - ito) <= 1, (kk, its, ito)
        if its == ito:
            check_equal_iterations(c["gs"], x.cpu().numpy(), xo, ito, twin(c))
        else:
            assert _rel(x.cpu().numpy(), xo) < 1e-8, kk
