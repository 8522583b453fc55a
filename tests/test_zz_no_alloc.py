"""mcs_solve_rhs_noalloc (the solve for callers that cannot allocate) against
mcs_solve_rhs through the C ABI: two no-alloc calls in a row, the second on a
smaller problem (and in the other precision), each bitwise equal to the
allocating entry point's solution, with the same iteration count."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problem(n, k, precision):
    from paper_2207_08481_amd import Problem
    mesh = W.unit_cube_mesh(n)
    nu = torch.as_tensor(W.lognormal_nu(mesh.n_elements, seed=4), device="cuda:0")
    f = torch.as_tensor(W.RandomForce(3, seed=3).f(W.lattice_points(mesh, k + 1)), device="cuda:0")
    pb = Problem(mesh.vertices, mesh.elements, mesh.lattice, k, precision=precision, tol=1e-10).bind("cuda:0")
    pb.condense(nu)
    return pb, pb.load(f)


def test_noalloc_solve_equals_solve_rhs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cases = [(3, 3, 0), (2, 2, 1)]   # the second input is smaller
    print(f"[no-alloc] cases (n, k, precision) {cases}", flush=True)
    probs = [_problem(*c) for c in cases]
    refs = [pb.solve_rhs(b) for pb, b in probs]
    outs = []
    for pb, b in probs:           # two no-alloc calls in a row
        x = pb.vector()
        si = pb.solve_rhs_noalloc(b, x)
        outs.append((x, si))
    torch.cuda.synchronize()
    for c, (xr, sr), (x, si) in zip(cases, refs, outs):
        print(f"[no-alloc] {c}: iterations {si['iterations']} in {si['outer_steps']} steps (allocating entry "
              f"{sr['iterations']} in {sr['outer_steps']})", flush=True)
        assert si["status"] == 0 and sr["status"] == 0
        assert si["iterations"] == sr["iterations"] and si["outer_steps"] == sr["outer_steps"]
        assert torch.equal(x, xr), (x - xr).abs().max().item()
        assert si["rel_residual"] == sr["rel_residual"]
        assert np.isfinite(si["rel_residual"]) and si["rel_residual"] < 1e-6
