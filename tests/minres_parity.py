"""Equal-iteration MINRES parity between the GPU and the oracle.

Two FP64 implementations of the same preconditioned Lanczos process agree
after N iterations up to rounding, amplified by the process.  How far that
amplification goes depends on the system, so it is measured on the oracle
itself: the same MINRES on the same system with the degrees of freedom
numbered in a random order (every sum then runs in another order; the
preconditioner is applied through the permutation, so the arithmetic is that
of a second FP64 implementation).  The GPU iterate must be within 1e-12
relative L2 of the oracle's (velocity and mean-free pressure), or, where the
oracle's own permuted run is further away than that, within ten times that
distance.
"""
import numpy as np

from tests.quadrature import element_rule


def l2_rel(gs, x, y):
    """Relative L2(Omega) differences of the velocity and pressure fields of
    coefficient vectors x and y (reference y), by quadrature."""
    du = nu_ = dp = np_ = 0.0
    for e in range(gs.n_e):
        X = gs.topo.element_coords(e)
        xq, lam, w = element_rule(X, gs.k + 2)
        u1, p1 = gs.eval_element(x, e, lam)
        u2, p2 = gs.eval_element(y, e, lam)
        du += np.sum(w[:, None] * (u1 - u2) ** 2)
        nu_ += np.sum(w[:, None] * u2 ** 2)
        dp += np.sum(w * (p1 - p2) ** 2)
        np_ += np.sum(w * p2 ** 2)
    return np.sqrt(du / nu_), np.sqrt(dp / np_)


def permuted_oracle_drift(gs, K, pc_apply, b, n_it, x_ref, seed=0):
    """(du, dp): the oracle's MINRES after n_it iterations with a random dof
    numbering, against x_ref (its run in the natural numbering)."""
    from oracle.minres import minres
    perm = np.random.default_rng(seed).permutation(gs.n_dof)
    inv = np.argsort(perm)
    Kp = K[perm][:, perm].tocsr()

    def Mp(r):
        z = np.zeros(gs.n_dof)
        z[perm] = r
        return pc_apply(z)[perm]

    xp, _ = minres(lambda v: Kp @ v, Mp, b[perm], tol=0.0, max_it=n_it)
    return l2_rel(gs, gs.normalize_pressure(xp[inv]), x_ref)


def check_equal_iterations(gs, K, pc_apply, x_gpu, x_oracle, n_it):
    """Asserts the equal-iteration bar; returns the differences it measured."""
    b = gs.assemble_rhs()
    eu, ep = l2_rel(gs, x_gpu, x_oracle)
    out = {"u": eu, "p": ep, "iterations": n_it}
    if eu < 1e-12 and ep < 1e-12:
        print(f"[parity] equal-iteration difference u {eu:.2e} p {ep:.2e} ({n_it} its)", flush=True)
        return out
    du, dp = permuted_oracle_drift(gs, K, pc_apply, b, n_it, x_oracle)
    out.update(oracle_u=du, oracle_p=dp)
    print(f"[parity] equal-iteration difference u {eu:.2e} p {ep:.2e} ({n_it} its); "
          f"oracle against itself, permuted numbering: u {du:.2e} p {dp:.2e}", flush=True)
    assert eu < max(1e-12, 10 * du) and ep < max(1e-12, 10 * dp), out
    return out
