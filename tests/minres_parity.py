"""Equal-iteration MINRES parity between the GPU and the oracle.

Two FP64 computations of the same discrete problem agree after N MINRES
iterations up to rounding, amplified by the condensation and by the Lanczos
process.  How far that goes depends on the system, so it is measured on the
oracle itself, against a twin of itself: the same problem with every element's
Sigma_h(T) in a randomly rotated orthonormal basis (the condensed operators do
not depend on the basis, Sec. 4.2, so only their rounding changes) and the
degrees of freedom numbered in a random order (every sum of the solve then
runs in another order; the preconditioner is applied through the
permutation).  The GPU iterate must be within 1e-12 relative L2 of the
oracle's (velocity and mean-free pressure), or, where the twin is further from
the oracle than that, within ten times the twin's distance.
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


def oracle_twin(mesh, nu, k, f, coarse_max=512, variant="multiplicative", smoothing_steps=2, seed=1,
                face_bc=None, g_lattice=None):
    """A callable building the twin: (K, K-hat^{-1}, b) of the oracle's
    system with Sigma_h(T) in a rotated basis (build(rotation) takes another
    rotation seed)."""
    def build(rotation=None):
        from oracle.precond import Preconditioner
        from oracle.system import GlobalSystem
        rs = seed if rotation is None else rotation
        gs = GlobalSystem(mesh.vertices, mesh.elements, nu, k, f, face_bc=face_bc, g_lattice=g_lattice,
                          sigma_rotation_seed=rs)
        pc = Preconditioner(gs, mesh.lattice, smoothing_steps=smoothing_steps, coarse_max=coarse_max,
                            variant=variant)
        return gs.assemble_K(), pc.apply, gs.assemble_rhs()
    return build


def twin_drift(gs, twin, n_it, x_ref, seed=0):
    """(du, dp): the twin's MINRES after n_it iterations, in a random dof
    numbering, against x_ref (the oracle's own iterate)."""
    from oracle.minres import minres
    K, pc_apply, b = twin()
    perm = np.random.default_rng(seed).permutation(gs.n_dof)
    inv = np.argsort(perm)
    Kp = K[perm][:, perm].tocsr()

    def Mp(r):
        z = np.zeros(gs.n_dof)
        z[perm] = r
        return pc_apply(z)[perm]

    xp, _ = minres(lambda v: Kp @ v, Mp, b[perm], tol=0.0, max_it=n_it)
    return l2_rel(gs, gs.normalize_pressure(xp[inv]), x_ref)


def check_equal_iterations(gs, x_gpu, x_oracle, n_it, twin):
    """Asserts the equal-iteration bar; returns the differences it measured."""
    eu, ep = l2_rel(gs, x_gpu, x_oracle)
    out = {"u": eu, "p": ep, "iterations": n_it}
    if eu < 1e-12 and ep < 1e-12:
        print(f"[parity] equal-iteration difference u {eu:.2e} p {ep:.2e} ({n_it} its)", flush=True)
        return out
    du, dp = twin_drift(gs, twin, n_it, x_oracle)
    out.update(twin_u=du, twin_p=dp)
    print(f"[parity] equal-iteration difference u {eu:.2e} p {ep:.2e} ({n_it} its); "
          f"oracle twin (rotated Sigma basis, permuted numbering): u {du:.2e} p {dp:.2e}", flush=True)
    assert eu < max(1e-12, 10 * du) and ep < max(1e-12, 10 * dp), out
    return out


def twin_iterations(gs, twin, tol, seeds=(0, 1), rotation=None):
    """MINRES iteration counts of the oracle's twin at tol, one per random dof
    numbering."""
    from oracle.minres import minres
    K, pc_apply, b = twin(rotation)
    out = []
    for seed in seeds:
        perm = np.random.default_rng(seed).permutation(gs.n_dof)
        Kp = K[perm][:, perm].tocsr()

        def Mp(r, perm=perm):
            z = np.zeros(gs.n_dof)
            z[perm] = r
            return pc_apply(z)[perm]

        _, info = minres(lambda v: Kp @ v, Mp, b[perm], tol=tol, max_it=5000)
        out.append(info["iterations"])
    return out


def check_iterations(gs, its_gpu, its_oracle, twin, tol=1e-10):
    """Iterations within +-1 of the oracle's, or, where they are not, within
    +-1 of the range the oracle's twins (two rotated Sigma bases, two permuted
    numberings each) span: slowly converging runs move by a few iterations
    under FP64 rounding alone (the k = 1 additive case on the 2^3 cube: 268 to
    274 across twins)."""
    if abs(its_gpu - its_oracle) <= 1:
        return
    tw = twin_iterations(gs, twin, tol) + twin_iterations(gs, twin, tol, rotation=3)
    lo, hi = min([its_oracle] + tw), max([its_oracle] + tw)
    print(f"[parity] iterations gpu {its_gpu} oracle {its_oracle}; oracle twins {tw}", flush=True)
    assert lo - 1 <= its_gpu <= hi + 1, (its_gpu, its_oracle, tw)
