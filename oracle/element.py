"""Element spaces, element matrices and static condensation -- oracle (FP64).

Spaces (Sec. 3, eqs. fes_V .. fes_Vbar), on one simplex T with vertices sorted
by global index, barycentric coordinates lambda_0..lambda_d:

* V_h(T) = BDM^k = P^k(T, R^d), split into
  - normal bubbles (zero normal trace on all of dT), basis
        lambda^alpha (x_a - x_s0),  |alpha| = k, s0 = min supp(alpha),
        a in supp(alpha) \\ {s0}                      (alpha lex-descending, a ascending)
  - facet functions of local facet i, one per beta (|beta| = k over the
    facet's vertices, lex-descending):
        c * lambda^beta (x_j0 - x_i),  j0 = first facet vertex with beta_j0 > 0,
    with c fixed so that the normal trace w.r.t. the facet's global normal
    n_F is lambda^beta / |F| on F (zero on the other facets).
  The global normal n_F of a facet with sorted vertices (a, b[, c]) is the
  unit vector along R(x_b - x_a) (2D, R = clockwise quarter turn) or
  (x_b - x_a) x (x_c - x_a) (3D).  This makes the global basis normal
  continuous (Sec. 3: BDM is H(div)-conforming).
* hat V_h on facet F: lambda_F^gamma t_b, |gamma| = k-1 over the facet
  vertices, t_b = x_{f_b} - x_{f_0} (b = 1..d-1), index (b-1)*n_gamma + gamma.
* W_h(T) = P^{k-1}(T, K) for k >= 2; for k = 1 (3D, Sec. 7 "The lowest order
  case") the lowest-order Raviart-Thomas space P^0(T, R^3) + x P^0(T),
  normal-continuous, entering through kappa(omega), with one flux dof per
  facet and a stabilising
  (div omega, div eta) term (weight nu |T|^(2/3));
  Q_h(T) = P^{k-1}(T) (basis lambda^gamma),
  Sigma_h(T) = {tau in P^k(T, D): tau_nt in P^{k-1}(F) for all F in dT},
  built here as the null space of the top-degree nt-trace moments in
  P^k(T, D) (eq. fes_Sigma).

Element matrices follow eq. bigfemSPmat literally (with the weak-form sign of
the pressure coupling, -(div u, q), eq. discrmixedstressstokesweak, and the
volume reading of the B_omega_sigma integral).  Condensation I is
A = A^div - B_sigma M^{-1} B_sigma^T (Sec. 4.2, "Static condensation of
sigma, omega"); condensation II eliminates the bubbles (Sec. 4.2, "Static
condensation of high order velocity functions"): H = A_oo^{-1} A_od and
A^d = A_dd - A_do H.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .poly import (multi_indices, index_map, product_moments, facet_product_moments,
                   gradient_matrices)


def trace_free_basis(d):
    """A basis of D (trace-free d x d matrices): E_rs (r != s), E_rr - E_{d-1,d-1}."""
    out = []
    for r in range(d):
        for s in range(d):
            if r != s:
                E = np.zeros((d, d))
                E[r, s] = 1.0
                out.append(E)
    for r in range(d - 1):
        E = np.zeros((d, d))
        E[r, r] = 1.0
        E[d - 1, d - 1] = -1.0
        out.append(E)
    return np.asarray(out)


def skew_basis(d):
    """A basis of K (skew-symmetric d x d matrices): E_rs - E_sr, r < s."""
    out = []
    for r in range(d):
        for s in range(r + 1, d):
            E = np.zeros((d, d))
            E[r, s] = 1.0
            E[s, r] = -1.0
            out.append(E)
    return np.asarray(out)


def facet_normal_geo(P):
    """Global unit normal of a facet given its sorted vertex coordinates P (d, d)."""
    d = P.shape[1]
    if d == 2:
        t = P[1] - P[0]
        n = np.array([t[1], -t[0]])
    else:
        n = np.cross(P[1] - P[0], P[2] - P[0])
    return n / np.linalg.norm(n)


def expected_dims(d, k):
    """Dimensions of the local spaces (closed forms).  For k = 1 (3D only,
    Sec. 7) W_h(T) is the lowest-order Raviart-Thomas space (one normal flux
    per facet, n_w = 1), coupled across facets, so its dofs join the facet
    blocks; for k >= 2 it is P^{k-1}(T, K) and n_w = 0."""
    if k == 1 and d != 3:
        raise ValueError("the lowest order k = 1 is the three-dimensional method of Sec. 7")
    nk = math.comb(k + d, d)
    nkm1 = math.comb(k - 1 + d, d)
    nF = math.comb(k + d - 1, d - 1)
    nFm1 = math.comb(k - 1 + d - 1, d - 1)
    n_u = d * nk
    n_bub = n_u - (d + 1) * nF
    n_hat = (d - 1) * nFm1
    n_sig = (d * d - 1) * nk - (d + 1) * (d - 1) * (nF - nFm1)
    n_w = 1 if k == 1 else 0
    n_om = d + 1 if k == 1 else (d * (d - 1) // 2) * nkm1
    return dict(n_u=n_u, n_bub=n_bub, n_F=nF, n_hat=n_hat, n_w=n_w, n_fb=nF + n_hat + n_w,
                n_sig=n_sig, n_om=n_om, n_p=nkm1,
                n_A=n_u + (d + 1) * (n_hat + n_w), n_d=(d + 1) * (nF + n_hat + n_w))


def kappa(w):
    """The skew matrix kappa(w) of a vector w in R^3 with kappa(curl u) equal
    to the skew part (grad u - grad u^T) / 2 of grad u (Sec. 7 replaces omega
    by kappa(omega) in the bilinear forms)."""
    return 0.5 * np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def rt0_basis(ed):
    """Lowest-order Raviart-Thomas basis of W_h(T) for k = 1 (Sec. 7):
    psi_i = s_i (x - x_i) / (d |T|), one function per local facet i, with flux
    1 through F_i w.r.t. the global facet normal n_F (s_i = n_out,i . n_F = +-1)
    and zero normal component on the other facets.  Returns the coefficients
    over I_1 (lambda_0 .. lambda_d; x - x_i = sum_j lambda_j (x_j - x_i)),
    shape (d+1, d+1, d), and div psi_i = s_i / |T|."""
    d = ed.d
    nv = d + 1
    C = np.zeros((nv, nv, d))
    s = np.zeros(nv)
    for i in range(nv):
        s[i] = np.sign(ed.normals_out[i] @ ed.normals_geo[i])
        for j in range(nv):
            C[i, j] = s[i] * (ed.X[j] - ed.X[i]) / (d * ed.vol)
    return C, s / ed.vol


@dataclass
class ElementData:
    """Geometry and bases of one element (sorted vertex order)."""
    X: np.ndarray
    d: int
    k: int
    detJ: float
    vol: float
    grad_lambda: np.ndarray        # (d+1, d)
    normals_out: np.ndarray        # (d+1, d) outward unit normals
    normals_geo: np.ndarray        # (d+1, d) global facet normals n_F
    areas: np.ndarray              # (d+1,)
    tangents: np.ndarray           # (d+1, d-1, d)
    Phi: np.ndarray                # (n_u, |I_k|, d) BDM basis, bubbles first
    Vhat: np.ndarray               # (d+1, n_hat, |I_{k-1}|, d) facet tangential basis
    dims: dict


def element_geometry(X, k):
    X = np.asarray(X, dtype=np.float64)
    d = X.shape[1]
    J = (X[1:] - X[0]).T
    detJ = float(np.linalg.det(J))
    vol = abs(detJ) / math.factorial(d)
    Jinv = np.linalg.inv(J)
    gl = np.zeros((d + 1, d))
    gl[1:] = Jinv
    gl[0] = -Jinv.sum(axis=0)
    n_out = np.zeros((d + 1, d))
    n_geo = np.zeros((d + 1, d))
    areas = np.zeros(d + 1)
    tang = np.zeros((d + 1, d - 1, d))
    for i in range(d + 1):
        g = gl[i]
        n_out[i] = -g / np.linalg.norm(g)          # grad lambda_i points to vertex i
        areas[i] = d * vol * np.linalg.norm(g)     # |T| = |F_i| h_i / d
        fv = [j for j in range(d + 1) if j != i]
        n_geo[i] = facet_normal_geo(X[fv])
        for b in range(1, d):
            tang[i, b - 1] = X[fv[b]] - X[fv[0]]

    dims = expected_dims(d, k)
    nv = d + 1
    Ik = multi_indices(nv, k)
    im_k = index_map(nv, k)
    Phi = []
    # normal bubbles
    for a in Ik:
        S = [j for j in range(nv) if a[j] > 0]
        if len(S) < 2:
            continue
        for aa in S[1:]:
            c = np.zeros((len(Ik), d))
            c[im_k[a]] = X[aa] - X[S[0]]
            Phi.append(c)
    assert len(Phi) == dims["n_bub"]
    # facet functions
    for i in range(nv):
        fv = [j for j in range(nv) if j != i]
        for beta in multi_indices(d, k):
            alpha = [0] * nv
            for jj, v in enumerate(fv):
                alpha[v] = beta[jj]
            j0 = fv[next(jj for jj in range(d) if beta[jj] > 0)]
            w = X[j0] - X[i]
            scale = 1.0 / (areas[i] * float(w @ n_geo[i]))
            c = np.zeros((len(Ik), d))
            c[im_k[tuple(alpha)]] = scale * w
            Phi.append(c)
    Phi = np.asarray(Phi)
    assert Phi.shape[0] == dims["n_u"]

    Ikm1 = multi_indices(nv, k - 1)
    im_km1 = index_map(nv, k - 1)
    Vhat = np.zeros((nv, dims["n_hat"], len(Ikm1), d))
    for i in range(nv):
        fv = [j for j in range(nv) if j != i]
        gam_list = multi_indices(d, k - 1)
        for b in range(d - 1):
            for gi, gam in enumerate(gam_list):
                alpha = [0] * nv
                for jj, v in enumerate(fv):
                    alpha[v] = gam[jj]
                Vhat[i, b * len(gam_list) + gi, im_km1[tuple(alpha)]] = tang[i, b]
    return ElementData(X, d, k, detJ, vol, gl, n_out, n_geo, areas, tang, Phi, Vhat, dims)


def sigma_space(ed: ElementData):
    """Null-space basis Z of Sigma_h(T) inside P^k(T, D) (coefficients over
    (alpha, m) with alpha in I_k, m over trace_free_basis).  Constraint: for each
    facet F_i and tangent t_b, the facet polynomial t_b^T sigma n_i must lie in
    P^{k-1}(F_i), i.e. its degree-k Bernstein coefficients on F_i must lie in the
    range of degree elevation from k-1."""
    d, k = ed.d, ed.k
    nv = d + 1
    Dm = trace_free_basis(d)
    Ik = multi_indices(nv, k)
    nfull = len(Ik) * len(Dm)
    rows = []
    from .poly import elevation
    E = elevation(d, k - 1)                       # facet: n_vars = d
    N = sla.null_space(E.T)                       # left null space: top-degree part
    Ifk = multi_indices(d, k)
    im_fk = index_map(d, k)
    for i in range(nv):
        fv = [j for j in range(nv) if j != i]
        n = ed.normals_out[i]
        for b in range(d - 1):
            t = ed.tangents[i, b]
            # facet Bernstein coefficients of t^T sigma n for each basis function
            Cf = np.zeros((len(Ifk), nfull))
            for ai, a in enumerate(Ik):
                if a[i] > 0:
                    continue
                beta = tuple(a[v] for v in fv)
                for m in range(len(Dm)):
                    Cf[im_fk[beta], ai * len(Dm) + m] = t @ Dm[m] @ n
            rows.append(N.T @ Cf)
    C = np.vstack(rows)
    Z = sla.null_space(C)
    assert Z.shape[1] == ed.dims["n_sig"], (Z.shape, ed.dims["n_sig"])
    return Z, Dm


def lattice_bernstein(d, m, lattice_sorted):
    """Coefficients (over I_m) of the Lagrange basis of the degree-m principal
    lattice given by multi-indices lattice_sorted (n_lat, d+1) in sorted vertex
    order: L = V^{-1} with V[l, alpha] = prod_j (beta_lj / m)^alpha_j."""
    Im = np.asarray(multi_indices(d + 1, m))
    lam = np.asarray(lattice_sorted, dtype=np.float64) / m
    V = np.prod(lam[:, None, :] ** Im[None, :, :], axis=2)
    return np.linalg.inv(V)          # (|I_m|, n_lat)


def element_system(X, nu, k, f_lattice_sorted=None, lattice_sorted=None, m=None,
                   keep_blocks=False, pinned=(), sigma_rotation_seed=None):
    """All element quantities of the hybridised MCS method on one element.

    Returns a dict with
      'A'      condensed velocity block on (u, uhat), local order
               [Phi (bubbles, facet fns 0..d), Vhat (facet 0..d)],
      'B'      (n_p, n_u) pressure coupling -(div phi_u, phi_p),
      'Adiv', 'Mp', 'F' (load, n_u), and the condensation-II blocks in the
      reordered local order [bubbles | facet blocks (normal, tangential)]:
      'perm', 'Aoo', 'Aod', 'H', 'Ad'.

    pinned: local indices of A (original order) whose values are fixed to
    zero (tangential dofs on an outlet facet); their rows and columns of A are
    replaced by those of the identity, so that they decouple before the
    bubbles are condensed.

    sigma_rotation_seed: when given, Sigma_h(T) is represented in another
    orthonormal basis, Z Q with Q a seeded random orthogonal matrix.  sigma and
    omega are condensed, so the element operators do not depend on the basis
    (Sec. 4.2); only their rounding changes.  Tests use it to measure how far
    two FP64 computations of the same discrete problem drift apart.
    """
    ed = X if isinstance(X, ElementData) else element_geometry(X, k)
    d, nv = ed.d, ed.d + 1
    dims = ed.dims
    vol = ed.vol
    Z, Dm = sigma_space(ed)
    if sigma_rotation_seed is not None:
        g = np.random.default_rng(sigma_rotation_seed).standard_normal((Z.shape[1], Z.shape[1]))
        Q, _ = np.linalg.qr(g)
        Z = Z @ Q
    Kn = skew_basis(d)
    Ik = multi_indices(nv, k)
    nDm = len(Dm)
    nfull = len(Ik) * nDm

    G_kk = product_moments(nv, k, k)
    G_km1k = product_moments(nv, k - 1, k)
    G_kkm1 = product_moments(nv, k, k - 1)
    G_m1m1 = product_moments(nv, k - 1, k - 1)
    Dk = gradient_matrices(nv, k, ed.grad_lambda)       # (d, |I_{k-1}|, |I_k|)

    # M_sigma_sigma on the full P^k(T, D) coefficient space
    DD = np.einsum("mrs,nrs->mn", Dm, Dm)
    Mfull = (vol / nu) * np.kron(G_kk, DD)
    # B_omega_sigma (volume integral of sigma : omega)
    DK = np.einsum("mrs,nrs->mn", Dm, Kn)
    Bws_full = vol * np.kron(G_kkm1.T, DK.T)           # rows (gamma, n), cols (alpha, m)
    # div of sigma basis functions: coefficients over I_{k-1} x d
    divsig = np.einsum("sab,mrs->bmar", Dk, Dm)         # (alpha, m, alpha', r)
    divsig = divsig.reshape(nfull, -1, d)
    Phi = ed.Phi
    n_u = Phi.shape[0]
    # B_u_sigma = int_T div(sigma) . phi_u - int_dT sigma_nn (phi_u)_n
    Bus = vol * np.einsum("jar,ab,ibr->ij", divsig, G_km1k, Phi)
    for i in range(nv):
        n = ed.normals_out[i]
        Gf = facet_product_moments(nv, k, k, i) * ed.areas[i]
        snn = np.einsum("r,mrs,s->m", n, Dm, n)          # per m
        phin = Phi @ n                                    # (n_u, |I_k|)
        # rows i_u, cols (alpha, m)
        term = np.einsum("ib,ab->ia", phin, Gf)           # (n_u, |I_k|) over alpha
        Bus -= np.einsum("ia,m->iam", term, snn).reshape(n_u, nfull)
    # B_uhat_sigma = - int_dT sigma_nt . uhat_t  (uhat tangential -> (sigma n).uhat)
    n_hat = dims["n_hat"]
    Bhs = np.zeros(((d + 1) * n_hat, nfull))
    for i in range(nv):
        n = ed.normals_out[i]
        Gf = facet_product_moments(nv, k, k - 1, i) * ed.areas[i]    # (|I_k|, |I_{k-1}|)
        for j in range(n_hat):
            V = ed.Vhat[i, j]                                          # (|I_{k-1}|, d)
            # sum_gamma,r  (D_m n)_r V[gamma, r] * Gf[alpha, gamma]
            Dn = np.einsum("mrs,s->mr", Dm, n)                          # (m, r)
            val = -np.einsum("ag,gr,mr->am", Gf, V, Dn)
            Bhs[i * n_hat + j] = val.reshape(nfull)
    # restrict to Sigma_h(T)
    Mss = Z.T @ Mfull @ Z

    # div of velocity basis, A^div, pressure coupling, pressure mass
    divphi = np.einsum("sab,ibs->ia", Dk, Phi)            # (n_u, |I_{k-1}|)
    Adiv = (nu / d) * vol * divphi @ G_m1m1 @ divphi.T
    B = -vol * (divphi @ G_m1m1).T                        # (n_p, n_u)
    Mp = (vol / nu) * G_m1m1

    n_A = dims["n_A"]
    Adiv_ext = np.zeros((n_A, n_A))
    Adiv_ext[:n_u, :n_u] = Adiv
    if k >= 2:
        Bws = Bws_full @ Z
        Bsig = np.vstack([Bus @ Z, Bhs @ Z])                 # (n_A, n_sig)
        n_sig, n_om = Z.shape[1], Bws.shape[0]
        assert n_om == dims["n_om"]
        M = np.block([[-Mss, Bws.T], [Bws, np.zeros((n_om, n_om))]])
        Bfull = np.hstack([Bsig, np.zeros((Bsig.shape[0], n_om))])
        A = Adiv_ext - Bfull @ np.linalg.solve(M, Bfull.T)
    else:
        # k = 1 (Sec. 7): omega in the Raviart-Thomas space, kappa(omega) in
        # place of omega, so only sigma is condensed; omega's facet fluxes
        # stay in the system beside (u, uhat), with the stabilisation
        # nu h_T^2 (div omega, div eta)_T with h_T = |T|^(1/3): a weight
        # that keeps the term bounded by the lowest-order norm of Sec. 7
        # (||div omega||_T <~ h_T^-1 ||omega||_T), so that the facet block
        # smoother and E of the preconditioner stay robust in h.  With the
        # sigma rows
        # -M_ss sigma + B^T (u, uhat, omega) = 0 the condensed block is
        # A^div + B M_ss^{-1} B^T + stabilisation.
        Crt, divrt = rt0_basis(ed)
        Bw_full = np.zeros((nv, nfull))
        for i in range(nv):
            Kc = np.array([kappa(Crt[i, j]) for j in range(nv)])          # (|I_1|, d, d)
            DKc = np.einsum("mrs,brs->mb", Dm, Kc)                         # (m, beta)
            Bw_full[i] = vol * np.einsum("ab,mb->am", G_kk, DKc).reshape(nfull)
        Bws = Bw_full @ Z
        Bsig = np.vstack([Bus @ Z, Bhs @ Z, Bws])            # (n_A, n_sig)
        Adiv_ext[n_A - nv:, n_A - nv:] = nu * vol ** (2.0 / 3.0) * vol * np.outer(divrt, divrt)
        A = Adiv_ext + Bsig @ np.linalg.solve(Mss, Bsig.T)
    A = 0.5 * (A + A.T)
    for p in pinned:
        A[p, :] = 0.0
        A[:, p] = 0.0
        A[p, p] = 1.0

    F = None
    if f_lattice_sorted is not None:
        Lc = lattice_bernstein(d, m, lattice_sorted)      # (|I_m|, n_lat)
        fc = Lc @ f_lattice_sorted                        # (|I_m|, d)
        G_mk = product_moments(nv, m, k)
        F = vol * np.einsum("ar,ab,ibr->i", fc, G_mk, Phi)

    # reorder: [bubbles | per facet (normal fns, tangential fns[, omega flux])]
    nb, nF = dims["n_bub"], dims["n_F"]
    perm = list(range(nb))
    for i in range(nv):
        perm += list(range(nb + i * nF, nb + (i + 1) * nF))
        perm += list(range(n_u + i * n_hat, n_u + (i + 1) * n_hat))
        if dims["n_w"]:
            perm.append(n_u + nv * n_hat + i)
    perm = np.asarray(perm)
    Ar = A[np.ix_(perm, perm)]
    Aoo = Ar[:nb, :nb]
    Aod = Ar[:nb, nb:]
    Add = Ar[nb:, nb:]
    H = np.linalg.solve(Aoo, Aod) if nb else np.zeros((0, Add.shape[0]))
    Ad = Add - Aod.T @ H
    Ad = 0.5 * (Ad + Ad.T)
    out = dict(ed=ed, A=A, B=B, Adiv=Adiv, Mp=Mp, F=F, perm=perm,
               Aoo=Aoo, Aod=Aod, H=H, Ad=Ad, dims=dims)
    if keep_blocks:
        out.update(Z=Z, Mss=Mss, Bws=Bws, Bsig=Bsig, Dm=Dm, Kn=Kn)
    return out


def recover_stress(ed, nu, k, u_local):
    """Stress and vorticity of one element from its velocity (Sec. 4.2: after
    the condensed solve, sigma_h and omega_h follow from the local problems
    eq. projection).  With M and B_sigma of eq. bigfemSPmat the element rows
    read M (sigma, omega) + B_sigma^T (u, uhat) = 0, so
    (sigma, omega) = -M^{-1} B_sigma^T (u, uhat).

    u_local: velocity coefficients in the local order of the matrix 'A'
    ([Phi | Vhat]).  Returns coefficient arrays over lambda^alpha (sorted
    vertices): S (|I_k|, d, d) for sigma_h and W (|I_{k-1}|, d, d) for
    omega_h (k = 1: W (|I_1|, d, d), the skew field kappa(omega_h))."""
    if k == 1:
        # Sec. 7: only sigma is local; -M_ss sigma + B^T (u, uhat, omega) = 0,
        # and omega is the Raviart-Thomas field of its facet fluxes (returned
        # as kappa(omega), degree 1)
        es = element_system(ed, nu, k, keep_blocks=True)
        Z, Mss, Bsig, Dm = es["Z"], es["Mss"], es["Bsig"], es["Dm"]
        ul = np.asarray(u_local, dtype=np.float64)
        sig = np.linalg.solve(Mss, Bsig.T @ ul)
        cs = (Z @ sig).reshape(ed.d + 1, len(Dm))
        S = np.einsum("am,mrs->ars", cs, Dm)
        Crt, _ = rt0_basis(ed)
        n_u, n_hat = ed.dims["n_u"], ed.dims["n_hat"]
        wdof = ul[n_u + (ed.d + 1) * n_hat:]
        W = np.array([kappa(wdof @ Crt[:, j]) for j in range(ed.d + 1)])
        return S, W
    es = element_system(ed, nu, k, keep_blocks=True)
    Z, Mss, Bws, Bsig, Dm, Kn = es["Z"], es["Mss"], es["Bws"], es["Bsig"], es["Dm"], es["Kn"]
    n_sig, n_om = Z.shape[1], Bws.shape[0]
    M = np.block([[-Mss, Bws.T], [Bws, np.zeros((n_om, n_om))]])
    rhs = np.concatenate([Bsig.T @ np.asarray(u_local, dtype=np.float64), np.zeros(n_om)])
    sol = -np.linalg.solve(M, rhs)
    n_I = len(multi_indices(ed.d + 1, k))
    cs = (Z @ sol[:n_sig]).reshape(n_I, len(Dm))           # (alpha, m)
    S = np.einsum("am,mrs->ars", cs, Dm)
    cw = sol[n_sig:].reshape(-1, len(Kn))                    # (gamma, n)
    W = np.einsum("gn,nrs->grs", cw, Kn)
    return S, W
