"""Global condensed saddle system K (eq. femSPmat) and its direct solution -- oracle.

Global vector layout (free degrees of freedom only, all of dOmega is Dirichlet):

    [ u_o : element-major, n_bub per element                        ]
    [ facet blocks : free facets in canonical order, each block is   ]
    [                (n_F normal-moment dofs, n_hat tangential dofs) ]
    [ p   : element-major, n_p per element                           ]

K = [[A, B^T], [B, 0]] with A the sigma/omega-condensed velocity block
(Sec. 4.2) and B the pressure coupling -(div u, q) (weak-form sign of eq.
discrmixedstressstokesweak).  The pressure is unique up to a constant when all
of the boundary is Dirichlet (Sec. 1); the direct solve fixes int p = 0 with a
Lagrange multiplier.  With an outlet Gamma_NT (eq. stokes_NT) it is unique.

Boundary conditions (eq. stokes_D, stokes_NT): faces of the bounding box are
Dirichlet (default) or outlets.  On an outlet facet the normal dofs are free
and the tangential dofs are fixed to zero (u_t = 0): they stay in the vector
layout with identity rows in K.  Dirichlet data g (values on the element
lattices, like f) is lifted: its facet dofs are the L2 projections of g.n_F
onto the normal traces and of g_t onto V-hat(F), and b -= K x_D.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import element_geometry, element_system, expected_dims
from .poly import multi_indices, simplex_moment
from .topology import Topology


def _lattice_indices(d, m):
    return np.asarray(multi_indices(d + 1, m), dtype=np.int64)


class GlobalSystem:
    def __init__(self, vertices, elements, nu, k, f_lattice=None, m=None, face_bc=None, g_lattice=None,
                 sigma_rotation_seed=None):
        self.topo = topo = Topology(vertices, elements, face_bc)
        d = self.d = topo.dim
        self.k = k
        n_e = topo.elements.shape[0]
        self.n_e = n_e
        nu = np.broadcast_to(np.asarray(nu, dtype=np.float64), (n_e,))
        self.nu = np.array(nu)
        dims = self.dims = expected_dims(d, k)
        self.nb, self.nF, self.nh, self.nfb = dims["n_bub"], dims["n_F"], dims["n_hat"], dims["n_fb"]
        self.np_ = dims["n_p"]
        self.off_f = n_e * self.nb
        self.off_p = self.off_f + topo.n_free_facets * self.nfb
        self.n_dof = self.off_p + n_e * self.np_
        self.m = m if m is not None else k + 1
        lat = _lattice_indices(d, self.m)

        self.elems = []
        self.xD = []
        n_u, nh = dims["n_u"], dims["n_hat"]
        for e in range(n_e):
            X = topo.element_coords(e)
            ed = element_geometry(X, k)
            fl = ls = None
            if f_lattice is not None:
                fl = np.asarray(f_lattice[e], dtype=np.float64)
                ls = lat[:, topo.perm[e]]
            pinned = [n_u + i * nh + j for i in range(d + 1) if topo.facet_outlet[topo.elem_facets[e, i]]
                      for j in range(nh)]
            es = element_system(ed, self.nu[e], k, fl, ls, self.m, pinned=pinned,
                                sigma_rotation_seed=sigma_rotation_seed)
            self.elems.append(es)
            xd = np.zeros(dims["n_A"])
            if g_lattice is not None:
                for i in range(d + 1):
                    if topo.facet_dirichlet[topo.elem_facets[e, i]]:
                        self._lift_facet(ed, np.asarray(g_lattice[e], dtype=np.float64), lat[:, topo.perm[e]], i, xd)
            self.xD.append(xd)

    def _lift_facet(self, ed, g_lat, lat_sorted, i, xd):
        """Dirichlet dofs of local facet i from g (values on the element
        lattice): the normal dofs c with sum_beta c_beta lambda^beta/|F| =
        L2 projection of g.n_F onto P^k(F), and the tangential dofs as the L2
        projection of g_t onto V-hat(F)."""
        from .element import lattice_bernstein
        from .poly import facet_product_moments
        d, k, m = self.d, self.k, self.m
        nv = d + 1
        gc = lattice_bernstein(d, m, lat_sorted) @ g_lat              # (|I_m|, d) over lambda^alpha
        nF, nb = self.nF, self.nb
        n_u = self.dims["n_u"]
        area = ed.areas[i]
        # normal part: rows beta of the facet functions of facet i (|beta| = k on the facet)
        Gmk = facet_product_moments(nv, m, k, i) * area               # int_F lambda^alpha lambda^beta
        Gkk = facet_product_moments(nv, k, k, i) * area
        Ik = multi_indices(nv, k)
        on = [j for j, a in enumerate(Ik) if a[i] == 0]                # facet monomials, lex-descending
        rhs = (gc @ ed.normals_geo[i]) @ Gmk[:, on]
        a = np.linalg.solve(Gkk[np.ix_(on, on)], rhs)
        xd[nb + i * nF: nb + (i + 1) * nF] = area * a
        # tangential part
        Gmk1 = facet_product_moments(nv, m, k - 1, i) * area
        Gk1 = facet_product_moments(nv, k - 1, k - 1, i) * area
        V = ed.Vhat[i]                                                 # (n_hat, |I_{k-1}|, d)
        Mf = np.einsum("jgr,gh,lhr->jl", V, Gk1, V)
        rf = np.einsum("ar,ag,jgr->j", gc, Gmk1, V)
        xd[n_u + i * self.nh: n_u + (i + 1) * self.nh] = np.linalg.solve(Mf, rf)
        if self.dims["n_w"]:
            # k = 1: the flux of curl g through F w.r.t. n_F (the value of
            # omega = curl u on the boundary, Sec. 7)
            from .poly import gradient_matrices
            D = gradient_matrices(nv, m, ed.grad_lambda)               # (d, |I_{m-1}|, |I_m|)
            G = np.einsum("sab,br->ars", D, gc)                        # d g_r / d x_s
            curl = np.stack([G[:, 2, 1] - G[:, 1, 2], G[:, 0, 2] - G[:, 2, 0], G[:, 1, 0] - G[:, 0, 1]], axis=1)
            mom = facet_product_moments(nv, m - 1, 0, i)[:, 0] * area
            xd[n_u + nv * self.nh + i] = mom @ (curl @ ed.normals_geo[i])

    # ------------------------------------------------------------------ maps
    def local_dofs(self, e):
        """Global indices of the reordered local velocity dofs of element e
        ([bubbles | facet blocks]); -1 marks Dirichlet dofs."""
        nb, nfb = self.nb, self.nfb
        out = list(range(e * nb, (e + 1) * nb))
        for i in range(self.d + 1):
            g = self.topo.free_facet_of[self.topo.elem_facets[e, i]]
            if g < 0:
                out += [-1] * nfb
            else:
                out += list(range(self.off_f + g * nfb, self.off_f + (g + 1) * nfb))
        return np.asarray(out, dtype=np.int64)

    def facet_dofs(self, g):
        return np.arange(self.off_f + g * self.nfb, self.off_f + (g + 1) * self.nfb)

    def pressure_dofs(self, e):
        return np.arange(self.off_p + e * self.np_, self.off_p + (e + 1) * self.np_)

    def u_to_reordered(self, e):
        """Map original local u index (bubbles, facet fns) -> reordered position."""
        perm = self.elems[e]["perm"]
        inv = np.empty(len(perm), dtype=np.int64)
        inv[perm] = np.arange(len(perm))
        return inv[: self.dims["n_u"]]

    # --------------------------------------------------------------- assembly
    def _scatter(self, blocks):
        rows, cols, vals = [], [], []
        for (gr, gc, M) in blocks:
            mr = gr >= 0
            mc = gc >= 0
            sub = M[np.ix_(mr, mc)]
            R, C = np.meshgrid(gr[mr], gc[mc], indexing="ij")
            rows.append(R.ravel())
            cols.append(C.ravel())
            vals.append(sub.ravel())
        r = np.concatenate(rows)
        c = np.concatenate(cols)
        v = np.concatenate(vals)
        return sp.csr_matrix((v, (r, c)), shape=(self.n_dof, self.n_dof))

    def assemble_K(self):
        blocks = []
        for e, es in enumerate(self.elems):
            ld = self.local_dofs(e)
            perm = es["perm"]
            blocks.append((ld, ld, es["A"][np.ix_(perm, perm)]))
            pd = self.pressure_dofs(e)
            Bl = np.zeros((self.np_, len(ld)))
            Bl[:, self.u_to_reordered(e)] = es["B"]
            blocks.append((pd, ld, Bl))
            blocks.append((ld, pd, Bl.T))
        return self._scatter(blocks)

    def assemble_rhs(self):
        """Load vector minus K x_D (the lifted Dirichlet data)."""
        b = np.zeros(self.n_dof)
        for e, es in enumerate(self.elems):
            ld = self.local_dofs(e)
            perm = es["perm"]
            loc = np.zeros(len(ld))
            loc[self.u_to_reordered(e)] = es["F"]
            xd = self.xD[e]
            if np.any(xd):
                loc -= (es["A"] @ xd)[perm]
                b[self.pressure_dofs(e)] -= es["B"] @ xd[: self.dims["n_u"]]
            msk = ld >= 0
            np.add.at(b, ld[msk], loc[msk])
        return b

    def pressure_mean_functional(self):
        """c with c.x = int_Omega p_h (p basis lambda^gamma, |gamma| = k-1)."""
        d = self.d
        Ig = multi_indices(d + 1, self.k - 1)
        mom = np.array([simplex_moment(g) for g in Ig])
        c = np.zeros(self.n_dof)
        for e, es in enumerate(self.elems):
            c[self.pressure_dofs(e)] = es["ed"].vol * mom
        return c

    def constant_pressure(self):
        """Coefficient vector of p = 1 (sum of multinomial coefficients)."""
        Ig = multi_indices(self.d + 1, self.k - 1)
        coef = np.array([math.factorial(self.k - 1) / np.prod([math.factorial(a) for a in g])
                         for g in Ig])
        c = np.zeros(self.n_dof)
        for e in range(self.n_e):
            c[self.pressure_dofs(e)] = coef
        return c

    def normalize_pressure(self, x):
        """Subtract the mean of p_h (Sec. 1: p unique up to a constant); with
        an outlet the pressure is unique and x is returned unchanged."""
        if self.topo.has_outlet:
            return x
        c = self.pressure_mean_functional()
        area = sum(es["ed"].vol for es in self.elems)
        mean = (c @ x) / area
        return x - mean * self.constant_pressure()

    def direct_solve(self, b=None):
        K = self.assemble_K()
        if b is None:
            b = self.assemble_rhs()
        if self.topo.has_outlet:
            return spla.splu(K.tocsc()).solve(b)
        c = self.pressure_mean_functional()
        Kc = sp.bmat([[K, sp.csr_matrix(c[:, None])], [sp.csr_matrix(c[None, :]), None]],
                     format="csc")
        rhs = np.concatenate([b, [0.0]])
        x = spla.splu(Kc).solve(rhs)
        return x[:-1]

    # ------------------------------------------------------------- evaluation
    def eval_element(self, x, e, lam):
        """Values (u, p) of the discrete solution in element e at barycentric
        points lam (n, d+1) w.r.t. the sorted vertices."""
        from .poly import evaluate
        es = self.elems[e]
        ed = es["ed"]
        ld = self.local_dofs(e)
        perm = es["perm"]
        coef = np.where(ld >= 0, x[np.maximum(ld, 0)], 0.0) + self.xD[e][perm]
        u_coef_reordered = coef
        orig = np.zeros(len(perm))
        orig[perm] = u_coef_reordered
        cu = orig[: self.dims["n_u"]]
        field = np.tensordot(cu, ed.Phi, axes=(0, 0))           # (|I_k|, d)
        u = evaluate(field, self.d + 1, self.k, lam)
        cp = x[self.pressure_dofs(e)]
        p = evaluate(cp, self.d + 1, self.k - 1, lam)
        return u, p

    def local_velocity(self, x, e):
        """Velocity coefficients of element e in the local order of its matrix
        'A' ([Phi | Vhat]); Dirichlet dofs are zero."""
        ld = self.local_dofs(e)
        coef = np.where(ld >= 0, x[np.maximum(ld, 0)], 0.0)
        orig = np.zeros(len(ld))
        orig[self.elems[e]["perm"]] = coef
        return orig + self.xD[e]

    def eval_stress_element(self, x, e, lam):
        """Values (sigma_h, omega_h) recovered in element e (eq. projection) at
        barycentric points lam (n, d+1) w.r.t. the sorted vertices; each of
        shape (n, d, d)."""
        from .element import recover_stress
        from .poly import evaluate
        es = self.elems[e]
        S, W = recover_stress(es["ed"], self.nu[e], self.k, self.local_velocity(x, e))
        return evaluate(S, self.d + 1, self.k, lam), evaluate(W, self.d + 1, max(self.k - 1, 1), lam)
