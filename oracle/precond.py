"""Block preconditioner for K with the multiplicative auxiliary-space preconditioner
for the double Schur complement A^d -- oracle (FP64, sequential).

* K-hat^{-1} (eq. mhatinvfactor, with its top-right block read as -A-hat^{-1} B^T
  and the pressure block +S-hat^{-1}, S-hat = M_p the nu^{-1}-scaled pressure
  mass matrix, Sec. 5.1), applied with two A-hat^{-1} applications.
* A-hat_ext (Sec. 6.1 "Preconditioning via the condense system"): A through its
  bubble factorisation (eq. factorSsigma) with A^d replaced by A-hat^d_m.
* A-hat^d_m (Theorem aux_pc_schur with Corollary aux_pc_mult and the
  multiplicative ASP of Sec. 5.2): block Gauss-Seidel over facet blocks (one
  block per free facet holding its normal and tangential dofs), s sweeps in
  colour order, then the coarse correction E^d C^{-1} E^d^T on the residual,
  then s sweeps in reverse colour order (the adjoint smoother).
* Additive variant (Sec. 5.2, the additive auxiliary-space preconditioner of
  Theorem aux_pc_schur): A-hat^d_a^{-1} = D^{-1} + E^d C^{-1} E^d^T with D the
  facet block Jacobi preconditioner, one block D_F per free facet.
* l1 variant (the l1 block smoothers of the numerics of Sec. 8, in the
  multiplicative ASP of Sec. 5.2): the facet block Gauss-Seidel sweeps are
  replaced by facet block l1-Jacobi sweeps x += M^{-1} (s - A^d x) with
  M = blockdiag(M_F), M_F = D_F + diag(l_F), l_i = sum over the free facet
  dofs j outside the block of i of |a_ij| sqrt(a_ii / a_jj): the l1 row sums
  of the diagonally scaled S^{-1} A^d S^{-1} (S = diag(A^d)^{1/2}) taken back
  to the unscaled dofs, so that M does not depend on the scaling of the basis
  (normal and tangential facet dofs scale differently in h).  A^d <= M.
* Full-system variant (Sec. 5.2, Theorem aux_pc with the Gauss-Seidel form of
  Corollary aux_pc_mult; the paper's Table ST_full_vs_cond compares it with the
  condensed one): A-hat is applied to the whole velocity block A without the
  bubble factorisation.  Overlapping blocks, one per facet F of the mesh
  (Dirichlet facets included), each holding the free dofs of F and the bubble
  dofs of the elements adjacent to F; s block Gauss-Seidel sweeps in colour
  order (a greedy colouring of all facets in canonical order in which facets
  of one element differ), the coarse correction E C^{-1} E^T with the full
  embedding (bubble rows included), s sweeps in reverse colour order.
* E^d: rows of the embedding E u = (u, u_t) of continuous P1 (eq. defE) for the
  facet dofs (eq. defED).  For k = 1 (Sec. 7) E u = (u, Pi^0 u_t, curl u): the
  facet mean of the tangential trace and the flux of curl u through the facet.
* C: one symmetric V(1,1) multigrid cycle for A-bar, the P1 form
  a(u, v) = nu int eps(u) : eps(v) (eq. defAhat, read with nu, not nu^{-1}),
  on the vertex lattice: coarse points every second index per axis plus the
  last one, linear interpolation in index space, Galerkin coarse operators,
  l1-Jacobi smoothing with d x d vertex blocks, a dense Cholesky solve on the
  coarsest level (free dofs <= coarse_max or <= 2 intervals on some axis).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .poly import elevate_to, multi_indices


# ---------------------------------------------------------------------------
# P1 space and multigrid
# ---------------------------------------------------------------------------

def p1_element_matrix(ed, nu):
    """A-bar_T[(v,c),(w,e)] = nu int_T eps(lambda_v e_c) : eps(lambda_w e_e)."""
    d = ed.d
    gl = ed.grad_lambda
    n = (d + 1) * d
    A = np.zeros((n, n))
    for v in range(d + 1):
        for c in range(d):
            Ev = 0.5 * (np.outer(np.eye(d)[c], gl[v]) + np.outer(gl[v], np.eye(d)[c]))
            for w in range(d + 1):
                for e in range(d):
                    Ew = 0.5 * (np.outer(np.eye(d)[e], gl[w]) + np.outer(gl[w], np.eye(d)[e]))
                    A[v * d + c, w * d + e] = nu * ed.vol * np.sum(Ev * Ew)
    return A


def coarse_points(n):
    """Coarse lattice positions (fine indices) for n intervals: 0, 2, 4, ... plus n."""
    pts = list(range(0, n + 1, 2))
    if pts[-1] != n:
        pts.append(n)
    return pts


def interp_1d(n):
    """(n+1) x (n_c+1) linear interpolation in index space."""
    cp = coarse_points(n)
    P = np.zeros((n + 1, len(cp)))
    cset = {c: j for j, c in enumerate(cp)}
    for i in range(n + 1):
        if i in cset:
            P[i, cset[i]] = 1.0
        else:
            P[i, cset[i - 1]] = 0.5
            P[i, cset[i + 1]] = 0.5
    return P


def kept_indices(n, lo_free, hi_free):
    """Lattice indices 0..n of one axis that carry P1 dofs: the interior ones,
    plus an end whose face is an outlet (not Dirichlet)."""
    return ([0] if lo_free else []) + list(range(1, n)) + ([n] if hi_free else [])


class P1Multigrid:
    def __init__(self, Abar, lattice, d, coarse_max=512, face_bc=None):
        """Abar over the free lattice vertices, dof = d*free_vertex + c: the
        interior ones, plus those on outlet faces (face_bc[2a + side] == 1)
        that lie on no Dirichlet face."""
        self.d = d
        fb = np.zeros(2 * d, dtype=int) if face_bc is None else np.asarray(face_bc)
        self.levels = []
        dims = [n - 1 for n in lattice]          # intervals per axis
        A = Abar.tocsr()
        while True:
            lvl = {"A": A, "dims": dims}
            self.levels.append(lvl)
            nfree = A.shape[0]
            if nfree <= coarse_max or min(dims) <= 2:
                lvl["chol"] = sla.cho_factor(A.toarray())
                break
            lvl["Dinv"] = self._l1_block_inverse(A)
            # prolongation restricted to the free points, tensor product (x fastest)
            Ps = []
            for a, n in enumerate(dims):
                nc = len(coarse_points(n)) - 1
                Ps.append(interp_1d(n)[np.ix_(kept_indices(n, fb[2 * a], fb[2 * a + 1]),
                                              kept_indices(nc, fb[2 * a], fb[2 * a + 1]))])
            P = sp.csr_matrix(Ps[0])
            for Pa in Ps[1:]:
                P = sp.kron(sp.csr_matrix(Pa), P, format="csr")
            P = sp.kron(P, sp.identity(d), format="csr")
            lvl["P"] = P
            A = (P.T @ A @ P).tocsr()
            dims = [len(coarse_points(n)) - 1 for n in dims]

    def _l1_block_inverse(self, A):
        d = self.d
        A = A.tocsr()
        nv = A.shape[0] // d
        Dinv = np.zeros((nv, d, d))
        absA = abs(A)
        for v in range(nv):
            rows = slice(v * d, (v + 1) * d)
            blk = A[rows, rows].toarray()
            rowsum = np.asarray(absA[rows, :].sum(axis=1)).ravel()
            inblock = np.abs(blk).sum(axis=1)
            Dv = blk + np.diag(rowsum - inblock)
            Dinv[v] = np.linalg.inv(Dv)
        return Dinv

    def _jacobi(self, lvl, r):
        """Block l1-Jacobi step; r is a vector or a matrix of columns."""
        d = self.d
        if r.ndim == 1:
            return np.einsum("vab,vb->va", lvl["Dinv"], r.reshape(-1, d)).ravel()
        m = r.shape[1]
        return np.einsum("vab,vbm->vam", lvl["Dinv"], r.reshape(-1, d, m)).reshape(-1, m)

    def vcycle(self, b, level=0):
        lvl = self.levels[level]
        if "chol" in lvl:
            return sla.cho_solve(lvl["chol"], b)
        A = lvl["A"]
        x = self._jacobi(lvl, b)
        r = b - A @ x
        x = x + lvl["P"] @ self.vcycle(lvl["P"].T @ r, level + 1)
        x = x + self._jacobi(lvl, b - A @ x)
        return x


# ---------------------------------------------------------------------------
# embedding E, E^d
# ---------------------------------------------------------------------------

def p1_in_element_basis(es, v_local, c):
    """Coefficients of lambda_v e_c (a P1 field on the element) in the element's
    BDM basis (original order) and, per facet, in the tangential basis of its
    tangential trace (eq. defE: E u = (u, u_t))."""
    ed = es["ed"]
    d, k = ed.d, ed.k
    nv = d + 1
    lin = np.zeros((nv, d))
    lin[v_local, c] = 1.0                       # coefficients over I_1 = {e_v}
    # I_1 in lex-descending order is e_0, e_1, ..., e_d
    target = elevate_to(lin, nv, 1, k)          # (|I_k|, d)
    Phi = ed.Phi                                # (n_u, |I_k|, d)
    M = Phi.reshape(Phi.shape[0], -1).T
    cu, *_ = np.linalg.lstsq(M, target.ravel(), rcond=None)
    assert np.allclose(M @ cu, target.ravel(), atol=1e-10 * max(1.0, np.abs(target).max()))
    ch = []
    if k == 1:
        # Sec. 7: the tangential trace of a P1 field is not in hat V_h (P^0):
        # E takes its facet mean Pi^0 (the L2 projection onto constants)
        for i in range(nv):
            n = ed.normals_out[i]
            Pt = np.eye(d) - np.outer(n, n)
            mean = (0.0 if v_local == i else 1.0 / d) * np.eye(d)[c]
            V = ed.Vhat[i][:, 0, :]                 # (n_hat, d): the tangents t_b
            chi, *_ = np.linalg.lstsq(V.T, Pt @ mean, rcond=None)
            assert np.allclose(V.T @ chi, Pt @ mean, atol=1e-12)
            ch.append(chi)
        return cu, ch
    tgt_t = elevate_to(lin, nv, 1, k - 1)       # (|I_{k-1}|, d)
    Ikm1 = multi_indices(nv, k - 1)
    for i in range(nv):
        n = ed.normals_out[i]
        Pt = np.eye(d) - np.outer(n, n)
        msk = np.array([a[i] == 0 for a in Ikm1])
        tgt = (tgt_t @ Pt.T)[msk]               # tangential part on facet i
        V = ed.Vhat[i][:, msk, :]               # (n_hat, n_fac, d)
        Mv = V.reshape(V.shape[0], -1).T
        chi, *_ = np.linalg.lstsq(Mv, tgt.ravel(), rcond=None)
        assert np.allclose(Mv @ chi, tgt.ravel(), atol=1e-10 * max(1.0, np.abs(tgt).max()))
        ch.append(chi)
    return cu, ch


def embedding(gs, full=False):
    """Sparse E (n_dof_velocity x n_P1) for the free P1 dofs.  With full=False
    only the facet rows (E^d) are nonzero; with full=True also the bubble rows.
    Facet rows are computed from the first neighbour of each facet; the test
    suite checks that the other neighbour gives the same rows."""
    topo = gs.topo
    d = gs.d
    rows, cols, vals = [], [], []
    done_facet = np.zeros(topo.n_free_facets, dtype=bool)
    nb, nF, nh = gs.nb, gs.nF, gs.nh
    for e in range(gs.n_e):
        es = gs.elems[e]
        verts = topo.elements[e]
        for vl in range(d + 1):
            fvi = topo.free_vertex_of[verts[vl]]
            if fvi < 0:
                continue
            for c in range(d):
                col = d * fvi + c
                cu, ch = p1_in_element_basis(es, vl, c)
                if full:
                    for j in range(nb):
                        rows.append(e * nb + j); cols.append(col); vals.append(cu[j])
                for i in range(d + 1):
                    g = topo.free_facet_of[topo.elem_facets[e, i]]
                    if g < 0 or done_facet[g]:
                        continue
                    base = gs.off_f + g * gs.nfb
                    for q in range(nF):
                        rows.append(base + q); cols.append(col); vals.append(cu[nb + i * nF + q])
                    if not topo.free_outlet[g]:  # pi_0: no tangential rows on outlets
                        for q in range(nh):
                            rows.append(base + nF + q); cols.append(col); vals.append(ch[i][q])
                    if gs.dims["n_w"]:
                        # k = 1 (Sec. 7): the omega component curl(u-bar); its
                        # flux through F w.r.t. n_F, |F| (grad lambda_v x e_c) . n_F
                        ed = es["ed"]
                        cv = np.cross(ed.grad_lambda[vl], np.eye(d)[c])
                        rows.append(base + nF + nh); cols.append(col)
                        vals.append(ed.areas[i] * cv @ ed.normals_geo[i])
        for i in range(d + 1):
            g = topo.free_facet_of[topo.elem_facets[e, i]]
            if g >= 0:
                done_facet[g] = True
    n_p1 = d * len(topo.free_vertices)
    E = sp.coo_matrix((vals, (rows, cols)), shape=(gs.n_dof, n_p1)).tocsr()
    E.sum_duplicates()
    return E


# Tangential penalty of A-bar on outlet facets (Lemma outflow): nu C k^2 / h with
# h = d |T| / |F| the height of the element over the facet.
OUTLET_PENALTY = 8.0


def p1_outlet_penalty(ed, nu, k, i):
    """nu C k^2/h int_F (lambda_v e_c)_t . (lambda_w e_e)_t over local facet i,
    as a ((d+1)d)^2 element block (zero outside the facet's vertices)."""
    d = ed.d
    n = ed.normals_out[i]
    Pt = np.eye(d) - np.outer(n, n)
    h = d * ed.vol / ed.areas[i]
    cf = nu * OUTLET_PENALTY * k * k / h
    A = np.zeros(((d + 1) * d, (d + 1) * d))
    for v in range(d + 1):
        for w in range(d + 1):
            if v == i or w == i:
                continue
            mass = ed.areas[i] * (2.0 if v == w else 1.0) / (d * (d + 1))
            A[v * d:(v + 1) * d, w * d:(w + 1) * d] = cf * mass * Pt
    return A


def assemble_p1(gs):
    topo = gs.topo
    d = gs.d
    rows, cols, vals = [], [], []
    for e in range(gs.n_e):
        Ae = p1_element_matrix(gs.elems[e]["ed"], gs.nu[e])
        for i in range(d + 1):
            if topo.facet_outlet[topo.elem_facets[e, i]]:
                Ae = Ae + p1_outlet_penalty(gs.elems[e]["ed"], gs.nu[e], gs.k, i)
        idx = []
        for v in topo.elements[e]:
            fv = topo.free_vertex_of[v]
            for c in range(d):
                idx.append(d * fv + c if fv >= 0 else -1)
        idx = np.asarray(idx)
        m = idx >= 0
        R, C = np.meshgrid(idx[m], idx[m], indexing="ij")
        rows.append(R.ravel()); cols.append(C.ravel()); vals.append(Ae[np.ix_(m, m)].ravel())
    n = d * len(topo.free_vertices)
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


# ---------------------------------------------------------------------------
# the preconditioner
# ---------------------------------------------------------------------------

class Preconditioner:
    def __init__(self, gs, lattice, smoothing_steps=2, coarse_max=512, variant="multiplicative"):
        assert variant in ("multiplicative", "additive", "full", "l1")
        self.gs = gs
        topo = gs.topo
        d = gs.d
        self.steps = smoothing_steps
        self.variant = variant
        nfb = gs.nfb
        # assembled double Schur complement A^d on the facet dofs
        blocks_r, blocks_c, blocks_v = [], [], []
        for e, es in enumerate(gs.elems):
            ld = gs.local_dofs(e)[gs.nb:]
            m = ld >= 0
            R, C = np.meshgrid(ld[m], ld[m], indexing="ij")
            blocks_r.append(R.ravel()); blocks_c.append(C.ravel())
            blocks_v.append(es["Ad"][np.ix_(m, m)].ravel())
        self.Ad = sp.csr_matrix((np.concatenate(blocks_v), (np.concatenate(blocks_r),
                                 np.concatenate(blocks_c))), shape=(gs.n_dof, gs.n_dof))
        # facet block inverses D_F^{-1}
        self.Dinv = []
        for g in range(topo.n_free_facets):
            fd = gs.facet_dofs(g)
            D = self.Ad[fd][:, fd].toarray()
            self.Dinv.append(np.linalg.inv(D))
        self.colour_lists = [np.nonzero(topo.colour == c)[0] for c in range(topo.n_colours)]
        # auxiliary space
        self.E = embedding(gs, full=False)
        self.Abar = assemble_p1(gs)
        self.mg = P1Multigrid(self.Abar, lattice, d, coarse_max=coarse_max, face_bc=topo.face_bc)
        # element-local pressure mass inverses
        self.Mp_inv = [np.linalg.inv(es["Mp"]) for es in gs.elems]
        if variant == "full":
            self._setup_full()
        if variant == "l1":
            self._setup_l1()

    def _setup_l1(self):
        """l1 facet block Jacobi blocks M_F = D_F + diag(l_F) and their
        inverses.  For two free dofs i, j of different blocks the pair adds
        |a_ij| [[s_i/s_j, -sgn], [-sgn, s_j/s_i]] (s = sqrt(diag A^d)), a
        positive semidefinite 2 x 2 form, to M - A^d: hence A^d <= M."""
        gs, topo = self.gs, self.gs.topo
        Ad = self.Ad.tocsr()
        sq = np.sqrt(np.maximum(Ad.diagonal(), 0.0))
        blk = np.full(gs.n_dof, -1)
        for g in range(topo.n_free_facets):
            blk[gs.facet_dofs(g)] = g
        lsum = np.zeros(gs.n_dof)
        for i in range(gs.off_f, gs.off_p):
            for jj in range(Ad.indptr[i], Ad.indptr[i + 1]):
                j = Ad.indices[jj]
                if blk[j] != blk[i]:
                    lsum[i] += abs(Ad.data[jj]) * sq[i] / sq[j]
        self.l1_diag = lsum
        self.Minv = []
        for g in range(topo.n_free_facets):
            fd = gs.facet_dofs(g)
            M = Ad[fd][:, fd].toarray() + np.diag(lsum[fd])
            self.Minv.append(np.linalg.inv(M))

    def _setup_full(self):
        """Velocity block A, overlapping facet blocks and their inverses, the
        all-facet colouring and the full embedding (full-system variant)."""
        gs, topo = self.gs, self.gs.topo
        nb = gs.nb
        K = gs.assemble_K().tocsr()
        self.Afull = K[:gs.off_p][:, :gs.off_p].tocsr()
        self.blocks, self.Binv = [], []
        for f in range(topo.n_facets):
            g = topo.free_facet_of[f]
            dofs = list(gs.facet_dofs(g)) if g >= 0 else []
            for (t, _i) in topo.facet_neighbors[f]:
                dofs += list(range(t * nb, (t + 1) * nb))
            dofs = np.asarray(sorted(dofs), dtype=np.int64)
            self.blocks.append(dofs)
            self.Binv.append(np.linalg.inv(self.Afull[dofs][:, dofs].toarray()))
        # greedy colouring of all facets: facets of one element differ
        colour = -np.ones(topo.n_facets, dtype=np.int64)
        for f in range(topo.n_facets):
            used = {int(colour[f2]) for (t, _i) in topo.facet_neighbors[f] for f2 in topo.elem_facets[t]
                    if f2 != f and colour[f2] >= 0}
            c = 0
            while c in used:
                c += 1
            colour[f] = c
        self.full_colour = colour
        self.full_colour_lists = [np.nonzero(colour == c)[0] for c in range(int(colour.max()) + 1)]
        self.Efull = embedding(gs, full=True)

    def full_smooth(self, x, s, order):
        for c in order:
            for f in self.full_colour_lists[c]:
                B = self.blocks[f]
                r = s[B] - self.Afull[B] @ x[:self.gs.off_p]
                x[B] += self.Binv[f] @ r
        return x

    def A_full_inv(self, r):
        """A-hat^{-1} r of the full-system variant (velocity parts; x^0 = 0;
        s forward sweeps; coarse correction on the residual; s backward
        sweeps).  r is a vector or a matrix whose columns are treated alike."""
        gs = self.gs
        s = np.zeros(r.shape)
        s[:gs.off_p] = r[:gs.off_p]
        x = np.zeros(r.shape)
        nc = len(self.full_colour_lists)
        for _ in range(self.steps):
            x = self.full_smooth(x, s, range(nc))
        res = np.zeros(r.shape)
        res[:gs.off_p] = s[:gs.off_p] - self.Afull @ x[:gs.off_p]
        x = x + self.Efull @ self.mg.vcycle(self.Efull.T @ res)
        for _ in range(self.steps):
            x = self.full_smooth(x, s, range(nc - 1, -1, -1))
        x[gs.off_p:] = 0.0
        return x

    def A_hat_inv(self, r):
        """The A-hat^{-1} inside K-hat^{-1}: through the condensed system
        (A-hat_ext) or, for the full-system variant, directly."""
        return self.A_full_inv(r) if self.variant == "full" else self.A_ext_inv(r)

    # ---- pieces ---------------------------------------------------------
    def smooth(self, x, s, order):
        gs = self.gs
        for c in order:
            for g in self.colour_lists[c]:
                fd = gs.facet_dofs(g)
                r = s[fd] - self.Ad[fd] @ x
                x[fd] += self.Dinv[g] @ r
        return x

    def forward_sweep(self, x, s):
        return self.smooth(x, s, range(len(self.colour_lists)))

    def backward_sweep(self, x, s):
        return self.smooth(x, s, range(len(self.colour_lists) - 1, -1, -1))

    def aux_correction(self, r):
        return self.E @ self.mg.vcycle(self.E.T @ r)

    def Ad_mult_inv(self, s):
        """A-hat^d_m^{-1} s (x^0 = 0; s forward sweeps; coarse correction;
        s backward sweeps).  s and the result live on the facet dofs."""
        x = np.zeros_like(s)
        for _ in range(self.steps):
            x = self.forward_sweep(x, s)
        r = s - self.Ad @ x
        x = x + self.aux_correction(r)
        for _ in range(self.steps):
            x = self.backward_sweep(x, s)
        return x

    def block_jacobi(self, s):
        """D^{-1} s, facet block by facet block (the additive variant's smoother)."""
        gs = self.gs
        z = np.zeros_like(s)
        for g in range(gs.topo.n_free_facets):
            fd = gs.facet_dofs(g)
            z[fd] = self.Dinv[g] @ s[fd]
        return z

    def Ad_add_inv(self, s):
        """A-hat^d_a^{-1} s = D^{-1} s + E^d C^{-1} E^d^T s."""
        return self.block_jacobi(s) + self.aux_correction(s)

    def l1_jacobi(self, r):
        """M^{-1} r, facet block by facet block (the l1 variant's smoother)."""
        gs = self.gs
        z = np.zeros_like(r)
        for g in range(gs.topo.n_free_facets):
            fd = gs.facet_dofs(g)
            z[fd] = self.Minv[g] @ r[fd]
        return z

    def l1_sweep(self, x, s):
        """One l1-Jacobi sweep x + M^{-1} (s - A^d x)."""
        return x + self.l1_jacobi(s - self.Ad @ x)

    def Ad_l1_inv(self, s):
        """A-hat^d^{-1} s of the l1 variant: x^0 = 0; s l1-Jacobi sweeps; the
        coarse correction on the residual; s l1-Jacobi sweeps (the smoother is
        its own adjoint, so the operator is symmetric)."""
        x = np.zeros_like(s)
        for _ in range(self.steps):
            x = self.l1_sweep(x, s)
        x = x + self.aux_correction(s - self.Ad @ x)
        for _ in range(self.steps):
            x = self.l1_sweep(x, s)
        return x

    def Ad_inv(self, s):
        if self.variant == "additive":
            return self.Ad_add_inv(s)
        if self.variant == "l1":
            return self.Ad_l1_inv(s)
        return self.Ad_mult_inv(s)

    def A_ext_inv(self, r):
        """A-hat_ext^{-1} r for a velocity vector r (pressure part ignored/zero):
        s = r_d - sum_T H_T^T r_o,T;  t = A-hat^d_m^{-1} s;
        y_o,T = A_oo,T^{-1} r_o,T - H_T t_T;  y_d = t."""
        gs = self.gs
        nb = gs.nb
        s = np.zeros(gs.n_dof)
        s[gs.off_f:gs.off_p] = r[gs.off_f:gs.off_p]
        for e, es in enumerate(gs.elems):
            ro = r[e * nb:(e + 1) * nb]
            ld = gs.local_dofs(e)[nb:]
            m = ld >= 0
            contrib = es["H"].T @ ro
            np.add.at(s, ld[m], -contrib[m])
        t = self.Ad_inv(s)
        y = np.zeros(gs.n_dof)
        y[gs.off_f:gs.off_p] = t[gs.off_f:gs.off_p]
        for e, es in enumerate(gs.elems):
            ro = r[e * nb:(e + 1) * nb]
            ld = gs.local_dofs(e)[nb:]
            td = np.where(ld >= 0, t[np.maximum(ld, 0)], 0.0)
            y[e * nb:(e + 1) * nb] = np.linalg.solve(es["Aoo"], ro) - es["H"] @ td
        return y

    def B_apply(self, u):
        gs = self.gs
        out = np.zeros(gs.n_dof)
        for e, es in enumerate(gs.elems):
            ld = gs.local_dofs(e)
            ul = np.where(ld >= 0, u[np.maximum(ld, 0)], 0.0)
            uo = np.zeros(gs.dims["n_u"])
            uo[:] = ul[gs.u_to_reordered(e)]
            out[gs.pressure_dofs(e)] = es["B"] @ uo
        return out

    def BT_apply(self, p):
        gs = self.gs
        out = np.zeros(gs.n_dof)
        for e, es in enumerate(gs.elems):
            ld = gs.local_dofs(e)
            loc = np.zeros(len(ld))
            loc[gs.u_to_reordered(e)] = es["B"].T @ p[gs.pressure_dofs(e)]
            m = ld >= 0
            np.add.at(out, ld[m], loc[m])
        return out

    def Mp_inv_apply(self, r):
        gs = self.gs
        out = np.zeros(gs.n_dof)
        for e in range(gs.n_e):
            pd = gs.pressure_dofs(e)
            out[pd] = self.Mp_inv[e] @ r[pd]
        return out

    def apply(self, r):
        """K-hat^{-1} r:  a = A^{-1} r_u;  y_p = M_p^{-1}(r_p - B a);
        y_u = a - A^{-1} B^T y_p."""
        gs = self.gs
        ru = r.copy()
        ru[gs.off_p:] = 0.0
        a = self.A_hat_inv(ru)
        rp = np.zeros(gs.n_dof)
        rp[gs.off_p:] = r[gs.off_p:]
        yp = self.Mp_inv_apply(rp - self.B_apply(a))
        yu = a - self.A_hat_inv(self.BT_apply(yp))
        y = yu
        y[gs.off_p:] = yp[gs.off_p:]
        return y
