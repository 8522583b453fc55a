"""Seeded synthetic inputs for the MCS Stokes solver (shared by the oracle, the tests and bench).

This module holds NO arithmetic of the discretisation or of the solver.  It only
produces what a caller hands to the solver:

* structured simplicial meshes of the unit square / cube (vertex coordinates,
  element vertex lists in generation order, lattice dimensions);
* per-element viscosities nu_T;
* the body force f sampled at the principal lattice of degree m of every element
  (the representation of f that the solver interface takes), for manufactured
  solutions (problem statement, eq. (1.1) of the paper: -div(nu eps(u)) + grad p = f,
  div u = 0, with nu "the double of the kinematic viscosity");
* the exact (u, p) of the manufactured solutions, for error measurement.

Lattice convention (part of the solver interface): for an element with vertices
v_0..v_d *in the order given in the element list*, the lattice points of degree m
are x = sum_i (beta_i / m) v_i for all multi-indices beta in N^{d+1} with
|beta| = m, enumerated in lexicographically descending order
(beta_0 from m down to 0, then beta_1 from m - beta_0 down to 0, ...).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Mesh", "unit_square_mesh", "unit_cube_mesh", "box_mesh", "PlaneChannel", "lattice_indices",
    "lattice_points", "Manufactured2D", "CurlModes3D", "RandomForce",
    "lognormal_nu", "workload",
]


@dataclass
class Mesh:
    dim: int
    vertices: np.ndarray          # (n_v, dim) float64
    elements: np.ndarray          # (n_e, dim+1) int32, generation order
    lattice: tuple                # vertices per axis, e.g. (n+1, n+1, n+1)
    meta: dict = field(default_factory=dict)

    @property
    def n_vertices(self):
        return self.vertices.shape[0]

    @property
    def n_elements(self):
        return self.elements.shape[0]


def unit_square_mesh(n: int) -> Mesh:
    """n x n squares, each split by the diagonal (x_i,y_j)-(x_{i+1},y_{j+1}).

    Vertex (i, j) has index i + (n+1) j.  Square (i, j) (i fastest) gives the
    triangles (v00, v10, v11) and (v00, v11, v01)."""
    xs = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    els = []
    for j in range(n):
        for i in range(n):
            v00 = i + (n + 1) * j
            v10 = v00 + 1
            v01 = v00 + (n + 1)
            v11 = v01 + 1
            els.append((v00, v10, v11))
            els.append((v00, v11, v01))
    return Mesh(2, verts, np.asarray(els, dtype=np.int32), (n + 1, n + 1))


_PERMS3 = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def unit_cube_mesh(n: int) -> Mesh:
    """n^3 cubes, each split into the 6 Kuhn (Freudenthal) tetrahedra around the
    (0,0,0)-(1,1,1) diagonal.  Vertex (i, j, l) has index i + (n+1)(j + (n+1) l).
    Tetrahedron for axis permutation p: corner, +e_p0, +e_p0+e_p1, far corner."""
    xs = np.linspace(0.0, 1.0, n + 1)
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    N = n + 1

    def vid(i, j, l):
        return i + N * (j + N * l)

    els = []
    for l in range(n):
        for j in range(n):
            for i in range(n):
                for p in _PERMS3:
                    c = [i, j, l]
                    tet = [vid(*c)]
                    for ax in p:
                        c = list(c)
                        c[ax] += 1
                        tet.append(vid(*c))
                    els.append(tuple(tet))
    return Mesh(3, verts, np.asarray(els, dtype=np.int32), (N, N, N))


def box_mesh(cells, lengths) -> Mesh:
    """Box [0, L_0] x ... split like unit_square_mesh / unit_cube_mesh, with
    cells[a] intervals on axis a (vertex index: x fastest)."""
    d = len(cells)
    if d == 2:
        m = unit_square_like(cells)
    else:
        m = unit_cube_like(cells)
    m.vertices = m.vertices * np.asarray(lengths, dtype=np.float64)[None, :]
    return m


def unit_square_like(cells) -> Mesh:
    nx, ny = cells
    xs, ys = np.linspace(0.0, 1.0, nx + 1), np.linspace(0.0, 1.0, ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    els = []
    for j in range(ny):
        for i in range(nx):
            v00 = i + (nx + 1) * j
            v10, v01 = v00 + 1, v00 + (nx + 1)
            v11 = v01 + 1
            els.append((v00, v10, v11))
            els.append((v00, v11, v01))
    return Mesh(2, verts, np.asarray(els, dtype=np.int32), (nx + 1, ny + 1))


def unit_cube_like(cells) -> Mesh:
    nx, ny, nz = cells
    xs, ys, zs = (np.linspace(0.0, 1.0, n + 1) for n in cells)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def vid(i, j, l):
        return i + (nx + 1) * (j + (ny + 1) * l)

    els = []
    for l in range(nz):
        for j in range(ny):
            for i in range(nx):
                for p in _PERMS3:
                    c = [i, j, l]
                    tet = [vid(*c)]
                    for ax in p:
                        c = list(c)
                        c[ax] += 1
                        tet.append(vid(*c))
                    els.append(tuple(tet))
    return Mesh(3, verts, np.asarray(els, dtype=np.int32), (nx + 1, ny + 1, nz + 1))


@dataclass
class PlaneChannel:
    """Flow between the plates y = 0 and y = 1 of a box [0, L] x [0, 1] (x
    [0, 1]): u = (4 y (1 - y), 0[, 0]), p = 4 nu (L - x), f = 0.  It solves
    -div(nu eps(u)) + grad p = 0, div u = 0, with u = 0 on the plates, the
    profile itself as Dirichlet data on the inlet x = 0 (and on z = 0, 1 in
    3D), and on the outlet x = L: u_t = 0 and ((sigma + p I) n).n = p = 0."""
    dim: int
    nu: float = 1.0
    L: float = 1.0

    def u(self, X):
        X = np.asarray(X, dtype=np.float64)
        out = np.zeros(X.shape)
        out[..., 0] = 4.0 * X[..., 1] * (1.0 - X[..., 1])
        return out

    def p(self, X):
        X = np.asarray(X, dtype=np.float64)
        return 4.0 * self.nu * (self.L - X[..., 0])

    def f(self, X):
        return np.zeros(np.asarray(X).shape)

    def face_bc(self):
        """x- inlet (Dirichlet), x+ outlet, all other faces Dirichlet."""
        return [0, 1] + [0] * (2 * self.dim - 2)


def lattice_indices(dim: int, m: int):
    """Multi-indices beta in N^{dim+1}, |beta| = m, lexicographically descending."""
    def rec(nv, deg):
        if nv == 1:
            return [(deg,)]
        out = []
        for a in range(deg, -1, -1):
            for rest in rec(nv - 1, deg - a):
                out.append((a,) + rest)
        return out
    return np.asarray(rec(dim + 1, m), dtype=np.int64)


def lattice_points(mesh: Mesh, m: int) -> np.ndarray:
    """(n_e, n_lat, dim) coordinates of the degree-m lattice of every element."""
    B = lattice_indices(mesh.dim, m).astype(np.float64) / m      # (n_lat, d+1)
    V = mesh.vertices[mesh.elements]                              # (n_e, d+1, d)
    return np.einsum("lk,ekd->eld", B, V)


# ----------------------------------------------------------------------------
# manufactured solutions
# ----------------------------------------------------------------------------

class Manufactured2D:
    """u = curl psi = (d_y psi, -d_x psi) with psi = sin^2(pi x) sin^2(pi y),
    p = x - 1/2.  Constant nu, div u = 0, so f = -(nu/2) Lap u + grad p."""

    def __init__(self, nu: float = 1.0):
        self.nu = nu

    @staticmethod
    def _g(t):
        s = np.sin(np.pi * t)
        return s * s

    @staticmethod
    def _g1(t):
        return np.pi * np.sin(2 * np.pi * t)

    @staticmethod
    def _g2(t):
        return 2 * np.pi ** 2 * np.cos(2 * np.pi * t)

    @staticmethod
    def _g3(t):
        return -4 * np.pi ** 3 * np.sin(2 * np.pi * t)

    def u(self, x):
        X, Y = x[..., 0], x[..., 1]
        g, g1 = self._g, self._g1
        return np.stack([g(X) * g1(Y), -g1(X) * g(Y)], axis=-1)

    def lap_u(self, x):
        X, Y = x[..., 0], x[..., 1]
        g, g1, g2, g3 = self._g, self._g1, self._g2, self._g3
        lap_u1 = g2(X) * g1(Y) + g(X) * g3(Y)
        lap_u2 = -(g3(X) * g(Y) + g1(X) * g2(Y))
        return np.stack([lap_u1, lap_u2], axis=-1)

    def p(self, x):
        return x[..., 0] - 0.5

    def grad_p(self, x):
        out = np.zeros(x.shape, dtype=np.float64)
        out[..., 0] = 1.0
        return out

    def f(self, x):
        return -0.5 * self.nu * self.lap_u(x) + self.grad_p(x)


class CurlModes3D:
    """u = curl Psi, Psi = sum_{m=1}^{8} a_m prod_i sin^2(kappa_{m,i} pi x_i),
    a_m ~ N(0, I_3), kappa in {1, 2}; p = x + y + z - 3/2.  u vanishes on the
    boundary of the unit cube and is divergence free; f = -(nu/2) Lap u + grad p."""

    def __init__(self, seed: int = 2, n_modes: int = 8, nu: float = 1.0):
        rng = np.random.default_rng(seed)
        self.a = rng.standard_normal((n_modes, 3))
        self.kappa = rng.integers(1, 3, size=(n_modes, 3))
        self.nu = nu

    @staticmethod
    def _d(t, kap, order):
        w = kap * np.pi
        if order == 0:
            s = np.sin(w * t)
            return s * s
        if order == 1:
            return w * np.sin(2 * w * t)
        if order == 2:
            return 2 * w * w * np.cos(2 * w * t)
        if order == 3:
            return -4 * w ** 3 * np.sin(2 * w * t)
        raise ValueError(order)

    def _G(self, x, m, orders):
        """prod_i g_i^{(orders[i])}(x_i) for mode m."""
        out = np.ones(x.shape[:-1])
        for i in range(3):
            out = out * self._d(x[..., i], self.kappa[m, i], orders[i])
        return out

    def _curl_of(self, x, m, extra):
        """curl of a_m * D^extra G (extra = derivative multi-index added)."""
        a = self.a[m]
        def dG(j):
            o = list(extra)
            o[j] += 1
            return self._G(x, m, o)
        gx, gy, gz = dG(0), dG(1), dG(2)
        return np.stack([a[2] * gy - a[1] * gz,
                         a[0] * gz - a[2] * gx,
                         a[1] * gx - a[0] * gy], axis=-1)

    def u(self, x):
        out = np.zeros(x.shape, dtype=np.float64)
        for m in range(self.a.shape[0]):
            out += self._curl_of(x, m, (0, 0, 0))
        return out

    def lap_u(self, x):
        out = np.zeros(x.shape, dtype=np.float64)
        for m in range(self.a.shape[0]):
            for j in range(3):
                e = [0, 0, 0]
                e[j] = 2
                out += self._curl_of(x, m, tuple(e))
        return out

    def p(self, x):
        return x[..., 0] + x[..., 1] + x[..., 2] - 1.5

    def grad_p(self, x):
        return np.ones(x.shape, dtype=np.float64)

    def f(self, x):
        return -0.5 * self.nu * self.lap_u(x) + self.grad_p(x)


class RandomForce:
    """f = sum_{m=1}^{8} b_m prod_i sin(kappa_{m,i} pi x_i + phi_{m,i}),
    b_m ~ N(0, I_d), kappa in {1,2,3}, phi ~ U[0, 2 pi)."""

    def __init__(self, dim: int, seed: int = 3, n_modes: int = 8):
        rng = np.random.default_rng(seed)
        self.dim = dim
        self.b = rng.standard_normal((n_modes, dim))
        self.kappa = rng.integers(1, 4, size=(n_modes, dim))
        self.phi = rng.uniform(0.0, 2 * np.pi, size=(n_modes, dim))

    def f(self, x):
        out = np.zeros(x.shape, dtype=np.float64)
        for m in range(self.b.shape[0]):
            s = np.ones(x.shape[:-1])
            for i in range(self.dim):
                s = s * np.sin(self.kappa[m, i] * np.pi * x[..., i] + self.phi[m, i])
            out += s[..., None] * self.b[m]
        return out


def lognormal_nu(n_elements: int, seed: int = 4, contrast: float = 1e3) -> np.ndarray:
    """nu_T = exp(clip(g, -ln(contrast)/2, +ln(contrast)/2)), g ~ N(0,1) i.i.d."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(n_elements)
    c = 0.5 * math.log(contrast)
    return np.exp(np.clip(g, -c, c))


def workload(name: str, **kw):
    """Named configurations.  Returns a dict with mesh, nu (per element), k,
    f_lattice (n_e, n_lat, d) on the degree k+1 lattice, and exact solution
    callables when known."""
    if name == "square8_k2":
        n = kw.get("n", 8)
        k = kw.get("k", 2)
        mesh = unit_square_mesh(n)
        sol = Manufactured2D(nu=1.0)
        nu = np.ones(mesh.n_elements)
        f = sol.f(lattice_points(mesh, k + 1))
        return dict(mesh=mesh, nu=nu, k=k, f_lattice=f, solution=sol, tol=1e-10)
    if name == "cube16_k3":
        n = kw.get("n", 16)
        k = kw.get("k", 3)
        mesh = unit_cube_mesh(n)
        sol = CurlModes3D(seed=2, nu=1.0)
        nu = np.ones(mesh.n_elements)
        f = sol.f(lattice_points(mesh, k + 1))
        return dict(mesh=mesh, nu=nu, k=k, f_lattice=f, solution=sol, tol=1e-10)
    if name == "cube64_k1":
        # the lowest-order method (k = 1, Sec. 7) on 64^3 x 6 tets
        n = kw.get("n", 64)
        mesh = unit_cube_mesh(n)
        sol = CurlModes3D(seed=2, nu=1.0)
        nu = np.ones(mesh.n_elements)
        f = sol.f(lattice_points(mesh, 2))
        return dict(mesh=mesh, nu=nu, k=1, f_lattice=f, solution=sol, tol=1e-10)
    if name == "channel_k3":
        # plane channel flow in a 4 x 1 x 1 box (40 x 10 x 10 cells, 24,000
        # tets), nu = 1e-3 as in the paper's channel runs: the profile as
        # Dirichlet data on the inlet and on z = 0, 1, no-slip plates y = 0, 1,
        # an outlet Gamma_NT at x = 4
        cells = kw.get("cells", (40, 10, 10))
        k = kw.get("k", 3)
        L = 4.0
        mesh = box_mesh(cells, (L, 1.0, 1.0))
        sol = PlaneChannel(3, nu=1e-3, L=L)
        nu = np.full(mesh.n_elements, sol.nu)
        pts = lattice_points(mesh, k + 1)
        return dict(mesh=mesh, nu=nu, k=k, f_lattice=sol.f(pts), g_lattice=sol.u(pts), face_bc=sol.face_bc(),
                    solution=sol, tol=1e-10)
    if name == "channel_k1":
        # the lowest-order method (k = 1, Sec. 7) on the plane channel of
        # channel_k3 with 16 times the cells (160 x 40 x 40, 1,536,000 tets):
        # the configuration of the paper's k = 1 runs (a channel with an
        # outlet, nu = 1e-3); the profile is quadratic, so the discrete flow
        # only approximates it
        cells = kw.get("cells", (160, 40, 40))
        L = 4.0
        mesh = box_mesh(cells, (L, 1.0, 1.0))
        sol = PlaneChannel(3, nu=1e-3, L=L)
        nu = np.full(mesh.n_elements, sol.nu)
        pts = lattice_points(mesh, 2)
        return dict(mesh=mesh, nu=nu, k=1, f_lattice=sol.f(pts), g_lattice=sol.u(pts), face_bc=sol.face_bc(),
                    solution=sol, tol=1e-10)
    if name == "cube32_k4_lognormal":
        n = kw.get("n", 32)
        k = kw.get("k", 4)
        mesh = unit_cube_mesh(n)
        nu = lognormal_nu(mesh.n_elements, seed=4)
        force = RandomForce(3, seed=3)
        f = force.f(lattice_points(mesh, k + 1))
        return dict(mesh=mesh, nu=nu, k=k, f_lattice=f, solution=None, tol=1e-8)
    raise KeyError(name)


def batch_members(n_members: int = 256, seed: int = 5, n_min: int = 4, n_max: int = 16, orders=(2, 3, 4),
                  nu_sigma: float = 0.5):
    """Member recipe of a batch of independent cube problems: n_i =
    round(exp(U[ln n_min, ln n_max])) cubes per axis (6 n_i^3 tets), k_i uniform
    in `orders`, nu_i = exp(N(0, nu_sigma^2)) constant per member, and the
    seed of the member's random smooth force.  Returns a list of dicts
    (n, k, nu, force_seed); meshes and forces are built on demand by
    batch_member()."""
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(n_min), math.log(n_max), n_members))).astype(int)
    ks = rng.choice(np.asarray(orders), size=n_members)
    nus = np.exp(nu_sigma * rng.standard_normal(n_members))
    return [dict(n=int(ns[i]), k=int(ks[i]), nu=float(nus[i]), force_seed=1000 + seed * 7919 + i)
            for i in range(n_members)]


def batch_member(spec: dict):
    """Mesh, per-element viscosity and degree-(k+1) lattice force of one batch member."""
    mesh = unit_cube_mesh(spec["n"])
    nu = np.full(mesh.n_elements, spec["nu"])
    f = RandomForce(3, seed=spec["force_seed"]).f(lattice_points(mesh, spec["k"] + 1))
    return dict(mesh=mesh, nu=nu, k=spec["k"], f_lattice=f)


def serving_requests(n_requests: int, seed: int = 6, t_min: float = 1e3, t_max: float = 2e5, orders=(2, 3, 4, 5),
                     contrast: float = 1e3):
    """Request recipe of the serving stream: T ~ logU[t_min, t_max] tets, a
    unit cube of n = max(2, round((T/6)^(1/3))) cubes per axis, k uniform in
    `orders`, per-tet lognormal viscosity clipped to `contrast`, random smooth
    force; each request carries its own seeds.  Returns a list of dicts."""
    rng = np.random.default_rng(seed)
    ts = np.exp(rng.uniform(math.log(t_min), math.log(t_max), n_requests))
    ns = np.maximum(2, np.rint(np.cbrt(ts / 6.0))).astype(int)
    ks = rng.choice(np.asarray(orders), size=n_requests)
    return [dict(n=int(ns[i]), k=int(ks[i]), nu_seed=20000 + seed * 7919 + i, force_seed=40000 + seed * 7919 + i,
                 contrast=contrast) for i in range(n_requests)]


def serving_request(spec: dict):
    """Mesh, per-element viscosity and degree-(k+1) lattice force of one request."""
    mesh = unit_cube_mesh(spec["n"])
    nu = lognormal_nu(mesh.n_elements, seed=spec["nu_seed"], contrast=spec["contrast"])
    f = RandomForce(3, seed=spec["force_seed"]).f(lattice_points(mesh, spec["k"] + 1))
    return dict(mesh=mesh, nu=nu, k=spec["k"], f_lattice=f)
