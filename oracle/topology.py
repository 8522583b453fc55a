"""Mesh topology for the oracle: facets, orientation, Dirichlet data, colouring.

Conventions (Sec. 3 of the paper defines the mesh, facets and traces; the
numbering below is the solver's documented convention):

* every element's vertices are sorted by ascending global index; local facet i
  is the facet opposite sorted local vertex i;
* a facet is the sorted tuple of its global vertices; facets are ordered
  lexicographically by that tuple ("canonical order");
* boundary facets lie on the faces of the box the mesh fills; each face is
  Dirichlet (Gamma_D, the default) or an outlet Gamma_NT (u_t = 0 and zero
  normal stress, eq. stokes_NT); Dirichlet facets carry no free degrees of
  freedom, outlet facets keep their normal dofs free (their tangential dofs
  are fixed to zero);
* free facets are the interior and the outlet facets in canonical order;
* free vertices (P1 auxiliary space) are those on no Dirichlet facet;
* facet colouring: greedy in canonical order, smallest colour not used by any
  already coloured free facet that shares an element (so facets of one colour
  never share an element and their smoother blocks are independent).
"""
from __future__ import annotations

import numpy as np


class Topology:
    def __init__(self, vertices: np.ndarray, elements: np.ndarray, face_bc=None):
        """face_bc: per face of the bounding box (x-, x+, y-, y+[, z-, z+]) 0
        for Dirichlet, 1 for an outlet Gamma_NT; default all Dirichlet."""
        self.vertices = np.asarray(vertices, dtype=np.float64)
        self.elements_in = np.asarray(elements, dtype=np.int64)
        self.dim = self.vertices.shape[1]
        d = self.dim
        self.perm = np.argsort(self.elements_in, axis=1, kind="stable")
        self.elements = np.take_along_axis(self.elements_in, self.perm, axis=1)
        n_e = self.elements.shape[0]

        facets = {}
        for t in range(n_e):
            ev = self.elements[t]
            for i in range(d + 1):
                key = tuple(int(v) for j, v in enumerate(ev) if j != i)
                facets.setdefault(key, []).append((t, i))
        keys = sorted(facets)
        self.facet_vertices = np.asarray(keys, dtype=np.int64)
        self.facet_neighbors = [sorted(facets[k]) for k in keys]
        nf = len(keys)
        self.n_facets = nf
        self.facet_boundary = np.array([len(nb) == 1 for nb in self.facet_neighbors])
        # face of the bounding box that holds each boundary facet
        lo, hi = self.vertices.min(axis=0), self.vertices.max(axis=0)
        self.facet_face = -np.ones(nf, dtype=np.int64)
        for f in np.nonzero(self.facet_boundary)[0]:
            X = self.vertices[list(keys[f])]
            for a in range(d):
                if np.all(X[:, a] == lo[a]):
                    self.facet_face[f] = 2 * a
                elif np.all(X[:, a] == hi[a]):
                    self.facet_face[f] = 2 * a + 1
            assert self.facet_face[f] >= 0, "boundary facet off the bounding box"
        bc = np.zeros(2 * d, dtype=np.int64) if face_bc is None else np.asarray(face_bc, dtype=np.int64)
        assert bc.shape == (2 * d,) and set(bc.tolist()) <= {0, 1}
        self.face_bc = bc
        self.facet_outlet = np.array([self.facet_boundary[f] and bc[self.facet_face[f]] == 1 for f in range(nf)])
        self.facet_dirichlet = self.facet_boundary & ~self.facet_outlet
        self.has_outlet = bool(self.facet_outlet.any())
        fid = {k: n for n, k in enumerate(keys)}
        self.elem_facets = np.zeros((n_e, d + 1), dtype=np.int64)
        for t in range(n_e):
            ev = self.elements[t]
            for i in range(d + 1):
                key = tuple(int(v) for j, v in enumerate(ev) if j != i)
                self.elem_facets[t, i] = fid[key]

        # free (interior and outlet) facets in canonical order
        self.free_facet_of = -np.ones(nf, dtype=np.int64)
        free = np.nonzero(~self.facet_dirichlet)[0]
        self.free_facet_of[free] = np.arange(len(free))
        self.free_facets = free
        self.n_free_facets = len(free)

        # boundary / free vertices
        bverts = set(int(v) for k in np.asarray(keys)[self.facet_dirichlet] for v in k)
        self.free_outlet = self.facet_outlet[free]          # per free facet
        nv = self.vertices.shape[0]
        self.vertex_boundary = np.zeros(nv, dtype=bool)
        self.vertex_boundary[list(bverts)] = True
        self.free_vertex_of = -np.ones(nv, dtype=np.int64)
        fv = np.nonzero(~self.vertex_boundary)[0]
        self.free_vertex_of[fv] = np.arange(len(fv))
        self.free_vertices = fv

        self._colour()

    def _colour(self):
        n = self.n_free_facets
        colour = -np.ones(n, dtype=np.int64)
        for g, f in enumerate(self.free_facets):
            used = set()
            for (t, _i) in self.facet_neighbors[f]:
                for f2 in self.elem_facets[t]:
                    g2 = self.free_facet_of[f2]
                    if g2 >= 0 and g2 != g and colour[g2] >= 0:
                        used.add(int(colour[g2]))
            c = 0
            while c in used:
                c += 1
            colour[g] = c
        self.colour = colour
        self.n_colours = int(colour.max()) + 1 if n else 0

    def element_coords(self, t: int) -> np.ndarray:
        """(d+1, d) coordinates of the sorted vertices of element t."""
        return self.vertices[self.elements[t]]
