"""Spatial mesh topology for the oracle (test infrastructure only).

A tent pitched at vertex V stands on the vertex patch of V: all elements
containing V (Sec. 2.2, Sec. 4.1).  Time-like faces inside a tent only occur
above facets that contain V: facets on the domain boundary (Dirichlet faces,
Sec. 4.1) and facets between elements of different wave speed (Sec. 4.2).
"""
from __future__ import annotations

from collections import defaultdict

import numpy as np


class Topology:
    def __init__(self, coords, elems, c):
        self.coords = np.asarray(coords, dtype=np.float64)
        self.elems = np.asarray(elems, dtype=np.int64)
        self.c = np.asarray(c, dtype=np.float64)
        self.nv, self.n = self.coords.shape
        self.ne = len(self.elems)
        n = self.n
        # vertex patches, ascending element index
        patch = [[] for _ in range(self.nv)]
        for e, vs in enumerate(self.elems):
            for v in vs:
                patch[v].append(e)
        self.patch = [sorted(p) for p in patch]
        # neighbours (vertices sharing an edge), ascending
        nb = [set() for _ in range(self.nv)]
        for vs in self.elems:
            for a in vs:
                for b in vs:
                    if a != b:
                        nb[a].add(int(b))
        self.nbrs = [sorted(s) for s in nb]
        # facets: sorted vertex tuple -> list of (element, local index of the opposite vertex)
        fac = defaultdict(list)
        for e, vs in enumerate(self.elems):
            for k in range(n + 1):
                f = tuple(sorted(int(v) for j, v in enumerate(vs) if j != k))
                fac[f].append((e, k))
        self.facets = dict(fac)
        # barycentric gradients and volume scale of each element
        self.grad_lam = np.empty((self.ne, n + 1, n))
        self.absdet = np.empty(self.ne)
        for e, vs in enumerate(self.elems):
            X = self.coords[vs]
            J = (X[1:] - X[0]).T  # n x n, columns X_k - X_0
            Jinv = np.linalg.inv(J)
            self.grad_lam[e, 1:, :] = Jinv
            self.grad_lam[e, 0, :] = -Jinv.sum(axis=0)
            self.absdet[e] = abs(np.linalg.det(J))

    def boundary_facets(self):
        """All boundary facets as (element, opposite local index), ascending:
        the order in which a per-boundary-facet kind (Dirichlet/Neumann) is
        given."""
        if not hasattr(self, "_bfall"):
            self._bfall = sorted((e, k) for f, sides in self.facets.items() if len(sides) == 1
                                 for (e, k) in sides)
        return self._bfall

    def boundary_facets_at(self, V):
        """Boundary facets containing V: list of (element, opposite local index)."""
        if not hasattr(self, "_bf"):
            self._bf = {}
        if V in self._bf:
            return self._bf[V]
        out = []
        for e in self.patch[V]:
            vs = self.elems[e]
            for k in range(self.n + 1):
                if vs[k] == V:
                    continue
                f = tuple(sorted(int(v) for j, v in enumerate(vs) if j != k))
                if len(self.facets[f]) == 1:
                    out.append((e, k))
        self._bf[V] = out
        return out

    def interface_facets_at(self, V):
        """Interior facets containing V whose two elements have different c:
        list of (e1, k1, e2, k2) with e1 < e2."""
        if not hasattr(self, "_if"):
            self._if = {}
        if V in self._if:
            return self._if[V]
        out = []
        for e in self.patch[V]:
            vs = self.elems[e]
            for k in range(self.n + 1):
                if vs[k] == V:
                    continue
                f = tuple(sorted(int(v) for j, v in enumerate(vs) if j != k))
                sides = self.facets[f]
                if len(sides) == 2:
                    (ea, ka), (eb, kb) = sides
                    if ea == e and self.c[ea] != self.c[eb]:
                        out.append((ea, ka, eb, kb) if ea < eb else (eb, kb, ea, ka))
        # each shared facet is found from both sides; keep one copy
        self._if[V] = sorted(set(out))
        return self._if[V]

    def outward_normal(self, e, k):
        """Unit outward normal of element e on the facet opposite local vertex k."""
        g = self.grad_lam[e, k]
        return -g / np.linalg.norm(g)
