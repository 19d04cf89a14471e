"""Advancing-front tent pitcher (oracle; test infrastructure only).

Sec. 2.2: the space-time mesh is built by stacking tents, each the union of
(n+1)-simplices over a vertex patch, whose height respects a local causality
(CFL) condition; tents that do not sit on top of each other are independent.
The paper delegates the algorithm to its reference [MTP] and states that tent
heights are limited by the slope of the mesh edges (Sec. 6).  The exact
reading used here:

  kappa_VW = (gamma * |X_W - X_V|) / c_VW,  c_VW = max c over elements on edge VW
  tau = 0 everywhere; repeat:
    R = { V : tau_V < T and tau_V <= tau_W for all neighbours W }  (local minima)
    stop if R is empty
    sort R by (tau_V, V); build the layer S greedily, skipping any V with a
    neighbour already in S
    for V in S: t_top(V) = min(T, min_W (tau_W + kappa_VW)) from the pre-layer tau
    then set tau_V = t_top(V) for every V in S; next layer
  post-condition: every element of every tent stays space-like,
  c_e |grad phi_e| < 1 (Sec. 2.2 face classification).

|X_W - X_V| is the square root of the sum of squared coordinate differences,
summed in coordinate order; every operation is a single IEEE double operation
so that an independent implementation can reproduce the tent list bit for bit.
"""
from __future__ import annotations

import math

import numpy as np

from .topology import Topology


class NonCausal(Exception):
    pass


def pitch(coords, elems, c, T: float, gamma: float, topo: Topology | None = None):
    """Returns (tents, layer_ptr): tents is a list of (V, t_bot, t_top) in
    layer order; tents of layer l are tents[layer_ptr[l]:layer_ptr[l+1]]."""
    topo = topo or Topology(coords, elems, c)
    X = [tuple(float(x) for x in row) for row in topo.coords]
    cl = [float(x) for x in topo.c]
    nv = topo.nv
    # c_VW: maximum speed over the elements containing edge VW
    cedge = {}
    for e, vs in enumerate(topo.elems):
        for a in vs:
            for b in vs:
                if a != b:
                    key = (int(a), int(b))
                    cedge[key] = max(cedge.get(key, 0.0), cl[e])
    kappa = {}
    for V in range(nv):
        for W in topo.nbrs[V]:
            s = 0.0
            for d in range(topo.n):
                diff = X[W][d] - X[V][d]
                s = s + diff * diff
            length = math.sqrt(s)
            kappa[(V, W)] = (gamma * length) / cedge[(V, W)]
    tau = [0.0] * nv
    tents = []
    layer_ptr = [0]
    while True:
        R = [V for V in range(nv)
             if tau[V] < T and all(tau[V] <= tau[W] for W in topo.nbrs[V])]
        if not R:
            break
        R.sort(key=lambda V: (tau[V], V))
        S = []
        in_S = set()
        for V in R:
            if not any(W in in_S for W in topo.nbrs[V]):
                S.append(V)
                in_S.add(V)
        tops = []
        for V in S:
            m = T
            for W in topo.nbrs[V]:
                cand = tau[W] + kappa[(V, W)]
                if cand < m:
                    m = cand
            tops.append(m)
        for V, tt in zip(S, tops):
            tents.append((V, tau[V], tt))
        for V, tt in zip(S, tops):
            tau[V] = tt
        # causality post-condition on every element touched by this layer
        for V in S:
            for e in topo.patch[V]:
                g = topo.grad_lam[e].T @ np.array([tau[w] for w in topo.elems[e]])
                if cl[e] * float(np.linalg.norm(g)) >= 1.0:
                    raise NonCausal(f"element {e} not space-like after tent at vertex {V}")
        layer_ptr.append(len(tents))
    return tents, layer_ptr
