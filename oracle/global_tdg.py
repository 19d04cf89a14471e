"""The global Trefftz-DG system (eq. 2.5) on a tent-pitched mesh, assembled
face by face (oracle; test infrastructure only).

Sec. 2.4 states that on a tent-pitched mesh the global method is
semi-explicit: each tent depends only on the tents below it, so solving tent
by tent reaches the global solution.  This module assembles the global
bilinear form A and right-hand side l of eq. 2.5 directly from the face
definitions, with the space-time normals computed from the face geometry and
the averages/jumps of Sec. 2.4, and solves the whole sparse system at once.
It shares the Trefftz basis (``tdg.Group``) with the tent-by-tent oracle but
none of its face algebra.

Faces handled: space-like faces between two tents (upwind flux: the lower
tent's trace), the initial face F^0, the final face F^T, Dirichlet faces F^D,
Neumann faces F^N and interior time-like faces F^time between speed groups.

Recovery of U (Sec. 5), optional: every group carries the constant as an
extra unknown and the terms  int_{F^space} -[[U]]_t V^+ dS + int_{F^0} U V dS
(left) and int_{F^0} U_0 V dS (right) are added, for every test function V
of U^p (recover="all", the paper's form) or for the constant test function
only (recover="mean").  With [[U]]_t = U^- n_t^- + U^+ n_t^+ on a space-like
face (n_t^+ = -n_t^-) and n_t^- dS = dx the first term is int (U^+ - U^-) V^+ dx.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .quadrature import simplex_rule
from .topology import Topology
from .trefftz import dim_U
from .tdg import Group


def _normal_up(P):
    """Unit normal of the n-simplex with vertices P (n+1, n+1) in space-time,
    oriented with a positive time component; also its n-volume scale."""
    E = P[1:] - P[0]
    _, _, vt = np.linalg.svd(E)
    nu = vt[-1]
    if nu[-1] < 0:
        nu = -nu
    meas = np.sqrt(np.linalg.det(E @ E.T))
    return nu / np.linalg.norm(nu), meas


def global_solve(coords, elems, c, tents, p, q, v0, sig0, alpha=0.5, beta=0.5, gD=None, gN=None, bface_kind=None,
                 U0=None, recover="off", seed="monomial", info=None):
    """Solve eq. 2.5 for all tents at once.  v0 (ne,Q), sig0 (ne,Q,n) are the
    initial values at the element quadrature points (U0 too with a recovery).
    bface_kind: 0 Dirichlet / 1 Neumann per boundary facet in the order of
    Topology.boundary_facets() (None: all Dirichlet).  Returns the final (v,
    sigma) at the element quadrature points at t = T, the solution vector and
    (with a recovery) the final U there.  seed: spatial seed basis of the
    Trefftz recursion (Sec. 3, Sec. 6.3).  info (a dict, optional) receives
    the assembled sparse matrix under "A"."""
    topo = Topology(coords, elems, c)
    n = topo.n
    lam, wref = simplex_rule(n, q)
    X = topo.coords
    NW = dim_U(n, p) - 1
    assert recover in ("off", "mean", "all")
    c0 = 0 if recover == "off" else 1   # the constant precedes the functions in each block
    NB = NW + c0
    bf = topo.boundary_facets()
    kinds = np.zeros(len(bf), np.int64) if bface_kind is None else np.asarray(bface_kind, np.int64)
    kind = {ek: int(kd) for ek, kd in zip(bf, kinds)}
    tau = np.zeros(topo.nv)
    # per tent: its groups (Trefftz bases) and block offsets
    blocks = []  # (tent index, group dict e -> (Group, offset))
    offset = 0
    # history: per element, list of (tent id, heights of the element's vertices after it)
    hist = [[] for _ in range(topo.ne)]
    tent_faces = []
    for ti, (V, tb, tt) in enumerate(tents):
        assert tau[V] == tb
        P = topo.patch[V]
        cvals = []
        for e in P:
            if float(topo.c[e]) not in cvals:
                cvals.append(float(topo.c[e]))
        verts = sorted({int(w) for e in P for w in topo.elems[e]})
        pts = [(X[w], tau[w]) for w in verts] + [(X[V], tt)]
        groups = {}
        for r, cr in enumerate(cvals):
            h = max(np.sqrt(((a[0] - b[0]) ** 2).sum() + cr * cr * (a[1] - b[1]) ** 2)
                    for a, b in itertools.combinations(pts, 2))
            groups[cr] = (Group(n, p, cr, X[V].copy(), 0.5 * (tb + tt), h, seed), offset)
            offset += NB
        emap = {e: groups[float(topo.c[e])] for e in P}
        # time-like faces of this tent (vertical; built from the pre-tent front)
        tfaces = []
        for e, k in topo.boundary_facets_at(V):
            fv = [int(topo.elems[e][j]) for j in range(n + 1) if j != k and topo.elems[e][j] != V]
            Pf = np.array([np.append(X[V], tb), np.append(X[V], tt)] + [np.append(X[W], tau[W]) for W in fv])
            tfaces.append(("D" if kind[(e, k)] == 0 else "N", e, k, None, None, Pf))
        for e1, k1, e2, k2 in topo.interface_facets_at(V):
            fv = [int(topo.elems[e1][j]) for j in range(n + 1) if j != k1 and topo.elems[e1][j] != V]
            Pf = np.array([np.append(X[V], tb), np.append(X[V], tt)] + [np.append(X[W], tau[W]) for W in fv])
            tfaces.append(("I", e1, k1, e2, k2, Pf))
        tent_faces.append((emap, tfaces))
        tau[V] = tt
        for e in P:
            hist[e].append((ti, tau[topo.elems[e]].copy()))
        blocks.append(emap)
    ndof = offset
    rows, cols, vals = [], [], []
    rhs = np.zeros(ndof)

    def add(i0, j0, M):
        ii, jj = np.meshgrid(np.arange(M.shape[0]) + i0, np.arange(M.shape[1]) + j0, indexing="ij")
        rows.append(ii.ravel())
        cols.append(jj.ravel())
        vals.append(M.ravel())

    xq = np.einsum("qk,ekd->eqd", lam, X[topo.elems])
    for e in range(topo.ne):
        ce = float(topo.c[e])
        vs = topo.elems[e]
        Xe = X[vs]
        prev = None  # (tent id, group, offset) of the tent below
        heights0 = np.zeros(n + 1)
        seq = hist[e]
        # F^0 under the first tent over e:  l += int c^-2 v0 w + sigma0.tau dS
        ti, _ = seq[0]
        G, off = blocks[ti][e]
        t0 = lam @ heights0
        Vb, Sb, _ = G.fields(xq[e], t0)
        _, meas = _normal_up(np.concatenate([Xe, heights0[:, None]], axis=1))
        dS = wref * meas
        rhs[off + c0:off + NB] += (dS * v0[e] / ce ** 2) @ Vb + np.einsum("qm,qim->i", sig0[e] * dS[:, None], Sb)
        if recover != "off":
            # int_{F^0} U V (left) and int_{F^0} U_0 V (right), F^0 flat: dS = dx
            _, _, Ub0 = G.fields(xq[e], t0)
            Uf = np.concatenate([np.ones((len(dS), 1)), Ub0], axis=1)
            Vt_ = Uf if recover == "all" else Uf[:, :1]
            add(off, off, np.einsum("q,qi,qj->ij", dS, Vt_, Uf))
            rhs[off:off + Vt_.shape[1]] += (dS * U0[e]) @ Vt_
        # interior space-like faces between consecutive tents over e
        for (ta, ha), (tb_, _) in zip(seq[:-1], seq[1:]):
            Ga, oa = blocks[ta][e]
            Gb, ob = blocks[tb_][e]
            Pf = np.concatenate([Xe, ha[:, None]], axis=1)
            nu, meas = _normal_up(Pf)  # outward normal of the lower tent
            nx, nt = nu[:n], nu[n]
            dS = wref * meas
            tq = lam @ ha
            Va, Sa, _ = Ga.fields(xq[e], tq)
            Vb_, Sb_, _ = Gb.fields(xq[e], tq)
            # trial u^- from the lower tent a; [[w]]_t = (w^- - w^+) nt, [[w]]_N = (w^- - w^+) nx
            san = Sa @ nx
            for (Gt, ot, Vt, St, sgn) in ((Ga, oa, Va, Sa, 1.0), (Gb, ob, Vb_, Sb_, -1.0)):
                stn = St @ nx
                M = (np.einsum("q,qi,qj->ij", dS * nt / ce ** 2, Vt, Va)
                     + np.einsum("q,qim,qjm->ij", dS * nt, St, Sa)
                     + np.einsum("q,qi,qj->ij", dS, stn, Va)
                     + np.einsum("q,qi,qj->ij", dS, Vt, san))
                add(ot + c0, oa + c0, sgn * M)
            if recover != "off":
                # int (U^+ - U^-) V^+ dx, V from the upper tent b
                dx = dS * nt
                _, _, Ua = Ga.fields(xq[e], tq)
                _, _, Ub_ = Gb.fields(xq[e], tq)
                Ufa = np.concatenate([np.ones((len(dx), 1)), Ua], axis=1)
                Ufb = np.concatenate([np.ones((len(dx), 1)), Ub_], axis=1)
                Vt_ = Ufb if recover == "all" else Ufb[:, :1]
                add(ob, ob, np.einsum("q,qi,qj->ij", dx, Vt_, Ufb))
                add(ob, oa, -np.einsum("q,qi,qj->ij", dx, Vt_, Ufa))
        # F^T above the last tent over e: A += int c^-2 v w + sigma.tau dS
        tl, hl = seq[-1]
        G, off = blocks[tl][e]
        tq = lam @ hl
        Vt, St, _ = G.fields(xq[e], tq)
        _, meas = _normal_up(np.concatenate([Xe, hl[:, None]], axis=1))
        dS = wref * meas
        add(off + c0, off + c0, np.einsum("q,qi,qj->ij", dS / ce ** 2, Vt, Vt) + np.einsum("q,qim,qjm->ij", dS, St, St))
    # time-like faces
    for ti, (emap, tfaces) in enumerate(tent_faces):
        for kind, e1, k1, e2, k2, Pf in tfaces:
            fp = lam @ Pf
            E = Pf[1:] - Pf[0]
            dS = wref * np.sqrt(np.linalg.det(E @ E.T))
            xs, ts = fp[:, :n], fp[:, n]
            nrm = topo.outward_normal(e1, k1)
            if kind == "D":
                G, off = emap[e1]
                Vf, Sf, _ = G.fields(xs, ts)
                sn = Sf @ nrm
                add(off + c0, off + c0, np.einsum("q,qi,qj->ij", dS, Vf, sn + alpha * Vf))
                g = gD(xs, ts) if gD is not None else np.zeros(len(ts))
                rhs[off + c0:off + NB] += (dS * g) @ (alpha * Vf - sn)
            elif kind == "N":
                # int_{F^N} v (tau.n) + beta (sigma.n)(tau.n)  and  int g_N (beta tau.n - w)
                G, off = emap[e1]
                Vf, Sf, _ = G.fields(xs, ts)
                sn = Sf @ nrm
                add(off + c0, off + c0, np.einsum("q,qi,qj->ij", dS, sn, Vf + beta * sn))
                g = gN(xs, ts) if gN is not None else np.zeros(len(ts))
                rhs[off + c0:off + NB] += (dS * g) @ (beta * sn - Vf)
            else:
                # K+ = e1's side (normal n), K- = e2's side; jumps with n_{K+} = n, n_{K-} = -n
                sides = ((emap[e1], 1.0), (emap[e2], -1.0))
                F = [(G.fields(xs, ts), off, s) for (G, off), s in sides]
                for (Va, Sa, _), oa, sa in F:
                    for (Vb_, Sb_, _), ob, sb_ in F:
                        # {v}[[tau]]_N + {sigma}.[[w]]_N + alpha [[v]].[[w]] + beta [[sigma]][[tau]]
                        M = (np.einsum("q,qi,qj->ij", dS * 0.5 * sb_, Sb_ @ nrm, Va)
                             + np.einsum("q,qi,qj->ij", dS * 0.5 * sb_, Vb_, Sa @ nrm)
                             + np.einsum("q,qi,qj->ij", dS * alpha * sa * sb_, Vb_, Va)
                             + np.einsum("q,qi,qj->ij", dS * beta * sa * sb_, Sb_ @ nrm, Sa @ nrm))
                        add(ob + c0, oa + c0, M)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(ndof, ndof))
    if info is not None:
        info["A"] = A
    sol = spla.spsolve(A.tocsc(), rhs)
    # final values at the element points from the last tent over each element
    vT = np.zeros((topo.ne, len(wref)))
    sT = np.zeros((topo.ne, len(wref), n))
    UT = np.zeros((topo.ne, len(wref)))
    for e in range(topo.ne):
        tl, hl = hist[e][-1]
        G, off = blocks[tl][e]
        Vt, St, Ut = G.fields(xq[e], lam @ hl)
        x = sol[off + c0:off + NB]
        vT[e] = Vt @ x
        sT[e] = np.einsum("qjm,j->qm", St, x)
        if c0:
            UT[e] = sol[off] + Ut @ x
    if recover == "off":
        return vT, sT, sol
    return vT, sT, sol, UT
