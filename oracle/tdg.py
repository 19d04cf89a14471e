"""Tent-by-tent Trefftz-DG solver (oracle; test infrastructure only).

What is computed, following the paper:

* Per tent at vertex V (Sec. 4.1, eq. 4.1): find (v, sigma) in the Trefftz
  space of the tent with
      top-face term(u, w) + Dirichlet term(u, w) [+ interface term, Sec. 4.2]
        = bottom-face term(u_bot, w) + Dirichlet data term(g_D, w)
  for every Trefftz test function w.  The bottom data u_bot is the most recent
  value stored at each spatial quadrature point (Sec. 4.1, Fig. 2): the
  initial data (v0, sigma0) on the first tent over an element, else the value
  written by the tent below.

  Top and bottom facets are graphs t = phi(x) of the piecewise-linear front.
  With the facet normals written out (n^t dS = +dx, n^x dS = -grad phi dx on
  the top; n^t dS = -dx, n^x dS = +grad phi dx on the bottom), both face terms
  of eq. 4.1 become the same form
      B_phi(u, w) = int c^-2 v w_v + sigma.w_sigma - (v w_sigma + w_v sigma).grad phi dx
  taken with phi_new on the top and phi_old (bottom data, bottom test values)
  on the bottom.  Dirichlet faces (vertical, above boundary facets containing
  V) add int (sigma.n + alpha v) w_v on the left and int g_D (alpha w_v -
  w_sigma.n) on the right (eq. 4.1).  With piecewise-constant c the patch
  elements are grouped by speed; each group carries its own Trefftz basis and
  the vertical interfaces between groups add the centred-flux-plus-penalty
  term of Sec. 4.2 (averages and jumps of Sec. 2.4).

* Trefftz basis (Sec. 3, Remark 3.1): U^p computed once for c = 1 (module
  ``trefftz``), shifted to x_K = X_V, t_K = mid-height of the tent, scaled by
  the anisotropic diameter h_K (eq. 3.3) over the tent's vertices:
  xh = (x - x_K)/h_K, th = c (t - t_K)/h_K; fields v = c dU/dth, sigma =
  -grad_xh U (a common 1/h_K factor dropped), U_j = h_K * Uhat_j.

* Recovery of U (Sec. 5): the constant basis function does not enter the
  first-order form; it is fixed per group by one extra row that matches the
  mean of U over the tent's bottom facets with the incoming U (bottom reading
  of the extra space-like term; recover="mean").  The paper's own recovery
  (recover="all") adds int_bot U V to the left and int_bot U_bot V to the
  right for every test function V of U^p (the constant included), with the
  Trefftz unknowns of U (the constant and the N-1 functions whose derivatives
  are the first-order basis) solved together: the extra term of Sec. 5 taken
  on the tent's bottom facets, where the upper element's test function lives.

* Neumann faces (eq. 4.1, T^N): vertical faces above boundary facets of kind
  1 add int v (tau.n) + beta (sigma.n)(tau.n) to the left and
  int g_N (beta tau.n - w) to the right.

* Solve: dense LU with partial pivoting (numpy.linalg.solve, LAPACK getrf/getrs).

* After the solve (v, sigma, U) is evaluated at the top points of every patch
  element and overwrites the stored values (Sec. 4.1), and tau_V = t_top.

* Error at T (Sec. 6): e = (sum c^-2 (v - v_ex)^2 + |sigma - sigma_ex|^2)^(1/2)
  over the flat front t = T.  Energy (Sec. 6.5) on a general front is taken in
  flux form E_phi = 1/2 int c^-2 v^2 + |sigma|^2 - 2 v sigma.grad phi dx,
  which equals the paper's E where phi is flat.
"""
from __future__ import annotations

import itertools
from functools import lru_cache

import numpy as np

from .quadrature import simplex_rule
from .topology import Topology
from .trefftz import SEED_KINDS, dim_U, first_order_fields, trefftz_basis


def _monomials(n: int, deg: int):
    """Exponent list (k, alpha) for all t^k x^alpha with k + |alpha| <= deg."""
    out = []
    for tot in range(deg + 1):
        for k in range(tot + 1):
            for alpha in itertools.product(range(tot - k + 1), repeat=n):
                if sum(alpha) == tot - k:
                    out.append((k, alpha))
    return out


@lru_cache(maxsize=None)
def _coef_mats(n: int, p: int, seed: str = "monomial"):
    """Dense coefficient matrices of the basis (seeded by `seed`, Sec. 6.3)
    over the monomials of degree <= p: returns (mono, Cv, Cs, CU) with Cv (M,
    NW), Cs (n, M, NW), CU (M, NW)."""
    mono = _monomials(n, p)
    idx = {m: i for i, m in enumerate(mono)}
    fo = first_order_fields(n, p, seed)
    basis = trefftz_basis(n, p, seed)
    NW = len(fo)
    M = len(mono)
    Cv = np.zeros((M, NW))
    Cs = np.zeros((n, M, NW))
    CU = np.zeros((M, NW))
    for j in range(NW):
        for key, c in fo[j][0].items():
            Cv[idx[key], j] = float(c)
        for m in range(n):
            for key, c in fo[j][1 + m].items():
                Cs[m, idx[key], j] = float(c)
        for key, c in basis[j + 1].items():
            CU[idx[key], j] = float(c)
    kexp = np.array([m[0] for m in mono])
    aexp = np.array([m[1] for m in mono]).reshape(M, n)
    return kexp, aexp, Cv, Cs, CU


class Group:
    """Scaled Trefftz basis of one wave-speed group of a tent (Remark 3.1)."""

    def __init__(self, n, p, c, xK, tK, hK, seed="monomial"):
        self.n, self.p, self.c, self.xK, self.tK, self.hK = n, p, c, xK, tK, hK
        self.seed = seed

    def fields(self, x, t):
        """Basis fields at physical points x (Q, n), t (Q,):
        returns v (Q, NW), sigma (Q, NW, n), U (Q, NW)."""
        kexp, aexp, Cv, Cs, CU = _coef_mats(self.n, self.p, self.seed)
        xh = (x - self.xK) / self.hK
        th = self.c * (t - self.tK) / self.hK
        mono = th[:, None] ** kexp[None, :]
        for m in range(self.n):
            mono = mono * xh[:, m:m + 1] ** aexp[None, :, m]
        v = self.c * (mono @ Cv)
        s = np.stack([mono @ Cs[m] for m in range(self.n)], axis=-1)
        U = self.hK * (mono @ CU)
        return v, s, U


class OracleTDG:
    def __init__(self, coords, elems, c, tents, layer_ptr, p: int, q: int,
                 alpha: float = 0.5, beta: float = 0.5, gD=None, gN=None, bface_kind=None, recover="mean",
                 seed: str = "monomial"):
        self.topo = Topology(coords, elems, c)
        assert seed in SEED_KINDS
        self.seed = seed  # spatial seed basis of the Trefftz recursion (Sec. 3, Sec. 6.3)
        self.n = self.topo.n
        self.tents = list(tents)
        self.layer_ptr = list(layer_ptr)
        self.p = int(p)
        self.q = int(q)
        self.alpha = float(alpha)
        self.beta = float(beta)
        self.gD = gD  # callable (x (Q,n), t (Q,)) -> (Q,), None means g_D = 0
        self.gN = gN  # same for g_N on Neumann faces
        assert recover in ("off", "mean", "all")
        self.recover = recover
        # kind of every boundary facet (0 Dirichlet, 1 Neumann), in the order of
        # Topology.boundary_facets(); None: all Dirichlet
        bf = self.topo.boundary_facets()
        kinds = np.zeros(len(bf), dtype=np.int64) if bface_kind is None else np.asarray(bface_kind, dtype=np.int64)
        assert kinds.shape == (len(bf),) and set(np.unique(kinds)) <= {0, 1}
        self.kind = {ek: int(kd) for ek, kd in zip(bf, kinds)}
        self.lam_ref, self.w_ref = simplex_rule(self.n, self.q)
        X = self.topo.coords[self.topo.elems]  # (ne, n+1, n)
        self.xq = np.einsum("qk,ekd->eqd", self.lam_ref, X)
        self.wq = self.w_ref[None, :] * self.topo.absdet[:, None]
        ne, Q = self.xq.shape[:2]
        self.v = np.zeros((ne, Q))
        self.sig = np.zeros((ne, Q, self.n))
        self.U = np.zeros((ne, Q))
        self.tau = np.zeros(self.topo.nv)
        self.next_tent = 0
        self.diag = []

    # -- data -----------------------------------------------------------------
    def set_initial(self, v0, sig0, U0):
        self.v[...] = v0
        self.sig[...] = sig0
        self.U[...] = U0
        self.tau[:] = 0.0
        self.next_tent = 0

    def quad_points(self):
        return self.xq

    # -- one tent ---------------------------------------------------------------
    def _face(self, P):
        """Map the reference n-simplex rule onto the space-time simplex with
        vertices P (n+1, n+1); returns points (Q, n+1) and weights (Q,)."""
        pts = self.lam_ref @ P
        E = P[1:] - P[0]
        meas = np.sqrt(np.linalg.det(E @ E.T))
        return pts, self.w_ref * meas

    def _face_simplex(self, V, tb, tt, facet_vertices):
        X = self.topo.coords
        P = [np.append(X[V], tb), np.append(X[V], tt)]
        for W in facet_vertices:
            if W != V:
                P.append(np.append(X[W], self.tau[W]))
        return np.array(P)

    def solve_tent(self, V, tb, tt, p=None, want_diag=False):
        topo = self.topo
        n = self.n
        p = self.p if p is None else int(p)
        al, be = self.alpha, self.beta
        assert self.tau[V] == tb, "tent does not start on the current front"
        P = topo.patch[V]
        cvals = []
        grp = {}
        for e in P:
            ce = float(topo.c[e])
            if ce not in cvals:
                cvals.append(ce)
            grp[e] = cvals.index(ce)
        m = len(cvals)
        NW = dim_U(n, p) - 1
        # anisotropic diameter (eq. 3.3) over the tent's space-time vertices
        verts = sorted({int(w) for e in P for w in topo.elems[e]})
        pts = [(topo.coords[w], self.tau[w]) for w in verts] + [(topo.coords[V], tt)]
        xK = topo.coords[V].copy()
        tK = 0.5 * (tb + tt)
        groups = []
        for cr in cvals:
            h = 0.0
            for (xa, ta), (xb, tb_) in itertools.combinations(pts, 2):
                h = max(h, np.sqrt(((xa - xb) ** 2).sum() + cr * cr * (ta - tb_) ** 2))
            groups.append(Group(n, p, cr, xK, tK, h, self.seed))

        A = np.zeros((m * NW, m * NW))
        rhs = np.zeros(m * NW)
        A0 = np.zeros((m, NW))
        A00 = np.zeros(m)
        r0 = np.zeros(m)
        lam = self.lam_ref
        cache = {}
        for e in P:
            r = grp[e]
            G = groups[r]
            cr = G.c
            b = slice(r * NW, (r + 1) * NW)
            vs = topo.elems[e]
            lV = int(np.where(vs == V)[0][0])
            tau_e = self.tau[vs]
            phi_old = lam @ tau_e
            phi_new = phi_old + lam[:, lV] * (tt - tb)
            g_old = topo.grad_lam[e].T @ tau_e
            g_new = g_old + topo.grad_lam[e][lV] * (tt - tb)
            x = self.xq[e]
            w = self.wq[e]
            Vt, St, Ut = G.fields(x, phi_new)
            Vb, Sb, Ub = G.fields(x, phi_old)
            # top face: B_phi_new(u_j, w_i)
            sgt = St @ g_new
            A[b, b] += ((Vt * (w / cr ** 2)[:, None]).T @ Vt
                        + np.einsum("qim,qjm->ij", St * w[:, None, None], St)
                        - (sgt * w[:, None]).T @ Vt - (Vt * w[:, None]).T @ sgt)
            # bottom face: B_phi_old(u_bot, w_i), test functions at the bottom points
            vb = self.v[e]
            sb = self.sig[e]
            sgb = Sb @ g_old
            sbg = sb @ g_old
            rhs[b] += ((w * vb / cr ** 2) @ Vb + np.einsum("qm,qim->i", sb * w[:, None], Sb)
                       - (w * vb) @ sgb - (w * sbg) @ Vb)
            # recovery row for the constant (mean of U over the bottom facets)
            A0[r] += w @ Ub
            A00[r] += w.sum()
            r0[r] += w @ self.U[e]
            cache[e] = (Vt, St, Ut, Vb, Sb, g_old, g_new, phi_new, Ub)
        # Dirichlet faces
        dfaces = []
        nfaces = []
        for e, k in topo.boundary_facets_at(V):
            r = grp[e]
            G = groups[r]
            b = slice(r * NW, (r + 1) * NW)
            fv = [int(topo.elems[e][j]) for j in range(n + 1) if j != k]
            Pf = self._face_simplex(V, tb, tt, fv)
            fp, fw = self._face(Pf)
            xs, ts = fp[:, :n], fp[:, n]
            Vf, Sf, _ = G.fields(xs, ts)
            nrm = topo.outward_normal(e, k)
            sn = Sf @ nrm
            if self.kind[(e, k)] == 0:
                # Dirichlet: (sigma.n + alpha v) w on the left, g_D (alpha w - tau.n) on the right
                A[b, b] += (Vf * fw[:, None]).T @ (sn + al * Vf)
                g = self.gD(xs, ts) if self.gD is not None else np.zeros(len(ts))
                rhs[b] += (fw * g) @ (al * Vf - sn)
                dfaces.append((r, fw, Vf, Sf, nrm, g))
            else:
                # Neumann: v (tau.n) + beta (sigma.n)(tau.n) on the left, g_N (beta tau.n - w) on the right
                A[b, b] += (sn * fw[:, None]).T @ (Vf + be * sn)
                g = self.gN(xs, ts) if self.gN is not None else np.zeros(len(ts))
                rhs[b] += (fw * g) @ (be * sn - Vf)
                nfaces.append((r, fw, Vf, Sf, nrm, g))
        # interface faces between speed groups (Sec. 4.2)
        ifaces = []
        for e1, k1, e2, k2 in topo.interface_facets_at(V):
            r, s = grp[e1], grp[e2]
            fv = [int(topo.elems[e1][j]) for j in range(n + 1) if j != k1]
            Pf = self._face_simplex(V, tb, tt, fv)
            fp, fw = self._face(Pf)
            xs, ts = fp[:, :n], fp[:, n]
            nrm = topo.outward_normal(e1, k1)
            F = {r: groups[r].fields(xs, ts), s: groups[s].fields(xs, ts)}
            for a, sa in ((r, 1.0), (s, -1.0)):
                Va, Sa, _ = F[a]
                sna = Sa @ nrm
                for bb, sb_ in ((r, 1.0), (s, -1.0)):
                    Vb_, Sb_, _ = F[bb]
                    tnb = Sb_ @ nrm
                    A[bb * NW:(bb + 1) * NW, a * NW:(a + 1) * NW] += (
                        (Vb_ * fw[:, None]).T @ (al * sa * sb_ * Va + 0.5 * sb_ * sna)
                        + (tnb * fw[:, None]).T @ (0.5 * sb_ * Va + be * sa * sb_ * sna))
            ifaces.append((r, s, fw, F, nrm))

        if self.recover == "all":
            # unknowns per group: the constant, then the N-1 functions; the
            # first-order form acts on the functions only (the constant has no
            # derivatives), the bottom mass int_bot U_j U_i couples all of them
            N = NW + 1
            Af = np.zeros((m * N, m * N))
            bf = np.zeros(m * N)
            for r in range(m):
                for s_ in range(m):
                    Af[r * N + 1:(r + 1) * N, s_ * N + 1:(s_ + 1) * N] = A[r * NW:(r + 1) * NW, s_ * NW:(s_ + 1) * NW]
                bf[r * N + 1:(r + 1) * N] = rhs[r * NW:(r + 1) * NW]
            for e in P:
                r = grp[e]
                w = self.wq[e]
                Ub = cache[e][8]  # U of the functions at the bottom points
                Ufull = np.concatenate([np.ones((len(w), 1)), Ub], axis=1)  # (Q, N)
                Af[r * N:(r + 1) * N, r * N:(r + 1) * N] += (Ufull * w[:, None]).T @ Ufull
                bf[r * N:(r + 1) * N] += (w * self.U[e]) @ Ufull
            full = np.linalg.solve(Af, bf)
            a0 = np.array([full[r * N] for r in range(m)])
            sol = np.concatenate([full[r * N + 1:(r + 1) * N] for r in range(m)])
        else:
            sol = np.linalg.solve(A, rhs)
            a0 = np.array([(r0[r] - A0[r] @ sol[r * NW:(r + 1) * NW]) / A00[r] if self.recover == "mean" else 0.0
                           for r in range(m)])

        diag = None
        if want_diag:
            diag = self._diagnostics(P, grp, groups, cache, sol, NW, dfaces, ifaces, nfaces)
        # overwrite the stored values with the top values
        for e in P:
            r = grp[e]
            Vt, St, Ut = cache[e][:3]
            x_r = sol[r * NW:(r + 1) * NW]
            self.v[e] = Vt @ x_r
            self.sig[e] = np.einsum("qjm,j->qm", St, x_r)
            self.U[e] = a0[r] + Ut @ x_r
        self.tau[V] = tt
        return sol, a0, diag

    def _diagnostics(self, P, grp, groups, cache, sol, NW, dfaces, ifaces, nfaces=()):
        """Terms of the per-tent energy balance (derived from eq. 4.1 with w = u
        and the divergence theorem for Trefftz fields)."""
        al, be = self.alpha, self.beta
        E_top = E_bot_in = E_jump = 0.0
        for e in P:
            r = grp[e]
            cr = groups[r].c
            x_r = sol[r * NW:(r + 1) * NW]
            Vt, St, Ut, Vb, Sb, g_old, g_new, _, _ = cache[e]
            w = self.wq[e]
            vt, st = Vt @ x_r, np.einsum("qjm,j->qm", St, x_r)
            E_top += 0.5 * (w * (vt ** 2 / cr ** 2 + (st ** 2).sum(-1) - 2 * vt * (st @ g_new))).sum()
            vb, sb = self.v[e], self.sig[e]
            E_bot_in += 0.5 * (w * (vb ** 2 / cr ** 2 + (sb ** 2).sum(-1) - 2 * vb * (sb @ g_old))).sum()
            dv = Vb @ x_r - vb
            ds = np.einsum("qjm,j->qm", Sb, x_r) - sb
            E_jump += 0.5 * (w * (dv ** 2 / cr ** 2 + (ds ** 2).sum(-1) - 2 * dv * (ds @ g_old))).sum()
        D_bnd = G_bnd = 0.0
        for r, fw, Vf, Sf, nrm, g in dfaces:
            x_r = sol[r * NW:(r + 1) * NW]
            vf = Vf @ x_r
            snf = np.einsum("qjm,j->qm", Sf, x_r) @ nrm
            D_bnd += al * (fw * vf ** 2).sum()
            G_bnd += (fw * g * (al * vf - snf)).sum()
        for r, fw, Vf, Sf, nrm, g in nfaces:
            x_r = sol[r * NW:(r + 1) * NW]
            vf = Vf @ x_r
            snf = np.einsum("qjm,j->qm", Sf, x_r) @ nrm
            D_bnd += self.beta * (fw * snf ** 2).sum()
            G_bnd += (fw * g * (self.beta * snf - vf)).sum()
        D_int = 0.0
        for r, s, fw, F, nrm in ifaces:
            xr = sol[r * NW:(r + 1) * NW]
            xs = sol[s * NW:(s + 1) * NW]
            jv = F[r][0] @ xr - F[s][0] @ xs
            js = (np.einsum("qjm,j->qm", F[r][1], xr) - np.einsum("qjm,j->qm", F[s][1], xs)) @ nrm
            D_int += (fw * (al * jv ** 2 + be * js ** 2)).sum()
        return dict(E_top=E_top, E_bot_in=E_bot_in, E_jump=E_jump, D_bnd=D_bnd,
                    D_int=D_int, G_bnd=G_bnd, D_T=E_jump + D_bnd + D_int)

    # -- sweeps -----------------------------------------------------------------
    def run_layers(self, l0: int, l1: int, p_per_tent=None, want_diag=False):
        out = []
        for l in range(l0, l1):
            for i in range(self.layer_ptr[l], self.layer_ptr[l + 1]):
                V, tb, tt = self.tents[i]
                p = None if p_per_tent is None else int(p_per_tent[i])
                _, _, d = self.solve_tent(V, tb, tt, p=p, want_diag=want_diag)
                if want_diag:
                    out.append(d)
        return out

    def run(self, p_per_tent=None, want_diag=False):
        return self.run_layers(0, len(self.layer_ptr) - 1, p_per_tent, want_diag)

    # -- functionals --------------------------------------------------------------
    def error(self, v_ex, sig_ex):
        """e (Sec. 6) against exact values at the quadrature points (flat front)."""
        c = self.topo.c[:, None]
        d2 = (self.v - v_ex) ** 2 / c ** 2 + ((self.sig - sig_ex) ** 2).sum(-1)
        e_abs = np.sqrt((self.wq * d2).sum())
        ref = np.sqrt((self.wq * (v_ex ** 2 / c ** 2 + (sig_ex ** 2).sum(-1))).sum())
        return e_abs, (e_abs / ref if ref > 0 else np.inf)

    def error_U(self, U_ex):
        """||U - U_ex||_L2 on the flat front (Sec. 6.6 reports it) and its
        ratio to ||U_ex||."""
        d = np.sqrt((self.wq * (self.U - U_ex) ** 2).sum())
        ref = np.sqrt((self.wq * U_ex ** 2).sum())
        return d, (d / ref if ref > 0 else np.inf)

    def energy(self):
        """E_phi on the current front (flux form; the paper's E where flat)."""
        topo = self.topo
        g = np.einsum("ekd,ek->ed", topo.grad_lam, self.tau[topo.elems])
        c = topo.c[:, None]
        dens = self.v ** 2 / c ** 2 + (self.sig ** 2).sum(-1) - 2 * self.v * np.einsum("eqd,ed->eq", self.sig, g)
        return 0.5 * (self.wq * dens).sum()
