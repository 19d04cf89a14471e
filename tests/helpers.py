"""Shared set-up for the library tests: build a problem on both sides from the
same seeded inputs (workloads), never from each other's outputs."""
import numpy as np

from oracle.pitcher import pitch
from oracle.tdg import OracleTDG


SEEDS = ("monomial", "legendre", "chebyshev")  # seed_basis 0, 1, 2


def oracle_for(pr, field=None, p=None, q=None, seed_basis=0):
    f = field or pr.data
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=p or pr.p, q=q or pr.qpts,
                  alpha=pr.alpha, beta=pr.beta, gD=lambda x, t: f.v(x, t), seed=SEEDS[seed_basis])
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    return o


def gpu_for(pr, field=None, p_max=None, q=None, precision=0, gram_mode=0, seed_basis=0):
    from paper_1907_02367_amd import tdg

    f = field or pr.data
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=p_max or pr.p, q=q or pr.qpts,
                      alpha=pr.alpha, beta=pr.beta, precision=precision, seed_basis=seed_basis)
    if gram_mode:
        ctx.set_gram_mode(gram_mode)
    xq, w = ctx.quad_points()
    ctx.set_initial(f.v(xq, 0.0), f.sigma(xq, 0.0), f.U(xq, 0.0))
    if ctx.nb:
        bx = ctx.boundary_points()
        ctx.set_boundary(f.v(bx[:, :-1], bx[:, -1]))
    return ctx, xq, w


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def elem_max_rel(a, b):
    """Largest per-element difference relative to the typical element: max over
    elements e of ||a_e - b_e|| / (||b|| / sqrt(ne)), arrays (ne, ...).  One
    element off by d (relative to its own size) shows up as ~d here, where the
    global relative L2 difference would dilute it by sqrt(ne)."""
    a = np.asarray(a).reshape(len(a), -1)
    b = np.asarray(b).reshape(len(b), -1)
    scale = max(np.linalg.norm(b) / np.sqrt(len(b)), 1e-300)
    return float(np.linalg.norm(a - b, axis=1).max() / scale)
