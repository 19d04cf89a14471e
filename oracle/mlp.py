"""Oracle of the per-tent degree network and its tent features.

Test infrastructure only: the library's kernels never call this module.

The network predicts, from eight features of a tent, the logarithm of the
tent's indicator eta_T(p) for p = 2..8; eta_T is the energy of the jump
between the tent solution of degree p and the incoming values on the bottom
facets, a term of the tent's energy balance (eq. 4.1 tested with w = u; the
oracle's solve_tent reports it as E_jump).  The degree used is the smallest p
whose prediction is below the tolerance.

Everything here is FP64 NumPy on BF16-rounded weights, written from the
definitions:
  forward   a1 = tanh(W1 x + b1), a2 = tanh(W2 a1 + b2), y = W3 a2 + b3
  loss      L = sum_s sum_o mask (y - t)^2 / norm
  backward  reverse-mode chain rule of the three layers
  Adam      Kingma and Ba, "Adam: a method for stochastic optimization" (2015),
            bias-corrected moments
  BF16      the upper 16 bits of an IEEE binary32 after round-to-nearest-even
"""
from __future__ import annotations

import numpy as np

N_FEAT, N_HID, N_OUT = 8, 64, 7
SHAPES = [("W1", (N_HID, N_FEAT)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_OUT, N_HID)), ("b3", (N_OUT,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    """Parameter vector -> dict of arrays (row-major, out x in)."""
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.size == N_PARAM
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = theta[o:o + k].reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_bits(x):
    """uint16 BF16 encodings of float32 values (round to nearest, ties to even;
    infinities and NaNs truncated)."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    special = (u & 0x7F800000) == 0x7F800000
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(special, u >> 16, r)
    return (r & 0xFFFF).astype(np.uint16)


def bf16_value(bits):
    """float64 values of uint16 BF16 encodings."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def forward(theta, x):
    """y (n x 7) and the activations, for parameters theta (float64 values)."""
    P = unpack(theta)
    x = np.asarray(x, dtype=np.float64)
    a1 = np.tanh(x @ P["W1"].T + P["b1"])
    a2 = np.tanh(a1 @ P["W2"].T + P["b2"])
    y = a2 @ P["W3"].T + P["b3"]
    return y, (x, a1, a2)


def loss(theta, x, target, mask, norm):
    y, _ = forward(theta, x)
    return float((mask * (y - target) ** 2).sum() / norm)


def backward(theta, x, target, mask, norm):
    """Gradient of loss() with respect to theta, and the loss."""
    P = unpack(theta)
    y, (x, a1, a2) = forward(theta, x)
    d3 = 2.0 * mask * (y - target) / norm          # dL/dy
    d2 = (d3 @ P["W3"]) * (1.0 - a2 ** 2)          # dL/dz2
    d1 = (d2 @ P["W2"]) * (1.0 - a1 ** 2)          # dL/dz1
    g = {"W3": d3.T @ a2, "b3": d3.sum(0), "W2": d2.T @ a1, "b2": d2.sum(0), "W1": d1.T @ x, "b1": d1.sum(0)}
    return pack(g), float((mask * (y - target) ** 2).sum() / norm)


def adam_step(w, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns new (w, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad ** 2
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def select_degree(y, log_tol, p_max):
    """Smallest p in 2..p_max whose predicted log indicator y[p-2] <= log_tol,
    else p_max."""
    y = np.atleast_2d(y)
    out = np.full(len(y), p_max, dtype=np.int64)
    for i, row in enumerate(y):
        for o in range(N_OUT):
            if o + 2 > p_max:
                break
            if row[o] <= log_tol:
                out[i] = o + 2
                break
    return out


def tent_features(o, V, tb, tt):
    """Features of tent (V, tb, tt) of an OracleTDG `o` before it is solved:
      0 log(dt c_max / h_V)   1 log h_V   2 |patch| / 16   3 log c_max
      4 log(c_max / c_min)    5 log(E_bot / |patch|)
      6 log(relative spread of (v/c, sigma) about their element means)
      7 1 if V lies on the Dirichlet boundary
    h_V = largest distance from X_V to a vertex of the patch; E_bot = the
    incoming energy 1/2 int c^-2 v^2 + |sigma|^2 - 2 v sigma.grad phi_old over
    the patch (the flux form on the current front); the spread is
    sum_e int |u - mean_e(u)|^2 / sum_e int |u|^2 with u = (v/c, sigma)."""
    topo = o.topo
    P = topo.patch[V]
    X = topo.coords
    hv = max(np.linalg.norm(X[w] - X[V]) for e in P for w in topo.elems[e])
    cs = topo.c[P]
    cmax, cmin = cs.max(), cs.min()
    area = E = spread = norm = 0.0
    for e in P:
        c = topo.c[e]
        g_old = topo.grad_lam[e].T @ o.tau[topo.elems[e]]
        w = o.wq[e]
        v, s = o.v[e], o.sig[e]
        E += 0.5 * (w * (v ** 2 / c ** 2 + (s ** 2).sum(-1) - 2.0 * v * (s @ g_old))).sum()
        area += w.sum()
        u = np.concatenate([(v / c)[:, None], s], axis=1)
        mean = (w[:, None] * u).sum(0) / w.sum()
        spread += (w[:, None] * (u - mean) ** 2).sum()
        norm += (w[:, None] * u ** 2).sum()
    on_bnd = 1.0 if len(topo.boundary_facets_at(V)) else 0.0
    return np.array([np.log((tt - tb) * cmax / hv), np.log(hv), len(P) / 16.0, np.log(cmax), np.log(cmax / cmin),
                     np.log(max(E, 0.0) / area + 1e-300), np.log(spread / (norm + 1e-300) + 1e-30), on_bnd])
