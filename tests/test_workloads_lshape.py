"""The L-shaped workload of Sec. 6.6 (input side only): the structured and
graded meshes cover the domain conformingly with the intended sizes, and the
corner Bessel data solve the wave equation with the stated first-order
fields and vanish on the two edges at the re-entrant corner."""
import numpy as np
import pytest

from workloads import configs as C
from workloads import fields as F


def _areas(coords, elems):
    P = coords[elems]
    return 0.5 * ((P[:, 1, 0] - P[:, 0, 0]) * (P[:, 2, 1] - P[:, 0, 1])
                  - (P[:, 2, 0] - P[:, 0, 0]) * (P[:, 1, 1] - P[:, 0, 1]))


@pytest.mark.parametrize("h_max,graded", [(0.2, False), (0.07, False), (0.3, True), (0.12, True)])
def test_lshape_mesh_covers_the_domain(h_max, graded):
    pr = C.lshape_2d(h_max, graded)
    X, E = pr.coords, pr.elems
    a = _areas(X, E)
    assert (a > 0).all()
    assert abs(a.sum() - 3.0) < 1e-12
    # no vertex inside the removed quadrant, all inside [-1,1]^2
    assert not ((X[:, 0] > 1e-14) & (X[:, 1] < -1e-14)).any()
    assert np.abs(X).max() <= 1.0 + 1e-14
    # conforming: every edge is shared by two triangles or lies on the boundary
    edges = np.sort(np.concatenate([E[:, [0, 1]], E[:, [1, 2]], E[:, [2, 0]]]), axis=1)
    uniq, cnt = np.unique(edges, axis=0, return_counts=True)
    assert cnt.max() == 2
    bnd = uniq[cnt == 1]
    P, Q = X[bnd[:, 0]], X[bnd[:, 1]]

    def on_boundary(Z):
        outer = np.isclose(np.abs(Z).max(axis=1), 1.0)
        corner_x = np.isclose(Z[:, 1], 0.0) & (Z[:, 0] >= -1e-14)
        corner_y = np.isclose(Z[:, 0], 0.0) & (Z[:, 1] <= 1e-14)
        return outer | corner_x | corner_y

    assert on_boundary(P).all() and on_boundary(Q).all() and on_boundary(0.5 * (P + Q)).all()
    d = np.max(np.linalg.norm(X[E[:, [1, 2, 0]]] - X[E], axis=2), axis=1)
    assert 0.8 * h_max < d.max() <= h_max * 1.0001
    if graded:
        # the paper's floor h_min = h_max^3, reached at the corner
        assert 0.5 * h_max ** 3 < d.min() < 2.0 * h_max ** 3


def test_corner_bessel_solves_the_wave_equation():
    f = F.CornerBessel(10.0, 2.0 / 3.0)
    rng = np.random.default_rng(3)
    r = rng.uniform(0.2, 0.9, 20)
    phi = rng.uniform(0.1, 1.5 * np.pi - 0.1, 20)
    x = np.stack([r * np.cos(phi), r * np.sin(phi)], axis=1)
    t = rng.uniform(0.0, 1.0, 20)
    h = 1e-4
    ex, ey = np.array([h, 0.0]), np.array([0.0, h])
    U = f.U(x, t)
    utt = (f.U(x, t + h) - 2 * U + f.U(x, t - h)) / h ** 2
    lap = (f.U(x + ex, t) + f.U(x - ex, t) + f.U(x + ey, t) + f.U(x - ey, t) - 4 * U) / h ** 2
    scale = 100.0 * np.abs(U).max()
    assert np.abs(utt - lap).max() < 1e-4 * scale
    # v = dU/dt, sigma = -grad U
    ut = (f.U(x, t + h) - f.U(x, t - h)) / (2 * h)
    gx = (f.U(x + ex, t) - f.U(x - ex, t)) / (2 * h)
    gy = (f.U(x + ey, t) - f.U(x - ey, t)) / (2 * h)
    assert np.abs(ut - f.v(x, t)).max() < 1e-6 * scale
    s = f.sigma(x, t)
    assert np.abs(s[:, 0] + gx).max() < 1e-6 * scale and np.abs(s[:, 1] + gy).max() < 1e-6 * scale


def test_corner_bessel_vanishes_on_the_reentrant_edges():
    f = F.CornerBessel()
    s = np.linspace(0.01, 1.0, 50)
    on_x = np.stack([s, np.zeros_like(s)], axis=1)        # phi = 0
    on_y = np.stack([np.zeros_like(s), -s], axis=1)       # phi = 3 pi / 2
    for pts in (on_x, on_y):
        assert np.abs(f.U(pts, 0.3)).max() < 1e-14
        assert np.abs(f.v(pts, 0.3)).max() < 1e-13
    # and is singular at the corner: |grad U| grows like r^(nu - 1)
    r = np.array([1e-4, 1e-6])
    g = np.linalg.norm(f.sigma(np.stack([-r, r], axis=1), 0.0), axis=1)
    assert 0.9 < (g[1] / g[0]) / (100.0 ** (1.0 / 3.0)) < 1.1
