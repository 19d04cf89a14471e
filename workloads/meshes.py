"""Seeded synthetic simplicial meshes of the unit interval, square and cube.

These generators produce the spatial meshes that the space-time tents are
pitched on (Sec. 2.2 of the paper: tents are erected over vertex patches of a
spatial simplicial mesh).  They contain no part of the method's arithmetic;
both the CPU oracle and the GPU library consume their output.

Every mesh is returned as ``(coords, elems)``:
  coords  float64 array (nv, n)      vertex coordinates
  elems   int32   array (ne, n + 1)  vertex indices of each simplex
"""
from __future__ import annotations

import numpy as np


def interval_mesh(n_elems: int, a: float = 0.0, b: float = 1.0):
    """Uniform partition of [a, b] into ``n_elems`` segments.

    Vertex i sits at a + i*(b-a)/n_elems, computed as i/n_elems scaled, so that
    for [0,1] and a power-of-two element count the coordinates are exact
    binary fractions."""
    i = np.arange(n_elems + 1, dtype=np.float64)
    coords = (a + (b - a) * (i / n_elems)).reshape(-1, 1)
    elems = np.stack([np.arange(n_elems), np.arange(1, n_elems + 1)], axis=1)
    return coords, elems.astype(np.int32)


def _jitter_grid_2d(m: int, jitter: float, rng, fixed_x_cols=()):
    """m x m grid on [0,1]^2 with spacing 1/(m-1), jittered.

    Interior points move by U[-jitter, jitter]*spacing in each coordinate,
    boundary points slide only along their edge, corners stay fixed.  Columns
    listed in ``fixed_x_cols`` keep their x coordinate (they move in y only)."""
    h = 1.0 / (m - 1)
    g = np.arange(m, dtype=np.float64) * h
    X, Y = np.meshgrid(g, g, indexing="ij")  # X[i, j] = i*h
    dx = rng.uniform(-jitter, jitter, size=(m, m)) * h
    dy = rng.uniform(-jitter, jitter, size=(m, m)) * h
    on_x_bnd = np.zeros((m, m), bool)
    on_y_bnd = np.zeros((m, m), bool)
    on_x_bnd[[0, -1], :] = True
    on_y_bnd[:, [0, -1]] = True
    dx[on_x_bnd] = 0.0
    dy[on_y_bnd] = 0.0
    for col in fixed_x_cols:
        dx[col, :] = 0.0
    X = X + dx
    Y = Y + dy
    return X, Y


def _delaunay(points):
    from scipy.spatial import Delaunay

    tri = Delaunay(points)
    simp = tri.simplices.astype(np.int64)
    p = points[simp]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1])
                  - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    keep = np.abs(area) > 1e-14
    simp = simp[keep]
    area = area[keep]
    # orient counter-clockwise
    neg = area < 0
    simp[neg] = simp[neg][:, [0, 2, 1]]
    return simp


def _sort_elems(elems):
    """Deterministic element order: by sorted vertex tuple."""
    key = np.sort(elems, axis=1)
    order = np.lexsort(key.T[::-1])
    return elems[order]


def jittered_square(m: int, jitter: float = 0.2, seed: int = 0):
    """Seeded Delaunay triangulation of a jittered m x m grid of [0,1]^2.

    m = 32 gives 1,922 triangles (h ~ 0.05); m = 100 gives 19,602."""
    rng = np.random.default_rng(seed)
    X, Y = _jitter_grid_2d(m, jitter, rng)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    simp = _delaunay(pts)
    return pts, _sort_elems(simp).astype(np.int32)


def split_square(m: int, jitter: float = 0.2, seed: int = 0):
    """Jittered m x m grid of [0,1]^2 whose middle column is held at x = 0.5
    (m odd) and triangulated separately on each side, so that no triangle
    crosses the line x = 0.5 (a mesh aligned with a wave-speed jump)."""
    assert m % 2 == 1, "m must be odd so that a grid column sits at x = 0.5"
    mid = (m - 1) // 2
    rng = np.random.default_rng(seed)
    X, Y = _jitter_grid_2d(m, jitter, rng, fixed_x_cols=(mid,))
    X[mid, :] = 0.5
    idx = np.arange(m * m).reshape(m, m)
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    parts = []
    for cols in (slice(0, mid + 1), slice(mid, m)):
        sub = idx[cols, :].ravel()
        simp = _delaunay(pts[sub])
        parts.append(sub[simp])
    simp = np.concatenate(parts, axis=0)
    return pts, _sort_elems(simp).astype(np.int32)


def lshape(m: int, graded: bool = False, beta: float = 3.0, rho0: float = 0.0):
    """Structured triangulation of the L-shaped domain [-1,1]^2 minus
    (0,1] x [-1,0) (the domain of Sec. 6.6): a grid of m x m squares of side
    2/m (m even, so that the axes are grid lines) without the squares of the
    removed quadrant, each square cut along a diagonal whose direction
    alternates like a checkerboard.  ``graded`` maps every vertex x to
    x |x|_inf^(beta - 1): rays from the re-entrant corner and the outer square
    are kept, and an element at distance r from the corner gets a size of
    about beta (2/m) r^(1 - 1/beta) (beta = 3 is the paper's mu = 1/3).
    Inside |x|_inf < rho0 the factor is held at rho0^(beta - 1), so the
    smallest elements there have the size rho0^(beta - 1) (2/m) sqrt 2 (the
    paper's floor h_min).  The map preserves orientation: with
    g = max(rho, rho0)^(beta - 1) > 0 its Jacobian determinant is
    g (g + rho g') > 0."""
    assert m % 2 == 0 and m >= 2
    g = np.linspace(-1.0, 1.0, m + 1)
    X, Y = np.meshgrid(g, g, indexing="ij")  # X[i, j] = g[i]
    half = m // 2
    keep_cell = np.ones((m, m), bool)
    keep_cell[half:, :half] = False  # cells with x > 0 and y < 0
    keep_vert = np.zeros((m + 1, m + 1), bool)
    for di in (0, 1):
        for dj in (0, 1):
            keep_vert[di:m + di, dj:m + dj] |= keep_cell
    vid = -np.ones((m + 1, m + 1), np.int64)
    vid[keep_vert] = np.arange(int(keep_vert.sum()))
    pts = np.stack([X[keep_vert], Y[keep_vert]], axis=1)
    tris = []
    for i in range(m):
        for j in range(m):
            if not keep_cell[i, j]:
                continue
            a, b, c, d = vid[i, j], vid[i + 1, j], vid[i + 1, j + 1], vid[i, j + 1]
            if (i + j) % 2 == 0:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    elems = np.array(tris, dtype=np.int64)
    if graded:
        rho = np.maximum(np.abs(pts).max(axis=1), rho0)
        pts = pts * (rho ** (beta - 1.0))[:, None]
    return pts, _sort_elems(elems).astype(np.int32)


# The six Kuhn simplices of the unit cube: each follows a monotone lattice path
# from corner (0,0,0) to (1,1,1), adding one unit vector per step.
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_cube(m: int, jitter: float = 0.15, seed: int = 0, planes=()):
    """Unit cube split into m^3 sub-cubes, each cut into 6 Kuhn tetrahedra.

    Interior vertices move by up to ``jitter`` * spacing per coordinate; a
    vertex whose grid coordinate lies on one of ``planes`` (values in (0,1))
    keeps that coordinate, so the mesh stays aligned with those planes.
    Boundary vertices slide only within their boundary face."""
    rng = np.random.default_rng(seed)
    h = 1.0 / m
    g = np.arange(m + 1, dtype=np.float64) * h
    I, J, K = np.meshgrid(np.arange(m + 1), np.arange(m + 1), np.arange(m + 1), indexing="ij")
    base = np.stack([g[I], g[J], g[K]], axis=-1).reshape(-1, 3)
    gi = np.stack([I, J, K], axis=-1).reshape(-1, 3)
    d = rng.uniform(-jitter, jitter, size=base.shape) * h
    fixed = (gi == 0) | (gi == m)
    plane_idx = [int(round(pl * m)) for pl in planes]
    for pi in plane_idx:
        fixed |= gi == pi
    d[fixed] = 0.0
    coords = base + d

    def vid(i, j, k):
        return (i * (m + 1) + j) * (m + 1) + k

    cubes = np.stack(np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij"), axis=-1).reshape(-1, 3)
    tets = []
    for perm in _KUHN_PERMS:
        cur = cubes.copy()
        vs = [vid(cur[:, 0], cur[:, 1], cur[:, 2])]
        for ax in perm:
            cur = cur.copy()
            cur[:, ax] += 1
            vs.append(vid(cur[:, 0], cur[:, 1], cur[:, 2]))
        tets.append(np.stack(vs, axis=1))
    elems = np.concatenate(tets, axis=0)
    return coords, _sort_elems(elems).astype(np.int32)


def element_centroids(coords, elems):
    return coords[elems].mean(axis=1)
