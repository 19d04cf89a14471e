"""The synthetic workloads (problem statements) of the tent-pitched Trefftz-DG
hot path.  Each builder returns a ``Problem``: mesh, per-element speed c,
degree p, analytic data, final time T and pitch safety factor gamma.

Sizes and data follow the paper's experiments where they exist (Sec. 6: unit
square/cube, standing and plane waves, alpha = beta = 0.5, T = 1;
Sec. 6.7: two materials with a Gaussian pulse) and synthetic stand-ins where
the paper gives no public data set (none is used by the paper).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import fields as F
from . import meshes as M


@dataclass
class Problem:
    name: str
    coords: np.ndarray
    elems: np.ndarray
    c: np.ndarray
    p: int
    T: float
    gamma: float
    data: F.Field
    q: int = 0  # points per direction of the simplex rule (0 -> p)
    alpha: float = 0.5
    beta: float = 0.5
    exact: bool = True  # data is an exact solution (error at T is meaningful)
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.coords.shape[1]

    @property
    def qpts(self):
        return self.q if self.q else self.p


def cfg1_standing_1d(n_elems: int = 16, p: int = 3):
    """1+1D: [0,1], uniform mesh of 16 elements, c = 1, p = 3, T = 1,
    U = sin(pi x) cos(pi t)."""
    coords, elems = M.interval_mesh(n_elems)
    return Problem("1d_standing", coords, elems, np.ones(len(elems)), p, 1.0, 0.5,
                   F.StandingWave1D())


def cfg2_plane_2d(m: int = 32, p: int = 4, seed: int = 0, T: float = 1.0):
    """2+1D FP64: seeded Delaunay of a jittered 32x32 grid (1,922 triangles,
    h ~ 0.05), c = 1, p = 4, T = 1, plane wave with |k| = 2 pi, seeded
    direction."""
    coords, elems = M.jittered_square(m, 0.2, seed)
    return Problem(f"2d_plane_m{m}_p{p}", coords, elems, np.ones(len(elems)), p, T, 0.5,
                   F.PlaneWave.seeded(2, 2 * np.pi, seed + 1))


def cfg3_precision_2d(p: int, m: int = 100, seed: int = 0, T: float = 1.0):
    """2+1D precision sweep: same generator at 100x100 (19,602 triangles),
    p in 2..8, plane-wave data, T = 1."""
    return cfg2_plane_2d(m=m, p=p, seed=seed, T=T)


def cfg4_interface_2d(m: int = 159, p: int = 4, seed: int = 0, T: float = 1.0,
                      delta: float = 0.05):
    """2+1D heterogeneous: mesh aligned with x = 0.5 (m = 159 gives 49,928
    triangles), c = 1 for x < 0.5 and c = 3 otherwise, Gaussian pulse of width
    0.05 at a seeded centre in [0.3,0.7]^2, v0 = 0, homogeneous Dirichlet."""
    coords, elems = M.split_square(m, 0.2, seed)
    cent = M.element_centroids(coords, elems)
    c = np.where(cent[:, 0] < 0.5, 1.0, 3.0)
    rng = np.random.default_rng(seed + 7)
    x0 = rng.uniform(0.3, 0.7, size=2)
    pr = Problem(f"2d_interface_m{m}_p{p}", coords, elems, c, p, T, 0.5,
                 F.GaussianPulse(x0, delta), exact=False)
    pr.meta["x0"] = x0
    return pr


def lshape_2d(h_max: float = 0.05, graded: bool = False, p: int = 3, T: float = 1.0, a: float = 10.0):
    """2+1D L-shaped domain of Sec. 6.6 (the paper's only timed experiment):
    Omega = [-1,1]^2 minus (0,1] x [-1,0), c = 1, p = 3, T = 1, the corner
    Bessel solution with nu = 2/3, a = 10 (g_D = its v on the boundary).
    The paper meshes with an unstructured generator; here a structured
    triangulation stands in: uniform with element diameter h_max, or graded
    towards the corner with the size law h_K ~ h_max r^(2/3) (mu = 1/3), the
    same largest diameter and the paper's smallest size h_min = h_max^3."""
    beta = 3.0
    rho0 = 0.0
    if graded:
        # the outermost squares are stretched by beta along the rays
        m = int(np.ceil(2.0 * beta * np.sqrt(2.0) / h_max))
        m += m % 2
        rho0 = (h_max ** beta / (2.0 / m * np.sqrt(2.0))) ** (1.0 / (beta - 1.0))
    else:
        m = int(np.ceil(2.0 * np.sqrt(2.0) / h_max))
        m += m % 2
    coords, elems = M.lshape(m, graded=graded, beta=beta, rho0=rho0)
    pr = Problem(f"2d_lshape_{'g' if graded else 'u'}_m{m}_p{p}", coords, elems, np.ones(len(elems)), p, T, 0.5,
                 F.CornerBessel(a))
    pr.meta.update(h_max=h_max, graded=graded, m=m)
    return pr


def cfg5_cube_3d(m: int = 25, p: int = 8, seed: int = 0, T: float = 0.5,
                 variant: str = "a", regions: int = 5):
    """3+1D: unit cube, m^3 cubes x 6 Kuhn tetrahedra (m = 25: 93,750 tets),
    jittered, aligned with the planes of a regions^3 partition.
    Variant a: c_r ~ U[1,2] per region, U0 = sin sin sin, v0 = 0, homogeneous
    Dirichlet.  Variant b: c = 1.5 everywhere, exact standing wave.  Variant e:
    c_e ~ U[1,2] per element (every tent has as many speed groups as patch
    elements), data as variant a."""
    planes = [k / regions for k in range(1, regions)]
    coords, elems = M.kuhn_cube(m, 0.15, seed, planes)
    cent = M.element_centroids(coords, elems)
    if variant == "a":
        rng = np.random.default_rng(seed + 11)
        cr = rng.uniform(1.0, 2.0, size=(regions,) * 3)
        ix = np.clip((cent * regions).astype(int), 0, regions - 1)
        c = cr[ix[:, 0], ix[:, 1], ix[:, 2]]
        data = F.SinProduct()
        exact = False
    elif variant == "e":
        rng = np.random.default_rng(seed + 13)
        c = rng.uniform(1.0, 2.0, size=len(elems))
        data = F.SinProduct()
        exact = False
    else:
        c = np.full(len(elems), 1.5)
        data = F.StandingWaveND(3, 1.5)
        exact = True
    return Problem(f"3d_cube{variant}_m{m}_p{p}", coords, elems, c, p, T, 0.4, data,
                   exact=exact)
