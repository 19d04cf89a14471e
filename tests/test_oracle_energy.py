"""Pins for the oracle's energy functional (Sec. 6.5; flux form on a general
front, E_phi = 1/2 int c^-2 v^2 + |sigma|^2 - 2 v sigma.grad phi dx).

Each expected value is computed here from the mesh vertices alone (element
measures from determinants, barycentric second moments of a simplex, front
gradients from the vertex times by a linear solve), not from the oracle's
quadrature or its barycentric gradients, so that a dropped 1/2, a flipped
sign of the flux term, a missing c^-2 or a wrong front gradient fails:

* flat front, state linear in x (v = a.x + b) and sigma constant: closed form
  through the covariance of the uniform distribution on a simplex,
  E[(x - xbar)(x - xbar)^T] = sum_i (P_i - xbar)(P_i - xbar)^T / ((n+1)(n+2));
* tilted front (tau linear in x, so grad phi = k on every element), constant
  state: E = 1/2 sum_e |e| (c_e^-2 v^2 + |s|^2 - 2 v s.k);
* the 1+1D standing wave on a flat front: E = pi^2 / 4 at any time;
* the balance of one layer: E(after) = E(before) - sum D_T + sum G_bnd, the
  per-tent terms of eq. 4.1 tested with w = u (their own identity is pinned in
  test_oracle_solver), summed over the tents of the layer.
"""
import numpy as np
import pytest

from oracle.pitcher import pitch
from oracle.tdg import OracleTDG
from workloads import configs as C
from workloads import meshes


def _measures_and_cov(coords, elems):
    """|e| and the covariance matrix of the uniform distribution on e."""
    n = coords.shape[1]
    P = coords[elems]                       # (ne, n+1, n)
    E = P[:, 1:, :] - P[:, :1, :]           # (ne, n, n)
    fact = float(np.prod(np.arange(1, n + 1)))
    meas = np.abs(np.linalg.det(E)) / fact
    xbar = P.mean(axis=1)
    D = P - xbar[:, None, :]
    cov = np.einsum("eid,eif->edf", D, D) / ((n + 1) * (n + 2))
    return meas, xbar, cov


def _oracle(pr, q):
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    return OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=max(pr.p, 1), q=q)


CASES = {
    "1d": lambda: C.cfg1_standing_1d(n_elems=7),
    "2d_two_speeds": lambda: C.cfg4_interface_2d(m=7, p=2),
    "3d_regions": lambda: C.cfg5_cube_3d(m=2, p=2, variant="a", regions=2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_energy_flat_front_linear_state(name):
    pr = CASES[name]()
    n = pr.n
    o = _oracle(pr, q=2)
    X = o.quad_points()
    rng = np.random.default_rng(3)
    a, b, s = rng.normal(size=n), 0.7, rng.normal(size=n)
    v = X @ a + b
    o.set_initial(v, np.broadcast_to(s, X.shape).copy(), np.zeros(X.shape[:2]))
    meas, xbar, cov = _measures_and_cov(pr.coords, pr.elems)
    c = np.asarray(pr.c)
    v2 = (xbar @ a + b) ** 2 + np.einsum("d,edf,f->e", a, cov, a)   # mean of v^2 over e
    expect = 0.5 * np.sum(meas * (v2 / c ** 2 + s @ s))
    assert abs(o.energy() - expect) <= 1e-13 * expect


@pytest.mark.parametrize("name", list(CASES))
def test_energy_tilted_front_constant_state(name):
    pr = CASES[name]()
    n = pr.n
    o = _oracle(pr, q=1)
    X = o.quad_points()
    rng = np.random.default_rng(4)
    k = 0.3 * rng.normal(size=n)
    v0, s = -0.8, rng.normal(size=n)
    o.set_initial(np.full(X.shape[:2], v0), np.broadcast_to(s, X.shape).copy(), np.zeros(X.shape[:2]))
    o.tau[:] = pr.coords @ k + 0.05
    # front gradient per element from the vertex times (linear solve), here = k
    P = pr.coords[pr.elems]
    tv = o.tau[pr.elems]
    g = np.linalg.solve(P[:, 1:, :] - P[:, :1, :], (tv[:, 1:] - tv[:, :1])[..., None])[..., 0]
    assert np.allclose(g, k, atol=1e-13)
    meas, _, _ = _measures_and_cov(pr.coords, pr.elems)
    c = np.asarray(pr.c)
    expect = 0.5 * np.sum(meas * (v0 ** 2 / c ** 2 + s @ s - 2.0 * v0 * (g @ s)))
    assert abs(o.energy() - expect) <= 1e-13 * np.sum(meas * (v0 ** 2 / c ** 2 + s @ s))
    # the flux term has the sign of -v sigma.grad phi: flipping grad phi changes E
    o.tau[:] = -(pr.coords @ k) + 0.05
    flipped = 0.5 * np.sum(meas * (v0 ** 2 / c ** 2 + s @ s + 2.0 * v0 * (g @ s)))
    assert abs(o.energy() - flipped) <= 1e-13 * np.sum(meas * (v0 ** 2 / c ** 2 + s @ s))


@pytest.mark.parametrize("t", [0.0, 0.37, 0.81])
def test_energy_standing_wave_1d(t):
    # U = sin(pi x) cos(pi t): 1/2 int v^2 + sigma^2 dx = pi^2 / 4 at any t
    pr = C.cfg1_standing_1d(n_elems=16)
    o = _oracle(pr, q=10)
    X = o.quad_points()
    f = pr.data
    o.set_initial(f.v(X, t), f.sigma(X, t), f.U(X, t))
    assert abs(o.energy() - np.pi ** 2 / 4) < 1e-13


@pytest.mark.parametrize("builder", [
    lambda: C.cfg2_plane_2d(m=6, p=3),          # inhomogeneous Dirichlet data (G_bnd != 0)
    lambda: C.cfg4_interface_2d(m=7, p=2),      # interface faces
    lambda: C.cfg1_standing_1d(n_elems=8, p=3),
])
def test_energy_layer_balance(builder):
    pr = builder()
    pr.T = min(pr.T, 0.3)
    f = pr.data
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta,
                  gD=lambda x, tt: f.v(x, tt))
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    worst = 0.0
    E0 = o.energy()
    for l in range(len(lp) - 1):
        before = o.energy()
        d = o.run_layers(l, l + 1, want_diag=True)
        after = o.energy()
        change = sum(-x["D_T"] + x["G_bnd"] for x in d)
        worst = max(worst, abs(after - before - change) / E0)
    assert worst < 1e-12, worst
