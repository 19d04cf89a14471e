"""Pins for the oracle's tent-by-tent solver (Sec. 4, Sec. 5, Sec. 6).

* polynomial reproduction: data from a Trefftz polynomial of degree <= p built
  from plane waves f(d.x - c t) (not from the recursion) is reproduced to
  round-off, including U (Sec. 5 recovery);
* two-material reproduction: U = t^2 + (x1 - xi)^2 / c(x)^2 solves the
  interface problem exactly (Sec. 4.2);
* energy identity per tent (eq. 4.1 tested with w = u plus the divergence
  theorem for Trefftz fields) and dissipativity (Sec. 6.5);
* global equivalence: the face-by-face global system (eq. 2.5) gives the same
  solution (Sec. 2.4: tents can be solved one after another);
* h-rate O(h^p) for U-degree p (the paper's O(h^(p+1)) for first-order fields
  of degree p, Sec. 6.4) and exponential decay in p (Sec. 6.4, Sec. 6.5);
* the error functional against the closed-form energy of the standing wave.
"""
import numpy as np
import pytest

from oracle.global_tdg import global_solve
from oracle.pitcher import pitch
from oracle.tdg import OracleTDG
from workloads import configs as C
from workloads import fields as F


def solve(pr, f=None, p=None, diag=False, q=None):
    f = f or pr.data
    p = p or pr.p
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=p, q=q or p, alpha=pr.alpha, beta=pr.beta,
                  gD=lambda x, t: f.v(x, t))
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    d = o.run(want_diag=diag)
    return o, d, tents


@pytest.mark.parametrize("case", [
    ("1d", 2), ("1d", 3), ("1d", 5), ("2d", 2), ("2d", 4), ("3d", 2), ("3d", 3)])
def test_polynomial_reproduction(case):
    dim, p = case
    if dim == "1d":
        pr = C.cfg1_standing_1d(n_elems=8, p=p)
        f = F.PolynomialPlaneWaves(1, p, 2, seed=p)
    elif dim == "2d":
        pr = C.cfg2_plane_2d(m=6, p=p)
        f = F.PolynomialPlaneWaves(2, p, 4, seed=p)
    else:
        pr = C.cfg5_cube_3d(m=2, p=p, variant="b", regions=2)
        pr.T = 0.3
        f = F.PolynomialPlaneWaves(3, p, 4, seed=p, c=1.5)
    o, _, _ = solve(pr, f)
    X = o.quad_points()
    e_abs, e_rel = o.error(f.v(X, pr.T), f.sigma(X, pr.T))
    assert e_rel < 1e-12
    assert np.abs(o.U - f.U(X, pr.T)).max() < 1e-12 * max(1.0, np.abs(o.U).max())


def test_lower_degree_does_not_reproduce():
    # the same data with one degree less is not reproduced (sanity of the pin)
    pr = C.cfg2_plane_2d(m=6, p=3)
    f = F.PolynomialPlaneWaves(2, 3, 4, seed=3)
    o, _, _ = solve(pr, f, p=2, q=3)
    X = o.quad_points()
    assert o.error(f.v(X, pr.T), f.sigma(X, pr.T))[1] > 1e-6


@pytest.mark.parametrize("p", [2, 3])
def test_interface_reproduction(p):
    pr = C.cfg4_interface_2d(m=9, p=p)
    pr.T = 0.5
    f = F.InterfaceQuadratic(0.5, 1.0, 3.0)
    o, d, _ = solve(pr, f, diag=True)
    X = o.quad_points()
    assert o.error(f.v(X, pr.T), f.sigma(X, pr.T))[1] < 1e-12
    assert np.abs(o.U - f.U(X, pr.T)).max() < 1e-12


def _balance(d):
    return max(abs(x["E_top"] - (x["E_bot_in"] - x["D_T"] + x["G_bnd"])) / abs(x["E_bot_in"]) for x in d)


@pytest.mark.parametrize("builder", [
    lambda: C.cfg2_plane_2d(m=8, p=3),
    lambda: C.cfg4_interface_2d(m=9, p=3),
    lambda: C.cfg5_cube_3d(m=3, p=2, variant="a", regions=3),
])
def test_energy_identity_per_tent(builder):
    pr = builder()
    pr.T = min(pr.T, 0.3)
    o, d, _ = solve(pr, diag=True)
    assert _balance(d) < 1e-12
    assert all(x["D_T"] >= -1e-15 for x in d)


def test_energy_non_increasing_homogeneous_dirichlet():
    pr = C.cfg4_interface_2d(m=9, p=3)
    pr.T = 0.3
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=3, q=3)
    X = o.quad_points()
    f = pr.data
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    E = [o.energy()]
    for l in range(len(lp) - 1):
        o.run_layers(l, l + 1)
        E.append(o.energy())
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-14 * E[0])
    assert E[-1] < E[0]


@pytest.mark.parametrize("builder", [
    lambda: C.cfg1_standing_1d(n_elems=4, p=3),
    lambda: C.cfg2_plane_2d(m=5, p=3),
    lambda: C.cfg4_interface_2d(m=7, p=2),
])
def test_global_system_equivalence(builder):
    pr = builder()
    f = pr.data
    o, _, tents = solve(pr)
    X = o.quad_points()
    vT, sT, _ = global_solve(pr.coords, pr.elems, pr.c, tents, pr.p, pr.qpts,
                             f.v(X, 0.0), f.sigma(X, 0.0), gD=lambda x, t: f.v(x, t))
    assert np.abs(vT - o.v).max() <= 1e-11 * np.abs(o.v).max()
    assert np.abs(sT - o.sig).max() <= 1e-11 * np.abs(o.sig).max()


@pytest.mark.parametrize("p", [2, 3])
def test_h_convergence_rate_1d(p):
    errs = []
    hs = [1 / 8, 1 / 16, 1 / 32]
    for ne in (8, 16, 32):
        pr = C.cfg1_standing_1d(n_elems=ne, p=p)
        o, _, _ = solve(pr)
        X = o.quad_points()
        errs.append(o.error(pr.data.v(X, 1.0), pr.data.sigma(X, 1.0))[0])
    rates = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(rates > p - 0.3), rates


def test_h_convergence_rate_2d():
    errs, hs = [], []
    for m in (6, 11, 21):
        pr = C.cfg2_plane_2d(m=m, p=2)
        pr.data = F.PlaneWave.seeded(2, np.pi, 1)
        o, _, _ = solve(pr)
        X = o.quad_points()
        errs.append(o.error(pr.data.v(X, 1.0), pr.data.sigma(X, 1.0))[0])
        hs.append(1.0 / (m - 1))
    rates = np.diff(np.log(errs)) / np.diff(np.log(hs))
    assert np.all(rates > 1.7), rates


def test_exponential_p_convergence_1d():
    errs = []
    for p in range(2, 8):
        pr = C.cfg1_standing_1d(n_elems=5, p=p)
        o, _, _ = solve(pr)
        X = o.quad_points()
        errs.append(o.error(pr.data.v(X, 1.0), pr.data.sigma(X, 1.0))[0])
    errs = np.array(errs)
    ratios = errs[1:] / errs[:-1]
    assert np.all(ratios < 0.15), ratios


def test_error_functional_closed_form():
    # zero numerical solution against the standing wave: e^2 = 2 E = pi^2 / 2 at any t
    pr = C.cfg1_standing_1d(n_elems=16, p=6)
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=6, q=6)
    X = o.quad_points()
    e_abs, _ = o.error(pr.data.v(X, 0.37), pr.data.sigma(X, 0.37))
    assert abs(e_abs - np.pi / np.sqrt(2.0)) < 1e-12


@pytest.mark.parametrize("name,builder,tol", [
    ("1d_p10_max_degree", lambda: C.cfg1_standing_1d(n_elems=8, p=10), 3e-9),
    ("2d_p10_max_degree", lambda: C.cfg2_plane_2d(m=3, p=10, T=0.2), 4e-8),
])
def test_parity_tolerance_is_fifty_times_the_one_ulp_floor(name, builder, tol, monkeypatch):
    """The GPU parity tolerance of the high-degree cases is derived from the
    oracle itself: its solution moves by its one-ulp floor when every tent
    matrix and right-hand side is perturbed by a random relative one ulp; the
    tolerance is 50x the largest floor over three perturbations."""
    import oracle.tdg as OT
    from helpers import oracle_for, rel_l2

    pr = builder()
    o = oracle_for(pr)
    o.run()
    ref = np.concatenate([o.v.ravel(), o.sig.ravel()])
    solve = np.linalg.solve
    floors = []
    for seed in (1, 2, 3):
        rng = np.random.default_rng(seed)

        def noisy(A, b):
            return solve(A * (1 + rng.uniform(-1, 1, A.shape) * 2.2e-16), b * (1 + rng.uniform(-1, 1, b.shape) * 2.2e-16))

        monkeypatch.setattr(OT.np.linalg, "solve", noisy)
        o2 = oracle_for(pr)
        o2.run()
        monkeypatch.setattr(OT.np.linalg, "solve", solve)
        floors.append(rel_l2(np.concatenate([o2.v.ravel(), o2.sig.ravel()]), ref))
    assert max(floors) > 0
    assert tol / 3 <= 50 * max(floors) <= tol * 1.5, (name, floors)


@pytest.mark.parametrize("case", ["2d", "2d_two_speeds"])
def test_order_inside_a_layer_is_free(case):
    # the tents of a layer sit at pairwise non-adjacent vertices, so their
    # patches share no element and no vertex (any two vertices of a simplex
    # are joined by an edge): solving a layer's tents in any order gives the
    # same state bit for bit (Sec. 2.2: independent tents in parallel)
    pr = C.cfg2_plane_2d(m=6, p=3) if case == "2d" else C.cfg4_interface_2d(m=9, p=3)
    pr.T = 0.4
    f = pr.data
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    rng = np.random.default_rng(11)
    runs = []
    for shuffle in (False, True):
        o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=pr.p, q=pr.p, gD=lambda x, t: f.v(x, t))
        X = o.quad_points()
        o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
        for l in range(len(lp) - 1):
            idx = np.arange(lp[l], lp[l + 1])
            if shuffle:
                rng.shuffle(idx)
            for i in idx:
                V, tb, tt = tents[i]
                o.solve_tent(V, tb, tt)
        runs.append((o.v.copy(), o.sig.copy(), o.U.copy(), o.tau.copy()))
    assert any(lp[l + 1] - lp[l] > 2 for l in range(len(lp) - 1))  # some layer is really reordered
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
