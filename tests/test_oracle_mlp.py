"""Pins of the degree-network oracle against definitions that do not use its
own code paths: central finite differences of the loss (the derivative's
definition), closed forms of special weights, published BF16 encodings, the
first Adam step in closed form, and tent features in closed form on a flat
front with constant values."""
import numpy as np
import pytest

from oracle import mlp as M
from oracle.pitcher import pitch
from oracle.tdg import OracleTDG
from workloads import meshes


def _rand(seed, n=13):
    rng = np.random.default_rng(seed)
    theta = rng.normal(0, 0.3, M.N_PARAM)
    x = rng.normal(0, 1, (n, M.N_FEAT))
    t = rng.normal(0, 1, (n, M.N_OUT))
    mask = (rng.uniform(size=(n, M.N_OUT)) < 0.8).astype(float)
    return theta, x, t, mask


def test_parameter_count():
    assert M.N_PARAM == 64 * 8 + 64 + 64 * 64 + 64 + 7 * 64 + 7 == 5191


@pytest.mark.parametrize("seed", [0, 1])
def test_gradient_matches_central_differences(seed):
    theta, x, t, mask = _rand(seed)
    g, L = M.backward(theta, x, t, mask, norm=7.0)
    assert np.isclose(L, M.loss(theta, x, t, mask, 7.0), rtol=1e-14)
    rng = np.random.default_rng(100 + seed)
    idx = np.concatenate([rng.choice(M.N_PARAM, 60, replace=False), [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736,
                                                                         5183, 5184, 5190]])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss(tp, x, t, mask, 7.0) - M.loss(tm, x, t, mask, 7.0)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, g[i])


def test_masked_outputs_carry_no_gradient():
    theta, x, t, mask = _rand(3)
    mask[:] = 0.0
    mask[:, 2] = 1.0
    g, _ = M.backward(theta, x, t, mask, 1.0)
    P = M.unpack(g)
    # only output 2's row of W3 and b3 may be non-zero in the last layer
    assert np.all(P["W3"][[0, 1, 3, 4, 5, 6]] == 0) and np.all(P["b3"][[0, 1, 3, 4, 5, 6]] == 0)
    assert np.any(P["W3"][2] != 0)


def test_forward_special_weights():
    theta = np.zeros(M.N_PARAM)
    P = M.unpack(theta.copy())
    d = {k: v.copy() for k, v in P.items()}
    d["b2"][:] = 0.5
    d["W3"][:] = 0.1
    d["b3"][:] = np.arange(7)
    th = M.pack(d)
    x = np.random.default_rng(0).normal(size=(5, 8))
    y, _ = M.forward(th, x)
    # W1 = W2 = 0: a2 = tanh(0.5) everywhere, y_o = o + 64 * 0.1 * tanh(0.5)
    assert np.allclose(y, np.arange(7)[None, :] + 6.4 * np.tanh(0.5), rtol=0, atol=1e-15)


def test_bf16_known_encodings():
    vals = np.array([1.0, -2.0, np.pi, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.0, np.inf, 65504.0], dtype=np.float32)
    # 1 + 2^-8 is a tie -> even (0x3F80); 1 + 3*2^-8 is a tie -> even (0x3F82)
    assert list(M.bf16_bits(vals)) == [0x3F80, 0xC000, 0x4049, 0x3F80, 0x3F82, 0x0000, 0x7F80, 0x4780]
    assert M.bf16_value(np.uint16(0x4049)) == 3.140625


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    w, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), step=1, lr=0.01)
    # bias-corrected moments at step 1 are g and g^2
    assert np.allclose(w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_select_degree():
    y = np.array([[0.0, -1.0, -3.0, -5.0, -9.0, -10.0, -11.0],
                  [1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 1.0],
                  [-9.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]])
    assert list(M.select_degree(y, -4.0, 8)) == [5, 8, 2]
    assert list(M.select_degree(y, -4.0, 4)) == [4, 4, 2]


def test_tent_features_closed_form_2d():
    coords, elems = meshes.jittered_square(4, 0.0, 0)
    c = np.full(len(elems), 2.0)
    tents, lp = pitch(coords, elems, c, 0.2, 0.5)
    o = OracleTDG(coords, elems, c, tents, lp, p=2, q=2)
    X = o.quad_points()
    v0, s0 = 0.6, np.array([0.3, -0.4])
    o.set_initial(np.full(X.shape[:2], v0), np.broadcast_to(s0, X.shape[:2] + (2,)).copy(), None)
    V, tb, tt = tents[0]
    f = M.tent_features(o, V, tb, tt)
    P = o.topo.patch[V]
    hv = max(np.linalg.norm(coords[w] - coords[V]) for e in P for w in elems[e])
    assert np.isclose(f[0], np.log((tt - tb) * 2.0 / hv)) and np.isclose(f[1], np.log(hv))
    assert f[2] == len(P) / 16.0 and f[3] == np.log(2.0) and f[4] == 0.0
    # flat front, constant values: E / area = 1/2 (v^2 / c^2 + |sigma|^2)
    assert np.isclose(f[5], np.log(0.5 * (v0 ** 2 / 4.0 + 0.25)), rtol=1e-13)
    # constant values have no spread (round-off only)
    assert f[6] < np.log(1e-25)
    on_bnd = np.any(np.isclose(coords[V], 0.0) | np.isclose(coords[V], 1.0))
    assert f[7] == (1.0 if on_bnd else 0.0)


def _patch_measures(coords, elems, P):
    """|e|, centroid and the covariance of the uniform distribution on each
    patch element, from the vertices alone (see test_oracle_energy)."""
    n = coords.shape[1]
    X = coords[elems[P]]
    E = X[:, 1:, :] - X[:, :1, :]
    meas = np.abs(np.linalg.det(E)) / float(np.prod(np.arange(1, n + 1)))
    xbar = X.mean(axis=1)
    D = X - xbar[:, None, :]
    return meas, xbar, np.einsum("eid,eif->edf", D, D) / ((n + 1) * (n + 2))


def _interface_oracle():
    from workloads import configs as C

    pr = C.cfg4_interface_2d(m=7, p=2)
    tents, lp = pitch(pr.coords, pr.elems, pr.c, 0.2, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=2, q=2)
    # a vertex on the interface x = 1/2 (both speeds in its patch), not on the boundary
    V = next(v for v in range(len(pr.coords)) if abs(pr.coords[v, 0] - 0.5) < 1e-12
             and 0.2 < pr.coords[v, 1] < 0.8)
    return pr, o, V


def test_tent_features_linear_field_spread_and_two_speeds():
    """Feature 6 (spread about the element means) for v = a.x + b, sigma = s:
    per element int |v/c - mean|^2 = |e| a^T Cov_e a / c^2, sigma has no
    spread; feature 4 = log(c_max / c_min) on an interface patch."""
    pr, o, V = _interface_oracle()
    X = o.quad_points()
    a, b, s = np.array([0.9, -1.3]), 0.4, np.array([0.2, 0.5])
    o.set_initial(X @ a + b, np.broadcast_to(s, X.shape).copy(), None)
    tb, tt = 0.0, 0.01
    f = M.tent_features(o, V, tb, tt)
    P = o.topo.patch[V]
    c = np.asarray(pr.c)[P]
    meas, xbar, cov = _patch_measures(pr.coords, pr.elems, P)
    var = np.einsum("d,edf,f->e", a, cov, a)
    spread = np.sum(meas * var / c ** 2)
    norm = np.sum(meas * (((xbar @ a + b) ** 2 + var) / c ** 2 + s @ s))
    assert np.isclose(f[6], np.log(spread / norm), rtol=0, atol=1e-12)
    assert set(np.round(c, 12)) == {1.0, 3.0}
    assert np.isclose(f[3], np.log(3.0)) and np.isclose(f[4], np.log(3.0))
    assert f[7] == 0.0


def test_tent_features_incoming_energy_on_a_tilted_front():
    """Feature 5 = log(E_bot / |patch|) with the flux form of the energy on a
    tilted front: constant (v, sigma), grad phi = k on every element, so
    E_bot = 1/2 sum_e |e| (v^2 / c_e^2 + |s|^2 - 2 v s.k)."""
    pr, o, V = _interface_oracle()
    X = o.quad_points()
    v0, s = 0.7, np.array([-0.6, 0.25])
    o.set_initial(np.full(X.shape[:2], v0), np.broadcast_to(s, X.shape).copy(), None)
    k = np.array([0.2, -0.15])
    o.tau[:] = pr.coords @ k + 0.3
    tb = o.tau[V]
    f = M.tent_features(o, V, tb, tb + 0.01)
    P = o.topo.patch[V]
    c = np.asarray(pr.c)[P]
    meas, _, _ = _patch_measures(pr.coords, pr.elems, P)
    E = 0.5 * np.sum(meas * (v0 ** 2 / c ** 2 + s @ s - 2.0 * v0 * (s @ k)))
    assert np.isclose(f[5], np.log(E / meas.sum()), rtol=0, atol=1e-12)
    # constant values: no spread
    assert f[6] < np.log(1e-25)
