"""Pins for the oracle's tent pitcher (Sec. 2.2).

* 1D closed form: on 16 uniform elements of [0,1] with gamma = 0.5, c = 1,
  every edge limit is kappa = 1/32 exactly; layers alternate between the even
  and the odd vertices, an even vertex reaches (2j+1)/32 after its (j+1)-th
  tent and an odd vertex 2j/32 after its j-th, capped at T = 1: 17 tents per
  even vertex, 16 per odd one, 281 tents in 33 layers.
* invariants on 2D/3D meshes: tents of one layer are pairwise non-adjacent,
  every tent starts on the current front and rises, no edge of the front is
  steeper than gamma / c_VW, every element stays space-like (c |grad phi| < 1),
  the front ends flat at T, and the tents' space-time volumes add up to
  |Omega| * T.
"""
import math

import numpy as np
import pytest

from oracle.pitcher import pitch
from oracle.topology import Topology
from workloads import configs as C


def test_1d_closed_form():
    pr = C.cfg1_standing_1d()
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    assert len(tents) == 281 and len(lp) - 1 == 33
    count = {}
    for l in range(33):
        layer = tents[lp[l]:lp[l + 1]]
        par = {V % 2 for V, _, _ in layer}
        assert par == {l % 2}
        for V, tb, tt in layer:
            j = count.get(V, 0)
            if V % 2 == 0:
                assert tt == min(1.0, (2 * j + 1) / 32)
            else:
                assert tt == min(1.0, (2 * j + 2) / 32)
            count[V] = j + 1
    assert all(count[V] == (17 if V % 2 == 0 else 16) for V in range(17))


def _check_invariants(pr):
    topo = Topology(pr.coords, pr.elems, pr.c)
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma, topo)
    tau = np.zeros(topo.nv)
    vol = 0.0
    for l in range(len(lp) - 1):
        layer = tents[lp[l]:lp[l + 1]]
        Vs = {V for V, _, _ in layer}
        assert len(Vs) == len(layer)
        for V, tb, tt in layer:
            assert not (set(topo.nbrs[V]) & Vs)
            assert tau[V] == tb and tt > tb and tt <= pr.T
        for V, tb, tt in layer:
            # tent volume: each patch element contributes |e| * (tt - tb) / (n + 1)
            vol += sum(topo.absdet[e] / math.factorial(topo.n) for e in topo.patch[V]) * (tt - tb) / (topo.n + 1)
            tau[V] = tt
        for V, _, _ in layer:
            for e in topo.patch[V]:
                g = topo.grad_lam[e].T @ tau[topo.elems[e]]
                assert topo.c[e] * np.linalg.norm(g) < 1.0
            for W in topo.nbrs[V]:
                cvw = max(topo.c[e] for e in topo.patch[V] if W in topo.elems[e])
                L = np.linalg.norm(topo.coords[W] - topo.coords[V])
                assert abs(tau[V] - tau[W]) <= pr.gamma * L / cvw * (1 + 1e-12)
    assert np.all(tau == pr.T)
    area = topo.absdet.sum() / math.factorial(topo.n)
    assert abs(vol - area * pr.T) < 1e-12 * area * pr.T
    return tents, lp


@pytest.mark.parametrize("builder", [
    lambda: C.cfg2_plane_2d(m=12),
    lambda: C.cfg4_interface_2d(m=11),
    lambda: C.cfg5_cube_3d(m=3, variant="a", regions=3),
])
def test_invariants(builder):
    _check_invariants(builder())


def test_too_large_gamma_is_not_causal():
    from oracle.pitcher import NonCausal
    pr = C.cfg2_plane_2d(m=8)
    with pytest.raises(NonCausal):
        pitch(pr.coords, pr.elems, pr.c, pr.T, 1.5)
