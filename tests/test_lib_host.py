"""Host-side checks of libtdg that need no GPU: the library loads and exports
every symbol of include/tdg.h, its pitcher reproduces the oracle's tent list
bit for bit (same rule, independent code), its quadrature points agree with
the oracle's, and invalid inputs are rejected with the documented codes."""
import os
import re

import numpy as np
import pytest

from oracle.pitcher import pitch
from oracle.quadrature import simplex_rule
from workloads import configs as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "tdg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    from paper_1907_02367_amd import tdg

    L = tdg.lib()
    names = header_functions()
    assert len(names) >= 18
    for nm in names:
        assert hasattr(L, nm), nm
        assert nm in tdg.EXPORTS, nm


@pytest.mark.parametrize("builder", [
    lambda: C.cfg1_standing_1d(),
    lambda: C.cfg2_plane_2d(),
    lambda: C.cfg4_interface_2d(m=21),
    lambda: C.cfg5_cube_3d(m=4, regions=2),
    lambda: C.cfg5_cube_3d(m=3, variant="b"),
])
def test_pitcher_bit_equal_to_oracle(builder):
    from paper_1907_02367_amd import tdg

    pr = builder()
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    tents, lp = pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    assert T.as_list() == tents
    assert T.layer_ptr.tolist() == lp
    assert 0 < T.max_slope < 1


def test_cfg1_tent_counts():
    from paper_1907_02367_amd import tdg

    pr = C.cfg1_standing_1d()
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    assert (T.n_tents, T.n_layers) == (281, 33)


@pytest.mark.parametrize("n,p,q", [(1, 3, 3), (2, 4, 4), (2, 3, 9), (3, 3, 3)])
def test_quadrature_points_match_oracle(n, p, q):
    from paper_1907_02367_amd import tdg

    pr = {1: C.cfg1_standing_1d(n_elems=5), 2: C.cfg2_plane_2d(m=6), 3: C.cfg5_cube_3d(m=2, variant="b")}[n]
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=p, q=q, bind=False)
    xq, w = ctx.quad_points()
    lam, wr = simplex_rule(n, q)
    X = np.einsum("qk,ekd->eqd", lam, pr.coords[pr.elems]).reshape(-1, n)
    assert np.abs(xq - X).max() < 1e-14
    vol = np.abs(np.linalg.det(pr.coords[pr.elems][:, 1:] - pr.coords[pr.elems][:, :1]))
    assert np.abs(w - (wr[None, :] * vol[:, None]).ravel()).max() < 1e-15 * max(1.0, vol.max())


def test_boundary_points_on_boundary_and_in_time():
    from paper_1907_02367_amd import tdg

    pr = C.cfg2_plane_2d(m=8)
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=3, bind=False)
    bx = ctx.boundary_points()
    assert ctx.nb > 0 and bx.shape == (ctx.nb, 3)
    on = (np.abs(bx[:, 0]) < 1e-12) | (np.abs(bx[:, 0] - 1) < 1e-12) | (np.abs(bx[:, 1]) < 1e-12) | (np.abs(bx[:, 1] - 1) < 1e-12)
    assert on.all()
    assert (bx[:, 2] > 0).all() and (bx[:, 2] < pr.T).all()


def test_errors_are_reported_not_raised_across_the_abi():
    from paper_1907_02367_amd import tdg

    pr = C.cfg2_plane_2d(m=8)
    with pytest.raises(tdg.TdgError) as ei:
        tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, 1.5)
    assert ei.value.name == "TDG_ENONCAUSAL"
    bad_c = pr.c.copy()
    bad_c[3] = 0.0
    with pytest.raises(tdg.TdgError) as ei:
        tdg.tent_pitch(pr.coords, pr.elems, bad_c, pr.T, pr.gamma)
    assert ei.value.name == "TDG_EINVAL"
    coords = pr.coords.copy()
    e0 = pr.elems[0]
    coords[e0[2]] = 0.5 * (coords[e0[0]] + coords[e0[1]])  # flatten one triangle
    with pytest.raises(tdg.TdgError) as ei:
        tdg.tent_pitch(coords, pr.elems, pr.c, pr.T, pr.gamma)
    assert ei.value.name == "TDG_EINVAL"
    with pytest.raises(tdg.TdgError) as ei:
        tdg.tent_pitch(pr.coords, pr.elems, pr.c, -1.0, pr.gamma)
    assert ei.value.name == "TDG_EINVAL"
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    for p in (0, 11):
        with pytest.raises(tdg.TdgError) as ei:
            tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=p, bind=False)
        assert ei.value.name == "TDG_EINVAL"
    # recovery of U: only the documented values are accepted; the paper's form
    # (2) only with the FP64 quadrature Gram
    for ru in (-1, 3, 7):
        with pytest.raises(tdg.TdgError) as ei:
            tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=3, recover_U=ru, bind=False)
        assert ei.value.name == "TDG_EINVAL"
    for ru in (0, 1, 2):
        tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=3, recover_U=ru, bind=False)
    with pytest.raises(tdg.TdgError) as ei:
        tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=3, recover_U=2, precision=1, bind=False)
    assert ei.value.name == "TDG_EINVAL"
    ctx2 = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=3, recover_U=2, bind=False)
    with pytest.raises(tdg.TdgError) as ei:
        ctx2.set_gram_mode(1)
    assert ei.value.name == "TDG_EINVAL"
    # seed basis of the recursion: 0, 1 or 2 only
    for sb in (-1, 3):
        with pytest.raises(tdg.TdgError) as ei:
            tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=3, seed_basis=sb, bind=False)
        assert ei.value.name == "TDG_EINVAL"
    # boundary-facet kinds must be 0 or 1
    nbf = len(tdg.boundary_facets(pr.coords, pr.elems))
    bad = np.zeros(nbf, np.int8)
    bad[0] = 2
    with pytest.raises(tdg.TdgError) as ei:
        tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=3, bface_kind=bad, bind=False)
    assert ei.value.name == "TDG_EINVAL"


@pytest.mark.parametrize("builder", [lambda: C.cfg1_standing_1d(n_elems=5), lambda: C.cfg2_plane_2d(m=6),
                                     lambda: C.cfg5_cube_3d(m=2, variant="b", regions=1)])
def test_boundary_facets_and_neumann_points(builder):
    """The library lists the boundary facets in the oracle's order (ascending
    (element, opposite local vertex)), and with Neumann facets the boundary
    points of each tent are its Dirichlet faces' then its Neumann faces', each
    point on a facet of its kind."""
    from oracle.topology import Topology
    from paper_1907_02367_amd import tdg

    pr = builder()
    bf = tdg.boundary_facets(pr.coords, pr.elems)
    topo = Topology(pr.coords, pr.elems, pr.c)
    assert [tuple(x) for x in bf.tolist()] == [tuple(map(int, x)) for x in topo.boundary_facets()]
    # Neumann on the facets whose centroid has x_0 < 1/2
    cen = np.array([pr.coords[[v for j, v in enumerate(pr.elems[e]) if j != k]].mean(axis=0) for e, k in bf])
    kinds = (cen[:, 0] < 0.5).astype(np.int8)
    assert 0 < kinds.sum() < len(kinds)
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, 0.2, pr.gamma)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=2, bind=False, bface_kind=kinds)
    ctx_d = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=2, bind=False)
    assert ctx.nb == ctx_d.nb  # the same faces, split by kind
    xt = ctx.boundary_points()
    bk = ctx.boundary_kinds()
    assert set(np.unique(bk)) == {0, 1}
    # every point lies within the x_0-range of the facets of its kind
    x0 = xt[:, 0]
    vx = np.array([[pr.coords[v, 0] for j, v in enumerate(pr.elems[e]) if j != k] for e, k in bf])
    for kd in (0, 1):
        sel = vx[kinds == kd]
        assert (x0[bk == kd] <= sel.max() + 1e-12).all() and (x0[bk == kd] >= sel.min() - 1e-12).all()
    if pr.n == 1:
        assert np.allclose(x0[bk == 1], 0.0) and np.allclose(x0[bk == 0], 1.0)


def test_gram_modes_and_shapes_are_planned_on_the_host():
    """The LDS plan is made on the host: both Gram modes fit the 160 KB of a
    compute unit for the workloads (3+1D p = 8 included), the moment Gram is
    refused in a mixed-precision context and unknown modes are rejected."""
    from paper_1907_02367_amd import tdg

    for pr, gamma in ((C.cfg2_plane_2d(m=8), None), (C.cfg5_cube_3d(m=3, p=8, variant="b"), 0.4 * 0.8 ** 2),
                      (C.lshape_2d(0.3, True, T=0.1), None)):
        T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, gamma or pr.gamma)
        ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=pr.p, bind=False)
        for mode in (0, 1):
            ctx.set_gram_mode(mode)
            assert ctx.get_gram_mode() == mode
            sh = ctx.get_tuning()
            assert 0 < sh["lds_bytes"] <= 160 * 1024
        with pytest.raises(tdg.TdgError) as ei:
            ctx.set_gram_mode(2)
        assert ei.value.name == "TDG_EINVAL"
        mixed = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=pr.p, precision=1, bind=False)
        with pytest.raises(tdg.TdgError) as ei:
            mixed.set_gram_mode(1)
        assert ei.value.name == "TDG_EINVAL"


def test_largest_degree_per_dimension():
    # the tables exist up to p = 10 in every dimension; in 3+1D the working
    # set of a tent at p = 10 exceeds the LDS of a compute unit, which create
    # reports instead of failing at launch
    from paper_1907_02367_amd import tdg

    pr = C.cfg5_cube_3d(m=1, variant="b")
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, 0.05, 0.16)
    tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=9, bind=False)
    with pytest.raises(tdg.TdgError) as ei:
        tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=10, bind=False)
    assert ei.value.name == "TDG_EINVAL" and "LDS" in str(ei.value)
    for pr in (C.cfg1_standing_1d(n_elems=4), C.cfg2_plane_2d(m=3)):
        T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, 0.05, 0.16)
        tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=10, bind=False)
