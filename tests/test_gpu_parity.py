"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Bar (FP64): relative L2 difference <= 1e-10 over every stored value (v,
sigma, U at every quadrature point), after full runs at sizes the oracle
finishes in seconds; at full workload size, sampled tents of selected layers
are re-solved by the oracle from the GPU's own state before that layer
(tents of a layer are independent, so each sampled tent is an exact check),
plus properties that hold at any size (polynomial reproduction, energy
decay)."""
import sys

import numpy as np
import pytest

from helpers import elem_max_rel, gpu_for, oracle_for, rel_l2
from workloads import configs as C
from workloads import fields as F

pytestmark = pytest.mark.gpu
TOL = 1e-10
# 3D p = 8: the tent systems reach condition number 3.6e17 (median 2.5e15) in
# the monomial Trefftz basis; the oracle's own result moves by 2.1e-11 under a
# random one-ulp relative perturbation of its matrix and right-hand side, so a
# backward-stable solve in another summation order (the matrix-core Gram sums
# thousands of products per entry) is expected to differ by tens of ulps of
# backward error: tolerance 50x the one-ulp floor.
# The same rule at the largest degree with tables (p = 10): the oracle's one-ulp
# floor is 2.1e-11 .. 6.1e-11 in 1D (condition numbers up to 1.1e14) and
# 6.9e-10 .. 8.5e-10 in 2D (up to 1.8e19) over three random perturbations, so
# the tolerances are 50x the largest floor.
TOL_CASE = {"3d_p8_b_multipass_gram": 1e-9, "1d_p10_max_degree": 3e-9, "2d_p10_max_degree": 4e-8}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


CASES = {
    "1d_p3_cfg1": lambda: (C.cfg1_standing_1d(), None, None),
    "1d_p8": lambda: (C.cfg1_standing_1d(n_elems=16, p=8), None, None),
    "2d_p4_m8": lambda: (C.cfg2_plane_2d(m=8, p=4), None, None),
    "2d_p4_q9_ragged": lambda: (C.cfg2_plane_2d(m=7, p=4), None, 9),
    "2d_p6_m6": lambda: (C.cfg2_plane_2d(m=6, p=6), None, None),
    "2d_interface_p3": lambda: (C.cfg4_interface_2d(m=9, p=3), None, None),
    "3d_p3_b": lambda: (C.cfg5_cube_3d(m=2, p=3, variant="b"), None, None),
    "3d_p2_a_groups": lambda: (C.cfg5_cube_3d(m=3, p=2, variant="a", regions=3), None, None),
    "2d_p8_m4": lambda: (C.cfg2_plane_2d(m=4, p=8), None, None),
    "3d_p5_b": lambda: (C.cfg5_cube_3d(m=2, p=5, variant="b"), None, None),
    "3d_p3_a_8groups_global_system": lambda: (C.cfg5_cube_3d(m=2, p=3, variant="a", regions=2), None, None),
    # speeds drawn per element (the literal reading): the central vertex's tent
    # has 24 speed groups, a system of 24 x NW unknowns
    "3d_p2_e_per_element_speeds": lambda: (C.cfg5_cube_3d(m=2, p=2, variant="e", T=0.15), None, None),
    "3d_p3_e_per_element_speeds": lambda: (C.cfg5_cube_3d(m=2, p=3, variant="e", T=0.15), None, None),
    "3d_p8_b_multipass_gram": lambda: (C.cfg5_cube_3d(m=2, p=8, variant="b"), None, None),
    # the coarse 6^3 cube (1,296 tetrahedra) in full, speeds drawn per region
    # (125 regions: tents with up to eight speed groups at region corners)
    "3d_p3_a_cube6_regions": lambda: (C.cfg5_cube_3d(m=6, p=3, variant="a", regions=5), None, None),
    # the largest degree with tables (p = 10)
    "1d_p10_max_degree": lambda: (C.cfg1_standing_1d(n_elems=8, p=10), None, None),
    "2d_p10_max_degree": lambda: (C.cfg2_plane_2d(m=3, p=10, T=0.2), None, None),
    # the L-shaped domain of Sec. 6.6 with the corner Bessel data, uniform and graded
    "2d_lshape_uniform_p3": lambda: (C.lshape_2d(0.5, False, T=0.5), None, None),
    "2d_lshape_graded_p3": lambda: (C.lshape_2d(0.4, True, T=0.2), None, None),
}


@pytest.mark.parametrize("gram_mode", [0, 1], ids=["quadrature_gram", "moment_gram"])
@pytest.mark.parametrize("name", list(CASES))
def test_full_run_matches_oracle(name, gram_mode):
    pr, field, q = CASES[name]()
    if pr.n == 3:
        pr.T = 0.25 if pr.p <= 3 else (0.1 if pr.p <= 5 else 0.03)
    say(f"[gpu parity] {name} gram mode {gram_mode}: n={pr.n} p={pr.p} ne={len(pr.elems)}")
    o = oracle_for(pr, field, q=q)
    o.run()
    ctx, xq, w = gpu_for(pr, field, q=q, gram_mode=gram_mode)
    ctx.layer_solve()
    v, s, U = ctx.read_state()
    ctx.status()
    r_vs = rel_l2(np.concatenate([v.ravel(), s.ravel()]), np.concatenate([o.v.ravel(), o.sig.ravel()]))
    r_U = rel_l2(U, o.U)
    # per element: no single element may carry a difference the global norm hides
    # (v and sigma together, as in the global norm: either alone may vanish, e.g.
    # v of the 1+1D standing wave at T = 1)
    m_vs = elem_max_rel(np.concatenate([v[..., None], s], -1), np.concatenate([o.v[..., None], o.sig], -1))
    m_U = elem_max_rel(U, o.U)
    say(f"  rel diff (v, sigma) {r_vs:.2e}, U {r_U:.2e}; largest per element {m_vs:.2e}, {m_U:.2e}")
    tol = TOL_CASE.get(name, TOL)
    assert r_vs <= tol and r_U <= tol, (r_vs, r_U)
    assert m_vs <= 10 * tol and m_U <= 10 * tol, (m_vs, m_U)
    if pr.exact:
        f = field or pr.data
        X = o.quad_points()
        eo = o.error(f.v(X, pr.T), f.sigma(X, pr.T))
        eg = ctx.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T))
        # reverse triangle inequality in the norm of e: |e_gpu - e_orc| <= ||u_gpu - u_orc||
        c = o.topo.c[:, None]
        d = np.sqrt((o.wq * ((v - o.v) ** 2 / c ** 2 + ((s - o.sig) ** 2).sum(-1))).sum())
        ref = np.sqrt((o.wq * (o.v ** 2 / c ** 2 + (o.sig ** 2).sum(-1))).sum())
        assert abs(eg[0] - eo[0]) <= d + 1e-13 * ref, (eg, eo, d)


def _front_before(tents, layer_ptr, l, nv):
    tau = np.zeros(nv)
    for V, tb, tt in tents[: layer_ptr[l]]:
        tau[V] = tt
    return tau


def test_cfg2_full_size_sampled_tents():
    pr = C.cfg2_plane_2d()
    say(f"[gpu parity] cfg2 full size sampled: ne={len(pr.elems)} p={pr.p}")
    ctx, xq, w = gpu_for(pr)
    o = oracle_for(pr)
    assert ctx.tents.as_list() == o.tents
    L = ctx.tents.n_layers
    lp = ctx.tents.layer_ptr
    rng = np.random.default_rng(0)
    checks = {0, 1, 2, 100, L // 2, L - 2, L - 1}
    worst = 0.0
    for l in range(L):
        if l not in checks:
            ctx.layer_solve(l, l + 1)
            continue
        v0, s0, U0 = ctx.read_state()
        ctx.layer_solve(l, l + 1)
        v1, s1, U1 = ctx.read_state()
        o.v[...] = v0
        o.sig[...] = s0
        o.U[...] = U0
        o.tau[:] = _front_before(o.tents, lp, l, len(pr.coords))
        idx = rng.choice(np.arange(lp[l], lp[l + 1]), size=min(6, lp[l + 1] - lp[l]), replace=False)
        for i in idx:
            V, tb, tt = o.tents[i]
            o.solve_tent(V, tb, tt)
            els = o.topo.patch[V]
            a = np.concatenate([v1[els].ravel(), s1[els].ravel()])
            b = np.concatenate([o.v[els].ravel(), o.sig[els].ravel()])
            r = max(rel_l2(a, b), rel_l2(U1[els], o.U[els]))
            worst = max(worst, r)
            assert r <= TOL, (l, V, r)
    ctx.status()
    f = pr.data
    ea, er = ctx.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T))
    say(f"  worst sampled rel diff {worst:.2e}; e_abs at T = {ea:.3e} (rel {er:.3e})")
    assert er < 1e-2


def test_cube_3d_p8_full_size_sampled_tents():
    """The 3+1D workload of the learned-degree comparison at full size (93,750
    tetrahedra, p = 8, moment Gram, FP64): the first 24 layers are swept on the
    GPU, and sampled tents of three of them are re-solved by the oracle from
    the GPU's state before that layer.  The oracle pitches only up to a time
    above the tops of those layers (its pitcher is slow on 1.4M tents); the
    tents of the first 24 layers do not depend on the final time, and the test
    checks that both tent lists agree there."""
    from paper_1907_02367_amd import tdg

    # this seeded mesh is pitched causally from gamma = 0.4 x 0.8^4 on (the
    # rule of the learned-degree tools: lower gamma by 0.8 until causal)
    gamma = 0.4 * 0.8 ** 4
    pr = C.cfg5_cube_3d(m=25, p=8, seed=7, T=0.5, variant="b", regions=1)
    window = 24
    say(f"[gpu parity] 3D cube full size sampled: ne={len(pr.elems)} p={pr.p}")
    f = pr.data
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, gamma)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta)
    ctx.set_gram_mode(1)
    xq, _ = ctx.quad_points()
    ctx.set_initial(f.v(xq, 0.0), f.sigma(xq, 0.0), f.U(xq, 0.0))
    if ctx.nb:
        bx = ctx.boundary_points()
        ctx.set_boundary(f.v(bx[:, :-1], bx[:, -1]))
    lp = ctx.tents.layer_ptr
    glist = ctx.tents.as_list()[: lp[window]]
    t_or = 1.5 * max(tt for _, _, tt in glist)
    pr_or = C.cfg5_cube_3d(m=25, p=8, seed=7, T=t_or, variant="b", regions=1)
    pr_or.gamma = gamma
    o = oracle_for(pr_or, field=f)
    assert o.tents[: lp[window]] == glist
    assert list(o.layer_ptr[: window + 1]) == [int(x) for x in lp[: window + 1]]
    rng = np.random.default_rng(1)
    worst = 0.0
    for l in range(window):
        if l not in (0, 11, window - 1):
            ctx.layer_solve(l, l + 1)
            continue
        v0, s0, U0 = ctx.read_state()
        ctx.layer_solve(l, l + 1)
        v1, s1, U1 = ctx.read_state()
        o.v[...] = v0
        o.sig[...] = s0
        o.U[...] = U0
        o.tau[:] = _front_before(o.tents, lp, l, len(pr.coords))
        for i in rng.choice(np.arange(lp[l], lp[l + 1]), size=2, replace=False):
            V, tb, tt = o.tents[i]
            o.solve_tent(V, tb, tt)
            els = o.topo.patch[V]
            a = np.concatenate([v1[els].ravel(), s1[els].ravel()])
            b = np.concatenate([o.v[els].ravel(), o.sig[els].ravel()])
            r = max(rel_l2(a, b), rel_l2(U1[els], o.U[els]))
            say(f"  layer {l} tent {i} (patch {len(els)}): rel diff {r:.2e}")
            worst = max(worst, r)
            assert r <= TOL_CASE["3d_p8_b_multipass_gram"], (l, V, r)
    ctx.status()
    say(f"  worst sampled rel diff {worst:.2e}")


def test_polynomial_reproduction_full_size():
    pr = C.cfg2_plane_2d()
    f = F.PolynomialPlaneWaves(2, pr.p, 5, seed=11)
    say("[gpu parity] polynomial reproduction cfg2 mesh")
    ctx, xq, w = gpu_for(pr, f)
    ctx.layer_solve()
    ea, er = ctx.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T))
    assert er < 1e-11, er
    v, s, U = ctx.read_state()
    assert np.abs(U.ravel() - f.U(xq, pr.T)).max() < 1e-10 * np.abs(U).max()


def test_energy_decays_with_homogeneous_dirichlet():
    pr = C.cfg4_interface_2d(m=21, p=3)
    pr.T = 0.2
    say("[gpu parity] energy decay, interface mesh")
    ctx, xq, w = gpu_for(pr)
    E = [ctx.energy()[0]]
    for l in range(ctx.tents.n_layers):
        ctx.layer_solve(l, l + 1)
        if l % 10 == 0 or l == ctx.tents.n_layers - 1:
            E.append(ctx.energy()[0])
    E = np.array(E)
    assert np.all(np.diff(E) <= 1e-13 * E[0])
    assert E[-1] < E[0]


def test_empty_range_and_invalid_degree():
    import torch
    from paper_1907_02367_amd import tdg

    pr = C.cfg2_plane_2d(m=6, p=3)
    say("[gpu parity] edge cases")
    ctx, xq, w = gpu_for(pr)
    before = ctx.read_state()[0].copy()
    ctx.layer_solve(3, 3)
    assert np.array_equal(ctx.read_state()[0], before)
    with pytest.raises(tdg.TdgError):
        ctx.layer_solve(0, ctx.tents.n_layers + 1)
    bad = torch.full((ctx.tents.n_tents,), 9, dtype=torch.int8, device="cuda")
    ctx.layer_solve(0, 1, p_per_tent=bad)
    with pytest.raises(tdg.TdgError) as ei:
        ctx.status()
    assert ei.value.name == "TDG_EINVAL"


@pytest.mark.parametrize("shape", [(16, 0), (32, 1), (64, 1)])
def test_kernel_shapes_give_the_same_answer(shape):
    pr = C.cfg2_plane_2d(m=10, p=4)
    say(f"[gpu parity] kernel shape {shape}")
    ctx, xq, w = gpu_for(pr)
    ctx.layer_solve()
    ref = ctx.read_state()
    ctx.set_tuning(*shape)
    ctx.reset()
    ctx.layer_solve()
    got = ctx.read_state()
    ctx.status()
    for a, b in zip(got, ref):
        assert rel_l2(a, b) <= 1e-13


def test_graph_replays_match_eager():
    import torch

    pr = C.cfg2_plane_2d(m=10, p=4)
    say("[gpu parity] graph capture and replay")
    ctx, xq, w = gpu_for(pr)
    ctx.layer_solve()
    ref = ctx.read_state()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ctx.capture_sweep(0, ctx.tents.n_layers, with_reset=True, stream=s.cuda_stream)
    for rep in range(3):
        # eager work between replays
        ctx.reset()
        ctx.layer_solve(0, 5)
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            ctx.replay_sweep(s.cuda_stream)
        torch.cuda.synchronize()
        got = ctx.read_state()
        for a, b in zip(got, ref):
            assert rel_l2(a, b) <= 1e-13, rep
    ctx.status()


MIXED_CASES = {
    "2d_p3_m8": lambda: (C.cfg2_plane_2d(m=8, p=3), None),
    "2d_p4_m8": lambda: (C.cfg2_plane_2d(m=8, p=4), None),
    "2d_p6_m6": lambda: (C.cfg2_plane_2d(m=6, p=6), None),
    "2d_interface_p3": lambda: (C.cfg4_interface_2d(m=9, p=3), None),
    "3d_p3_b": lambda: (C.cfg5_cube_3d(m=2, p=3, variant="b"), None),
    # degrees where the FP32 Gram is too ill-conditioned for refinement on most
    # tents: the per-tent FP64 fallback carries them
    "2d_p7_m4_fallback": lambda: (C.cfg2_plane_2d(m=4, p=7), None),
    "2d_p8_m4_fallback": lambda: (C.cfg2_plane_2d(m=4, p=8), None),
}


@pytest.mark.parametrize("name", list(MIXED_CASES))
def test_mixed_precision_matches_oracle(name):
    """FP32 matrix-core Gram + FP64 LU + FP64 refinement (or per-tent FP64
    fallback) must reach the FP64 bar against the oracle."""
    pr, field = MIXED_CASES[name]()
    if pr.n == 3:
        pr.T = 0.25
    say(f"[gpu mixed] {name}")
    o = oracle_for(pr, field)
    o.run()
    ctx, xq, w = gpu_for(pr, field, precision=1)
    ctx.layer_solve()
    v, s, U = ctx.read_state()
    ctx.status()
    ir, _ = ctx.tent_stats()
    fb = (ir >= 1000).mean()
    steps = (ir % 1000)
    r_vs = rel_l2(np.concatenate([v.ravel(), s.ravel()]), np.concatenate([o.v.ravel(), o.sig.ravel()]))
    r_U = rel_l2(U, o.U)
    m_vs = elem_max_rel(np.concatenate([v[..., None], s], -1), np.concatenate([o.v[..., None], o.sig], -1))
    say(f"  rel diff (v, sigma) {r_vs:.2e}, U {r_U:.2e}, per element {m_vs:.2e}; refinement steps mean "
        f"{steps.mean():.2f}, FP64 fallback {100 * fb:.1f} %")
    assert (steps >= 1).all()
    assert r_vs <= TOL and r_U <= TOL, (r_vs, r_U)
    assert m_vs <= 10 * TOL, m_vs
    if "fallback" in name:
        assert fb > 0, fb
