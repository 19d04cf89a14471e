"""GPU paths against the oracle beyond the plain eager sweep: the energy and
the per-tent indicator (Sec. 6.5; eq. 4.1 tested with w = u), the persistent
grid on layers far wider than the resident grid, replayed as HIP graphs
(two-speed tents of Sec. 4.2 at the two-material workload's full size), and
the release of a recorded sweep when the kernel shape changes."""
import sys

import numpy as np
import pytest

from helpers import elem_max_rel, gpu_for, oracle_for, rel_l2
from workloads import configs as C

pytestmark = pytest.mark.gpu
TOL = 1e-10


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _front_before(tents, layer_ptr, l, nv):
    tau = np.zeros(nv)
    for V, tb, tt in tents[: layer_ptr[l]]:
        tau[V] = tt
    return tau


@pytest.mark.parametrize("gram_mode", [0, 1], ids=["quadrature_gram", "moment_gram"])
def test_energy_and_indicator_match_oracle(gram_mode):
    """E on every intermediate (non-flat) front and eta_T of every tent.
    eta_T = 1/2 B_phi_old(u - u_b, u - u_b) is a squared norm, so by the
    reverse triangle inequality |sqrt(eta_gpu) - sqrt(eta_orc)| is at most the
    energy norm of the solution difference on the tent's bottom (<= TOL
    relative to the solution, by the parity bar)."""
    pr = C.cfg4_interface_2d(m=9, p=3)
    pr.T = 0.3
    say(f"[gpu paths] energy and indicator, gram mode {gram_mode}")
    o = oracle_for(pr)
    ctx, xq, w = gpu_for(pr, gram_mode=gram_mode)
    ctx.set_indicator(True)
    E0 = o.energy()
    assert abs(ctx.energy()[0] - E0) <= 1e-13 * E0
    L = ctx.tents.n_layers
    jumps = []
    worst_E = 0.0
    for l in range(L):
        ctx.layer_solve(l, l + 1)
        d = o.run_layers(l, l + 1, want_diag=True)
        jumps.extend(x["E_jump"] for x in d)
        if l % 5 == 0 or l == L - 1:
            Eg, Dg = ctx.energy()
            Eo = o.energy()
            worst_E = max(worst_E, abs(Eg - Eo) / E0)
            assert abs(Eg - Eo) <= TOL * E0, (l, Eg, Eo)
            assert abs(Dg - sum(jumps)) <= TOL * E0, (l, Dg, sum(jumps))
    ctx.status()
    _, eta = ctx.tent_stats()
    jumps = np.array(jumps)
    dev = np.abs(np.sqrt(np.maximum(eta, 0)) - np.sqrt(np.maximum(jumps, 0))).max()
    say(f"  energy: worst |E_gpu - E_orc| / E0 = {worst_E:.2e}; indicator: worst sqrt difference "
        f"{dev:.2e} (sqrt(E0) = {np.sqrt(E0):.2e}); total dissipated {jumps.sum():.3e}")
    assert (eta >= 0).all()
    assert dev <= 10 * TOL * np.sqrt(E0), dev
    assert jumps.sum() > 1e-6 * E0  # the check is not vacuous


def test_persistent_grid_and_graph_replay_wide_layers_vs_oracle():
    """Two-material workload at full size (49,928 triangles, c = 1 | 3, p = 4,
    interface tents with 48 unknowns) up to t = 0.003: 27 layers of up to 7,127
    tents, far more than the resident grid of the persistent kernel, so each
    workgroup solves many tents in a row (LDS and shared state reused).  The
    sweep runs as HIP graphs on a side stream; at sampled layers the state
    before and after the layer is read and sampled tents (interface tents
    among them) are re-solved by the oracle from the state before."""
    import torch

    pr = C.cfg4_interface_2d(p=4)
    pr.T = 0.003
    say(f"[gpu paths] persistent grid + graph replay: ne={len(pr.elems)} p={pr.p} T={pr.T}")
    ctx, xq, w = gpu_for(pr)
    ctx.set_tuning(0, 1)
    assert ctx.get_tuning()["persistent"] == 1
    o = oracle_for(pr)
    assert ctx.tents.as_list() == o.tents
    lp = ctx.tents.layer_ptr
    L = ctx.tents.n_layers
    width = int(np.diff(lp).max())
    assert width > 4 * 256, width
    # eager (one workgroup per tent) reference of the whole sweep
    ctx.set_tuning(0, 0)
    ctx.reset()
    ctx.layer_solve()
    ref = ctx.read_state()
    ctx.set_tuning(0, 1)
    s = torch.cuda.Stream()
    iface = set(int(v) for v in range(len(pr.coords)) if abs(pr.coords[v, 0] - 0.5) < 1e-12)
    rng = np.random.default_rng(5)
    worst = worst_el = 0.0
    n_iface = 0
    for l in (0, 1, L // 2, L - 1):
        with torch.cuda.stream(s):
            if l > 0:
                ctx.capture_sweep(0, l, with_reset=True, stream=s.cuda_stream)
                ctx.replay_sweep(s.cuda_stream)
            else:
                ctx.reset(s.cuda_stream)
        torch.cuda.synchronize()
        v0, s0, U0 = ctx.read_state()
        with torch.cuda.stream(s):
            ctx.capture_sweep(l, l + 1, with_reset=False, stream=s.cuda_stream)
            ctx.replay_sweep(s.cuda_stream)
        torch.cuda.synchronize()
        v1, s1, U1 = ctx.read_state()
        o.v[...] = v0
        o.sig[...] = s0
        o.U[...] = U0
        o.tau[:] = _front_before(o.tents, lp, l, len(pr.coords))
        ids = np.arange(lp[l], lp[l + 1])
        on_if = [i for i in ids if o.tents[i][0] in iface]
        pick = list(rng.choice(ids, size=min(6, len(ids)), replace=False)) + on_if[:3]
        for i in pick:
            V, tb, tt = o.tents[i]
            o.solve_tent(V, tb, tt)
            els = o.topo.patch[V]
            n_iface += V in iface
            a = np.concatenate([v1[els].ravel(), s1[els].ravel()])
            b = np.concatenate([o.v[els].ravel(), o.sig[els].ravel()])
            r = max(rel_l2(a, b), rel_l2(U1[els], o.U[els]))
            m = max(elem_max_rel(np.concatenate([v1[els][..., None], s1[els]], -1),
                                 np.concatenate([o.v[els][..., None], o.sig[els]], -1)),
                    elem_max_rel(U1[els], o.U[els]))
            worst, worst_el = max(worst, r), max(worst_el, m)
            assert r <= TOL and m <= 10 * TOL, (l, V, r, m)
    ctx.status()
    assert n_iface > 0
    # the whole sweep replayed as one graph (persistent) against the eager sweep
    with torch.cuda.stream(s):
        ctx.capture_sweep(0, L, with_reset=True, stream=s.cuda_stream)
        for _ in range(2):
            ctx.replay_sweep(s.cuda_stream)
    torch.cuda.synchronize()
    got = ctx.read_state()
    ctx.status()
    for a, b in zip(got, ref):
        assert rel_l2(a, b) <= 1e-13
    say(f"  widest layer {width} tents; sampled tents (interface: {n_iface}): worst rel diff {worst:.2e}, "
        f"per element {worst_el:.2e}")


def test_retuning_releases_the_recorded_sweep():
    import torch
    from paper_1907_02367_amd import tdg

    pr = C.cfg2_plane_2d(m=6, p=3)
    say("[gpu paths] retuning releases a recorded sweep")
    ctx, xq, w = gpu_for(pr)
    s = torch.cuda.Stream()
    for change in (lambda: ctx.set_tuning(16, 1), lambda: ctx.set_gram_mode(1)):
        with torch.cuda.stream(s):
            ctx.capture_sweep(0, ctx.tents.n_layers, with_reset=True, stream=s.cuda_stream)
            ctx.replay_sweep(s.cuda_stream)
        torch.cuda.synchronize()
        change()
        with pytest.raises(tdg.TdgError) as ei:
            ctx.replay_sweep(s.cuda_stream)
        assert ei.value.name == "TDG_ESTATE"
    ctx.status()
