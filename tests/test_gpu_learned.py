"""GPU parity of the per-tent degree path: the network kernels (forward,
backward, Adam, BF16 rounding) against the FP64 oracle of the network, the
tent features and the indicator against the oracle's, and degree-adaptive
sweeps against the oracle run with the same degrees.

Tolerances: the network runs in FP32 on BF16 weights; each output is a sum of
at most 64 products after two tanh layers, so its FP32 rounding error is below
64 * 2^-24 relative to the sum of absolute terms (about 4e-6); we allow 2e-5
of max(1, |value|).  Gradients sum over up to n samples per block and block
sums in order: 1e-4 of the largest gradient entry.  BF16 rounding and Adam's
BF16 copy are bit-exact (integer results, decided in FP32 on both sides).
Features are FP32 casts of FP64 quantities: 1e-5 of max(1, |value|).
The indicator is an FP64 energy of a difference: |d eta| <= 1e-8 eta +
1e-12 E_bot (E_bot the tent's incoming energy)."""
import sys

import numpy as np
import pytest

from helpers import gpu_for, oracle_for, rel_l2
from oracle import mlp as OM
from workloads import configs as C

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch

    return torch


def _weights(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    w32 = rng.normal(0, scale, OM.N_PARAM).astype(np.float32)
    bits = OM.bf16_bits(w32)
    return w32, bits


def _dev_bits(bits):
    torch = _torch()
    return torch.from_numpy(bits.view(np.int16).copy()).cuda()


def test_mlp_forward_matches_oracle():
    from paper_1907_02367_amd import tdg

    torch = _torch()
    assert tdg.mlp_nparam() == OM.N_PARAM
    _, bits = _weights(0)
    for n in (1, 63, 64, 65, 1000):
        say(f"[mlp forward] n={n}")
        x = np.random.default_rng(n).normal(0, 1.5, (n, 8)).astype(np.float32)
        y = tdg.mlp_forward(_dev_bits(bits), torch.from_numpy(x).cuda()).cpu().numpy()
        yo, _ = OM.forward(OM.bf16_value(bits), x.astype(np.float64))
        err = np.abs(y - yo) / np.maximum(1.0, np.abs(yo))
        assert err.max() <= 2e-5, err.max()


def test_mlp_backward_matches_oracle():
    from paper_1907_02367_amd import tdg

    torch = _torch()
    _, bits = _weights(1)
    for n in (5, 32, 1000):
        say(f"[mlp backward] n={n}")
        rng = np.random.default_rng(10 + n)
        x = rng.normal(0, 1.5, (n, 8)).astype(np.float32)
        t = rng.normal(0, 2.0, (n, 7)).astype(np.float32)
        mask = (rng.uniform(size=(n, 7)) < 0.7).astype(np.float32)
        norm = float(mask.sum())
        g, _ = tdg.mlp_backward(_dev_bits(bits), torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda(),
                                torch.from_numpy(mask).cuda(), norm)
        g = g.cpu().numpy().astype(np.float64)
        go, Lo = OM.backward(OM.bf16_value(bits), x.astype(np.float64), t.astype(np.float64),
                             mask.astype(np.float64), norm)
        assert abs(g[-1] - Lo) <= 2e-5 * max(1.0, abs(Lo)), (g[-1], Lo)
        err = np.abs(g[:-1] - go).max() / np.abs(go).max()
        assert err <= 1e-4, err


def test_mlp_adam_and_round_match_oracle():
    from paper_1907_02367_amd import tdg

    torch = _torch()
    P = OM.N_PARAM
    rng = np.random.default_rng(5)
    w32 = rng.normal(0, 0.3, P).astype(np.float32)
    m = rng.normal(0, 0.01, P).astype(np.float32)
    v = rng.uniform(0, 1e-3, P).astype(np.float32)
    grad = np.concatenate([rng.normal(0, 0.1, P), [0.0]]).astype(np.float32)
    dw, dm, dv = (torch.from_numpy(a.copy()).cuda() for a in (w32, m, v))
    wb = torch.zeros(P, dtype=torch.int16, device="cuda")
    tdg.mlp_adam(dw, wb, torch.from_numpy(grad).cuda(), dm, dv, step=3, lr=1e-3)
    # the kernel receives the hyper-parameters as FP32: the oracle takes the same values
    f32 = lambda a: float(np.float32(a))  # noqa: E731
    b1, b2 = f32(0.9), f32(0.999)
    g64, m64, v64 = grad[:P].astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    wo, mo, vo = OM.adam_step(w32.astype(np.float64), g64, m64, v64, 3, f32(1e-3), b1, b2, f32(1e-8))
    w_gpu = dw.cpu().numpy()
    assert np.abs(w_gpu - wo).max() <= 1e-6 * np.abs(wo).max() + 1e-9
    # a few FP32 ulps of the sum of the absolute terms
    assert np.all(np.abs(dm.cpu().numpy() - mo) <= 1e-6 * (b1 * np.abs(m64) + (1 - b1) * np.abs(g64)))
    assert np.all(np.abs(dv.cpu().numpy() - vo) <= 1e-6 * vo)
    # the BF16 copy is the rounding of the FP32 master weights, bit for bit
    assert np.array_equal(wb.cpu().numpy().view(np.uint16), OM.bf16_bits(w_gpu))
    # rounding of ties and specials
    special = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -0.0, np.inf, -np.inf, 3.3895314e38, 1e-40],
                       dtype=np.float32)
    w_sp = np.concatenate([special, rng.normal(0, 1, P - len(special)).astype(np.float32)])
    tdg.mlp_round(torch.from_numpy(w_sp).cuda(), wb)
    assert np.array_equal(wb.cpu().numpy().view(np.uint16), OM.bf16_bits(w_sp))


def _advance(pr, layers):
    """Oracle and library contexts advanced through the first `layers` layers."""
    o = oracle_for(pr)
    o.run_layers(0, layers)
    ctx, xq, w = gpu_for(pr)
    ctx.layer_solve(0, layers)
    ctx.status()
    return o, ctx


FEATURE_CASES = {
    "2d_p4": lambda: C.cfg2_plane_2d(m=8, p=4),
    "2d_interface_p3": lambda: C.cfg4_interface_2d(m=9, p=3),
    "3d_a_p3": lambda: C.cfg5_cube_3d(m=3, p=3, variant="a", regions=3, T=0.2),
}


@pytest.mark.parametrize("name", list(FEATURE_CASES))
def test_features_and_indicator_match_oracle(name):
    torch = _torch()
    pr = FEATURE_CASES[name]()
    o, ctx = _advance(pr, 3)
    l = 3
    say(f"[features/indicator] {name}: layer {l}")
    nt = ctx.tents.n_tents
    feats = torch.zeros((nt, 8), dtype=torch.float32, device="cuda")
    ctx.tent_features(l, feats)
    f_gpu = feats.cpu().numpy()
    lp = o.layer_ptr
    for i in range(lp[l], lp[l + 1]):
        V, tb, tt = o.tents[i]
        fo = OM.tent_features(o, V, tb, tt)
        err = np.abs(f_gpu[i] - fo) / np.maximum(1.0, np.abs(fo))
        assert err.max() <= 1e-5, (i, f_gpu[i], fo)
    # indicator at two degrees, state untouched
    before = ctx.read_state()
    eta = torch.zeros(nt, dtype=torch.float64, device="cuda")
    for p in sorted({2, pr.p}):
        ctx.layer_indicator(l, p, eta)
        ctx.status()
        e_gpu = eta.cpu().numpy()
        for i in range(lp[l], lp[l + 1]):
            V, tb, tt = o.tents[i]
            saved = (o.v.copy(), o.sig.copy(), o.U.copy(), o.tau.copy())
            _, _, d = o.solve_tent(V, tb, tt, p=p, want_diag=True)
            o.v[...], o.sig[...], o.U[...], o.tau[...] = saved
            assert abs(e_gpu[i] - d["E_jump"]) <= 1e-8 * d["E_jump"] + 1e-12 * d["E_bot_in"], \
                (p, i, e_gpu[i], d["E_jump"])
    after = ctx.read_state()
    for a, b in zip(before, after):
        assert np.array_equal(a, b)


def test_adaptive_sweep_matches_oracle_with_same_degrees():
    """A network that reads the patch size gives a spread of degrees; the
    library records the degree each tent was solved with (after any re-solves
    at higher degrees), and the oracle run with exactly those degrees must
    agree to the FP64 bar.  Each layer's tents are drawn in decreasing chosen
    degree (the queue order the library builds after the degree choice)."""
    torch = _torch()
    pr = C.cfg2_plane_2d(m=8, p=5)
    o = oracle_for(pr)
    ctx, xq, w = gpu_for(pr)
    nt = ctx.tents.n_tents
    # a network that reads the patch size (feature 2): y_o = 10 tanh(tanh(4 f_2)) + b3_o,
    # b3 = -2.5, -5, -7, -100: degrees 2..5 from small to large patches (weights exact in BF16)
    d = OM.unpack(np.zeros(OM.N_PARAM))
    d = {k: v.copy() for k, v in d.items()}
    d["W1"][0, 2] = 4.0
    d["W2"][0, 0] = 1.0
    d["W3"][:, 0] = 10.0
    d["b3"][:] = [-2.5, -5.0, -7.0, -100.0, -100.0, -100.0, -100.0]
    bits = OM.bf16_bits(OM.pack(d).astype(np.float32))
    assert np.array_equal(OM.bf16_value(bits), OM.pack(d))
    wb = _dev_bits(bits)
    feats = torch.zeros((nt, 8), dtype=torch.float32, device="cuda")
    p_sel = torch.zeros(nt, dtype=torch.int8, device="cuda")
    p_used = torch.zeros(nt, dtype=torch.int8, device="cuda")
    eta = torch.zeros(nt, dtype=torch.float64, device="cuda")
    log_tol, eta_tol = 0.0, 1e-6
    ctx.layer_solve_adaptive(wb, log_tol, eta_tol, feats, p_sel, p_used, eta)
    ctx.status()
    ps, pu, et = p_sel.cpu().numpy(), p_used.cpu().numpy(), eta.cpu().numpy()
    f = feats.cpu().numpy()
    say(f"  selected degrees {np.bincount(ps, minlength=6)[2:]}, used {np.bincount(pu, minlength=6)[2:]}")
    assert len(set(ps.tolist())) >= 2, "weights should give several degrees"
    # selection: the oracle's FP64 forward on the library's features, except
    # where the prediction sits within FP32 rounding of the threshold
    yo, _ = OM.forward(OM.bf16_value(bits), f.astype(np.float64))
    so = OM.select_degree(yo, log_tol, pr.p)
    near = np.any(np.abs(yo[:, : pr.p - 1] - log_tol) < 1e-4, axis=1)
    assert np.array_equal(ps[~near], so[~near])
    # re-solve rule: degrees only go up, and a tent below p_max was accepted
    # only with its realised indicator within the tolerance
    assert np.all(pu >= ps)
    assert np.all(et[pu < pr.p] <= eta_tol)
    assert np.all(et >= 0)
    # the queue of every layer: a permutation of its tents, chosen degree not
    # increasing along it, tent index increasing inside a degree
    import ctypes
    from paper_1907_02367_amd import tdg

    fq = tdg.lib().tdg_debug_queue_order
    fq.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    fq.restype = ctypes.c_int
    lp = np.asarray(ctx.tents.layer_ptr)
    for layer in range(ctx.tents.n_layers):
        t0, t1 = int(lp[layer]), int(lp[layer + 1])
        q = np.zeros(t1 - t0, np.int32)
        assert fq(ctx._h, layer, q.ctypes.data, tdg._stream()) == 0
        assert np.array_equal(np.sort(q), np.arange(t0, t1))
        key = -ps[q].astype(np.int64) * (nt + 1) + q
        assert np.all(np.diff(key) > 0)
    o.run(p_per_tent=pu)
    v, s, U = ctx.read_state()
    r_vs = rel_l2(np.concatenate([v.ravel(), s.ravel()]), np.concatenate([o.v.ravel(), o.sig.ravel()]))
    r_U = rel_l2(U, o.U)
    say(f"  rel diff (v, sigma) {r_vs:.2e}, U {r_U:.2e}")
    assert r_vs <= 1e-10 and r_U <= 1e-10


@pytest.mark.parametrize("seed_basis", [0, 1, 2], ids=["monomial", "legendre", "chebyshev"])
def test_adaptive_3d_one_pass_matches_fixed_degree_solve(seed_basis):
    """3+1D degree-adaptive sweep in moment mode: below p_max the indicator and
    the tent's top values come from one pass of the matrix-core evaluation
    (kept in the workgroup's global slot until the tent is accepted).  A plain
    solve at the recorded degrees (write-back only, no indicator) must leave
    the same stored values bit for bit, with each seed basis of the Trefftz
    recursion (Sec. 6.3)."""
    torch = _torch()
    pr = C.cfg5_cube_3d(m=3, p=5, variant="b", regions=1, T=0.2)
    pr.gamma = 0.4 * 0.8 ** 4  # (the jittered cube needs the lower edge slope to pitch)
    ctx, xq, w = gpu_for(pr, gram_mode=1, seed_basis=seed_basis)
    nt = ctx.tents.n_tents
    # a network that reads the patch size: degrees 3..5 (weights exact in BF16)
    d = OM.unpack(np.zeros(OM.N_PARAM))
    d = {k: v.copy() for k, v in d.items()}
    d["W1"][0, 2] = 4.0
    d["W2"][0, 0] = 1.0
    d["W3"][:, 0] = 10.0
    d["b3"][:] = [100.0, -7.0, -7.5, -100.0, -100.0, -100.0, -100.0]
    bits = OM.bf16_bits(OM.pack(d).astype(np.float32))
    assert np.array_equal(OM.bf16_value(bits), OM.pack(d))
    wb = _dev_bits(bits)
    feats = torch.zeros((nt, 8), dtype=torch.float32, device="cuda")
    p_sel = torch.zeros(nt, dtype=torch.int8, device="cuda")
    p_used = torch.zeros(nt, dtype=torch.int8, device="cuda")
    eta = torch.zeros(nt, dtype=torch.float64, device="cuda")
    ctx.layer_solve_adaptive(wb, 0.0, 1e-7, feats, p_sel, p_used, eta)
    ctx.status()
    ps, pu = p_sel.cpu().numpy(), p_used.cpu().numpy()
    say(f"  3D selected degrees {np.bincount(ps, minlength=6)[2:]}, used {np.bincount(pu, minlength=6)[2:]}")
    assert (pu < pr.p).sum() > 0 and len(set(pu.tolist())) >= 2
    ref, _, _ = gpu_for(pr, gram_mode=1, seed_basis=seed_basis)
    ref.layer_solve(p_per_tent=p_used)
    ref.status()
    for a, b in zip(ctx.read_state(), ref.read_state()):
        assert np.array_equal(a, b)


def test_adaptive_without_network_is_fixed_pmax():
    torch = _torch()
    pr = C.cfg2_plane_2d(m=6, p=4)
    ref, _, _ = gpu_for(pr)
    ref.layer_solve()
    ref.status()
    ctx, _, _ = gpu_for(pr)
    nt = ctx.tents.n_tents
    feats = torch.zeros((nt, 8), dtype=torch.float32, device="cuda")
    p_sel = torch.zeros(nt, dtype=torch.int8, device="cuda")
    ctx.layer_solve_adaptive(None, 0.0, 0.0, feats, p_sel)
    ctx.status()
    assert np.all(p_sel.cpu().numpy() == pr.p)
    for a, b in zip(ref.read_state(), ctx.read_state()):
        assert np.array_equal(a, b)


def test_indicator_rejects_bad_degree():
    from paper_1907_02367_amd import tdg

    torch = _torch()
    pr = C.cfg2_plane_2d(m=4, p=3)
    ctx, _, _ = gpu_for(pr)
    eta = torch.zeros(ctx.tents.n_tents, dtype=torch.float64, device="cuda")
    with pytest.raises(tdg.TdgError):
        ctx.layer_indicator(0, 4, eta)
    with pytest.raises(tdg.TdgError):
        ctx.layer_indicator(ctx.tents.n_layers, 2, eta)
    with pytest.raises(ValueError):
        ctx.layer_indicator(0, 2, eta[:-1])


def test_trained_network_gains_over_fixed_pmax():
    """What the packaged network buys on a 3+1D mesh (18 cells per side, 34,992
    tetrahedra, p_max = 8, exact standing wave; layers are wider than the
    GPU has compute units): over the first 12 layers, the degree-adaptive sweep
    does fewer DOF-updates and takes less time than fixed p = 8, with the
    error against the exact solution on the reached front and against the
    fixed-p solution both below 1e-6."""
    import time

    torch = _torch()
    from paper_1907_02367_amd import learned_p as LP
    from workloads import configs as Cf

    pr = Cf.cfg5_cube_3d(m=18, p=8, seed=7, T=0.5, variant="b", regions=1)
    net = LP.load_default()
    ctx, xq = LP.make_context(pr)  # FP64, moment Gram
    W = 12
    nt = int(ctx.tents.layer_ptr[W])
    say(f"[learned gain] m=18: {nt} tents in the first {W} layers")

    def run(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    # both paths warmed up once before they are timed (first launches, caches)
    ctx.layer_solve(0, W)
    ctx.reset()
    LP.adaptive_sweep(ctx, net, -40.0, 10 * np.exp(-40.0), layer_end=W)
    ctx.reset()
    t_fixed = run(lambda: ctx.layer_solve(0, W))
    ctx.status()
    v_ref, s_ref, _ = ctx.read_state()
    e_fixed = LP.front_error(ctx, pr.coords, pr.elems, xq, field=pr.data)[0]
    ctx.reset()
    holder = {}
    t_learned = run(lambda: holder.update(b=LP.adaptive_sweep(ctx, net, -40.0, 10 * np.exp(-40.0), layer_end=W)))
    ctx.status()
    pu = holder["b"][2].cpu().numpy()[:nt]
    ps = holder["b"][1].cpu().numpy()[:nt]
    e_learned = LP.front_error(ctx, pr.coords, pr.elems, xq, field=pr.data)[0]
    e_vs_fixed = LP.front_error(ctx, pr.coords, pr.elems, xq, ref=(v_ref, s_ref))[0]
    dof_fixed = nt * ctx.table_info(8)["N"]
    dof_learned = LP.dof_count(ctx, pu)
    say(f"  fixed p=8: {t_fixed:.2f} s, e {e_fixed:.2e}; learned: {t_learned:.2f} s, e {e_learned:.2e} "
        f"(vs fixed {e_vs_fixed:.2e}), DOF-updates {dof_learned / dof_fixed:.3f} of fixed, degrees "
        f"{np.bincount(pu, minlength=9)[2:]}, re-solved higher {int((pu > ps).sum())}")
    assert e_fixed <= 1e-6 and e_learned <= 1e-6 and e_vs_fixed <= 1e-6
    assert dof_learned <= 0.9 * dof_fixed
    assert t_learned < 0.9 * t_fixed


def test_training_loop_steps_match_oracle_and_fit_a_teacher():
    """DegreeNet.train end to end on the GPU (full batch, so deterministic):
    each of two single steps against the oracle's gradient and Adam step from
    the GPU's own state (the second with the step counter carried over, so the
    bias correction is that of step 2), then 400 steps on the outputs of a
    teacher of the same architecture must cut the oracle's own loss at the
    trained BF16 weights tenfold (the oracle's run of the same loop: 0.84 to
    0.017).  Compared are the updates of the weights whose gradient is at
    least 1e-2 of the largest: the kernels' gradient is accurate to 1e-4 of
    the largest entry, so to 1 % there, and each update must be within 2 % of
    the oracle's (a wrong learning rate or bias correction is off by a factor
    of two or more); elsewhere FP32 rounding may flip the sign of a tiny
    gradient, and the first Adam step moves every weight by at most lr."""
    from paper_1907_02367_amd.learned_p import DegreeNet

    torch = _torch()
    n = 2048
    rng = np.random.default_rng(21)
    x = rng.normal(0, 1.0, (n, 8)).astype(np.float32)
    tw = np.random.default_rng(22).normal(0, 0.2, OM.N_PARAM).astype(np.float32)
    t, _ = OM.forward(OM.bf16_value(OM.bf16_bits(tw)), x.astype(np.float64))
    t = t.astype(np.float32)
    mask = (rng.uniform(size=(n, 7)) < 0.8).astype(np.float32)
    X, Y, Mk = (torch.from_numpy(a).cuda() for a in (x, t, mask))
    x64, t64, m64 = x.astype(np.float64), t.astype(np.float64), mask.astype(np.float64)
    f32 = lambda a: float(np.float32(a))  # noqa: E731
    net = DegreeNet(seed=3)
    say("[mlp train] two single steps against the oracle")
    for step, lr in ((1, 3e-3), (2, 1e-3)):
        w_before = net.w32.cpu().numpy().astype(np.float64)
        m_before = net.m.cpu().numpy().astype(np.float64)
        v_before = net.v.cpu().numpy().astype(np.float64)
        bits = net.wb.cpu().numpy().view(np.uint16)
        assert np.array_equal(bits, OM.bf16_bits(w_before.astype(np.float32)))
        net.train(X, Y, Mk, steps=1, lr=lr, lr_end=lr)
        assert net.step == step
        go, _ = OM.backward(OM.bf16_value(bits), x64, t64, m64, float(mask.size))
        wo, _, _ = OM.adam_step(w_before, go, m_before, v_before, step, f32(lr), f32(0.9), f32(0.999), f32(1e-8))
        w_gpu = net.w32.cpu().numpy().astype(np.float64)
        big = np.abs(go) >= 1e-2 * np.abs(go).max()
        assert big.sum() > 1000
        du = np.abs((w_gpu - w_before) - (wo - w_before))
        assert (du <= 2e-2 * np.abs(wo - w_before) + 1e-6 * np.abs(w_before).max())[big].all()
        if step == 1:
            assert np.abs(w_gpu - w_before).max() <= lr * (1 + 1e-5) + 1e-7 * np.abs(w_before).max()
    L0 = OM.loss(OM.bf16_value(OM.bf16_bits(w_gpu.astype(np.float32))), x64, t64, m64, float(mask.size))
    say(f"[mlp train] 400 steps from loss {L0:.3e}")
    hist = net.train(X, Y, Mk, steps=400, lr=3e-3, lr_end=3e-4, log_every=100)
    bits = net.wb.cpu().numpy().view(np.uint16)
    L1 = OM.loss(OM.bf16_value(bits), x64, t64, m64, float(mask.size))
    say(f"  loss {L0:.3e} -> {L1:.3e} (oracle at the trained weights); GPU history {hist}")
    assert np.isfinite(L1) and L1 <= 0.1 * L0, (L0, L1)
