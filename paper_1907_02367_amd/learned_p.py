"""Learned degree per tent: data from the method's own indicator, training on
the GPU with the library's network kernels, and degree-adaptive sweeps.

Indicator.  For a tent solved at degree p, eta_T(p) is the energy of the jump
between the tent solution and the incoming values on its bottom facets, the
term of the tent's energy balance that the Trefftz space of degree p cannot
match (eq. 4.1 tested with w = u).  The library computes it without writing
anything (trefftz_layer_indicator), so one sweep at p_max yields, for every
tent, its features and eta_T(p) for all p at once.

Network.  8 features -> 64 -> 64 -> 7 (tanh), BF16 weights, FP32 arithmetic;
output o predicts log eta_T(o + 2).  Training minimises the masked mean
squared error of the log indicator with Adam; forward, backward and the Adam
step are the library's kernels (tdg_mlp_*), the host only slices mini-batches.

Use.  Per layer the library computes the features, evaluates the network and
gives each tent the smallest degree whose predicted log indicator is below
log_eta_tol (else p_max); a tent whose realised indicator exceeds eta_tol is
solved again one degree higher (up to p_max, where it is accepted) before
anything is written, so fixed p_max is both the fallback and the yardstick.
"""
from __future__ import annotations

import os
import time

import numpy as np

from . import tdg

N_FEAT, N_OUT = 8, 7
# network trained by paper_1907_02367_amd.studies.learned on 3+1D unit-cube
# meshes (p_max = 8; sizes 3, 5 and the first layers of 25 cells per side)
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "degree_net_3d.npz")


def _torch():
    import torch

    return torch


class DegreeNet:
    """FP32 master weights, their BF16 copy and the Adam moments, on the GPU."""

    def __init__(self, seed=0, device="cuda"):
        torch = _torch()
        P = tdg.mlp_nparam()
        rng = np.random.default_rng(seed)
        parts = []
        for fan_out, fan_in in ((64, 8), (64, 64), (7, 64)):
            lim = np.sqrt(6.0 / (fan_in + fan_out))  # Glorot uniform
            parts += [rng.uniform(-lim, lim, fan_out * fan_in), np.zeros(fan_out)]
        w = np.concatenate(parts).astype(np.float32)
        assert w.size == P
        self.P = P
        self.w32 = torch.from_numpy(w).to(device)
        self.wb = torch.zeros(P, dtype=torch.int16, device=device)
        self.m = torch.zeros(P, dtype=torch.float32, device=device)
        self.v = torch.zeros(P, dtype=torch.float32, device=device)
        self.step = 0
        tdg.mlp_round(self.w32, self.wb)

    def set_output_bias(self, b):
        """Sets b3 (the last 7 parameters) and refreshes the BF16 copy."""
        torch = _torch()
        self.w32[-N_OUT:] = torch.as_tensor(np.asarray(b, dtype=np.float32), device=self.w32.device)
        tdg.mlp_round(self.w32, self.wb)

    def predict(self, x):
        return tdg.mlp_forward(self.wb, x)

    def train(self, X, Y, M, steps=2000, batch=4096, lr=3e-3, lr_end=3e-4, seed=0, log_every=0):
        """Adam on the masked MSE of log eta over (X, Y, M) (device tensors).
        Returns the loss history (one value per step)."""
        torch = _torch()
        n = X.shape[0]
        g = torch.Generator(device="cpu").manual_seed(seed)
        partial = None
        grad = torch.empty(self.P + 1, dtype=torch.float32, device=X.device)
        hist = []
        for it in range(steps):
            if n > batch:
                idx = torch.randint(0, n, (batch,), generator=g).to(X.device)
                xb, yb, mb = X[idx].contiguous(), Y[idx].contiguous(), M[idx].contiguous()
            else:
                xb, yb, mb = X, Y, M
            # mean over the batch's entries (masked ones count as zero error)
            grad, partial = tdg.mlp_backward(self.wb, xb, yb, mb, float(mb.numel()), partial, grad)
            self.step += 1
            frac = it / max(1, steps - 1)
            lr_t = lr * (lr_end / lr) ** frac
            tdg.mlp_adam(self.w32, self.wb, grad, self.m, self.v, self.step, lr_t)
            if log_every and (it % log_every == 0 or it == steps - 1):
                hist.append((it, float(grad[-1].item())))
        return hist

    def state_dict(self):
        return {"w32": self.w32.cpu().numpy()}

    def load_state_dict(self, d):
        torch = _torch()
        self.w32.copy_(torch.from_numpy(np.asarray(d["w32"], dtype=np.float32)))
        tdg.mlp_round(self.w32, self.wb)


def load_default():
    """The packaged degree network (FP32 master weights and their BF16 copy)."""
    net = DegreeNet(seed=0)
    net.load_state_dict(np.load(DEFAULT_WEIGHTS))
    return net


def make_context(pr, p_max=None, precision=0, device=None, gram_mode=None):
    """Library context of a workload (synthetic inputs resident on the GPU).
    gram_mode None: the moment Gram in FP64 contexts, where it fits."""
    f = pr.data
    gamma = pr.gamma
    while True:  # a strongly jittered mesh may need a smaller edge-slope factor
        try:
            T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, gamma)
            break
        except tdg.TdgError as e:
            if e.name != "TDG_ENONCAUSAL" or gamma < 0.05:
                raise
            gamma *= 0.8
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=p_max or pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta,
                      precision=precision)
    mode = (1 if precision == 0 else 0) if gram_mode is None else gram_mode
    if mode:
        try:
            ctx.set_gram_mode(mode)
        except tdg.TdgError:
            if gram_mode is not None:
                raise
    xq, w = ctx.quad_points()
    ctx.set_initial(f.v(xq, 0.0), f.sigma(xq, 0.0), f.U(xq, 0.0))
    if ctx.nb:
        bx = ctx.boundary_points()
        ctx.set_boundary(f.v(bx[:, :-1], bx[:, -1]))
    return ctx, xq


def collect(ctx, p_list=range(2, 9), layer_stride=1, progress=None, max_layers=None):
    """Sweeps the context at p_max (the first max_layers layers, default all);
    before every `layer_stride`-th layer, records the features and eta_T(p)
    for p in p_list of its tents.  Returns device tensors X (n x 8),
    Y = log eta (n x 7), M (n x 7 mask).  progress(l, L), if given, is called
    after every tenth layer."""
    torch = _torch()
    nt = ctx.tents.n_tents
    L = ctx.tents.n_layers if max_layers is None else min(max_layers, ctx.tents.n_layers)
    lp = ctx.tents.layer_ptr
    feats = torch.zeros((nt, N_FEAT), dtype=torch.float32, device="cuda")
    eta = torch.full((N_OUT, nt), -1.0, dtype=torch.float64, device="cuda")
    taken = torch.zeros(nt, dtype=torch.bool, device="cuda")
    p_list = [p for p in p_list if 2 <= p < ctx.p_max]
    # eta_T(p_max) comes with the sweep's own solve
    ctx.set_indicator(True)
    eta_top = ctx.indicator_tensor()
    for l in range(L):
        a, b = lp[l], lp[l + 1]
        if l % layer_stride == 0:
            ctx.tent_features(l, feats)
            for p in p_list:
                ctx.layer_indicator(l, p, eta[p - 2])
            taken[a:b] = True
        ctx.layer_solve(l, l + 1)
        if l % layer_stride == 0 and ctx.p_max >= 2:
            eta[ctx.p_max - 2, a:b] = eta_top[a:b]
        if progress is not None and (l % 10 == 9 or l == L - 1):
            torch.cuda.synchronize()
            progress(l + 1, L)
    ctx.status()
    ctx.set_indicator(False)
    X = feats[taken].contiguous()
    E = eta[:, taken].T.contiguous()
    M = (E > 0) & torch.isfinite(E)
    Y = torch.where(M, torch.log(torch.where(M, E, torch.ones_like(E))), torch.zeros_like(E)).float().contiguous()
    return X, Y, M.float().contiguous()


def adaptive_sweep(ctx, net, log_eta_tol, eta_tol, stream=None, buffers=None, want_eta=False, block=0,
                   progress=None, layer_end=None):
    """One degree-adaptive sweep of all layers (from the current state).
    net = None: fixed p_max (the fallback).  want_eta: also record eta_T of
    every tent (costs an evaluation at the bottom points of each tent).
    block > 0: launch in blocks of that many layers, calling progress(l, L)
    after each (synchronised).  Returns the buffers (feats, p_sel, p_used, eta)
    as device tensors."""
    torch = _torch()
    nt = ctx.tents.n_tents
    if buffers is None:
        buffers = (torch.zeros((nt, N_FEAT), dtype=torch.float32, device="cuda"),
                   torch.zeros(nt, dtype=torch.int8, device="cuda"),
                   torch.zeros(nt, dtype=torch.int8, device="cuda"),
                   torch.zeros(nt, dtype=torch.float64, device="cuda"))
    feats, p_sel, p_used, eta = buffers
    L = ctx.tents.n_layers if layer_end is None else layer_end
    step = block if block > 0 else L
    for l0 in range(0, L, max(step, 1)):
        l1 = min(L, l0 + step)
        ctx.layer_solve_adaptive(None if net is None else net.wb, log_eta_tol, eta_tol, feats, p_sel, p_used,
                                 eta if want_eta else None, layer_begin=l0, layer_end=l1, stream=stream)
        if progress is not None and block > 0:
            torch.cuda.synchronize()
            progress(l1, L)
    return buffers


def fixed_sweep(ctx, block=0, progress=None, layer_end=None):
    """Plain sweep at p_max, optionally in blocks of layers with progress."""
    torch = _torch()
    L = ctx.tents.n_layers if layer_end is None else layer_end
    step = block if block > 0 else L
    for l0 in range(0, L, max(step, 1)):
        l1 = min(L, l0 + step)
        ctx.layer_solve(l0, l1)
        if progress is not None and block > 0:
            torch.cuda.synchronize()
            progress(l1, L)


def front_error(ctx, coords, elems, xq, field=None, ref=None):
    """Error e (the c^-2-weighted L2 norm of Sec. 6) of the stored values on
    the current front, against the exact field at each point's own time on
    the front (field) or against reference values at the same points (ref =
    (v, sigma) of another sweep over the same layers).  Returns (e_abs, e_rel)."""
    if ref is not None:
        return ctx.eval_error(ref[0], ref[1])
    coords = np.asarray(coords, dtype=np.float64)
    elems = np.asarray(elems)
    n, Q = ctx.n, ctx.Q
    # barycentric coordinates of the reference points (the same in every element)
    B = np.vstack([coords[elems[0]].T, np.ones(n + 1)])
    lam = np.linalg.solve(B, np.vstack([xq[:Q].T, np.ones(Q)])).T  # Q x (n+1)
    tq = (ctx.front()[elems] @ lam.T).reshape(-1)  # ne*Q, element-major
    return ctx.eval_error(field.v(xq, tq), field.sigma(xq, tq))


def dof_count(ctx, p_used):
    """sum over tents of dim U^p for the degrees used."""
    N = np.array([0] + [ctx.table_info(p)["N"] for p in range(1, ctx.p_max + 1)])
    return int(N[np.asarray(p_used, dtype=np.int64)].sum())


def timed(fn, reps=1):
    torch = _torch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps
