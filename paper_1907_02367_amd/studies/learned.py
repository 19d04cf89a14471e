"""Learned degree on 3+1D: train the degree network on the method's own
indicator and compare degree-adaptive sweeps with fixed p_max.

  python -m paper_1907_02367_amd.studies.learned --out results.jsonl

Training data: coarse unit-cube meshes (Kuhn tetrahedra, jittered), both
speed variants (c per region drawn from U[1,2], or c = 1.5 with an exact
standing wave), several seeds; each is swept at p_max and, before every
layer, the features and eta_T(p), p = 2..p_max, of its tents are recorded.
The network is trained on the GPU with the library's kernels.

Evaluation (held-out seed and mesh size): fixed p_max in FP64 is the
reference; degree-adaptive sweeps at several indicator tolerances, in FP64
and in mixed precision, report wall time, DOF-updates done, the degrees used
and the error e (Sec. 6) against the fixed-p_max solution and, where the data
is an exact solution, against it.  The rate at equal error counts the
DOF-updates of the fixed-p_max sweep (the work it replaces) per second.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def say(*a):
    print(*a, flush=True)


def problem(m, p_max, seed, T, variant):
    """3+1D unit cube.  'b': c = 1.5, exact standing wave; 'a': one speed
    drawn from U[1,2] (seeded), U0 = sin sin sin, homogeneous Dirichlet.
    (Several speeds per tent multiply the unknowns by the number of speed
    groups, up to 8 x 284 at p = 8, beyond a one-workgroup LU.)"""
    from workloads import configs as C

    return C.cfg5_cube_3d(m=m, p=p_max, seed=seed, T=T, variant=variant, regions=1)


def train_problems(ms, seeds, p_max, T):
    return [problem(m, p_max, seed, T, v) for m in ms for seed in seeds for v in ("a", "b")]


def build_dataset(problems, layer_stride=1, max_layers=None):
    import torch

    from paper_1907_02367_amd import learned_p as LP

    Xs, Ys, Ms = [], [], []
    for pr in problems:
        t0 = time.perf_counter()
        ctx, _ = LP.make_context(pr)
        X, Y, M = LP.collect(ctx, range(2, pr.p + 1), layer_stride,
                             progress=lambda l, L: say(f"[data] {pr.name}: layer {l}/{L} "
                                                       f"{time.perf_counter() - t0:.1f} s"),
                             max_layers=max_layers)
        Xs.append(X)
        Ys.append(Y)
        Ms.append(M)
        say(f"[data] {pr.name}: {ctx.tents.n_tents} tents, {ctx.tents.n_layers} layers, {X.shape[0]} samples, "
            f"{time.perf_counter() - t0:.1f} s")
        del ctx
    return torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous(), torch.cat(Ms).contiguous()


def evaluate(pr, net, tols, precisions=(0, 1), block=20, window=None):
    """Fixed p_max FP64 reference, then adaptive sweeps over the first
    `window` layers (all by default), one timed sweep each, launched in blocks
    of layers with a progress line per block; yields result dicts.  Errors are
    taken on the front reached (flat at T for a full sweep), against the
    exact field at each point's time where there is one, and against the
    fixed-p_max values."""
    from paper_1907_02367_amd import learned_p as LP

    f = pr.data
    ctx, xq = LP.make_context(pr)
    L = ctx.tents.n_layers if window is None else min(window, ctx.tents.n_layers)
    nt = int(ctx.tents.layer_ptr[L])
    N = {p: ctx.table_info(p)["N"] for p in range(1, pr.p + 1)}
    dof_fixed = nt * N[pr.p]

    def prog(tag):
        t0 = time.perf_counter()
        return lambda l, LL: say(f"[{tag}] layer {l}/{LL} {time.perf_counter() - t0:.1f} s")

    def errs(c, ref=None):
        e_ex = LP.front_error(c, pr.coords, pr.elems, xq, field=f)[0] if pr.exact else None
        e_ref = LP.front_error(c, pr.coords, pr.elems, xq, ref=ref)[0] if ref is not None else 0.0
        return e_ex, e_ref

    t_fixed = LP.timed(lambda: LP.fixed_sweep(ctx, block, prog(f"{pr.name} fixed"), layer_end=L))
    ctx.status()
    v_ref, s_ref, _ = ctx.read_state()
    e_ex, _ = errs(ctx)
    base = dict(workload=pr.name, ne=len(pr.elems), tents=nt, layers=L, layers_total=ctx.tents.n_layers,
                p_max=pr.p)
    yield dict(base, run="fixed_pmax_fp64", time_s=t_fixed, dof_updates=dof_fixed,
               rate_equiv=dof_fixed / t_fixed, e_vs_exact=e_ex, e_vs_fixed=0.0)
    for prec in precisions:
        c2 = ctx if prec == 0 else LP.make_context(pr, precision=1)[0]
        bufs = None
        for log_tol in tols:
            eta_tol = float(np.exp(log_tol)) * 10.0
            c2.reset()
            holder = {}

            def sweep():
                holder["b"] = LP.adaptive_sweep(c2, net, log_tol, eta_tol, buffers=bufs, block=block,
                                                progress=prog(f"{pr.name} learned {log_tol}"), layer_end=L)

            t = LP.timed(sweep)
            bufs = holder["b"]
            c2.status()
            pu = bufs[2].cpu().numpy()[:nt]
            ps = bufs[1].cpu().numpy()[:nt]
            dofs = LP.dof_count(c2, pu)
            e_ex, e_fixed = errs(c2, (v_ref, s_ref))
            yield dict(base, run=f"learned_{'fp64' if prec == 0 else 'mixed'}", log_eta_tol=log_tol,
                       eta_tol=eta_tol, time_s=t, dof_updates=dofs, rate_equiv=dof_fixed / t,
                       speedup=t_fixed / t, e_vs_exact=e_ex, e_vs_fixed=e_fixed,
                       p_hist={int(p): int((pu == p).sum()) for p in range(2, pr.p + 1)},
                       resolved=int((pu > ps).sum()))
        if prec == 1:
            c2.reset()
            t = LP.timed(lambda: LP.fixed_sweep(c2, block, prog(f"{pr.name} fixed mixed"), layer_end=L))
            c2.status()
            e_ex, e_fixed = errs(c2, (v_ref, s_ref))
            yield dict(base, run="fixed_pmax_mixed", time_s=t, dof_updates=dof_fixed, rate_equiv=dof_fixed / t,
                       speedup=t_fixed / t, e_vs_exact=e_ex, e_vs_fixed=e_fixed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-m", default="3,5,7")
    ap.add_argument("--train-seeds", default="1,2")
    ap.add_argument("--train-T", type=float, default=0.3)
    ap.add_argument("--eval-m", default="4")
    ap.add_argument("--eval-T", type=float, default=0.5)
    ap.add_argument("--p-max", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--layer-stride", type=int, default=1)
    ap.add_argument("--tols", default="-30,-34,-38,-42")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--eval-variants", default="b,a")
    ap.add_argument("--eval-window", type=int, default=0, help="layers per evaluation sweep (0: all)")
    ap.add_argument("--train-window-m", default="", help="mesh sizes sampled over their first layers only")
    ap.add_argument("--train-window", type=int, default=16)
    ap.add_argument("--save-data", default="", help="write the training set (npz)")
    ap.add_argument("--load-data", default="", help="training sets (npz, comma-separated) to add")
    ap.add_argument("--save", default="")
    ap.add_argument("--load", default="")
    ap.add_argument("--out", default="")
    args = ap.parse_args()

    import torch

    from paper_1907_02367_amd import learned_p as LP
    from workloads import configs as C

    torch.cuda.set_device(0)
    out = open(args.out, "a") if args.out else None

    def emit(d):
        line = json.dumps(d)
        say(line)
        if out:
            out.write(line + "\n")
            out.flush()

    net = LP.DegreeNet(seed=0)
    if args.load:
        net.load_state_dict(np.load(args.load))
    else:
        ints = lambda a: [int(x) for x in a.split(",")] if a else []  # noqa: E731
        parts = []
        probs = train_problems(ints(args.train_m), ints(args.train_seeds), args.p_max, args.train_T)
        if probs:
            parts.append(build_dataset(probs, args.layer_stride))
        wprobs = train_problems(ints(args.train_window_m), ints(args.train_seeds), args.p_max, args.eval_T)
        if wprobs:
            parts.append(build_dataset(wprobs, args.layer_stride, max_layers=args.train_window))
        if args.load_data:
            for path in args.load_data.split(","):
                d = np.load(path)
                parts.append(tuple(torch.from_numpy(d[k]).cuda() for k in ("X", "Y", "M")))
        X, Y, M = (torch.cat([pt[i] for pt in parts]).contiguous() for i in range(3))
        if args.save_data:
            np.savez(args.save_data, X=X.cpu().numpy(), Y=Y.cpu().numpy(), M=M.cpu().numpy())
        # output bias at the per-degree mean of the targets
        mean = ((Y * M).sum(0) / M.sum(0).clamp(min=1)).cpu().numpy()
        net.set_output_bias(mean)
        n = X.shape[0]
        perm = torch.randperm(n, generator=torch.Generator().manual_seed(0)).cuda()
        nval = max(1, n // 10)
        va, tr = perm[:nval], perm[nval:]
        t0 = time.perf_counter()
        hist = net.train(X[tr].contiguous(), Y[tr].contiguous(), M[tr].contiguous(), steps=args.steps,
                         log_every=max(1, args.steps // 10))
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t0
        yv = net.predict(X[va].contiguous())
        mv = M[va]
        rmse = float(torch.sqrt(((yv - Y[va]) ** 2 * mv).sum() / mv.sum()).item())
        emit(dict(run="train", samples=int(n), steps=args.steps, train_s=t_train, loss_hist=hist,
                  val_rmse_log_eta=rmse, mean_log_eta_by_p=[float(x) for x in mean]))
        if args.save:
            np.savez(args.save, **net.state_dict())
    tols = [float(x) for x in args.tols.split(",")] if args.tols else []
    for m in ([int(x) for x in args.eval_m.split(",")] if args.eval_m else []):
        for variant in args.eval_variants.split(","):
            pr = problem(m, args.p_max, 7, args.eval_T, variant)
            for d in evaluate(pr, net, tols, precisions=(0,) if args.no_mixed else (0, 1),
                              window=args.eval_window or None):
                emit(d)


if __name__ == "__main__":
    main()
