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


def build_dataset(problems, layer_stride=1):
    import torch

    from paper_1907_02367_amd import learned_p as LP

    Xs, Ys, Ms = [], [], []
    for pr in problems:
        t0 = time.perf_counter()
        ctx, _ = LP.make_context(pr)
        X, Y, M = LP.collect(ctx, range(2, pr.p + 1), layer_stride,
                             progress=lambda l, L: say(f"[data] {pr.name}: layer {l}/{L} "
                                                       f"{time.perf_counter() - t0:.1f} s"))
        Xs.append(X)
        Ys.append(Y)
        Ms.append(M)
        say(f"[data] {pr.name}: {ctx.tents.n_tents} tents, {ctx.tents.n_layers} layers, {X.shape[0]} samples, "
            f"{time.perf_counter() - t0:.1f} s")
        del ctx
    return torch.cat(Xs).contiguous(), torch.cat(Ys).contiguous(), torch.cat(Ms).contiguous()


def evaluate(pr, net, tols, precisions=(0, 1), reps=1):
    """Fixed p_max FP64 reference, then adaptive sweeps; yields result dicts."""
    import torch

    from paper_1907_02367_amd import learned_p as LP

    f = pr.data
    ctx, xq = LP.make_context(pr)
    nt = ctx.tents.n_tents
    N = {p: ctx.table_info(p)["N"] for p in range(1, pr.p + 1)}
    dof_fixed = nt * N[pr.p]

    def sweep_fixed():
        ctx.reset()
        ctx.layer_solve()

    sweep_fixed()
    ctx.status()
    t_fixed = LP.timed(sweep_fixed, reps)
    ctx.status()
    v_ref, s_ref, _ = ctx.read_state()
    e_exact_fixed = ctx.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T)) if pr.exact else (None, None)
    base = dict(workload=pr.name, ne=len(pr.elems), tents=nt, layers=ctx.tents.n_layers, p_max=pr.p)
    yield dict(base, run="fixed_pmax_fp64", time_s=t_fixed, dof_updates=dof_fixed,
               rate_equiv=dof_fixed / t_fixed, e_vs_exact=e_exact_fixed[0], e_vs_fixed=0.0)
    for prec in precisions:
        c2 = ctx if prec == 0 else LP.make_context(pr, precision=1)[0]
        bufs = None
        for log_tol in tols:
            eta_tol = float(np.exp(log_tol)) * 10.0

            def sweep():
                nonlocal bufs
                c2.reset()
                bufs = LP.adaptive_sweep(c2, net, log_tol, eta_tol, buffers=bufs)

            sweep()
            c2.status()
            t = LP.timed(sweep, reps)
            c2.status()
            pu = bufs[2].cpu().numpy()
            ps = bufs[1].cpu().numpy()
            dofs = LP.dof_count(c2, pu)
            e_fixed = c2.eval_error(v_ref, s_ref)[0]
            e_ex = c2.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T))[0] if pr.exact else None
            yield dict(base, run=f"learned_{'fp64' if prec == 0 else 'mixed'}", log_eta_tol=log_tol,
                       eta_tol=eta_tol, time_s=t, dof_updates=dofs, rate_equiv=dof_fixed / t,
                       speedup=t_fixed / t, e_vs_exact=e_ex, e_vs_fixed=e_fixed,
                       p_hist={int(p): int((pu == p).sum()) for p in range(2, pr.p + 1)},
                       resolved=int(((pu == pr.p) & (ps < pr.p)).sum()))
        if prec == 1:
            # fixed p_max in mixed precision
            def sweep_m():
                c2.reset()
                c2.layer_solve()

            sweep_m()
            c2.status()
            t = LP.timed(sweep_m, reps)
            c2.status()
            e_fixed = c2.eval_error(v_ref, s_ref)[0]
            yield dict(base, run="fixed_pmax_mixed", time_s=t, dof_updates=dof_fixed, rate_equiv=dof_fixed / t,
                       speedup=t_fixed / t, e_vs_fixed=e_fixed)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train-m", default="2,3")
    ap.add_argument("--train-seeds", default="1,2")
    ap.add_argument("--train-T", type=float, default=0.3)
    ap.add_argument("--eval-m", default="4")
    ap.add_argument("--eval-T", type=float, default=0.5)
    ap.add_argument("--p-max", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--layer-stride", type=int, default=1)
    ap.add_argument("--tols", default="-30,-34,-38,-42")
    ap.add_argument("--no-mixed", action="store_true")
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
        probs = train_problems([int(x) for x in args.train_m.split(",")], [int(x) for x in args.train_seeds.split(",")],
                               args.p_max, args.train_T)
        X, Y, M = build_dataset(probs, args.layer_stride)
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
    tols = [float(x) for x in args.tols.split(",")]
    for m in [int(x) for x in args.eval_m.split(",")]:
        for variant in ("b", "a"):
            pr = problem(m, args.p_max, 7, args.eval_T, variant)
            for d in evaluate(pr, net, tols, precisions=(0,) if args.no_mixed else (0, 1)):
                emit(d)


if __name__ == "__main__":
    main()
