"""Mixed-precision study on the 2+1D precision workload (jittered Delaunay of
a 100x100 grid, plane wave): for each degree p, the FP64 path and the mixed
path (FP32 matrix-core Gram, FP64 LU and refinement) solve the same layers;
reported per p: time, DOF-updates/s, e_abs at the last solved time against
the exact solution for both, the relative difference of the two solutions,
refinement steps and the share of tents that fell back to the FP64 Gram.

    python -m paper_1907_02367_amd.studies.precision [--layers N] [--m 100] [--p 2 3 ...]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np


def run_one(pr, precision, layers, stream=None):
    import torch

    from paper_1907_02367_amd import tdg
    from paper_1907_02367_amd.autotune import autotune

    f = pr.data
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=pr.p, precision=precision)
    xq, _ = ctx.quad_points()
    ctx.set_initial(f.v(xq, 0.0), f.sigma(xq, 0.0), f.U(xq, 0.0))
    bx = ctx.boundary_points()
    ctx.set_boundary(f.v(bx[:, :-1], bx[:, -1]))
    L = T.n_layers if layers is None else min(layers, T.n_layers)
    autotune(ctx, n_layers=min(16, L), use_cache=False)
    ctx.reset()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.layer_solve(0, L)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ctx.status()
    v, s, U = ctx.read_state()
    nt = int(T.layer_ptr[L])
    ir, _ = ctx.tent_stats(0, nt)
    info = ctx.table_info(pr.p)
    out = dict(time_s=el, tents=nt, layers=L, dof_per_s=nt * info["N"] / el, shape=ctx.get_tuning())
    if L == T.n_layers:
        out["e_abs"], out["e_rel"] = ctx.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T))
    if precision:
        out["ir_steps_mean"] = float((ir % 1000).mean())
        out["fp64_fallback_pct"] = float(100 * (ir >= 1000).mean())
    return out, (v, s, U)


def main():
    from workloads import configs as C

    ap = argparse.ArgumentParser()
    ap.add_argument("--m", type=int, default=100)
    ap.add_argument("--layers", type=int, default=None)
    ap.add_argument("--p", type=int, nargs="*", default=[2, 3, 4, 5, 6, 7, 8])
    args = ap.parse_args()
    for p in args.p:
        pr = C.cfg3_precision_2d(p=p, m=args.m)
        r64, s64 = run_one(pr, 0, args.layers)
        r32, s32 = run_one(pr, 1, args.layers)
        vs64 = np.concatenate([s64[0].ravel(), s64[1].ravel()])
        vs32 = np.concatenate([s32[0].ravel(), s32[1].ravel()])
        diff = float(np.linalg.norm(vs32 - vs64) / np.linalg.norm(vs64))
        print(json.dumps(dict(p=p, mesh_triangles=len(pr.elems), fp64=r64, mixed=r32,
                              rel_diff_mixed_vs_fp64=diff)), flush=True)


if __name__ == "__main__":
    main()
