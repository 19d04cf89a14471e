"""The L-shaped domain of Sec. 6.6 on one MI355X: the corner Bessel solution
(nu = 2/3, a = 10, T = 1, p = 3) on uniform and corner-graded meshes of the
largest element diameters of the paper's Table 1.  Per mesh: triangles, tents,
layers, DOF-updates (16 per tent), wall time of the sweep (recorded once as a
HIP graph and replayed; inputs resident), DOF-updates/s, the error e of
(v, sigma) at T and the L2 error of the recovered U at T, beside the paper's
own figures for the same h_max (context only: its mesher, pitcher and U
recovery differ, and it ran on 24 CPU threads).

    python -m paper_1907_02367_amd.studies.lshape [--out results.jsonl] [--meshes u0.07,g0.12,...]
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

# Table 1 of the paper (Sec. 6.6): h_max -> (total DOFs, L2 error of U at T, runtime [s])
PAPER_TABLE1 = {
    ("u", 0.07): (320112, 0.0178, 0.6234),
    ("u", 0.05): (875696, 0.0117, 1.5916),
    ("u", 0.03): (3894752, 0.0067, 7.9157),
    ("u", 0.01): (102320048, 0.0021, 255.3233),
    ("g", 0.12): (1138256, 0.0218, 3.276),
    ("g", 0.10): (2003536, 0.0083, 4.6809),
    ("g", 0.08): (3832624, 0.0030, 8.0069),
    ("g", 0.06): (9777536, 0.0008, 23.4588),
}


def say(*a):
    print(*a, flush=True)


def run_mesh(kind, h_max, repeats=2):
    import torch

    from paper_1907_02367_amd import tdg
    from paper_1907_02367_amd.autotune import autotune
    from workloads import configs as C

    pr = C.lshape_2d(h_max, graded=(kind == "g"))
    f = pr.data
    t0 = time.perf_counter()
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    t_pitch = time.perf_counter() - t0
    say(f"[lshape] {pr.name}: {len(pr.elems)} triangles, {T.n_tents} tents, {T.n_layers} layers "
        f"(pitched in {t_pitch:.1f} s)")
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta)
    xq, w = ctx.quad_points()
    ctx.set_initial(f.v(xq, 0.0), f.sigma(xq, 0.0), f.U(xq, 0.0))
    bx = ctx.boundary_points()
    ctx.set_boundary(f.v(bx[:, :-1], bx[:, -1]))
    L = T.n_layers
    autotune(ctx, n_layers=min(16, L), use_cache=False)
    say(f"[lshape] {pr.name}: shape {ctx.get_tuning()} gram mode {ctx.get_gram_mode()}")
    g = torch.cuda.Stream()
    with torch.cuda.stream(g):
        ctx.capture_sweep(0, L, with_reset=True, stream=g.cuda_stream)
        ctx.replay_sweep(g.cuda_stream)
        torch.cuda.synchronize()
        say(f"[lshape] {pr.name}: warm sweep done")
        t0 = time.perf_counter()
        for _ in range(repeats):
            ctx.replay_sweep(g.cuda_stream)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / repeats
    ctx.status()
    e_abs, e_rel = ctx.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T))
    _, _, U = ctx.read_state()
    ue = f.U(xq.reshape(U.shape + (2,)), pr.T)
    wq = w.reshape(U.shape)
    u_err = float(np.sqrt((wq * (U - ue) ** 2).sum()))
    dofs = 16.0 * T.n_tents
    out = dict(workload=pr.name, kind=kind, h_max=h_max, triangles=int(len(pr.elems)), tents=int(T.n_tents),
               layers=int(L), dof_updates=dofs, time_s=t, dof_updates_per_s=dofs / t, e_abs=e_abs, e_rel=e_rel,
               u_l2_error=u_err, shape=ctx.get_tuning(), gram_mode=ctx.get_gram_mode())
    paper = PAPER_TABLE1.get((kind, h_max))
    if paper:
        out["paper_table1"] = dict(dofs=paper[0], u_l2_error=paper[1], runtime_s=paper[2],
                                   dof_per_s=paper[0] / paper[2], threads=24)
    del ctx
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--meshes", default="u0.07,u0.05,u0.03,u0.01,g0.12,g0.10,g0.08,g0.06")
    ap.add_argument("--repeats", type=int, default=2)
    ap.add_argument("--out", default="")
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    fh = open(args.out, "a") if args.out else None
    for item in args.meshes.split(","):
        d = run_mesh(item[0], float(item[1:]), args.repeats)
        line = json.dumps(d)
        say(line)
        if fh:
            fh.write(line + "\n")
            fh.flush()


if __name__ == "__main__":
    main()
