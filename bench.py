#!/usr/bin/env python3
"""Throughput of the tent-pitched Trefftz-DG layer solve on one MI355X.

One step = one pass of the whole hot path over the workload: restore the
initial values and the flat front (device to device), then solve every layer
of tents from t = 0 to T (one launch per layer; all tents of a layer in that
launch).  The step is recorded once as a HIP graph and replayed; the same
sweep launched layer by layer from the host is timed too (informational).
Inputs (mesh tables, initial values, boundary data) are resident in HBM
before the timed region starts.

value = DOF-updates per second = sum over tents of dim U^p / wall time of a step.
The roofline object reports the tent kernel: algorithmic FP64 flops per launch
(the operation count of the method, not the kernel's padded work) divided by
its average launch duration: HIP events on the replay stream around every
timed replay, divided by the launches of the sweep.

cpu_baseline: the CPU oracle (plain NumPy, one process) on a bounded prefix of
the same workload, on this machine's host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tent DOF-updates/sec at fixed L2 error (FP64 plain vs mixed+learned-p); % matrix peak"
FP64_PEAK = 78.6e12   # MI355X FP64 (vector and matrix), FLOP/s
HBM_PEAK = 8.0e12     # B/s


def workload(name):
    from workloads import configs as C

    if name == "cfg2":
        pr = C.cfg2_plane_2d()
        desc = ("2+1D plain FP64 batched: unit square, seeded Delaunay of a jittered 32x32 grid "
                f"({len(pr.elems)} triangles, h~0.05), c=1, p=4 (25 basis functions), plane wave |k|=2pi, T=1")
    elif name == "cfg1":
        pr = C.cfg1_standing_1d()
        desc = "1+1D plain: [0,1], 16 elements, c=1, p=3, standing wave, T=1"
    elif name == "cfg4":
        pr = C.cfg4_interface_2d()
        desc = ("2+1D heterogeneous uneven batch: unit square, mesh aligned with x=0.5 "
                f"({len(pr.elems)} triangles), c=1 (x<0.5) / 3 (x>0.5), p=4 (25 per speed group, 50 on "
                "interface tents), Gaussian pulse width 0.05 at a seeded centre, homogeneous Dirichlet, T=1")
    elif name in ("lshape", "lshape_graded"):
        graded = name == "lshape_graded"
        pr = C.lshape_2d(0.06 if graded else 0.01, graded)
        desc = (f"2+1D L-shaped domain (Sec. 6.6), {'corner-graded' if graded else 'uniform'} structured mesh, "
                f"h_max={pr.meta['h_max']} ({len(pr.elems)} triangles), c=1, p=3, corner Bessel solution "
                "nu=2/3, a=10, T=1")
    elif name.startswith("cfg3"):
        p = int(name.split("p")[-1]) if "p" in name else 8
        pr = C.cfg3_precision_2d(p=p)
        desc = f"2+1D: seeded Delaunay of a jittered 100x100 grid ({len(pr.elems)} triangles), c=1, p={p}, plane wave, T=1"
    else:
        raise SystemExit(f"unknown workload {name}")
    return pr, desc


def op_counts(ctx, pr, tents):
    """Algorithmic flops, HBM bytes and unknowns per tent (point-value layout):
    flops = 2*(2 Q_T nnz) [fields at top and bottom points] + K NW (NW+1) [symmetric Gram]
          + 4 K NW [right-hand side and top evaluation] + 2/3 S^3 + 2 S^2 [LU and solve],
    K = Q_T (n+1), Q_T = patch size * points per element, S = groups * NW (one
    Trefftz space per speed group); face terms are not counted.
    bytes = 2 Q_T (n+2) 8; unknowns (DOFs) = groups * N."""
    info = ctx.table_info(pr.p)
    NW = info["N"] - 1
    n = pr.n
    nv = len(pr.coords)
    patch = np.bincount(pr.elems.ravel(), minlength=nv)
    # speed groups per vertex: distinct speeds among the patch elements
    _, cid = np.unique(pr.c, return_inverse=True)
    pairs = np.unique(np.stack([pr.elems.ravel(), np.repeat(cid, n + 1)], axis=1), axis=0)
    groups = np.bincount(pairs[:, 0], minlength=nv)
    QT = patch[tents.vertex].astype(np.float64) * info["Q"]
    m = groups[tents.vertex].astype(np.float64)
    K = QT * (n + 1)
    S = m * NW
    flops = 4.0 * QT * info["nnz_fields"] + K * NW * (NW + 1) + 4.0 * K * NW + (2.0 / 3.0) * S ** 3 + 2.0 * S ** 2
    bytes_ = 2.0 * QT * (n + 2) * 8
    return flops, bytes_, m * info["N"]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for f in ("tent_kernel.hip", "tdg_internal.h"):
        with open(os.path.join(ROOT, "paper_1907_02367_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_name):
    """HBM bytes per tent-kernel launch from the committed rocprofv3 counter
    summary of this workload, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"tent_layer_kernel_{workload_name}_traffic.json")
    try:
        with open(path) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(d["hbm_bytes_per_launch"])


def learned_3d(m=25, window=24, log_tol=-40.0):
    """Degree-adaptive (packaged network) vs fixed p = 8 on the 3+1D unit cube
    (m cells per side, 6 m^3 jittered Kuhn tetrahedra, c = 1.5, exact standing
    wave), over the first `window` layers, both in FP64 with the moment Gram.
    Errors: the paper's e on the reached front against the exact field at each
    point's time.  The fixed run also reports its algorithmic FLOP rate."""
    import torch

    from paper_1907_02367_amd import learned_p as LP
    from workloads import configs as C

    pr = C.cfg5_cube_3d(m=m, p=8, seed=7, T=0.5, variant="b", regions=1)
    net = LP.load_default()
    ctx, xq = LP.make_context(pr)
    nt = int(ctx.tents.layer_ptr[window])
    flops, _, N = op_counts(ctx, pr, ctx.tents)
    wflops = float(flops[:nt].sum())
    dof_fixed = float(N[:nt].sum())
    out = {"workload": f"3+1D unit cube, {m}^3 x 6 jittered Kuhn tets ({len(pr.elems)}), c=1.5, standing wave, "
                       f"p_max=8, first {window} of {ctx.tents.n_layers} layers ({nt} tents)",
           "log_eta_tol": log_tol, "gram_mode": ctx.get_gram_mode()}
    t = LP.timed(lambda: ctx.layer_solve(0, window))
    ctx.status()
    e = LP.front_error(ctx, pr.coords, pr.elems, xq, field=pr.data)[0]
    out["fixed_fp64"] = {"time_s": t, "dof_updates_per_s": dof_fixed / t, "e": e,
                         "alg_tflops": wflops / t / 1e12, "alg_frac_fp64_peak": wflops / t / FP64_PEAK}
    ctx.reset()
    holder = {}
    t = LP.timed(lambda: holder.update(b=LP.adaptive_sweep(ctx, net, log_tol, 10 * np.exp(log_tol), layer_end=window)))
    ctx.status()
    pu = holder["b"][2].cpu().numpy()[:nt]
    e = LP.front_error(ctx, pr.coords, pr.elems, xq, field=pr.data)[0]
    out["learned_fp64"] = {"time_s": t, "equiv_dof_updates_per_s": dof_fixed / t,
                           "dof_updates_done": LP.dof_count(ctx, pu), "e": e,
                           "speedup_vs_fixed_fp64": out["fixed_fp64"]["time_s"] / t,
                           "degrees": {int(p): int((pu == p).sum()) for p in range(2, 9) if (pu == p).any()}}
    del ctx
    torch.cuda.empty_cache()
    return out


def cpu_baseline(pr, budget_s: float, dofs_per_tent, n_tents_gpu):
    """The oracle on the first layers of the same workload.  For large
    workloads the oracle pitches only up to a shorter final time (the first
    layers are the same tents; the pure-Python pitcher would otherwise take
    longer than the whole budget)."""
    from oracle.pitcher import pitch
    from oracle.tdg import OracleTDG

    f = pr.data
    T_or = pr.T * min(1.0, 60000.0 / max(n_tents_gpu, 1))
    tents, lp = pitch(pr.coords, pr.elems, pr.c, T_or, pr.gamma)
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lp, p=pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta,
                  gD=lambda x, t: f.v(x, t))
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    t0 = time.perf_counter()
    layers = 0
    while layers < len(lp) - 1 and time.perf_counter() - t0 < budget_s:
        o.run_layers(layers, layers + 1)
        layers += 1
    el = time.perf_counter() - t0
    ntents = lp[layers]
    # unknowns per tent of the oracle's own tents (speed groups x dim U^p)
    dofs = float(np.sum(dofs_per_tent[:ntents])) if T_or == pr.T else None
    if dofs is None:
        from oracle.trefftz import dim_U

        groups = [len({pr.c[e] for e in o.topo.patch[V]}) for V, _, _ in tents[:ntents]]
        dofs = float(sum(groups)) * dim_U(pr.n, pr.p)
    return {"value": dofs / el, "unit": "DOF-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {layers} of {len(lp) - 1} layers ({ntents} tents) in {el:.1f} s, one Python/NumPy "
                      f"process (FP64, LAPACK LU)"}


def say(msg):
    """Progress of the run (stderr; the JSON line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (automatic shape)")
    ap.add_argument("--no-learned", action="store_true", help="skip the 3+1D learned-degree comparison")
    ap.add_argument("--gram", type=int, default=-1, choices=(-1, 0, 1),
                    help="Gram mode: 0 basis values on the matrix cores, 1 monomial moments, -1 autotuned")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); domain-decomposed runs over several "
              "GPUs are not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1907_02367_amd import tdg

    torch.cuda.set_device(0)
    pr, desc = workload(args.workload)
    f = pr.data
    say(f"workload {args.workload}: {len(pr.elems)} elements")
    tents = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    say(f"pitched: {tents.n_tents} tents in {tents.n_layers} layers")
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, tents, p_max=pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta)
    xq, _ = ctx.quad_points()
    ctx.set_initial(f.v(xq, 0.0), f.sigma(xq, 0.0), f.U(xq, 0.0))
    if ctx.nb:
        bx = ctx.boundary_points()
        ctx.set_boundary(f.v(bx[:, :-1], bx[:, -1]))
    say("context bound, initial and boundary data uploaded")
    tuned, tune_ms = None, {}
    if not args.no_tune:
        from paper_1907_02367_amd.autotune import autotune

        tuned, tune_ms = autotune(ctx, use_cache=False, modes=None if args.gram < 0 else (args.gram,))
    elif args.gram > 0:
        ctx.set_gram_mode(args.gram)
    shape = ctx.get_tuning()
    shape["gram_mode"] = ctx.get_gram_mode()
    flops, bytes_, N = op_counts(ctx, pr, tents)
    L = tents.n_layers
    lp = tents.layer_ptr
    layer_flops = np.array([flops[lp[l]:lp[l + 1]].sum() for l in range(L)])
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream

    def step(events=None):
        ctx.reset(sptr)
        for l in range(L):
            if events is not None:
                events[l][0].record(stream)
            ctx.layer_solve(l, l + 1, stream=sptr)
            if events is not None:
                events[l][1].record(stream)

    # a plain device copy of known size (256 MiB), outside the timed region: the
    # reference for scaling hardware byte counters in profiles of this command
    calib = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    calib2 = torch.empty_like(calib)
    calib2.copy_(calib)
    torch.cuda.synchronize()
    del calib, calib2
    say(f"shape {ctx.get_tuning()}")
    # The step: the whole sweep (reset to the initial data, then every layer,
    # one launch each) recorded once as a HIP graph on a side stream and
    # replayed; HIP events on that stream bracket every replay, and the average
    # launch duration is a replay's event time over its launches (the gaps
    # between the graph's kernels included).
    gstream = torch.cuda.Stream()
    gptr = gstream.cuda_stream
    with torch.cuda.stream(gstream):
        ctx.capture_sweep(0, L, with_reset=True, stream=gptr)
        for _ in range(args.warmup):
            ctx.replay_sweep(gptr)
        torch.cuda.synchronize()
        say("graph captured, warm-up done")
        gev = [[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            gev[s][0].record(gstream)
            ctx.replay_sweep(gptr)
            gev[s][1].record(gstream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    say(f"{args.steps} timed steps done")
    ctx.status()
    ms_per_step = 1e3 * wall / args.steps
    step_ev_ms = np.array([gev[s][0].elapsed_time(gev[s][1]) for s in range(args.steps)])
    avg_launch_s = step_ev_ms.mean() * 1e-3 / L
    flops_per_launch = layer_flops.mean()
    achieved = flops_per_launch / avg_launch_s
    if pr.exact:
        e_abs, e_rel = ctx.eval_error(f.v(xq, pr.T), f.sigma(xq, pr.T))
    else:  # no closed-form solution: report the energy on the final front instead
        e_abs = e_rel = None
    E_T, _ = ctx.energy()
    # the same sweep launched layer by layer from the host, with events around
    # every launch (informational: launch gaps and per-launch kernel times)
    for _ in range(args.warmup):
        step()
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(L)]
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    e0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - e0) / args.steps
    kern_ms = np.array([[ev[s][l][0].elapsed_time(ev[s][l][1]) for l in range(L)] for s in range(args.steps)])
    ctx.status()
    dofs = float(N.sum())
    out = {
        "metric": METRIC,
        "value": dofs / (wall / args.steps),
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": desc,
            "tents": int(tents.n_tents), "layers": int(L), "dofs_per_tent_mean": float(N.mean()),
            "dof_updates_per_step": dofs, "e_abs_at_T": e_abs, "e_rel_at_T": e_rel, "energy_at_T": E_T,
            "step": "HIP-graph replay of the sweep (reset + one launch per layer)",
            "eager_ms_per_step": eager_ms,
            "eager_kernel_ms_per_step": float(kern_ms.sum(axis=1).mean()),
            "eager_avg_launch_us": float(kern_ms.mean() * 1e3),
            "kernel_shape": shape, "autotuned": tuned is not None,
            "autotune_ms_first_layers": tune_ms,
            "parallelism": "single GPU, all tents of a layer in one launch",
        },
        "roofline": {
            "bound": "alu", "achieved": achieved / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": achieved / FP64_PEAK, "traffic": measured_traffic(args.workload),
            "kernel": f"tent_layer_kernel<{pr.n}>", "launches_per_step": int(L),
            "avg_launch_us": avg_launch_s * 1e6, "alg_flops_per_launch": float(flops_per_launch),
            "alg_bytes_per_launch": float(bytes_.sum() / L),
        },
    }
    if not args.no_learned:
        say("learned-degree comparison (3+1D)")
        out["learned_3d"] = learned_3d()
    if not args.no_cpu_baseline:
        say("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(pr, args.cpu_seconds, N, tents.n_tents)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
