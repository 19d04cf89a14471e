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


def op_counts_deg(ctx, pr, tents, p_of_tent):
    """op_counts with a degree per tent (the learned path): per-tent algorithmic
    flops (the same formula at each tent's own degree), bytes and unknowns."""
    n = pr.n
    nv = len(pr.coords)
    patch = np.bincount(pr.elems.ravel(), minlength=nv)
    _, cid = np.unique(pr.c, return_inverse=True)
    pairs = np.unique(np.stack([pr.elems.ravel(), np.repeat(cid, n + 1)], axis=1), axis=0)
    groups = np.bincount(pairs[:, 0], minlength=nv)
    p_of_tent = np.asarray(p_of_tent, dtype=np.int64)
    tab = {p: ctx.table_info(p) for p in np.unique(p_of_tent)}
    NW = np.array([tab[p]["N"] - 1 for p in p_of_tent], dtype=np.float64)
    nnz = np.array([tab[p]["nnz_fields"] for p in p_of_tent], dtype=np.float64)
    Q = tab[int(p_of_tent[0])]["Q"]
    V = np.asarray(tents.vertex)[: len(p_of_tent)]
    QT = patch[V].astype(np.float64) * Q
    m = groups[V].astype(np.float64)
    K = QT * (n + 1)
    S = m * NW
    flops = 4.0 * QT * nnz + K * NW * (NW + 1) + 4.0 * K * NW + (2.0 / 3.0) * S ** 3 + 2.0 * S ** 2
    return flops, 2.0 * QT * (n + 2) * 8, m * (NW + 1)


def moment_exec_flops(ctx, pr, tents, p_of_tent):
    """Operations the moment form actually executes per tent (its own count,
    for comparison with the quadrature count of op_counts): top moments of the
    M2 monomials of degree <= 2p-2 weighted by w and w grad phi_d (n+1 FMAs
    each per point), bottom moments (M monomials of degree <= p by w, M1 of
    degree <= p-1 by the n+1 data terms), the contraction with the sparse field
    tables (one pass of (n+1) M1 FMAs per table term and test function), the
    LU, and the top evaluation ((n+2) fields over the M monomials per point)."""
    from math import comb

    n = pr.n
    nv = len(pr.coords)
    patch = np.bincount(pr.elems.ravel(), minlength=nv)
    p_of_tent = np.asarray(p_of_tent, dtype=np.int64)
    V = np.asarray(tents.vertex)[: len(p_of_tent)]
    out = np.zeros(len(p_of_tent))
    for p in np.unique(p_of_tent):
        t = ctx.table_info(int(p))
        NW, nnz, M, Q = t["N"] - 1, t["nnz_fields"], t["n_mono"], t["Q"]
        M1 = comb(p - 1 + n + 1, n + 1)
        M2 = comb(2 * p - 2 + n + 1, n + 1)
        sel = p_of_tent == p
        QT = patch[V[sel]].astype(np.float64) * Q
        per_pt = 2.0 * (n + 1) * M2 + 2.0 * (M + (n + 1) * M1) + 2.0 * (n + 2) * M
        out[sel] = QT * per_pt + 2.0 * nnz * (n + 1) * M1 + NW * nnz + (2.0 / 3.0) * NW ** 3
    return out


def bench_cube_3d(args):
    """3+1D learned-degree workload: unit cube, 25^3 x 6 jittered Kuhn
    tetrahedra (93,750), c = 1.5, exact standing wave, p_max = 8, FP64 moment
    Gram.  One step = reset + the degree-adaptive sweep (features, network,
    degree choice, tent solves, indicator re-solves) over the first `window`
    layers; the same window is swept at fixed p = 8 (the plain method, the
    fallback and the reference for the error) as the comparison."""
    import torch

    from paper_1907_02367_amd import learned_p as LP
    from paper_1907_02367_amd import tdg
    from workloads import configs as C

    m, window, log_tol = 25, args.window, args.log_tol
    pr = C.cfg5_cube_3d(m=m, p=8, seed=7, T=0.5, variant="b", regions=1)
    say(f"workload cube_3d: {len(pr.elems)} tetrahedra")
    ctx, xq = LP.make_context(pr)
    tents = ctx.tents
    L = tents.n_layers
    window = min(window, L)
    nt = int(tents.layer_ptr[window])
    lp = tents.layer_ptr
    say(f"pitched: {tents.n_tents} tents in {L} layers; window {window} layers ({nt} tents); "
        f"gram mode {ctx.get_gram_mode()}, shape {ctx.get_tuning()}")
    net = LP.load_default()
    stream = torch.cuda.current_stream()
    sptr = stream.cuda_stream
    bufs = (torch.zeros((tents.n_tents, 8), dtype=torch.float32, device="cuda"),
            torch.zeros(tents.n_tents, dtype=torch.int8, device="cuda"),
            torch.zeros(tents.n_tents, dtype=torch.int8, device="cuda"),
            torch.zeros(tents.n_tents, dtype=torch.float64, device="cuda"))
    eta_tol = 10.0 * np.exp(log_tol)

    def learned_step(events=None):
        ctx.reset(sptr)
        for l in range(window):
            if events is not None:
                events[l][0].record(stream)
            ctx.layer_solve_adaptive(net.wb, log_tol, eta_tol, bufs[0], bufs[1], bufs[2], None,
                                     layer_begin=l, layer_end=l + 1, stream=sptr)
            if events is not None:
                events[l][1].record(stream)

    def fixed_step(events=None):
        ctx.reset(sptr)
        for l in range(window):
            if events is not None:
                events[l][0].record(stream)
            ctx.layer_solve(l, l + 1, stream=sptr)
            if events is not None:
                events[l][1].record(stream)

    def run(step_fn, K, Wm):
        for _ in range(Wm):
            step_fn()
        torch.cuda.synchronize()
        ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in range(window)]
              for _ in range(K)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(K):
            step_fn(ev[k])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / K
        lay_ms = np.array([[ev[k][l][0].elapsed_time(ev[k][l][1]) for l in range(window)] for k in range(K)])
        return wall, lay_ms

    # a plain device copy of known size (256 MiB), outside the timed regions: the
    # reference for scaling hardware byte counters in profiles of this command
    calib = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
    torch.empty_like(calib).copy_(calib)
    torch.cuda.synchronize()
    del calib
    out_paths = {}
    if args.path in ("both", "learned"):
        wall_l, lay_l = run(learned_step, args.steps, args.warmup)
        ctx.status()
        pu = bufs[2].cpu().numpy()[:nt].astype(np.int64)
        e_l = LP.front_error(ctx, pr.coords, pr.elems, xq, field=pr.data)[0]
        say(f"learned: {wall_l * 1e3:.1f} ms per step, e = {e_l:.2e}")
        out_paths["learned"] = (wall_l, lay_l, pu, e_l)
    if args.path in ("both", "fixed"):
        wall_f, lay_f = run(fixed_step, args.steps, args.warmup)
        ctx.status()
        e_f = LP.front_error(ctx, pr.coords, pr.elems, xq, field=pr.data)[0]
        say(f"fixed p=8: {wall_f * 1e3:.1f} ms per step, e = {e_f:.2e}")
        out_paths["fixed"] = (wall_f, lay_f, np.full(nt, 8, np.int64), e_f)
    dof8 = float(op_counts_deg(ctx, pr, tents, np.full(nt, 8))[2].sum())
    res = {}
    for name, (wall, lay, pt, e) in out_paths.items():
        fl, by, N = op_counts_deg(ctx, pr, tents, pt)
        ex = moment_exec_flops(ctx, pr, tents, pt)
        lay_fl = np.array([fl[lp[l]:lp[l + 1]].sum() for l in range(window)])
        lay_ex = np.array([ex[lp[l]:lp[l + 1]].sum() for l in range(window)])
        launch_s = lay.mean(axis=0) * 1e-3  # per layer, averaged over the timed steps
        res[name] = dict(
            time_s=wall, dof_updates=float(N.sum()), dof_updates_per_s=float(N.sum()) / wall, e_abs=e,
            p8_equivalent_dof_updates_per_s=dof8 / wall,
            degrees={int(p): int((pt == p).sum()) for p in range(2, 9) if (pt == p).any()},
            alg_flops_per_launch=float(lay_fl.mean()), exec_flops_per_launch=float(lay_ex.mean()),
            avg_launch_us=float(launch_s.mean() * 1e6),
            achieved_alg=float(lay_fl.sum() / launch_s.sum()), achieved_exec=float(lay_ex.sum() / launch_s.sum()),
            alg_bytes_per_launch=float(np.array([by[lp[l]:lp[l + 1]].sum() for l in range(window)]).mean()))
    main_path = "learned" if "learned" in res else "fixed"
    r = res[main_path]
    desc = (f"3+1D learned degree: unit cube, {m}^3 x 6 jittered Kuhn tetrahedra ({len(pr.elems)}), speed variant b "
            f"(c = 1.5 everywhere; exact standing wave sin sin sin cos), p in 2..8 per tent by the packaged "
            f"8-64-64-7 network (log eta_tol = {log_tol}) vs fixed p = 8, FP64 moment Gram, T = 0.5 pitched in "
            f"{L} layers; window = the first {window} layers ({nt} tents)")
    out = {
        "metric": METRIC,
        "value": r["p8_equivalent_dof_updates_per_s"],
        "unit": "DOF-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["time_s"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {
            "workload": desc,
            "value_is": (f"{main_path} path, counted in the DOF-updates of the plain fixed p = 8 method over the same "
                         "window (the work the plain method needs for the same front at the same error bar) per "
                         "second of the step"),
            "step": f"reset + {main_path} sweep of the window, one launch per layer (plus features and degree "
                    "selection per layer on the learned path)",
            "tents_in_window": nt, "layers_total": int(L), "p8_dof_updates_per_step": dof8,
            "paths": res, "kernel_shape": ctx.get_tuning(), "gram_mode": ctx.get_gram_mode(),
            "parallelism": "single GPU, all tents of a layer in one launch",
        },
        "roofline": {
            "bound": "alu", "achieved": r["achieved_alg"] / 1e12, "peak": FP64_PEAK / 1e12, "unit": "TFLOP/s",
            "frac": r["achieved_alg"] / FP64_PEAK, "traffic": measured_traffic(f"cube_3d_{main_path}"),
            "kernel": "tent_layer_kernel<3,1,false,true> (moment Gram, FP64)",
            "count": "quadrature-form operation count of eq. 4.1 per tent at its degree (op_counts_deg)",
            "achieved_executed": r["achieved_exec"] / 1e12, "frac_executed": r["achieved_exec"] / FP64_PEAK,
            "count_executed": "operations the moment form executes (bench.moment_exec_flops)",
            "launches_per_step": window, "avg_launch_us": r["avg_launch_us"],
            "alg_flops_per_launch": r["alg_flops_per_launch"], "exec_flops_per_launch": r["exec_flops_per_launch"],
            "alg_bytes_per_launch": r["alg_bytes_per_launch"],
        },
    }
    if "learned" in res and "fixed" in res:
        out["config"]["speedup_learned_vs_fixed_p8_at_equal_error"] = res["fixed"]["time_s"] / res["learned"]["time_s"]
    if not args.no_cpu_baseline:
        say("cpu baseline (oracle, all host cores)")
        out["cpu_baseline"] = cpu_baseline_cube(pr, ctx, args.cpu_seconds)
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


def _host_cpu():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


_CUBE = {}


def _cube_worker(args):
    """Solves tents of the first layer from the initial state (tents of a layer
    are independent) until the shared deadline; returns (tents, DOFs)."""
    from threadpoolctl import threadpool_limits

    ids, deadline = args
    o = _CUBE["oracle"]
    done = dofs = 0
    with threadpool_limits(1):
        for i in ids:
            if time.time() >= deadline:
                break
            V, tb, tt = o.tents[i]
            o.solve_tent(V, tb, tt)
            done += 1
            dofs += _CUBE["dofs"][i]
    return done, dofs


def cpu_baseline_cube(pr, ctx, budget_s):
    """The oracle (NumPy, FP64, LAPACK LU) on tents of the first layer of the
    3+1D workload at p = 8, one process per host core (fork, copy-on-write
    oracle state), each process with one BLAS thread, for about budget_s of
    wall time.  The oracle pitches only to just above the first layer's tops
    (the first layer's tents do not depend on the final time; checked)."""
    import multiprocessing as mp

    from oracle.pitcher import pitch
    from oracle.tdg import OracleTDG
    from oracle.trefftz import dim_U

    lp = ctx.tents.layer_ptr
    first = ctx.tents.as_list()[: lp[1]]
    gamma = ctx.tents.gamma
    t_or = 1.01 * max(tt for _, _, tt in first)
    tents, lpo = pitch(pr.coords, pr.elems, pr.c, t_or, gamma)
    assert tents[: lp[1]] == first, "oracle and library pitch different first layers"
    f = pr.data
    o = OracleTDG(pr.coords, pr.elems, pr.c, tents, lpo, p=pr.p, q=pr.qpts, alpha=pr.alpha, beta=pr.beta,
                  gD=lambda x, t: f.v(x, t))
    X = o.quad_points()
    o.set_initial(f.v(X, 0.0), f.sigma(X, 0.0), f.U(X, 0.0))
    _CUBE["oracle"] = o
    _CUBE["dofs"] = [dim_U(pr.n, pr.p)] * lp[1]
    model, avail = _host_cpu()
    workers = max(1, min(avail, 16, lp[1]))
    ids = np.arange(lp[1])
    chunks = [ids[k::workers].tolist() for k in range(workers)]
    ctx_mp = mp.get_context("fork")
    t0 = time.time()
    deadline = t0 + budget_s
    with ctx_mp.Pool(workers) as pool:
        res = pool.map(_cube_worker, [(c, deadline) for c in chunks])
    el = time.time() - t0
    done = sum(r[0] for r in res)
    dofs = float(sum(r[1] for r in res))
    _CUBE.clear()
    return {"value": dofs / el, "unit": "DOF-updates/s", "cores": workers, "kind": "oracle",
            "sample": f"{done} tents of the first layer at p = 8 (the fixed-degree method) solved from the initial "
                      f"state in {el:.1f} s by {workers} processes with one BLAS thread each (fork, tents split "
                      f"round-robin); host: {avail} usable CPUs, {model}"}


def say(msg):
    """Progress of the run (stderr; the JSON line is the only stdout output)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube_3d",
                    help="cube_3d (default: 3+1D learned degree vs fixed p = 8), cfg1, cfg2, cfg3[_pP], cfg4, "
                         "lshape, lshape_graded")
    ap.add_argument("--window", type=int, default=24, help="cube_3d: layers per step")
    ap.add_argument("--log-tol", type=float, default=-40.0, help="cube_3d: log eta_tol of the degree choice")
    ap.add_argument("--path", default="both", choices=("both", "learned", "fixed"),
                    help="cube_3d: which sweeps to time (the step is the learned one when run)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="cube_3d: skip the extra 2+1D (config 2) line")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (automatic shape)")
    ap.add_argument("--gram", type=int, default=-1, choices=(-1, 0, 1),
                    help="Gram mode: 0 basis values on the matrix cores, 1 monomial moments, -1 autotuned")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); domain-decomposed runs over several "
              "GPUs are not implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    torch.cuda.set_device(0)
    if args.workload == "cube_3d":
        out = bench_cube_3d(args)
        if not args.no_extra:
            say("extra line: 2+1D plain FP64 batched (config 2)")
            sub = argparse.Namespace(**vars(args))
            sub.workload, sub.steps, sub.warmup, sub.no_cpu_baseline = "cfg2", 5, 2, True
            out["extra_cfg2"] = bench_sweep(sub)
        print(json.dumps(out), flush=True)
        return
    print(json.dumps(bench_sweep(args)), flush=True)


def bench_sweep(args):
    """A whole sweep (reset + every layer) of a 1+1D/2+1D workload, recorded
    as a HIP graph and replayed."""
    import torch

    from paper_1907_02367_amd import tdg

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
    if not args.no_cpu_baseline:
        say("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(pr, args.cpu_seconds, N, tents.n_tents)
    del ctx
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
