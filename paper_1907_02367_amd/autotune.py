"""Autotuner for the execution shape of the tent kernel.

The shape is (Gram mode, points per chunk, persistent grid or one workgroup
per tent); it changes speed, not results beyond rounding.  Each feasible shape
is timed with HIP events on the first layers of the sweep (from the initial
state), the fastest is kept, and the choice is cached in a JSON file keyed by
the problem class (dimension, degree, speed groups, mesh size, tents per
layer) and by a hash of the kernel sources, so that a shape tuned for an
earlier kernel is not reused after the kernel changes.  Gram modes: 0 = basis
values at the points on the matrix cores, 1 = monomial moments (FP64 contexts
only).
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

CACHE = os.environ.get("TDG_TUNING_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "tdg_tuning.json"))
SHAPES = [(pch, pers) for pch in (64, 32, 16, 8, 4) for pers in (0, 1)]


def kernel_source_hash():
    """First 16 hex digits of the SHA-256 of the tent kernel's sources."""
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in ("tent_kernel.hip", "tdg_internal.h", "api.cpp"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def problem_key(ctx, p_max):
    t = ctx.tents
    width = int(np.diff(t.layer_ptr).mean()) if t.n_layers else 0
    return f"n{ctx.n}_p{p_max}_ne{ctx.ne}_Q{ctx.Q}_w{width}_prec{ctx.precision}_k{kernel_source_hash()}"


def _load():
    try:
        with open(CACHE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(cache):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        with open(CACHE, "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    except OSError:
        pass


def autotune(ctx, n_layers=24, reps=2, use_cache=True, p_per_tent=None, verbose=False, modes=None):
    """Picks the fastest feasible shape for ctx and applies it.  Leaves the
    context reset to its initial state.  Returns (shape dict, timings)."""
    import torch

    key = problem_key(ctx, ctx.p_max)
    cache = _load() if use_cache else {}
    if key in cache:
        sh = cache[key]
        try:
            ctx.set_gram_mode(sh.get("gram_mode", 0))
            ctx.set_tuning(sh["pts_per_chunk"], sh["persistent"])
            ctx.reset()
            return dict(sh, cached=True), {}
        except Exception:
            pass
    L = min(n_layers, ctx.tents.n_layers)
    timings = {}
    shapes = [(mode, pch, pers) for mode in (modes if modes is not None else (0, 1)) for pch, pers in SHAPES]
    for mode, pch, pers in shapes:
        try:
            ctx.set_tuning(0, 0)
            ctx.set_gram_mode(mode)
            ctx.set_tuning(pch, pers)
        except Exception:
            continue
        best = np.inf
        for _ in range(reps + 1):
            ctx.reset()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            ctx.layer_solve(0, L, p_per_tent=p_per_tent)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        timings[(mode, pch, pers)] = best
        if verbose:
            print(f"  shape gram={mode} pts_per_chunk={pch} persistent={pers}: {best:.3f} ms for {L} layers",
                  file=sys.stderr, flush=True)
    if not timings:
        raise RuntimeError("no feasible kernel shape")
    (mode, pch, pers), ms = min(timings.items(), key=lambda kv: kv[1])
    ctx.set_tuning(0, 0)
    ctx.set_gram_mode(mode)
    ctx.set_tuning(pch, pers)
    ctx.reset()
    torch.cuda.synchronize()
    sh = dict(gram_mode=mode, pts_per_chunk=pch, persistent=pers, ms=ms, layers=L)
    cache[key] = sh
    if use_cache:
        _save(cache)
    return dict(sh, cached=False), {f"{k[0]}/{k[1]}/{k[2]}": v for k, v in timings.items()}
