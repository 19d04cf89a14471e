"""Choice of the spatial seed basis of the Trefftz recursion (Sec. 6.3) on one
MI355X: the 1+1D standing wave of Sec. 6 (U = cos(pi x) sin(pi t) / pi on
[0, 1], c = 1, alpha = beta = 0.5, T = 1), tent-pitched, solved tent by tent
by the library with monomial, Legendre and Chebyshev seeds for p = 1..10.
Per degree and seed: the error e of (v, sigma) at T.  The three seeds span
the same Trefftz space, so the errors agree until the conditioning of the
tent systems in the seeded basis limits the accuracy.

    python -m paper_1907_02367_amd.studies.seeds [--elems 8] [--pmax 10] [--out results.jsonl]
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SEEDS = ("monomial", "legendre", "chebyshev")  # tdg_opts.seed_basis 0, 1, 2


def say(*a):
    print(*a, flush=True)


def run(n_elems, p, seed_basis):
    from paper_1907_02367_amd import tdg
    from workloads import fields as F
    from workloads import meshes as M

    coords, elems = M.interval_mesh(n_elems)
    c = np.ones(len(elems))
    f = F.PaperStandingWave(1)
    T = tdg.tent_pitch(coords, elems, c, 1.0, 0.5)
    ctx = tdg.Trefftz(coords, elems, c, T, p_max=p, q=p, alpha=0.5, beta=0.5, seed_basis=seed_basis)
    xq, w = ctx.quad_points()
    ctx.set_initial(f.v(xq, 0.0), f.sigma(xq, 0.0), f.U(xq, 0.0))
    bx = ctx.boundary_points()
    ctx.set_boundary(f.v(bx[:, :-1], bx[:, -1]))
    ctx.layer_solve()
    ctx.status()
    e_abs, e_rel = ctx.eval_error(f.v(xq, 1.0), f.sigma(xq, 1.0))
    return T.n_tents, float(e_abs), float(e_rel)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--elems", type=int, default=8)
    ap.add_argument("--pmax", type=int, default=10)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    rows = []
    say(f"{'p':>3} " + " ".join(f"{s:>12}" for s in SEEDS))
    for p in range(1, a.pmax + 1):
        errs = []
        for sb in range(3):
            nt, e_abs, _ = run(a.elems, p, sb)
            errs.append(e_abs)
            rows.append({"p": p, "seed": SEEDS[sb], "tents": nt, "e_abs": e_abs, "elems": a.elems})
        say(f"{p:>3} " + " ".join(f"{e:>12.3e}" for e in errs))
    if a.out:
        with open(a.out, "w") as fh:
            for r in rows:
                fh.write(json.dumps(r) + "\n")


if __name__ == "__main__":
    main()
