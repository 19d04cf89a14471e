"""Host-side checks of bench.py that need no GPU: the one-GPU guard, the
traffic record keyed by the kernel source, and the algorithmic operation
counts against their closed form on a tiny mesh."""
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_is_used_only_for_the_same_kernel_source(monkeypatch):
    import bench

    path = os.path.join(ROOT, "profiles", "tent_layer_kernel_cfg2_traffic.json")
    rec = json.load(open(path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: rec["kernel_source_sha256_16"])
    assert bench.measured_traffic("cfg2") == float(rec["hbm_bytes_per_launch"])
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 16)
    assert bench.measured_traffic("cfg2") is None
    assert bench.measured_traffic("no_such_workload") is None


def test_operation_counts_follow_the_closed_form():
    import bench
    from paper_1907_02367_amd import tdg
    from workloads import configs as C

    pr = C.cfg2_plane_2d(m=4, p=3)
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, pr.T, pr.gamma)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=pr.p, bind=False)
    flops, bytes_, N = bench.op_counts(ctx, pr, T)
    info = ctx.table_info(pr.p)
    assert info["N"] == 16  # dim U^3 in 2+1D
    patch = np.bincount(pr.elems.ravel(), minlength=len(pr.coords))[T.vertex]
    QT = patch * info["Q"]
    NW = info["N"] - 1
    K = QT * 3
    expect = 4.0 * QT * info["nnz_fields"] + K * NW * (NW + 1) + 4.0 * K * NW + (2.0 / 3.0) * NW ** 3 + 2.0 * NW ** 2
    assert np.allclose(flops, expect)
    assert np.allclose(bytes_, 2.0 * QT * 4 * 8)
    assert (N == 16).all()


def test_per_tent_degree_counts_reduce_to_the_fixed_degree_counts():
    """op_counts_deg (the learned path: a degree per tent) gives op_counts at a
    uniform degree, and the moment form's executed count is below the
    quadrature count at 3+1D p = 8 (its reason to exist) but positive."""
    import bench
    from paper_1907_02367_amd import tdg
    from workloads import configs as C

    pr = C.cfg5_cube_3d(m=2, p=8, variant="b", regions=1)
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, 0.05, 0.4 * 0.8 ** 4)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=8, bind=False)
    f8, b8, N8 = bench.op_counts(ctx, pr, T)
    fd, bd, Nd = bench.op_counts_deg(ctx, pr, T, np.full(T.n_tents, 8))
    assert np.allclose(fd, f8) and np.allclose(bd, b8) and np.allclose(Nd, N8)
    assert (N8 == 285).all()
    ex = bench.moment_exec_flops(ctx, pr, T, np.full(T.n_tents, 8))
    assert (ex > 0).all() and (ex < 0.5 * f8).all()
    p = np.where(np.arange(T.n_tents) % 2 == 0, 5, 8)
    fm, _, Nm = bench.op_counts_deg(ctx, pr, T, p)
    assert (fm[p == 5] < f8[p == 5]).all() and np.allclose(fm[p == 8], f8[p == 8])
    assert set(np.unique(Nm)) == {91, 285}
