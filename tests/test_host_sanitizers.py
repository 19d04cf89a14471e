"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU): tests/host_sanitize_driver.cpp is built with g++ together with the
table builder, the topology, the pitcher and the simplex rule, and run over
every Trefftz table (all dimensions, degrees and seed bases) and over meshes
of the workload generators (1D, 2D, two speeds, 3D with region and
per-element speeds, a graded L-shape).  Any invalid access or undefined
operation aborts the driver; the tent counts must equal the library's."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

from workloads import configs as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1907_02367_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_code_is_clean_under_sanitizers(tmp_path):
    from paper_1907_02367_amd import tdg

    exe = str(tmp_path / "drv")
    srcs = [os.path.join(ROOT, "tests", "host_sanitize_driver.cpp")] + \
        [os.path.join(CSRC, f) for f in ("trefftz_table.cpp", "topology.cpp", "pitch.cpp", "quadrature.cpp")]
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"), "-I", CSRC] + srcs + ["-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    cases = [C.cfg1_standing_1d(), C.cfg2_plane_2d(), C.cfg4_interface_2d(m=41),
             C.cfg5_cube_3d(m=6, variant="a"), C.cfg5_cube_3d(m=3, variant="e", T=0.15),
             C.lshape_2d(0.12, True, T=0.2)]
    files, expect = [], []
    for i, pr in enumerate(cases):
        T = min(pr.T, 0.3)
        gamma = pr.gamma * (0.8 ** 4 if pr.n == 3 else 1.0)
        path = str(tmp_path / f"mesh{i}.bin")
        with open(path, "wb") as fh:
            fh.write(struct.pack("<iiidd", pr.n, len(pr.coords), len(pr.elems), T, gamma))
            fh.write(np.ascontiguousarray(pr.coords, np.float64).tobytes())
            fh.write(np.ascontiguousarray(pr.elems, np.int32).tobytes())
            fh.write(np.ascontiguousarray(pr.c, np.float64).tobytes())
        files.append(path)
        tl = tdg.tent_pitch(pr.coords, pr.elems, pr.c, T, gamma)
        expect.append((tl.n_tents, tl.n_layers))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe] + files, capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, (r.returncode, r.stderr[-3000:])
    got = [tuple(int(x) for x in ln.split()[2:4]) for ln in r.stdout.splitlines() if ln.startswith("mesh")]
    assert got == expect
