"""Host replay of the index arithmetic of the moment-phase loads of the tent
kernel (no GPU): for every degree of 3+1D contexts, the task words of the VALU
moment loops, the matrix-core top-moment tiles and the LDS regions they address
are read from the library (its own tables and plan) and every address a lane
computes is checked against the bounds of the array or region it reads, for
full and ragged chunks.  The tile list is also rebuilt here independently
(smallest degrees of 16-blocks of the two monomial lists) and the tiles must
cover every moment monomial of degree <= 2p-2 exactly once."""
import ctypes
from math import comb

import numpy as np
import pytest

from workloads import configs as C

K_TASK_SLOTS, K_TASK_SLOTS1, K_BLOCK, K_MOM_SLOTS = 6, 2, 256, 6


def _tables(ctx, p):
    from paper_1907_02367_amd import tdg

    L = tdg.lib()
    f = L.tdg_debug_moment_tables
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 5
    f.restype = ctypes.c_int
    info = np.zeros(16, np.int32)
    assert f(ctx._h, p, info.ctypes.data, None, None, None, None) == 0
    M, M1, M2, nt2, nt1, ntile = (int(x) for x in info[:6])
    task2 = np.zeros(max(nt2 * 3, 1), np.int32)
    task1 = np.zeros(max(nt1 * 3, 1), np.int32)
    ex = np.zeros(max(ntile * 16, 1), np.int32)
    mp = np.zeros(max(ntile * 256, 1), np.int32)
    assert f(ctx._h, p, info.ctypes.data, task2.ctypes.data, task1.ctypes.data, ex.ctypes.data, mp.ctypes.data) == 0
    keys = ["M", "M1", "M2", "ntask2", "ntask1", "ntile", "Q", "pch", "off_pt", "off_pow", "off_W1", "off_fg",
            "total", "moment", "n", "pmax"]
    d = dict(zip(keys, (int(x) for x in info)))
    return d, task2[: nt2 * 3].view(np.uint32), task1[: nt1 * 3].view(np.uint32), ex[: ntile * 16], mp[: ntile * 256]


def _check_tasks(task, ntask, slots, n_idx, max_exp, n):
    """load_tasks / task_idx: words of task t < ntask only; exponents of the
    prefix and the run start, run indices < n_idx or 0xFFFF past the run; the
    runs cover 0..n_idx-1 exactly once."""
    assert ntask <= slots * K_BLOCK
    seen = np.zeros(n_idx, np.int64)
    for t in range(ntask):
        w0, w1, w2 = (int(x) for x in task[3 * t:3 * t + 3])
        exps = [(w0 >> (5 * v)) & 31 for v in range(n)]
        d0 = (w0 >> 15) & 31
        idx = [w1 & 0xFFFF, w1 >> 16, w2 & 0xFFFF, w2 >> 16]
        run = [i for i in idx if i != 0xFFFF]
        assert idx[:len(run)] == run  # no gap inside a run
        assert sum(exps) + d0 + len(run) - 1 <= max_exp
        for i in run:
            assert 0 <= i < n_idx
            seen[i] += 1
    assert (seen == 1).all()


def _check_bottom_groups(ntask1, Q, pch):
    """Bottom moments of the 3+1D moment loop: with at most 64 (128) tasks they
    are repeated over 4 (2) groups of waves; thread tid is group tid // span,
    task tid % span (+ slot * span) and takes the points group, group +
    nsplit, ... of a chunk.  Every (task, point) pair is summed exactly once,
    and with more than one group every task sits in slot 0 (the slot whose sums
    the groups add one after another after the last chunk)."""
    nwt = max(1, (ntask1 + 63) // 64)
    nsplit = 4 // nwt if nwt <= 2 else 1
    span = K_BLOCK // nsplit
    if nsplit > 1:
        assert ntask1 <= span
    for nc in {pch, Q % pch or pch, 1}:
        seen = np.zeros((ntask1, nc), np.int64)
        for tid in range(K_BLOCK):
            g, tt = tid // span, tid % span
            for sl in range(K_TASK_SLOTS1):
                t = tt + sl * span
                if t >= ntask1:
                    break
                assert sl == 0 or nsplit == 1
                for pt in range(g, nc, nsplit):
                    seen[t, pt] += 1
        assert (seen == 1).all()


def _degree_blocks(D):
    lst = [(a, d - a) for d in range(D + 1) for a in range(d, -1, -1)]
    nb = (len(lst) + 15) // 16
    return lst, [sum(lst[16 * i]) for i in range(nb)]


@pytest.mark.parametrize("seed_basis", [0, 2], ids=["monomial_seeds", "chebyshev_seeds"])
@pytest.mark.parametrize("p_max", [8, 5])
def test_moment_phase_indices_stay_in_bounds_3d(p_max, seed_basis):
    # (a seeded basis has about twice the table terms, which moves the LDS plan)
    from paper_1907_02367_amd import tdg

    pr = C.cfg5_cube_3d(m=3, p=p_max, variant="b", regions=1)
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, 0.05, 0.4 * 0.8 ** 4)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=p_max, bind=False, seed_basis=seed_basis)
    ctx.set_gram_mode(1)
    n = 3
    checked_tiles = 0
    for p in range(1, p_max + 1):
        d, task2, task1, ex, mp = _tables(ctx, p)
        assert d["moment"] == 1 and d["n"] == 3
        M, M1, M2, Q, PCH = d["M"], d["M1"], d["M2"], d["Q"], d["pch"]
        assert M == comb(p + n + 1, n + 1) and M1 == comb(p - 1 + n + 1, n + 1)
        assert M2 == comb(max(2 * p - 2, 0) + n + 1, n + 1)
        E2 = 2 * p - 1
        # VALU moment tasks (moment_points, face moments, write-back runs)
        _check_tasks(task2, d["ntask2"], K_TASK_SLOTS, M2, max(2 * p - 2, 0), n)
        _check_tasks(task1, d["ntask1"], K_TASK_SLOTS1, M, p, n)
        _check_bottom_groups(d["ntask1"], Q, PCH)
        # LDS regions: powers of the top (E2) and bottom (p+1) points, moments
        pow_region = d["off_W1"] - d["off_pow"]
        assert PCH * (n + 1) * E2 + PCH * (n + 1) * (p + 1) <= pow_region
        assert (n + 1) * M2 + (n + 1) * M1 + M <= d["off_fg"] - d["off_W1"]
        assert d["total"] * 8 <= 160 * 1024
        ntile = d["ntile"]
        if p < 2:
            assert ntile == 0
            continue
        # independent tile list
        D = 2 * p - 2
        lst, mins = _degree_blocks(D)
        expect = [(I, J) for I in range(len(mins)) for J in range(len(mins)) if mins[I] + mins[J] <= D]
        if len(expect) > 4 * K_MOM_SLOTS:
            assert ntile == 0
            continue
        assert ntile == len(expect)
        checked_tiles += ntile
        assert PCH % 4 == 0
        exps = ex.reshape(ntile, 16)
        for field, sh in (("a0", 0), ("a1", 5), ("c0", 10), ("c1", 15)):
            assert ((exps >> sh) & 31).max() < E2, field
        # rows/columns of each tile carry the exponents of the degree lists
        for t, (I, J) in enumerate(expect):
            for l in range(16):
                i, j = 16 * I + l, 16 * J + l
                a = lst[i] if i < len(lst) else (0, 0)
                c = lst[j] if j < len(lst) else (0, 0)
                assert int(exps[t, l]) == a[0] | a[1] << 5 | c[0] << 10 | c[1] << 15
        # every moment monomial exactly once in the fold map; entries in range
        assert mp.min() >= -1 and mp.max() < M2
        cnt = np.bincount(mp[mp >= 0], minlength=M2)
        assert (cnt == 1).all()
        # k-step reads of a full chunk and of the ragged last chunk of an element
        for nc in {PCH, Q % PCH or PCH, 1}:
            nks = (nc + 3) // 4
            lane = np.arange(64)
            for ks in range(nks):
                pt = ks * 4 + lane // 16
                assert pt.max() < PCH  # inside the chunk's regions even for padded points
                for w in range(4):
                    for s in range(K_MOM_SLOTS):
                        # every slot's operands are loaded (a slot past the wave's
                        # tiles has exponents 0), only valid slots reach the MFMA
                        t = w + 4 * s
                        e = exps[t, lane % 16] if t < ntile else np.zeros(64, np.int64)
                        base = pt * (n + 1) * E2
                        for v, sh in enumerate((0, 5, 10, 15)):
                            addr = base + v * E2 + ((e >> sh) & 31)
                            assert addr.max() < PCH * (n + 1) * E2
        # fold reads of mt_map
        lane = np.arange(64)
        for t in range(ntile):
            for r in range(4):
                idx = t * 256 + ((lane >> 4) + 4 * r) * 16 + (lane & 15)
                assert idx.max() < ntile * 256
    assert checked_tiles > 0


@pytest.mark.parametrize("gram_mode", [0, 1])
@pytest.mark.parametrize("seed_basis", [0, 2], ids=["monomial_seeds", "chebyshev_seeds"])
@pytest.mark.parametrize("p_max", [8, 3])
def test_matrix_core_evaluation_indices_3d(p_max, gram_mode, seed_basis):
    """The matrix-core evaluation of the solution at points (indicator and
    write-back, 3+1D): every monomial of degree <= p is one (L, R) pair of the
    two-variable list, each pair at most once; the k-steps of tile I cover the
    R entries of degree <= p - (smallest degree of the tile); every LDS read of
    the evaluation (dense coefficients, the 4 waves' point powers, the entry
    list) lies inside the W1 region of the plan, and every read index is
    inside its array."""
    import ctypes
    from paper_1907_02367_amd import tdg

    pr = C.cfg5_cube_3d(m=3, p=p_max, variant="b", regions=1)
    T = tdg.tent_pitch(pr.coords, pr.elems, pr.c, 0.05, 0.4 * 0.8 ** 4)
    ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, T, p_max=p_max, bind=False, seed_basis=seed_basis)
    ctx.set_gram_mode(gram_mode)
    L = tdg.lib()
    f = L.tdg_debug_eval_tables
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    for p in range(1, p_max + 1):
        info = np.zeros(22, np.int32)
        assert f(ctx._h, p, info.ctypes.data, None, None) == 0
        nl, nat, nks, M, w1 = int(info[0]), int(info[1]), info[2:10], int(info[10]), int(info[11])
        mpch, moff = int(info[12]), int(info[13])
        nkv = info[14:22]
        if moff >= 0:
            # the larger moment chunk of this degree sits behind its moments in W1:
            # points (2 (n+1) + 1 + (n+2) doubles each) and powers (E2 + p + 1 per
            # variable); the moments themselves take (n+1) M2 + (n+1) M1 + M
            assert gram_mode == 1 and mpch % 4 == 0 and mpch in (32, 64)
            M1, M2 = comb(p - 1 + 4, 4), comb(2 * p - 2 + 4, 4)
            assert moff >= 4 * M2 + 4 * M1 + M
            assert moff + mpch * (8 + 1 + 5) + mpch * 4 * ((2 * p - 1) + (p + 1)) <= w1
        assert nl == (p + 1) * (p + 2) // 2 and nat == (nl + 15) // 16
        ab = np.zeros(M, np.int32)
        ex = np.zeros(nl, np.int32)
        assert f(ctx._h, p, info.ctypes.data, ab.ctypes.data, ex.ctypes.data) == 0
        lst = [(int(e) & 255, int(e) >> 8) for e in ex]
        assert lst == [(a, d - a) for d in range(p + 1) for a in range(d, -1, -1)]
        pairs = [(int(x) & 0xFFFF, int(x) >> 16) for x in ab]
        assert len(set(pairs)) == M
        for k, (a, b) in enumerate(pairs):
            assert a < nl and b < nl and sum(lst[a]) + sum(lst[b]) <= p
            # the pair is reached by the k-steps of a's tile; the monomials of
            # degree <= p - 1 (those of v and sigma: the first C(p+3, 4)) by the
            # shorter step count of the tile
            assert b < 4 * nks[a // 16]
            if k < comb(p - 1 + 4, 4):
                assert b < 4 * nkv[a // 16]
        assert all(nkv[I] <= nks[I] for I in range(nat))
        ldb = nl | 1
        nA16 = 16 * nat
        dense = 5 * nA16 * ldb
        P1 = p + 1
        pww = 4 * 16 * 4 * P1
        if dense + pww + (nl + 1) // 2 + 1 > w1:
            continue  # the kernel keeps the VALU evaluation at this degree (its fit test)
        # the evaluation at two times (indicator and write-back in one pass):
        # 5 power rows per point, its fit test, and every power read inside the
        # wave's rows (R at rows 2, 3 of point l%16; L at rows 0, 1 and 4 of the
        # points l/16 + 4r)
        pww5 = 4 * 16 * 5 * P1
        if dense + pww5 + (nl + 1) // 2 + 1 <= w1:
            lane = np.arange(64)
            e = np.array([int(x) for x in ex])
            for r in range(4):
                pt = (lane >> 4) + 4 * r
                for row in (0, 1, 4):
                    addr = pt[:, None] * 5 * P1 + row * P1 + (e[None, :] & 255 if row != 1 else e[None, :] >> 8)
                    assert addr.max() < 16 * 5 * P1
            for row in (2, 3):
                addr = (lane & 15)[:, None] * 5 * P1 + row * P1 + (e[None, :] & 255 if row == 2 else e[None, :] >> 8)
                assert addr.max() < 16 * 5 * P1
        # reads of eval16_mfma: coefficients, powers (pt <= 15, exponents <= p)
        lane = np.arange(64)
        for I in range(nat):
            a = I * 16 + (lane & 15)
            for ks in range(int(nks[I])):
                b = ks * 4 + (lane >> 4)
                ok = b < nl
                idx = ((4 * nA16 + a) * ldb + b)[ok]
                assert idx.max(initial=0) < dense
                e = np.array([int(ex[bb]) for bb in b[ok]])
                addr = (lane & 15)[ok] * 4 * P1 + 3 * P1 + (e >> 8)
                assert addr.max(initial=0) < 16 * 4 * P1
