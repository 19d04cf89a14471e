"""The library's Trefftz tables for each seed basis (Sec. 3, Sec. 6.3) against
the oracle's, on the host (no GPU): both are exact rationals rounded once to
double, built by different routes (the library combines monomial-seeded
functions with closed-form Legendre and Chebyshev coefficients, the oracle
runs the recursion of eq. 3.1 from the seed itself), so the rows of the
first-order fields (v, sigma) and of U must agree bit for bit, term by term."""
import ctypes

import numpy as np
import pytest

from oracle.trefftz import SEED_KINDS, first_order_fields, trefftz_basis
from workloads import configs as C


def _lib_tables(ctx, p):
    from paper_1907_02367_amd import tdg

    f = tdg.lib().tdg_debug_field_tables
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32] + [ctypes.c_void_p] * 8
    f.restype = ctypes.c_int
    info = np.zeros(5, np.int32)
    assert f(ctx._h, p, info.ctypes.data, *([None] * 7)) == 0
    M, NW, n, nfo, nu = (int(x) for x in info)
    expo = np.zeros(M * (n + 1), np.int32)
    fp = np.zeros(NW * (n + 1) + 1, np.int32)
    fi, fc = np.zeros(max(nfo, 1), np.int32), np.zeros(max(nfo, 1))
    up = np.zeros(NW + 1, np.int32)
    ui, uc = np.zeros(max(nu, 1), np.int32), np.zeros(max(nu, 1))
    assert f(ctx._h, p, info.ctypes.data, expo.ctypes.data, fp.ctypes.data, fi.ctypes.data, fc.ctypes.data,
             up.ctypes.data, ui.ctypes.data, uc.ctypes.data) == 0
    ex = expo.reshape(M, n + 1)

    def key(i):
        return (int(ex[i, 0]), tuple(int(x) for x in ex[i, 1:]))

    fo = [[{key(fi[e]): fc[e] for e in range(fp[j * (n + 1) + c], fp[j * (n + 1) + c + 1])}
           for c in range(n + 1)] for j in range(NW)]
    U = [{key(ui[e]): uc[e] for e in range(up[j], up[j + 1])} for j in range(NW)]
    return fo, U


@pytest.mark.parametrize("dim,p_max,degrees", [("1d", 10, range(1, 11)), ("2d", 10, (1, 2, 3, 4, 5, 6, 10)),
                                                ("3d", 9, (1, 2, 3, 4, 8, 9))])
def test_library_tables_equal_the_oracle_for_every_seed(dim, p_max, degrees):
    from paper_1907_02367_amd import tdg

    pr = {"1d": lambda: C.cfg1_standing_1d(n_elems=4), "2d": lambda: C.cfg2_plane_2d(m=3),
          "3d": lambda: C.cfg5_cube_3d(m=1, variant="b")}[dim]()
    tents = tdg.tent_pitch(pr.coords, pr.elems, pr.c, 0.05, 0.16)
    for sb, name in enumerate(SEED_KINDS):
        ctx = tdg.Trefftz(pr.coords, pr.elems, pr.c, tents, p_max=p_max, bind=False, seed_basis=sb)
        for p in degrees:
            fo, U = _lib_tables(ctx, p)
            ofo = first_order_fields(pr.n, p, name)
            oU = trefftz_basis(pr.n, p, name)[1:]
            assert len(fo) == len(ofo) == len(oU)
            for j in range(len(fo)):
                for c in range(pr.n + 1):
                    assert fo[j][c] == {k: float(v) for k, v in ofo[j][c].items()}, (name, p, j, c)
                assert U[j] == {k: float(v) for k, v in oU[j].items()}, (name, p, j)
