"""Python binding of libtdg (ctypes).  Argument marshalling only: every step
of the tent-pitched Trefftz-DG path runs inside libtdg (host C++ for the
pitcher and tables, HIP kernels for the solve).  Device buffers are PyTorch
tensors handed to the library as raw pointers; work is queued on PyTorch's
current HIP stream.

The names follow the C-ABI in include/tdg.h.  There is no fallback: if the
shared library is missing the import of this module's functions raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdg.so")

TDG_NBUF = 8
ERRORS = {
    -1: "TDG_EINVAL", -2: "TDG_ENONCAUSAL", -3: "TDG_ESINGULAR", -4: "TDG_ENOCONV",
    -5: "TDG_ENAN", -6: "TDG_EHIP", -7: "TDG_ENOMEM", -8: "TDG_ESTATE",
}


class TdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nv", ctypes.c_int32), ("ne", ctypes.c_int32),
                ("coords", ctypes.c_void_p), ("elems", ctypes.c_void_p), ("bface_kind", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("p_max", ctypes.c_int32), ("q", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("beta", ctypes.c_double), ("precision", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("recover_U", ctypes.c_int32), ("seed_basis", ctypes.c_int32)]


_lib = None

EXPORTS = {
    "tent_pitch": [ctypes.POINTER(_Mesh), ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.POINTER(ctypes.c_void_p)],
    "tdg_boundary_facets": [ctypes.POINTER(_Mesh), ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p],
    "trefftz_boundary_kinds": [ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_eval_u_error": [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.c_void_p],
    "tent_info": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)],
    "tent_export": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "tent_free": [ctypes.c_void_p],
    "trefftz_create": [ctypes.POINTER(_Mesh), ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_void_p)],
    "trefftz_quad_points": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_boundary_points": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p],
    "trefftz_buffer_sizes": [ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_bind": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_set_initial": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_set_boundary": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_reset": [ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_layer_solve": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_eval_error": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.c_void_p],
    "trefftz_energy": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), ctypes.c_void_p],
    "trefftz_status": [ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_read_state": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_table_info": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "trefftz_set_tuning": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32],
    "trefftz_set_gram_mode": [ctypes.c_void_p, ctypes.c_int32],
    "trefftz_get_gram_mode": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)],
    "trefftz_get_tuning": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32)],
    "trefftz_capture_sweep": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                              ctypes.c_void_p],
    "trefftz_replay_sweep": [ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_tent_stats": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                           ctypes.c_void_p],
    "trefftz_set_indicator": [ctypes.c_void_p, ctypes.c_int32],
    "trefftz_tent_features": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_layer_indicator": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_layer_solve_adaptive": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_float,
                                     ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p],
    "tdg_mlp_nparam": [],
    "tdg_mlp_forward": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p],
    "tdg_mlp_backward": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                         ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "tdg_mlp_backward_noalloc": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                 ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p],
    "tdg_mlp_adam": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_void_p],
    "tdg_mlp_round": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
    "trefftz_destroy": [ctypes.c_void_p],
    "tdg_last_error": [],
}


def _hip_runtimes():
    """Paths of the HIP runtime libraries mapped into this process."""
    paths = set()
    try:
        with open("/proc/self/maps") as fh:
            for line in fh:
                if "libamdhip64" in line:
                    paths.add(line.split()[-1])
    except OSError:
        pass
    return paths


def lib():
    """Loads libtdg.so (built by paper_1907_02367_amd.build); raises if absent.

    PyTorch is imported first so that its HIP runtime (same soname as the one
    libtdg links against) is the only one in the process: the library then
    shares PyTorch's device memory, streams and events."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads PyTorch's HIP runtime first)

        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libtdg.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        rts = _hip_runtimes()
        if len(rts) > 1:
            raise RuntimeError(f"two HIP runtimes loaded in one process: {sorted(rts)}")
        for name, args in EXPORTS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = None if name in ("tent_free", "trefftz_destroy") else ctypes.c_int
        L.tdg_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _dptr(t, dtype, shape):
    """Device pointer of a contiguous CUDA tensor of the given dtype and shape
    (argument checks only)."""
    import torch

    if not (t.is_cuda and t.is_contiguous() and t.dtype == getattr(torch, dtype) and tuple(t.shape) == tuple(shape)):
        raise ValueError(f"expected a contiguous CUDA {dtype} tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")
    return ctypes.c_void_p(t.data_ptr())


# ---- degree network (C-ABI tdg_mlp_*; device tensors, argument marshalling only)
def mlp_nparam():
    return int(lib().tdg_mlp_nparam())


def mlp_forward(w_bf16, x, stream=None):
    """y (n x 7 float32) = network(x (n x 8 float32)) with BF16 weights (stored as int16)."""
    import torch

    n = x.shape[0]
    y = torch.empty((n, 7), dtype=torch.float32, device=x.device)
    _check(lib().tdg_mlp_forward(_dptr(w_bf16, "int16", (mlp_nparam(),)), _dptr(x, "float32", (n, 8)), n,
                                 _dptr(y, "float32", (n, 7)), _stream(stream)))
    return y


def mlp_backward(w_bf16, x, target, mask, norm, partial=None, grad=None, stream=None):
    """Gradient of sum mask (y - target)^2 / norm: returns grad (nparam+1
    float32, last entry the loss) and the scratch used."""
    import torch

    n, P = x.shape[0], mlp_nparam()
    nb = (n + 31) // 32
    if partial is None or partial.numel() < nb * (P + 1):
        partial = torch.empty(nb * (P + 1), dtype=torch.float32, device=x.device)
    if grad is None:
        grad = torch.empty(P + 1, dtype=torch.float32, device=x.device)
    _check(lib().tdg_mlp_backward(_dptr(w_bf16, "int16", (P,)), _dptr(x, "float32", (n, 8)),
                                  _dptr(target, "float32", (n, 7)), _dptr(mask, "float32", (n, 7)), n, float(norm),
                                  ctypes.c_void_p(partial.data_ptr()), _dptr(grad, "float32", (P + 1,)),
                                  _stream(stream)))
    return grad, partial


def mlp_backward_noalloc(w_bf16, x, target, mask, norm, grad, stream=None):
    """tdg_mlp_backward_noalloc: the gradient into the caller's grad (nparam+1
    float32) with the library's fixed scratch (n <= 8192 samples)."""
    n, P = x.shape[0], mlp_nparam()
    _check(lib().tdg_mlp_backward_noalloc(_dptr(w_bf16, "int16", (P,)), _dptr(x, "float32", (n, 8)),
                                          _dptr(target, "float32", (n, 7)), _dptr(mask, "float32", (n, 7)), n,
                                          float(norm), _dptr(grad, "float32", (P + 1,)), _stream(stream)))
    return grad


def mlp_adam(w32, w_bf16, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, stream=None):
    P = mlp_nparam()
    _check(lib().tdg_mlp_adam(_dptr(w32, "float32", (P,)), _dptr(w_bf16, "int16", (P,)),
                              ctypes.c_void_p(grad.data_ptr()), _dptr(m, "float32", (P,)), _dptr(v, "float32", (P,)),
                              int(step), float(lr), float(b1), float(b2), float(eps), _stream(stream)))


def mlp_round(w32, w_bf16, stream=None):
    P = mlp_nparam()
    _check(lib().tdg_mlp_round(_dptr(w32, "float32", (P,)), _dptr(w_bf16, "int16", (P,)), _stream(stream)))


def _check(rc):
    if rc != 0:
        raise TdgError(rc, lib().tdg_last_error().decode())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _mesh(coords, elems, bface_kind=None):
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    elems = np.ascontiguousarray(elems, dtype=np.int32)
    kinds = None if bface_kind is None else np.ascontiguousarray(bface_kind, dtype=np.int8)
    m = _Mesh(coords.shape[1], coords.shape[0], elems.shape[0], _ptr(coords), _ptr(elems), _ptr(kinds))
    return m, (coords, elems, kinds)


def boundary_facets(coords, elems):
    """(nbf, 2) int32: (element, local index of the opposite vertex) of every
    boundary facet, in the order of the per-facet kinds (tdg_boundary_facets)."""
    m, keep = _mesh(coords, elems)
    nbf = ctypes.c_int64()
    _check(lib().tdg_boundary_facets(ctypes.byref(m), ctypes.byref(nbf), None))
    out = np.zeros((nbf.value, 2), np.int32)
    _check(lib().tdg_boundary_facets(ctypes.byref(m), ctypes.byref(nbf), _ptr(out)))
    return out


def _stream(stream=None):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Tents:
    """A pitched tent mesh (library-owned)."""

    def __init__(self, handle):
        self._h = handle
        nl, nt, ms = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().tent_info(handle, ctypes.byref(nl), ctypes.byref(nt), ctypes.byref(ms)))
        self.n_layers, self.n_tents, self.max_slope = nl.value, nt.value, ms.value
        self.vertex = np.empty(self.n_tents, np.int32)
        self.t_bot = np.empty(self.n_tents)
        self.t_top = np.empty(self.n_tents)
        self.layer_ptr = np.empty(self.n_layers + 1, np.int64)
        _check(lib().tent_export(handle, _ptr(self.vertex), _ptr(self.t_bot), _ptr(self.t_top), _ptr(self.layer_ptr)))

    def as_list(self):
        return list(zip(self.vertex.tolist(), self.t_bot.tolist(), self.t_top.tolist()))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.tent_free(self._h)
            self._h = None


def tent_pitch(coords, elems, c, T, gamma) -> Tents:
    m, keep = _mesh(coords, elems)
    c = np.ascontiguousarray(c, dtype=np.float64)
    h = ctypes.c_void_p()
    _check(lib().tent_pitch(ctypes.byref(m), _ptr(c), float(T), float(gamma), ctypes.byref(h)))
    t = Tents(h)
    t.T, t.gamma = float(T), float(gamma)
    return t


class Trefftz:
    """Solver context: trefftz_create + buffers (PyTorch) + trefftz_bind."""

    def __init__(self, coords, elems, c, tents: Tents, p_max: int, q: int = 0, alpha: float = 0.5,
                 beta: float = 0.5, precision: int = 0, recover_U: int = 1, device=None, bind: bool = True,
                 bface_kind=None, seed_basis: int = 0):
        self.n = int(np.asarray(coords).shape[1])
        self.nv = int(np.asarray(coords).shape[0])
        self.ne = int(np.asarray(elems).shape[0])
        self.tents = tents
        m, keep = _mesh(coords, elems, bface_kind)
        c = np.ascontiguousarray(c, dtype=np.float64)
        opts = _Opts(int(p_max), int(q), float(alpha), float(beta), int(precision), 1, int(recover_U),
                     int(seed_basis))
        h = ctypes.c_void_p()
        _check(lib().trefftz_create(ctypes.byref(m), _ptr(c), tents._h, ctypes.byref(opts), ctypes.byref(h)))
        self._h = h
        self.p_max = int(p_max)
        self.precision = int(precision)
        nq = ctypes.c_int64()
        _check(lib().trefftz_quad_points(h, ctypes.byref(nq), None, None))
        self.nq = nq.value
        self.Q = self.nq // self.ne
        nb = ctypes.c_int64()
        _check(lib().trefftz_boundary_points(h, ctypes.byref(nb), None))
        self.nb = nb.value
        sizes = np.zeros(TDG_NBUF, np.int64)
        _check(lib().trefftz_buffer_sizes(h, _ptr(sizes)))
        self.buffer_sizes = sizes
        self.buffers = None
        if bind:
            self.bind(device)

    def quad_points(self):
        xq = np.empty((self.nq, self.n))
        w = np.empty(self.nq)
        nq = ctypes.c_int64()
        _check(lib().trefftz_quad_points(self._h, ctypes.byref(nq), _ptr(xq), _ptr(w)))
        return xq, w

    def boundary_points(self):
        xt = np.empty((self.nb, self.n + 1))
        nb = ctypes.c_int64()
        _check(lib().trefftz_boundary_points(self._h, ctypes.byref(nb), _ptr(xt)))
        return xt

    def boundary_kinds(self):
        """Per boundary point: 0 on a Dirichlet face (g_D), 1 on a Neumann face (g_N)."""
        k = np.zeros(max(self.nb, 1), np.int8)
        _check(lib().trefftz_boundary_kinds(self._h, _ptr(k)))
        return k[: self.nb]

    def bind(self, device=None):
        import torch

        device = device or torch.device("cuda", torch.cuda.current_device())
        self.buffers = [torch.empty(max(int(s), 256), dtype=torch.uint8, device=device) for s in self.buffer_sizes]
        ptrs = (ctypes.c_void_p * TDG_NBUF)(*[b.data_ptr() for b in self.buffers])
        _check(lib().trefftz_bind(self._h, ptrs, _stream()))

    def state_tensor(self):
        """Device view (ne, n+2, Q) float64 of the stored (v, sigma, U) values."""
        import torch

        return self.buffers[2][: self.nq * (self.n + 2) * 8].view(torch.float64).view(self.ne, self.n + 2, self.Q)

    def front(self):
        """Host copy of the advancing front (one time per vertex)."""
        import torch

        torch.cuda.synchronize()
        return self.buffers[4][: self.nv * 8].view(torch.float64).cpu().numpy()

    def indicator_tensor(self):
        """Device view (n_tents,) float64 of the per-tent indicator written by
        solves with the indicator on (trefftz_set_indicator)."""
        import torch

        return self.buffers[7][: self.tents.n_tents * 8].view(torch.float64)

    def set_initial(self, v0, sigma0, U0=None):
        v0 = np.ascontiguousarray(v0, dtype=np.float64).reshape(-1)
        s0 = np.ascontiguousarray(sigma0, dtype=np.float64).reshape(-1)
        U0 = None if U0 is None else np.ascontiguousarray(U0, dtype=np.float64).reshape(-1)
        assert v0.size == self.nq and s0.size == self.nq * self.n
        _check(lib().trefftz_set_initial(self._h, _ptr(v0), _ptr(s0), _ptr(U0), _stream()))

    def set_boundary(self, gD):
        gD = np.ascontiguousarray(gD, dtype=np.float64).reshape(-1)
        assert gD.size == self.nb
        _check(lib().trefftz_set_boundary(self._h, _ptr(gD), _stream()))

    def reset(self, stream=None):
        _check(lib().trefftz_reset(self._h, _stream(stream)))

    def layer_solve(self, layer_begin=0, layer_end=None, p_per_tent=None, stream=None):
        if layer_end is None:
            layer_end = self.tents.n_layers
        pp = None if p_per_tent is None else ctypes.c_void_p(p_per_tent.data_ptr())
        _check(lib().trefftz_layer_solve(self._h, int(layer_begin), int(layer_end), pp, _stream(stream)))

    def eval_error(self, v_ex, sigma_ex):
        v_ex = np.ascontiguousarray(v_ex, dtype=np.float64).reshape(-1)
        s_ex = np.ascontiguousarray(sigma_ex, dtype=np.float64).reshape(-1)
        ea, er = ctypes.c_double(), ctypes.c_double()
        _check(lib().trefftz_eval_error(self._h, _ptr(v_ex), _ptr(s_ex), ctypes.byref(ea), ctypes.byref(er), _stream()))
        return ea.value, er.value

    def eval_u_error(self, U_ex):
        U_ex = np.ascontiguousarray(U_ex, dtype=np.float64).reshape(-1)
        assert U_ex.size == self.nq
        ea, er = ctypes.c_double(), ctypes.c_double()
        _check(lib().trefftz_eval_u_error(self._h, _ptr(U_ex), ctypes.byref(ea), ctypes.byref(er), _stream()))
        return ea.value, er.value

    def energy(self):
        E, D = ctypes.c_double(), ctypes.c_double()
        _check(lib().trefftz_energy(self._h, ctypes.byref(E), ctypes.byref(D), _stream()))
        return E.value, D.value

    def status(self):
        _check(lib().trefftz_status(self._h, _stream()))

    def read_state(self):
        v = np.empty(self.nq)
        s = np.empty(self.nq * self.n)
        U = np.empty(self.nq)
        _check(lib().trefftz_read_state(self._h, _ptr(v), _ptr(s), _ptr(U), _stream()))
        return v.reshape(self.ne, self.Q), s.reshape(self.ne, self.Q, self.n), U.reshape(self.ne, self.Q)

    def set_tuning(self, pts_per_chunk=0, persistent=0):
        _check(lib().trefftz_set_tuning(self._h, int(pts_per_chunk), int(persistent)))

    def set_gram_mode(self, mode):
        _check(lib().trefftz_set_gram_mode(self._h, int(mode)))

    def get_gram_mode(self):
        m = ctypes.c_int32()
        _check(lib().trefftz_get_gram_mode(self._h, ctypes.byref(m)))
        return m.value

    def get_tuning(self):
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().trefftz_get_tuning(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return dict(pts_per_chunk=a.value, persistent=b.value, lds_bytes=c.value)

    def capture_sweep(self, layer_begin=0, layer_end=None, p_per_tent=None, with_reset=True, stream=None):
        if layer_end is None:
            layer_end = self.tents.n_layers
        pp = None if p_per_tent is None else ctypes.c_void_p(p_per_tent.data_ptr())
        _check(lib().trefftz_capture_sweep(self._h, int(layer_begin), int(layer_end), pp, int(bool(with_reset)),
                                           _stream(stream)))

    def replay_sweep(self, stream=None):
        _check(lib().trefftz_replay_sweep(self._h, _stream(stream)))

    def tent_stats(self, first=0, count=None):
        if count is None:
            count = self.tents.n_tents - first
        ir = np.zeros(count, np.int32)
        dis = np.zeros(count)
        _check(lib().trefftz_tent_stats(self._h, int(first), int(count), _ptr(ir), _ptr(dis), _stream()))
        return ir, dis

    def set_indicator(self, on=True):
        _check(lib().trefftz_set_indicator(self._h, int(bool(on))))

    def tent_features(self, layer, feats, stream=None):
        """Writes the features of the tents of `layer` into the device tensor
        feats (n_tents x 8 float32)."""
        _check(lib().trefftz_tent_features(self._h, int(layer), _dptr(feats, "float32", (self.tents.n_tents, 8)),
                                           _stream(stream)))

    def layer_indicator(self, layer, p, eta, stream=None):
        """eta_T at degree p of the tents of `layer` into the device tensor eta
        (n_tents float64); nothing else changes."""
        _check(lib().trefftz_layer_indicator(self._h, int(layer), int(p), _dptr(eta, "float64", (self.tents.n_tents,)),
                                             _stream(stream)))

    def layer_solve_adaptive(self, w_bf16, log_eta_tol, eta_tol, feats, p_sel, p_used=None, eta=None,
                             layer_begin=0, layer_end=None, stream=None):
        if layer_end is None:
            layer_end = self.tents.n_layers
        nt = self.tents.n_tents
        w = None if w_bf16 is None else _dptr(w_bf16, "int16", (mlp_nparam(),))
        _check(lib().trefftz_layer_solve_adaptive(
            self._h, int(layer_begin), int(layer_end), w, float(log_eta_tol), float(eta_tol),
            _dptr(feats, "float32", (nt, 8)), _dptr(p_sel, "int8", (nt,)),
            None if p_used is None else _dptr(p_used, "int8", (nt,)),
            None if eta is None else _dptr(eta, "float64", (nt,)), _stream(stream)))

    def table_info(self, p):
        N, nnz, M, Q = (ctypes.c_int32() for _ in range(4))
        _check(lib().trefftz_table_info(self._h, int(p), ctypes.byref(N), ctypes.byref(nnz), ctypes.byref(M), ctypes.byref(Q)))
        return dict(N=N.value, nnz_fields=nnz.value, n_mono=M.value, Q=Q.value)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.trefftz_destroy(self._h)
            self._h = None
