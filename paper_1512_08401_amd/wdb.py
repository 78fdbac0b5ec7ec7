"""Thin Python binding of the wdb C ABI (``include/wdb.h``).

Argument marshalling only: every numerical step runs in libwdb's HIP
kernels.  Device buffers are torch tensors on a ROCm device (float32,
contiguous); the current torch stream is passed to the library.  If
``libwdb.so`` is missing, importing this module raises ImportError: there is
no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwdb.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1512_08401_amd.build`")

_lib = C.CDLL(LIB_PATH)

WAVELETS = {"haar": 0, "db4": 1, "sym6": 2}
VALTYPES = {"f32": 0, "bf16": 1, "f16": 2}
PRECOND = {"none": 0, "spai": 1, "spai_scale": 2, "jacobi": 3}

WDB_OK = 0
WDB_ERR_ARG, WDB_ERR_SIZE, WDB_ERR_LEVELS, WDB_ERR_NONFINITE = -1, -2, -3, -4
WDB_ERR_OOM, WDB_ERR_HIP, WDB_ERR_DIVERGED, WDB_ERR_NOT_CONVERGED, WDB_ERR_FORMAT = -5, -6, -7, -8, -9


class WdbError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code
        self.msg = msg


class PsfFieldC(C.Structure):
    _fields_ = [("n", C.c_int32), ("sig_major", C.POINTER(C.c_double)),
                ("sig_minor", C.POINTER(C.c_double)), ("angle", C.POINTER(C.c_double)),
                ("trunc", C.c_double)]


class ThetaDesc(C.Structure):
    _fields_ = [("n", C.c_int32), ("levels", C.c_int32), ("wavelet", C.c_int32),
                ("has_lipschitz", C.c_int32), ("nnz", C.c_int64), ("stored", C.c_int64),
                ("lipschitz", C.c_double), ("threshold", C.c_double), ("lipschitz_p", C.c_double),
                ("precond", C.c_int32), ("valtype", C.c_int32), ("slice", C.c_int32), ("group", C.c_int32),
                ("group16", C.c_int32), ("escapes", C.c_int64), ("conv_build", C.c_int32),
                ("l1_weights", C.c_int32), ("rule", C.c_int32), ("circulant", C.c_int64),
                ("tile_waves", C.c_int32), ("tile_slots", C.c_int64), ("tile_waves16", C.c_int32),
                ("tile_unroll", C.c_int32), ("tile_unroll16", C.c_int32), ("tile_escapes", C.c_int64),
                ("tile_kept", C.c_int32), ("reserved", C.c_int32), ("tile_kept_values", C.c_int64)]


class SolveOpts(C.Structure):
    _fields_ = [("max_iters", C.c_int32), ("check_every", C.c_int32), ("tol_rel_gap", C.c_double),
                ("x_init", C.c_void_p), ("k0", C.c_int32), ("use_precond", C.c_int32),
                ("stream", C.c_void_p), ("trace", C.POINTER(C.c_double)), ("trace_cap", C.c_int32),
                ("use_graph", C.c_int32), ("target_objective", C.c_double), ("ista", C.c_int32),
                ("plain_iterate", C.c_int32), ("x64_out", C.c_void_p)]


class ProblemC(C.Structure):
    _fields_ = [("theta", C.c_void_p), ("u", C.c_void_p), ("lam", C.c_float), ("x_init", C.c_void_p),
                ("x_out", C.c_void_p), ("target_objective", C.c_double), ("x0", C.c_void_p),
                ("x64_out", C.c_void_p)]


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int32), ("checks", C.c_int32), ("objective", C.c_double),
                ("rel_gap", C.c_double), ("lipschitz", C.c_double), ("tau", C.c_double)]


_vp, _i32, _i64, _f32, _f64 = C.c_void_p, C.c_int32, C.c_int64, C.c_float, C.c_double
_pd = C.POINTER(C.c_double)

_SIGS = {
    "wdb_build_theta": [C.POINTER(PsfFieldC), _i32, _i32, _i64, _vp, C.POINTER(_vp)],
    "wdb_build_theta_rule": [C.POINTER(PsfFieldC), _i32, _i32, _i64, _i32, _vp, C.POINTER(_vp)],
    "wdb_theta_import": [_i32, _i32, _i32, _i64, _vp, _vp, _vp, _vp, C.POINTER(_vp)],
    "wdb_theta_export": [_vp, _vp, _vp, _vp],
    "wdb_theta_info": [_vp, C.POINTER(ThetaDesc)],
    "wdb_theta_lipschitz": [_vp, _vp, _f64, _i32, _pd, C.POINTER(_i32)],
    "wdb_theta_lipschitz_lanczos": [_vp, _vp, _f64, _i32, _pd, C.POINTER(_i32), _pd],
    "wdb_exact_create": [C.POINTER(PsfFieldC), _i32, _i32, _vp, C.POINTER(_vp)],
    "wdb_exact_apply": [_vp, _i32, _vp, _vp, _vp],
    "wdb_exact_lipschitz": [_vp, _vp, _f64, _i32, _pd, C.POINTER(_i32), _pd],
    "wdb_exact_solve": [_vp, _vp, _f32, C.POINTER(SolveOpts), _vp, C.POINTER(SolveInfo)],
    "wdb_set_precond": [_vp, _i32, _f64, _vp, _f64, _i32],
    "wdb_get_precond": [_vp, _vp],
    "wdb_solve": [_vp, _vp, _f32, C.POINTER(SolveOpts), _vp, C.POINTER(SolveInfo)],
    "wdb_solve_coeffs": [_vp, _vp, _f32, C.POINTER(SolveOpts), _vp, C.POINTER(SolveInfo)],
    "wdb_objective": [_vp, _vp, _vp, _f32, _vp, _pd, _pd],
    "wdb_theta_apply": [_vp, _i32, _vp, _vp, _vp, _i32, _vp],
    "wdb_prox_step": [_vp, _vp, _vp, _vp, _f32, _f32, _f32, _i32, _vp],
    "wdb_synthesize": [_vp, _vp, _vp, _vp],
    "wdb_dwt": [_i32, _i32, _i32, _vp, _vp, _i32, _vp],
    "wdb_dwt_batched": [_i32, _i32, _i32, _i32, _vp, _vp, _i32, _vp],
    "wdb_blur": [C.POINTER(PsfFieldC), _vp, _vp, _vp],
    "wdb_wavelet_filter": [_i32, _pd, _i32, C.POINTER(_i32)],
    "wdb_set_precision": [_vp, _i32],
    "wdb_set_kernel_layout": [_vp, _i32, _i32],
    "wdb_set_packed_group": [_vp, _i32],
    "wdb_set_tile_shape": [_vp, _i32, _i32],
    "wdb_set_tile_values": [_vp, _i32],
    "wdb_set_l1_weights": [_vp, _i32, _vp],
    "wdb_autotune": [_vp, C.c_char_p, _i32, C.POINTER(_i32), C.POINTER(_i32), _pd],
    "wdb_cnn_create": [_i32, _i32, _i32, C.c_uint64, C.POINTER(_vp)],
    "wdb_cnn_param_count": [_vp, C.POINTER(_i64)],
    "wdb_cnn_set_params": [_vp, _vp, _i64],
    "wdb_cnn_get_params": [_vp, _vp, _i32],
    "wdb_cnn_predict": [_vp, _vp, _i32, _vp, _vp],
    "wdb_cnn_loss_grad": [_vp, _vp, _vp, _i32, _pd, _vp, _vp],
    "wdb_cnn_train_step": [_vp, _vp, _vp, _i32, _f32, _pd, _vp],
    "wdb_solve_batched": [_i32, C.POINTER(ProblemC), C.POINTER(SolveOpts), C.POINTER(SolveInfo)],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = C.c_int
_lib.wdb_cnn_free.argtypes = [_vp]
_lib.wdb_cnn_free.restype = None
_lib.wdb_theta_free.argtypes = [_vp]
_lib.wdb_theta_free.restype = None
_lib.wdb_exact_free.argtypes = [_vp]
_lib.wdb_exact_free.restype = None
_lib.wdb_last_error.restype = C.c_char_p
_lib.wdb_version.restype = C.c_char_p


def _check(fn: str, status: int) -> None:
    if status != WDB_OK:
        raise WdbError(fn, status, _lib.wdb_last_error().decode(errors="replace"))


def version() -> str:
    return _lib.wdb_version().decode()


def wavelet_filter(name: str) -> np.ndarray:
    """Low-pass analysis filter the library derives for ``name`` (host only)."""
    ln = C.c_int32(0)
    _check("wdb_wavelet_filter", _lib.wdb_wavelet_filter(WAVELETS[name], None, 0, C.byref(ln)))
    h = np.zeros(ln.value)
    _check("wdb_wavelet_filter", _lib.wdb_wavelet_filter(WAVELETS[name], h.ctypes.data_as(_pd), ln.value,
                                                         C.byref(ln)))
    return h


# --------------------------------------------------------------------------
# helpers
# --------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream(stream=None):
    if stream is not None:
        return C.c_void_p(int(stream))
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, numel=None, name="tensor"):
    """Device pointer of a contiguous float32 ROCm tensor (checked)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float32")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


def _dev64(t, numel=None, name="tensor"):
    """Device pointer of a contiguous float64 ROCm tensor (checked)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous float64")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return C.c_void_p(t.data_ptr())


def _field_struct(field):
    n = int(field.n)
    arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float64).reshape(n * n))
            for a in (field.sig_major, field.sig_minor, field.angle)]
    st = PsfFieldC(n, arrs[0].ctypes.data_as(_pd), arrs[1].ctypes.data_as(_pd),
                   arrs[2].ctypes.data_as(_pd), float(getattr(field, "trunc", 3.0)))
    return st, arrs   # keep arrays alive with the struct


def _f64ptr(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return C.c_void_p(arr.ctypes.data), arr


# --------------------------------------------------------------------------
# operator handle
# --------------------------------------------------------------------------
class Theta:
    """Owns a wdb_theta handle."""

    def __init__(self, handle: C.c_void_p):
        self._h = handle

    # The free routine is bound at class creation: at interpreter exit the
    # module's globals may already be cleared when a handle is collected.
    def __del__(self, _free=_lib.wdb_theta_free):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _free(h)
            self._h = None

    def free(self):
        self.__del__()

    @property
    def handle(self):
        return self._h

    @classmethod
    def build(cls, field, wavelet: str, levels: int, nnz_budget: int, stream=None, rule: str = "naive") -> "Theta":
        """Theta_K of a PSF field; rule "naive" (K largest |Theta|) or "scale"
        (K largest 2^-k |Theta[a, b]| for column b of scale k, Sec. 3.7)."""
        st, keep = _field_struct(field)
        out = C.c_void_p()
        _check("wdb_build_theta_rule", _lib.wdb_build_theta_rule(C.byref(st), WAVELETS[wavelet], levels,
                                                                 int(nnz_budget), {"naive": 0, "scale": 1}[rule],
                                                                 _stream(stream), C.byref(out)))
        del keep
        return cls(out)

    @classmethod
    def from_csr(cls, n: int, wavelet: str, levels: int, rowptr, col, val, stream=None) -> "Theta":
        rp = np.ascontiguousarray(np.asarray(rowptr, dtype=np.int64))
        cc = np.ascontiguousarray(np.asarray(col, dtype=np.int32))
        vv = np.ascontiguousarray(np.asarray(val, dtype=np.float64))
        out = C.c_void_p()
        _check("wdb_theta_import", _lib.wdb_theta_import(n, WAVELETS[wavelet], levels, int(vv.size),
                                                         C.c_void_p(rp.ctypes.data), C.c_void_p(cc.ctypes.data),
                                                         C.c_void_p(vv.ctypes.data), _stream(stream), C.byref(out)))
        return cls(out)

    def info(self) -> dict:
        d = ThetaDesc()
        _check("wdb_theta_info", _lib.wdb_theta_info(self._h, C.byref(d)))
        return {k: getattr(d, k) for k, _ in ThetaDesc._fields_}

    def export(self):
        """(rowptr int64, col int32, val float64) host arrays."""
        d = self.info()
        N = d["n"] * d["n"]
        rp = np.zeros(N + 1, dtype=np.int64)
        cc = np.zeros(max(d["nnz"], 1), dtype=np.int32)
        vv = np.zeros(max(d["nnz"], 1), dtype=np.float64)
        _check("wdb_theta_export", _lib.wdb_theta_export(self._h, C.c_void_p(rp.ctypes.data),
                                                         C.c_void_p(cc.ctypes.data), C.c_void_p(vv.ctypes.data)))
        return rp, cc[: d["nnz"]], vv[: d["nnz"]]

    def lipschitz(self, start=None, tol: float = 1e-12, max_iters: int = 20000, require: bool = True):
        """L by the power iteration; returns (L, iterations).  A run that hits
        max_iters raises unless require=False (the handle keeps the quotient)."""
        p, keep = _f64ptr(start)
        L = C.c_double(0.0)
        it = C.c_int32(0)
        st = _lib.wdb_theta_lipschitz(self._h, p, tol, max_iters, C.byref(L), C.byref(it))
        if not (st == WDB_ERR_NOT_CONVERGED and not require):
            _check("wdb_theta_lipschitz", st)
        return L.value, it.value

    def lipschitz_lanczos(self, start=None, tol: float = 1e-12, max_steps: int = 2000) -> dict:
        """L = theta + resid by restarted Lanczos (the solver's default)."""
        p, keep = _f64ptr(start)
        L, res = C.c_double(0.0), C.c_double(0.0)
        st = C.c_int32(0)
        status = _lib.wdb_theta_lipschitz_lanczos(self._h, p, tol, max_steps, C.byref(L), C.byref(st), C.byref(res))
        if status != WDB_ERR_NOT_CONVERGED:
            _check("wdb_theta_lipschitz_lanczos", status)
        return {"L": L.value, "theta": L.value - res.value, "resid": res.value, "method": "lanczos",
                "steps": st.value, "converged": status == 0}

    def lipschitz_info(self, start=None, tol: float = 1e-12, max_steps: int = 2000) -> dict:
        return self.lipschitz_lanczos(start, tol, max_steps)

    def set_precond(self, kind: str, eps: float = 0.0, start=None, tol: float = 1e-12, max_iters: int = 20000):
        p, keep = _f64ptr(start)
        _check("wdb_set_precond", _lib.wdb_set_precond(self._h, PRECOND[kind], eps, p, tol, max_iters))

    def set_kernel_layout(self, slice: int = 64, group: int = 0):
        _check("wdb_set_kernel_layout", _lib.wdb_set_kernel_layout(self._h, slice, group))

    def set_l1_weights(self, kind="uniform", w=None):
        """l1 weights: "uniform", "scale" (w[i] = j(i), Sec. 5) or "given" with a host array of N floats."""
        k = {"uniform": 0, "scale": 1, "given": 2}[kind]
        arr = None
        if k == 2:
            arr = np.ascontiguousarray(w, dtype=np.float32)
            if arr.size != self.N:
                raise ValueError(f"weights have {arr.size} entries, expected {self.N}")
        _check("wdb_set_l1_weights", _lib.wdb_set_l1_weights(self._h, k, None if arr is None else
                                                             arr.ctypes.data_as(C.c_void_p)))

    def set_packed_group(self, group: int = 0):
        """Lanes per row of the packed 16-bit kernels (2/4/8/16; 0 = default)."""
        _check("wdb_set_packed_group", _lib.wdb_set_packed_group(self._h, int(group)))

    def set_tile_shape(self, waves: int = 4, unroll: int = 0):
        """Tiled kernels of the current value type: wavefronts per tile (1/2/4/8) and
        code groups in flight per wavefront (1/2/4; 0 = default)."""
        _check("wdb_set_tile_shape", _lib.wdb_set_tile_shape(self._h, int(waves), int(unroll)))

    def set_tile_values(self, kept: bool):
        """Value layout of the float32 tiled kernels: kept values with row masks
        (True) or the dense values (False)."""
        _check("wdb_set_tile_values", _lib.wdb_set_tile_values(self._h, 1 if kept else 0))

    def autotune(self, cache_path: str | None = None, reps: int = 20):
        """Pick the fastest iteration layout for this operator; returns (slice, group, us)."""
        c, g, us = C.c_int32(), C.c_int32(), C.c_double()
        _check("wdb_autotune", _lib.wdb_autotune(self._h, cache_path.encode() if cache_path else None, reps,
                                                 C.byref(c), C.byref(g), C.byref(us)))
        return c.value, g.value, us.value

    def set_precision(self, valtype: str):
        """Iteration values in float32, bfloat16 or binary16 ("f32" | "bf16" | "f16")."""
        _check("wdb_set_precision", _lib.wdb_set_precision(self._h, VALTYPES[valtype]))

    def precond(self) -> np.ndarray:
        d = self.info()
        out = np.zeros(d["n"] * d["n"])
        _check("wdb_get_precond", _lib.wdb_get_precond(self._h, C.c_void_p(out.ctypes.data)))
        return out

    @property
    def N(self) -> int:
        d = self.info()
        return d["n"] * d["n"]

    def apply(self, x, b=None, transpose: bool = False, out=None, repeat: int = 1, stream=None):
        torch = _torch()
        N = self.N
        y = torch.empty(N, device=x.device, dtype=torch.float32) if out is None else out
        _check("wdb_theta_apply", _lib.wdb_theta_apply(self._h, 1 if transpose else 0, _dev(x, N, "x"),
                                                       None if b is None else _dev(b, N, "b"), _dev(y, N, "out"),
                                                       repeat, _stream(stream)))
        return y

    def prox_step(self, r, x, y, tau: float, lam: float, beta: float, use_precond: bool = False, stream=None):
        N = self.N
        _check("wdb_prox_step", _lib.wdb_prox_step(self._h, _dev(r, N, "r"), _dev(x, N, "x"), _dev(y, N, "y"),
                                                   tau, lam, beta, 1 if use_precond else 0, _stream(stream)))

    def objective(self, x, x0, lam: float, stream=None):
        N = self.N
        E = C.c_double(0.0)
        g = C.c_double(0.0)
        _check("wdb_objective", _lib.wdb_objective(self._h, _dev(x, N, "x"), _dev(x0, N, "x0"), lam,
                                                   _stream(stream), C.byref(E), C.byref(g)))
        return E.value, g.value

    def _solve(self, fn, src, lam, iters, check_every, tol, x_init, k0, precond, use_graph, trace_cap, out,
               stream, target=0.0, ista=False, plain_iterate=False, x64_out=None):
        torch = _torch()
        N = self.N
        x = torch.empty(N, device=src.device, dtype=torch.float32) if out is None else out
        trace = np.zeros(3 * max(trace_cap, 1))
        o = SolveOpts(int(iters), int(check_every), float(tol),
                      None if x_init is None else _dev(x_init, N, "x_init").value, int(k0),
                      1 if precond else 0, _stream(stream).value, trace.ctypes.data_as(_pd), int(trace_cap),
                      1 if use_graph else 0, float(target), 1 if ista else 0, 1 if plain_iterate else 0,
                      None if x64_out is None else _dev64(x64_out, N, "x64_out").value)
        info = SolveInfo()
        st = getattr(_lib, fn)(self._h, _dev(src, name="input"), float(lam), C.byref(o), _dev(x, N, "x_out"),
                               C.byref(info))
        res = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
        res["trace"] = trace[: 3 * min(info.checks, trace_cap)].reshape(-1, 3)
        if st == WDB_ERR_NOT_CONVERGED:
            res["converged"] = False
            return x, res
        _check(fn, st)
        res["converged"] = tol > 0 or target > 0
        return x, res

    def solve(self, u, lam: float, iters: int, check_every: int = 20, tol: float = 0.0, x_init=None, k0: int = 1,
              precond: bool = False, use_graph: bool = False, trace_cap: int = 0, out=None, stream=None,
              target: float = 0.0, ista: bool = False, plain_iterate: bool = False, x64_out=None):
        """FISTA (ISTA with ista=True) from a blurred image u (device n*n float32); returns (x, info).
        plain_iterate=True keeps the float32 iterate without its float64 anchor; x64_out (device
        float64, N) receives the float64 iterate the last check scored."""
        return self._solve("wdb_solve", u, lam, iters, check_every, tol, x_init, k0, precond, use_graph,
                           trace_cap, out, stream, target, ista, plain_iterate, x64_out)

    def solve_coeffs(self, x0, lam: float, iters: int, check_every: int = 20, tol: float = 0.0, x_init=None,
                     k0: int = 1, precond: bool = False, use_graph: bool = False, trace_cap: int = 0, out=None,
                     stream=None, target: float = 0.0, ista: bool = False, plain_iterate: bool = False,
                     x64_out=None):
        """FISTA (ISTA with ista=True) from wavelet-domain data x0 (device N float32); returns (x, info)."""
        return self._solve("wdb_solve_coeffs", x0, lam, iters, check_every, tol, x_init, k0, precond, use_graph,
                           trace_cap, out, stream, target, ista, plain_iterate, x64_out)

    def synthesize(self, x, out=None, stream=None):
        torch = _torch()
        d = self.info()
        n = d["n"]
        u = torch.empty((n, n), device=x.device, dtype=torch.float32) if out is None else out
        _check("wdb_synthesize", _lib.wdb_synthesize(self._h, _dev(x, n * n, "x"), _dev(u, n * n, "u_hat"),
                                                     _stream(stream)))
        return u


class Exact:
    """Owns a wdb_exact handle: Alg. 1 with the exact-operator gradient (the baseline)."""

    def __init__(self, field, wavelet: str, levels: int, stream=None):
        self._h = C.c_void_p()
        st, keep = _field_struct(field)
        _check("wdb_exact_create", _lib.wdb_exact_create(C.byref(st), WAVELETS[wavelet], levels, _stream(stream),
                                                         C.byref(self._h)))
        self.n, self.N, self.levels = int(field.n), int(field.n) ** 2, levels

    def __del__(self, _free=_lib.wdb_exact_free):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _free(h)
            self._h = None

    def apply(self, u, adjoint: bool = False, out=None, stream=None):
        """H u (or H^* u) on an image (device float32, n*n)."""
        torch = _torch()
        y = torch.empty(self.N, device=u.device, dtype=torch.float32) if out is None else out
        _check("wdb_exact_apply", _lib.wdb_exact_apply(self._h, 1 if adjoint else 0, _dev(u, self.N, "in"),
                                                       _dev(y, self.N, "out"), _stream(stream)))
        return y

    def lipschitz(self, start=None, tol: float = 1e-12, max_steps: int = 2000) -> dict:
        p, keep = _f64ptr(start)
        L, res = C.c_double(0.0), C.c_double(0.0)
        st = C.c_int32(0)
        status = _lib.wdb_exact_lipschitz(self._h, p, tol, max_steps, C.byref(L), C.byref(st), C.byref(res))
        if status != WDB_ERR_NOT_CONVERGED:
            _check("wdb_exact_lipschitz", status)
        return {"L": L.value, "theta": L.value - res.value, "resid": res.value, "steps": st.value,
                "converged": status == 0}

    def solve(self, u, lam: float, iters: int, check_every: int = 20, tol: float = 0.0, x_init=None, k0: int = 1,
              trace_cap: int = 0, out=None, stream=None, target: float = 0.0, ista: bool = False):
        """Alg. 1 with the exact gradient from a blurred image u (device n*n float32); returns (x, info)."""
        torch = _torch()
        x = torch.empty(self.N, device=u.device, dtype=torch.float32) if out is None else out
        trace = np.zeros(3 * max(trace_cap, 1))
        o = SolveOpts(int(iters), int(check_every), float(tol),
                      None if x_init is None else _dev(x_init, self.N, "x_init").value, int(k0), 0,
                      _stream(stream).value, trace.ctypes.data_as(_pd), int(trace_cap), 0, float(target),
                      1 if ista else 0)
        info = SolveInfo()
        st = _lib.wdb_exact_solve(self._h, _dev(u, self.N, "u"), float(lam), C.byref(o), _dev(x, self.N, "x_out"),
                                  C.byref(info))
        res = {k: getattr(info, k) for k, _ in SolveInfo._fields_}
        res["trace"] = trace[: 3 * min(info.checks, trace_cap)].reshape(-1, 3)
        if st == WDB_ERR_NOT_CONVERGED:
            res["converged"] = False
            return x, res
        _check("wdb_exact_solve", st)
        res["converged"] = tol > 0 or target > 0
        return x, res


class Cnn:
    """Owns a wdb_cnn handle (warm-start network)."""

    def __init__(self, n: int, levels: int, features: int = 32, seed: int = 0):
        self._h = C.c_void_p()
        _check("wdb_cnn_create", _lib.wdb_cnn_create(n, levels, features, seed, C.byref(self._h)))
        self.n, self.N = n, n * n
        cnt = C.c_int64()
        _check("wdb_cnn_param_count", _lib.wdb_cnn_param_count(self._h, C.byref(cnt)))
        self.nparam = cnt.value

    def __del__(self, _free=_lib.wdb_cnn_free):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            _free(h)
            self._h = None

    def set_params(self, p):
        a = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
        _check("wdb_cnn_set_params", _lib.wdb_cnn_set_params(self._h, C.c_void_p(a.ctypes.data), a.size))

    def get_params(self, rounded: bool = False) -> np.ndarray:
        out = np.zeros(self.nparam, dtype=np.float32)
        _check("wdb_cnn_get_params", _lib.wdb_cnn_get_params(self._h, C.c_void_p(out.ctypes.data), int(rounded)))
        return out

    def predict(self, x0, out=None, stream=None):
        torch = _torch()
        B = x0.numel() // self.N
        y = torch.empty_like(x0) if out is None else out
        _check("wdb_cnn_predict", _lib.wdb_cnn_predict(self._h, _dev(x0, B * self.N, "x0"), B,
                                                       _dev(y, B * self.N, "out"), _stream(stream)))
        return y

    def loss_grad(self, x0, target, stream=None):
        B = x0.numel() // self.N
        loss = C.c_double()
        g = np.zeros(self.nparam, dtype=np.float32)
        _check("wdb_cnn_loss_grad", _lib.wdb_cnn_loss_grad(self._h, _dev(x0, B * self.N, "x0"),
                                                           _dev(target, B * self.N, "target"), B, C.byref(loss),
                                                           C.c_void_p(g.ctypes.data), _stream(stream)))
        return loss.value, g

    def train_step(self, x0, target, lr: float, stream=None) -> float:
        B = x0.numel() // self.N
        loss = C.c_double()
        _check("wdb_cnn_train_step", _lib.wdb_cnn_train_step(self._h, _dev(x0, B * self.N, "x0"),
                                                             _dev(target, B * self.N, "target"), B, lr,
                                                             C.byref(loss), _stream(stream)))
        return loss.value


def solve_batched(problems, iters: int, check_every: int = 20, tol: float = 0.0, k0: int = 1,
                  precond: bool = False, use_graph: bool = False, outs=None, stream=None, coeffs: bool = False,
                  outs64=None):
    """Batched Alg. 1.  ``problems``: list of (theta, u, lam[, x_init[, target_objective]]).
    With ``coeffs`` the second entry of every problem is the wavelet-domain
    data x0 = Psi^* u (N coefficients) instead of the image.  ``outs64``
    (optional list of float64 device tensors) receive the float64 iterates the
    last checks scored.  Returns (list of x tensors, list of info dicts)."""
    torch = _torch()
    n = len(problems)
    arr = (ProblemC * n)()
    xs = []
    for i, p in enumerate(problems):
        th, u, lam = p[0], p[1], p[2]
        xi = p[3] if len(p) > 3 else None
        tgt = float(p[4]) if len(p) > 4 else 0.0
        N = th.N
        x = torch.empty(N, device=u.device, dtype=torch.float32) if outs is None else outs[i]
        xs.append(x)
        data = _dev(u, N, "x0" if coeffs else "u").value
        arr[i] = ProblemC(th.handle.value, None if coeffs else data, float(lam),
                          None if xi is None else _dev(xi, N, "x_init").value, _dev(x, N, "x_out").value, tgt,
                          data if coeffs else None,
                          None if outs64 is None or outs64[i] is None else _dev64(outs64[i], N, "x64_out").value)
    o = SolveOpts(int(iters), int(check_every), float(tol), None, int(k0), 1 if precond else 0,
                  _stream(stream).value, None, 0, 1 if use_graph else 0, 0.0, 0)
    infos = (SolveInfo * n)()
    st = _lib.wdb_solve_batched(n, arr, C.byref(o), infos)
    res = [{k: getattr(inf, k) for k, _ in SolveInfo._fields_} for inf in infos]
    if st != WDB_ERR_NOT_CONVERGED:
        _check("wdb_solve_batched", st)
    # per problem: met its own stopping test (tolerance, or its objective target)
    for p, r in zip(problems, res):
        tgt = float(p[4]) if len(p) > 4 else 0.0
        r["converged"] = (tol > 0 and r["rel_gap"] <= tol) or (tgt > 0 and r["objective"] <= tgt)
    return xs, res


def build_theta(field, wavelet: str, levels: int, nnz_budget: int, stream=None, rule: str = "naive") -> Theta:
    return Theta.build(field, wavelet, levels, nnz_budget, stream, rule)


def dwt(u, wavelet: str, levels: int, inverse: bool = False, out=None, stream=None):
    torch = _torch()
    n = int(round(u.numel() ** 0.5))
    y = torch.empty(n * n, device=u.device, dtype=torch.float32) if out is None else out
    _check("wdb_dwt", _lib.wdb_dwt(n, WAVELETS[wavelet], levels, _dev(u, n * n, "in"), _dev(y, n * n, "out"),
                                   1 if inverse else 0, _stream(stream)))
    return y


def dwt_batched(u, wavelet: str, levels: int, inverse: bool = False, out=None, stream=None):
    """The transform of every row of a (count, n*n) float32 device tensor."""
    torch = _torch()
    count, N = u.shape
    n = int(round(N ** 0.5))
    y = torch.empty((count, N), device=u.device, dtype=torch.float32) if out is None else out
    _check("wdb_dwt_batched", _lib.wdb_dwt_batched(n, WAVELETS[wavelet], levels, count, _dev(u, count * N, "in"),
                                                   _dev(y, count * N, "out"), 1 if inverse else 0,
                                                   _stream(stream)))
    return y


def blur(field, u, out=None, stream=None):
    torch = _torch()
    n = int(field.n)
    y = torch.empty((n, n), device=u.device, dtype=torch.float32) if out is None else out
    st, keep = _field_struct(field)
    _check("wdb_blur", _lib.wdb_blur(C.byref(st), _dev(u, n * n, "u"), _dev(y, n * n, "out"), _stream(stream)))
    return y
