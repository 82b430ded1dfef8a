"""Python binding of libappga (ctypes).  Argument marshalling only.

Every function named ``appga_*`` calls the C entry point of the same name in
``libappga.so`` (declared in include/appga.h) and raises ``AppgaError`` when
it returns a negative status.  Host arrays are numpy arrays; device arrays are
torch tensors on a HIP device (their ``data_ptr()`` is passed), with torch's
current stream unless another one is given.  Nothing here computes any part of
the reconstruction, and there is no fallback: if the library is missing the
import of this module's functions fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libappga.so")

APPGA_OK = 0
STATUS_NAMES = {
    0: "APPGA_OK", -1: "APPGA_E_INVALID_ARG", -2: "APPGA_E_SHAPE", -3: "APPGA_E_DOMAIN",
    -4: "APPGA_E_OOM", -5: "APPGA_E_DEVICE", -6: "APPGA_E_NONFINITE", -7: "APPGA_E_BUSY",
    -8: "APPGA_E_NOT_FOUND", -9: "APPGA_E_TIMEOUT",
}
APPGA_F32, APPGA_BF16, APPGA_F16, APPGA_FP8_E4M3_ROWSCALE = 1, 2, 3, 4
DTYPES = {"f32": APPGA_F32, "bf16": APPGA_BF16, "f16": APPGA_F16, "fp8": APPGA_FP8_E4M3_ROWSCALE}
APPGA_MOMENTUM_GN, APPGA_MOMENTUM_NONE, APPGA_MOMENTUM_NESTEROV = 0, 1, 2
APPGA_PRECOND_EM, APPGA_PRECOND_EM_FROZEN, APPGA_PRECOND_FIXED = 0, 1, 2


class AppgaError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__("%s: %s (%s)" % (where, STATUS_NAMES.get(status, status), message))


class appga_geometry(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_angles", C.c_int32), ("n_bins", C.c_int32)]


class appga_params(C.Structure):
    _fields_ = [("lambda1", C.c_double), ("lambda2", C.c_double), ("eps", C.c_double),
                ("omega", C.c_double), ("a", C.c_double), ("b", C.c_double),
                ("beta", C.c_double), ("iterations", C.c_int32), ("momentum", C.c_int32),
                ("precond", C.c_int32), ("precond_freeze_iter", C.c_int32),
                ("monitor_every", C.c_int32), ("fixed_p", C.c_double),
                ("gamma_scalar", C.c_double)]


class appga_stats(C.Structure):
    _fields_ = [("iterations_done", C.c_int32), ("objective0", C.c_double),
                ("objective", C.c_double), ("re", C.c_double), ("guard_clamps", C.c_int64),
                ("seconds", C.c_double)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class appga_server_cfg(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("slots_per_matrix", C.c_int32),
                ("reserved", C.c_int32)]


_lib = None
P, I32, I64, D, U64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
PP = C.POINTER(C.c_void_p)

_SIGS = {
    "appga_params_default": [C.POINTER(appga_params)],
    "appga_validate_params": [C.POINTER(appga_params)],
    "appga_validate_system_matrix": [C.POINTER(appga_geometry), I64, P, P, P],
    "appga_create": [PP, C.c_int],
    "appga_destroy": [P],
    "appga_load_system_matrix": [P, C.POINTER(appga_geometry), I64, P, P, P, C.c_int, PP],
    "appga_free_system_matrix": [P, P],
    "appga_load_system_matrix_factored": [P, C.POINTER(appga_geometry), I64, P, P, P, C.c_int, P, D, PP],
    "appga_matrix_psf": [P, C.POINTER(D), C.POINTER(I32)],
    "appga_matrix_symmetry": [P, C.POINTER(I32), C.POINTER(I64)],
    "appga_matrix_info": [P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I64), C.POINTER(I32)],
    "appga_matrix_dequantized": [P, P],
    "appga_reconstruct": [P, P, P, P, C.POINTER(appga_params), P, P, C.POINTER(appga_stats)],
    "appga_reconstruct_simple": [P, P, P, P, D, D, D, I32, P],
    "appga_reconstruct_batch": [P, P, I32, P, P, C.POINTER(appga_params), P, P,
                                C.POINTER(appga_stats)],
    "appga_reconstruct_batch_device": [P, P, I32, P, P, C.POINTER(appga_params), P, P, P],
    "appga_solve_begin": [P, P, I32, P, P, C.POINTER(appga_params), P, P, PP],
    "appga_afppa_batch": [P, P, I32, P, P, C.POINTER(appga_params), P, P, P, C.POINTER(appga_stats)],
    "appga_afppa_batch_device": [P, P, I32, P, P, C.POINTER(appga_params), P, P, P, P],
    "appga_afppa_begin": [P, P, I32, P, P, C.POINTER(appga_params), P, P, PP],
    "appga_solve_duals": [P, P],
    "appga_solve_image": [P, P],
    "appga_solve_step": [P, I32],
    "appga_solve_end": [P, P, C.POINTER(appga_stats)],
    "appga_op_forward": [P, P, I32, P, P, P, P],
    "appga_op_ratio": [P, P, I32, P, P, P, P, P],
    "appga_op_back": [P, P, I32, P, P, P],
    "appga_op_grad_reg": [P, I32, I32, P, P, P, P, P, P],
    "appga_op_step": [P, P, I32, P, P, P, P, P, P, P, P, P, P, P],
    "appga_set_kernel_timing": [P, I32],
    "appga_kernel_times": [P, I32, P, I32, P, P, C.POINTER(I32)],
    "appga_server_footprint": [P, C.POINTER(I64)],
    "appga_tune": [P, P, I32, P],
    "appga_solve_history": [P, I32, I32, P, P, C.POINTER(I32)],
    "appga_server_start": [P, C.POINTER(appga_server_cfg), PP],
    "appga_submit": [P, P, P, P, C.POINTER(appga_params), C.POINTER(U64)],
    "appga_wait": [P, U64, P, C.POINTER(appga_stats), I32],
    "appga_server_stop": [P],
    "appga_matrix_tiles": [P, I32, P],
    "appga_tiles_emulate": [C.POINTER(appga_geometry), I64, P, P, P, C.c_int, I32, I32, P, P, P],
}


def load_library(path: str = LIB_PATH):
    """Loads libappga.so (built by ``paper_2409_13344_amd.build``); raises if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError("libappga.so not found at %s: build the HIP library first "
                               "(python -m paper_2409_13344_amd.build)" % path)
        lib = C.CDLL(path)
        for name, args in _SIGS.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = C.c_int
        lib.appga_last_error.argtypes = []
        lib.appga_last_error.restype = C.c_char_p
        _lib = lib
    return _lib


def appga_last_error() -> str:
    return load_library().appga_last_error().decode()


def _check(st: int, where: str):
    if st != APPGA_OK:
        raise AppgaError(st, where, appga_last_error())


def _call(name: str, *args):
    st = getattr(load_library(), name)(*args)
    _check(st, name)


def _np(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if hasattr(a, "data_ptr"):          # torch tensor (device memory)
        return a.data_ptr()
    return a.ctypes.data


def _stream(stream) -> Optional[int]:
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ------------------------------------------------------------- parameters ---

def appga_params_default() -> appga_params:
    p = appga_params()
    _call("appga_params_default", C.byref(p))
    return p


def make_params(**kw) -> appga_params:
    """appga_params_default() with fields overridden; ``lam`` sets lambda1 = lambda2."""
    p = appga_params_default()
    lam = kw.pop("lam", None)
    if lam is not None:
        p.lambda1 = p.lambda2 = lam
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def appga_validate_params(p: appga_params) -> None:
    _call("appga_validate_params", C.byref(p))


def appga_validate_system_matrix(n, n_angles, n_bins, row_ptr, col, val) -> None:
    geom = appga_geometry(n, n_angles, n_bins)
    rp, cl, vl = _np(row_ptr, np.int64), _np(col, np.int32), _np(val, np.float64)
    _call("appga_validate_system_matrix", C.byref(geom), len(cl), _ptr(rp), _ptr(cl), _ptr(vl))


# --------------------------------------------------------- context, matrix ---

def appga_create(device: int = 0) -> int:
    h = C.c_void_p()
    _call("appga_create", C.byref(h), device)
    return h.value


def appga_destroy(ctx: int) -> None:
    _call("appga_destroy", ctx)


# (m, d) of every loaded matrix and (B, m, d) of every open session: the device
# entry points cannot see the length of a caller's buffer, so the wrappers
# below check tensor sizes against them before any call reaches the device.
_MAT_DIMS: Dict[int, tuple] = {}
_SESS_DIMS: Dict[int, tuple] = {}


def _need(t, count: int, what: str) -> None:
    """A device tensor (or None) must be float32, contiguous and hold >= count elements."""
    if t is None:
        return
    if str(getattr(t, "dtype", "")) != "torch.float32" or not t.is_contiguous():
        raise ValueError("%s must be a contiguous float32 tensor" % what)
    if t.numel() < count:
        raise ValueError("%s holds %d elements, needs %d" % (what, t.numel(), count))


def _dims(mat):
    if mat not in _MAT_DIMS:
        raise ValueError("unknown matrix handle")
    return _MAT_DIMS[mat]


def _host_shapes(mat, d, g, gm, fi) -> None:
    """Host batch inputs: g (B, m), gamma (B, m) or None, f_init (B, d) or None."""
    m, dm = _dims(mat)
    B = g.shape[0]
    if d != dm or g.size != B * m or (gm is not None and gm.size != B * m) or \
            (fi is not None and fi.size != B * d):
        raise ValueError("batch shapes do not match the matrix (m = %d, d = %d)" % (m, dm))


def appga_load_system_matrix(ctx, n, n_angles, n_bins, row_ptr, col, val, storage="f32") -> int:
    geom = appga_geometry(n, n_angles, n_bins)
    rp, cl, vl = _np(row_ptr, np.int64), _np(col, np.int32), _np(val, np.float64)
    h = C.c_void_p()
    _call("appga_load_system_matrix", ctx, C.byref(geom), len(cl), _ptr(rp), _ptr(cl), _ptr(vl),
          DTYPES.get(storage, storage), C.byref(h))
    _MAT_DIMS[h.value] = (n_angles * n_bins, n * n)
    return h.value


def appga_load_system_matrix_factored(ctx, n, n_angles, n_bins, row_ptr, col, val, storage="f32",
                                      row_factors=None, psf_fwhm_px=0.0) -> int:
    """A = diag(row_factors) G H (G the given CSR, H a Gaussian PSF of psf_fwhm_px pixels)."""
    geom = appga_geometry(n, n_angles, n_bins)
    rp, cl, vl = _np(row_ptr, np.int64), _np(col, np.int32), _np(val, np.float64)
    rf = None if row_factors is None else _np(row_factors, np.float64)
    if rf is not None and rf.size != n_angles * n_bins:
        raise ValueError("row_factors needs one entry per ray")
    h = C.c_void_p()
    _call("appga_load_system_matrix_factored", ctx, C.byref(geom), len(cl), _ptr(rp), _ptr(cl), _ptr(vl),
          DTYPES.get(storage, storage), _ptr(rf), float(psf_fwhm_px), C.byref(h))
    _MAT_DIMS[h.value] = (n_angles * n_bins, n * n)
    return h.value


def appga_matrix_symmetry(mat) -> tuple:
    """(folds, stored bytes of the single-solve operators): folds = 2 when the B = 1
    kernels read a half-stored matrix (quarter-turn symmetry), else 1."""
    f, b = I32(), I64()
    _call("appga_matrix_symmetry", mat, C.byref(f), C.byref(b))
    return f.value, b.value


def appga_matrix_psf(mat) -> tuple:
    """(FWHM in pixels, tap radius R) of a matrix's PSF; (0.0, -1) without one."""
    fw, R = D(), I32()
    _call("appga_matrix_psf", mat, C.byref(fw), C.byref(R))
    return fw.value, R.value


def appga_free_system_matrix(ctx, mat) -> None:
    _call("appga_free_system_matrix", ctx, mat)
    _MAT_DIMS.pop(mat, None)


def appga_matrix_info(mat) -> dict:
    nnz, ba, bt, stg = I64(), I64(), I64(), I32()
    _call("appga_matrix_info", mat, C.byref(nnz), C.byref(ba), C.byref(bt), C.byref(stg))
    return dict(nnz=nnz.value, bytes_a=ba.value, bytes_at=bt.value, storage=stg.value)


class appga_tile_info(C.Structure):
    _fields_ = [("valid", I32), ("tiles", I32), ("split", I32), ("pad0", I32), ("windows", I64),
                ("records", I64), ("entries", I64), ("bytes", I64)]


APPGA_TILES_FORWARD, APPGA_TILES_BACK = 0, 1


def appga_matrix_tiles(mat, which: int) -> dict:
    """Counts of the tile form of `mat` for A x (APPGA_TILES_FORWARD) or A^T e (APPGA_TILES_BACK)."""
    info = appga_tile_info()
    _call("appga_matrix_tiles", mat, which, C.byref(info))
    return {k: getattr(info, k) for k, _ in info._fields_ if k != "pad0"}


def appga_tiles_emulate(A, geom, storage: str, which: int, split: int, x) -> tuple:
    """Host emulation of the tile form of a synth.SparseMatrix: (out, counts)."""
    g = appga_geometry(geom.n, geom.n_angles, geom.n_bins)
    rp = _np(A.row_ptr, np.int64)
    col = _np(A.col, np.int32)
    val = _np(A.val, np.float64)
    xin = _np(x, np.float32)
    n_out = geom.m if which == APPGA_TILES_FORWARD else geom.d
    out = np.zeros(n_out, dtype=np.float32)
    info = appga_tile_info()
    _call("appga_tiles_emulate", C.byref(g), A.nnz, _ptr(rp), _ptr(col), _ptr(val), DTYPES[storage],
          which, split, _ptr(xin), _ptr(out), C.byref(info))
    return out, {k: getattr(info, k) for k, _ in info._fields_ if k != "pad0"}


def appga_matrix_dequantized(mat, nnz: int) -> np.ndarray:
    out = np.empty(nnz, dtype=np.float64)
    _call("appga_matrix_dequantized", mat, _ptr(out))
    return out


# ---------------------------------------------------------------- solvers ---

def appga_reconstruct(ctx, mat, d, g, gamma, params: appga_params, f_init=None):
    """Returns (f_out (d,) float32, stats dict)."""
    g = _np(g, np.float32)
    gm = None if gamma is None else _np(gamma, np.float32)
    fi = None if f_init is None else _np(f_init, np.float32)
    out = np.empty(d, dtype=np.float32)
    st = appga_stats()
    _call("appga_reconstruct", ctx, mat, _ptr(g), _ptr(gm), C.byref(params), _ptr(fi), _ptr(out),
          C.byref(st))
    return out, st.to_dict()


def appga_reconstruct_simple(ctx, mat, d, g, gamma, lam, eps, omega, iterations) -> np.ndarray:
    g = _np(g, np.float32)
    gm = None if gamma is None else _np(gamma, np.float32)
    out = np.empty(d, dtype=np.float32)
    _call("appga_reconstruct_simple", ctx, mat, _ptr(g), _ptr(gm), lam, eps, omega, iterations,
          _ptr(out))
    return out


def _param_array(params: Sequence[appga_params]):
    arr = (appga_params * len(params))()
    for i, p in enumerate(params):
        arr[i] = p
    return arr


def appga_reconstruct_batch(ctx, mat, d, g, gamma, params: Sequence[appga_params], f_init=None):
    """g: (B, m); gamma: (B, m) or None.  Returns (f (B, d) float32, [stats dicts])."""
    g = _np(g, np.float32)
    B = g.shape[0]
    gm = None if gamma is None else _np(gamma, np.float32)
    fi = None if f_init is None else _np(f_init, np.float32)
    _host_shapes(mat, d, g, gm, fi)
    out = np.empty((B, d), dtype=np.float32)
    stats = (appga_stats * B)()
    _call("appga_reconstruct_batch", ctx, mat, B, _ptr(g), _ptr(gm), _param_array(params), _ptr(fi),
          _ptr(out), stats)
    return out, [s.to_dict() for s in stats]


def appga_reconstruct_batch_device(ctx, mat, g_t, gamma_t, params: Sequence[appga_params],
                                   f_init_t, out_t, stream=None) -> None:
    """torch tensors on the device, solve-major (B, m) / (B, d)."""
    B = len(params)
    m, d = _dims(mat)
    _need(g_t, B * m, "g"), _need(gamma_t, B * m, "gamma"), _need(f_init_t, B * d, "f_init")
    _need(out_t, B * d, "out")
    _call("appga_reconstruct_batch_device", ctx, mat, B, _ptr(g_t), _ptr(gamma_t),
          _param_array(params), _ptr(f_init_t), _ptr(out_t), _stream(stream))


def appga_afppa_batch(ctx, mat, d, g, gamma, params: Sequence[appga_params], f_init=None,
                      duals=False):
    """AFPPA on the nonsmooth model.  g: (B, m); gamma: (B, m) or None.  Returns
    (f (B, d), duals (B, 6 d) or None, [stats dicts])."""
    g = _np(g, np.float32)
    B = g.shape[0]
    gm = None if gamma is None else _np(gamma, np.float32)
    fi = None if f_init is None else _np(f_init, np.float32)
    _host_shapes(mat, d, g, gm, fi)
    out = np.empty((B, d), dtype=np.float32)
    du = np.empty((B, 6 * d), dtype=np.float32) if duals else None
    stats = (appga_stats * B)()
    _call("appga_afppa_batch", ctx, mat, B, _ptr(g), _ptr(gm), _param_array(params), _ptr(fi),
          _ptr(out), _ptr(du), stats)
    return out, du, [s.to_dict() for s in stats]


def appga_afppa_batch_device(ctx, mat, g_t, gamma_t, params: Sequence[appga_params], f_init_t,
                             out_t, duals_t=None, stream=None) -> None:
    B = len(params)
    m, d = _dims(mat)
    _need(g_t, B * m, "g"), _need(gamma_t, B * m, "gamma"), _need(f_init_t, B * d, "f_init")
    _need(out_t, B * d, "out"), _need(duals_t, B * 6 * d, "duals")
    _call("appga_afppa_batch_device", ctx, mat, B, _ptr(g_t), _ptr(gamma_t), _param_array(params),
          _ptr(f_init_t), _ptr(out_t), _ptr(duals_t), _stream(stream))


def appga_afppa_begin(ctx, mat, g_t, gamma_t, params: Sequence[appga_params], f_init_t=None,
                      stream=None) -> int:
    B = len(params)
    m, d = _dims(mat)
    _need(g_t, B * m, "g"), _need(gamma_t, B * m, "gamma"), _need(f_init_t, B * d, "f_init")
    h = C.c_void_p()
    _call("appga_afppa_begin", ctx, mat, B, _ptr(g_t), _ptr(gamma_t),
          _param_array(params), _ptr(f_init_t), _stream(stream), C.byref(h))
    _SESS_DIMS[h.value] = (B, m, d)
    return h.value


def appga_solve_duals(sess, duals_t) -> None:
    if sess in _SESS_DIMS:
        B, _, d = _SESS_DIMS[sess]
        _need(duals_t, B * 6 * d, "duals")
    _call("appga_solve_duals", sess, _ptr(duals_t))


def appga_solve_image(sess, out_t) -> None:
    """The session's current image f^k into out_t (B, d)."""
    if sess in _SESS_DIMS:
        B, _, d = _SESS_DIMS[sess]
        _need(out_t, B * d, "out")
    _call("appga_solve_image", sess, _ptr(out_t))


def appga_solve_begin(ctx, mat, g_t, gamma_t, params: Sequence[appga_params], f_init_t=None,
                      stream=None) -> int:
    B = len(params)
    m, d = _dims(mat)
    _need(g_t, B * m, "g"), _need(gamma_t, B * m, "gamma"), _need(f_init_t, B * d, "f_init")
    h = C.c_void_p()
    _call("appga_solve_begin", ctx, mat, B, _ptr(g_t), _ptr(gamma_t),
          _param_array(params), _ptr(f_init_t), _stream(stream), C.byref(h))
    _SESS_DIMS[h.value] = (B, m, d)
    return h.value


def appga_solve_step(sess, n_iters: int) -> None:
    _call("appga_solve_step", sess, n_iters)


def appga_solve_history(sess, solve: int):
    """(iterations k, Phi(f^k)) of one solve of a session with monitor_every > 0."""
    n = I32()
    _call("appga_solve_history", sess, solve, 0, None, None, C.byref(n))
    ks = np.empty(n.value, dtype=np.int32)
    obj = np.empty(n.value, dtype=np.float64)
    _call("appga_solve_history", sess, solve, n.value, _ptr(ks), _ptr(obj), C.byref(n))
    return ks, obj


def appga_solve_end(sess, out_t, B: int) -> List[dict]:
    if sess in _SESS_DIMS:
        Bs, _, d = _SESS_DIMS[sess]
        if B != Bs:
            raise ValueError("session has %d solves, not %d" % (Bs, B))
        _need(out_t, B * d, "out")
    stats = (appga_stats * B)()
    _call("appga_solve_end", sess, _ptr(out_t), stats)
    _SESS_DIMS.pop(sess, None)
    return [s.to_dict() for s in stats]


# -------------------------------------------------------------- operators ---

def appga_op_forward(ctx, mat, x_t, gamma_t, y_t, stream=None) -> None:
    _call("appga_op_forward", ctx, mat, x_t.shape[0] if x_t.dim() == 2 else 1, _ptr(x_t),
          _ptr(gamma_t), _ptr(y_t), _stream(stream))


def appga_op_ratio(ctx, mat, x_t, g_t, gamma_t, e_t, stream=None) -> None:
    _call("appga_op_ratio", ctx, mat, x_t.shape[0] if x_t.dim() == 2 else 1, _ptr(x_t), _ptr(g_t),
          _ptr(gamma_t), _ptr(e_t), _stream(stream))


def appga_op_back(ctx, mat, r_t, out_t, stream=None) -> None:
    _call("appga_op_back", ctx, mat, r_t.shape[0] if r_t.dim() == 2 else 1, _ptr(r_t), _ptr(out_t),
          _stream(stream))


def _dbl(vals) -> np.ndarray:
    return _np(vals, np.float64)


def appga_op_grad_reg(ctx, n, lambda1, lambda2, eps, x_t, out_t, stream=None) -> None:
    B = x_t.shape[0] if x_t.dim() == 2 else 1
    l1, l2, ep = _dbl(np.broadcast_to(lambda1, B)), _dbl(np.broadcast_to(lambda2, B)), \
        _dbl(np.broadcast_to(eps, B))
    _call("appga_op_grad_reg", ctx, n, B, _ptr(l1), _ptr(l2), _ptr(ep), _ptr(x_t), _ptr(out_t),
          _stream(stream))


def appga_op_step(ctx, mat, g_t, gamma_t, lambda1, lambda2, eps, beta, theta_next, f_t, ft_t,
                  ft_next_t, stream=None) -> None:
    B = f_t.shape[0] if f_t.dim() == 2 else 1
    arrs = [_dbl(np.broadcast_to(v, B)) for v in (lambda1, lambda2, eps, beta, theta_next)]
    _call("appga_op_step", ctx, mat, B, _ptr(g_t), _ptr(gamma_t), *[_ptr(a) for a in arrs],
          _ptr(f_t), _ptr(ft_t), _ptr(ft_next_t), _stream(stream))


# ----------------------------------------------------------------- timing ---

def appga_set_kernel_timing(ctx, enable: bool) -> None:
    _call("appga_set_kernel_timing", ctx, 1 if enable else 0)


def appga_kernel_times(ctx) -> Dict[str, dict]:
    cap = 64
    names = C.create_string_buffer(cap * 64)
    counts = np.zeros(cap, dtype=np.int64)
    ms = np.zeros(cap, dtype=np.float64)
    nk = I32()
    _call("appga_kernel_times", ctx, cap, names, len(names), _ptr(counts), _ptr(ms), C.byref(nk))
    raw = names.raw.split(b"\0")
    return {raw[i].decode(): dict(count=int(counts[i]), total_ms=float(ms[i]))
            for i in range(min(nk.value, cap))}


# ---------------------------------------------------------------- serving ---

class appga_tuning(C.Structure):
    _fields_ = [("group_fwd", I32), ("group_back", I32), ("fwd_wgs", I32), ("xcd_remap", I32),
                ("us_fwd_single", D), ("us_back_single", D), ("us_fwd_batch", D),
                ("us_step_batch", D)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


APPGA_TUNE_SINGLE, APPGA_TUNE_BATCH = 1, 2


def appga_tune(ctx, mat, flags: int = APPGA_TUNE_SINGLE | APPGA_TUNE_BATCH) -> dict:
    t = appga_tuning()
    _call("appga_tune", ctx, mat, flags, C.byref(t))
    return t.to_dict()


def appga_server_footprint(mat) -> int:
    b = I64()
    _call("appga_server_footprint", mat, C.byref(b))
    return b.value


def appga_server_start(ctx, hbm_budget_bytes: int, slots_per_matrix: int) -> int:
    cfg = appga_server_cfg(hbm_budget_bytes, slots_per_matrix, 0)
    h = C.c_void_p()
    _call("appga_server_start", ctx, C.byref(cfg), C.byref(h))
    return h.value


def appga_submit(srv, mat, g, gamma, params: appga_params) -> int:
    g = _np(g, np.float32)
    gm = None if gamma is None else _np(gamma, np.float32)
    t = U64()
    _call("appga_submit", srv, mat, _ptr(g), _ptr(gm), C.byref(params), C.byref(t))
    return t.value


def appga_wait(srv, ticket: int, d: int, timeout_ms: int = -1):
    out = np.empty(d, dtype=np.float32)
    st = appga_stats()
    _call("appga_wait", srv, ticket, _ptr(out), C.byref(st), timeout_ms)
    return out, st.to_dict()


def appga_server_stop(srv) -> None:
    _call("appga_server_stop", srv)


# -------------------------------------------------------------- utilities ---

def load_matrix(ctx, A, geom, storage="f32") -> int:
    """Uploads a synth.SparseMatrix with its geometry."""
    return appga_load_system_matrix(ctx, geom.n, geom.n_angles, geom.n_bins, A.row_ptr, A.col,
                                    A.val, storage)
