"""ctypes front end of the FP64 C oracle (``appga_oracle.c``).

Test infrastructure only (see the package docstring).  Every function takes
numpy arrays and converts them to float64 / int64 / int32 C arrays; each one
forwards to the C routine of the same name, which cites the passage of the
paper it follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

__all__ = [
    "build_oracle", "load", "forward", "back", "b1", "b2", "b1t", "b2t", "s_eps", "reg_value",
    "grad_reg", "grad_fidelity", "objective", "em_lambda", "init_image", "theta", "appga",
    "t_nesterov", "theta_nesterov", "hoitv_value", "objective_hoitv", "afppa",
    "MOMENTUM_GN", "MOMENTUM_NONE", "MOMENTUM_NESTEROV", "psf_radius", "psf_taps", "psf_apply",
    "attenuation", "factored_matrix", "PRECOND_EM", "PRECOND_EM_FROZEN", "PRECOND_FIXED",
]

MOMENTUM_GN, MOMENTUM_NONE, MOMENTUM_NESTEROV = 0, 1, 2
PRECOND_EM, PRECOND_EM_FROZEN, PRECOND_FIXED = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "appga_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# A prebuilt copy may be substituted (the mutation tests load planted-mistake builds).
_LIB_OVERRIDE = os.environ.get("APPGA_ORACLE_LIB")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (no fast-math, strict IEEE double)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = C.CDLL(_LIB_OVERRIDE)
            _declare(_lib)
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = C.c_void_p
I64, I32, D = C.c_int64, C.c_int, C.c_double


def _declare(lib):
    sig = {
        "orc_forward": (None, [I64, P, P, P, P, P]),
        "orc_back": (None, [I64, I64, P, P, P, P, P]),
        "orc_b1": (I32, [I32, P, P]),
        "orc_b2": (I32, [I32, P, P]),
        "orc_b1t": (I32, [I32, P, P]),
        "orc_b2t": (I32, [I32, P, P]),
        "orc_s_eps": (D, [P, I32, D]),
        "orc_reg_value": (I32, [I32, D, D, D, P, P]),
        "orc_grad_reg": (I32, [I32, D, D, D, P, P]),
        "orc_ratio": (None, [I64, P, P, P, P, P]),
        "orc_grad_fidelity": (I32, [I64, I64, P, P, P, P, P, P, P, P]),
        "orc_objective": (I32, [I32, I64, P, P, P, P, P, D, D, D, P, P]),
        "orc_em_lambda": (I32, [I64, I64, P, P, P, P]),
        "orc_init_image": (I32, [I32, I64, I32, P, P, P]),
        "orc_theta": (D, [I32, D, D, D]),
        "orc_appga": (I32, [I32, I64, P, P, P, I32, P, P, D, D, D, D, D, D, D, I32, I32, I32, I32,
                            P, D, P, P, P, P, P, P, I32]),
        "orc_t_nesterov": (D, [I32]),
        "orc_theta_nesterov": (D, [I32]),
        "orc_hoitv_value": (I32, [I32, D, D, P, P]),
        "orc_objective_hoitv": (I32, [I32, I64, P, P, P, P, P, D, D, P, P]),
        "orc_afppa": (I32, [I32, I64, P, P, P, I32, P, P, D, D, D, D, D, D, I32, I32, I32, D, P, P, P, P,
                            P, P, P, P, I32]),
        "orc_psf_taps": (I32, [D, I32, P]),
        "orc_psf_apply": (I32, [I32, I32, P, P, P]),
        "orc_attenuation": (I32, [I64, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args


def _f64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _csr(A):
    rp = np.ascontiguousarray(A.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(A.col, dtype=np.int32)
    val = _f64(A.val)
    return rp, col, val


def _check(st: int, name: str):
    if st != 0:
        raise RuntimeError("oracle %s failed with status %d" % (name, st))


def forward(A, x) -> np.ndarray:
    """y = A x."""
    rp, col, val = _csr(A)
    x = _f64(x)
    y = np.empty(A.n_rows, dtype=np.float64)
    load().orc_forward(A.n_rows, _ptr(rp), _ptr(col), _ptr(val), _ptr(x), _ptr(y))
    return y


def back(A, r) -> np.ndarray:
    """A^T r (by scattering rows; no stored transpose)."""
    rp, col, val = _csr(A)
    r = _f64(r)
    out = np.empty(A.n_cols, dtype=np.float64)
    load().orc_back(A.n_rows, A.n_cols, _ptr(rp), _ptr(col), _ptr(val), _ptr(r), _ptr(out))
    return out


def _img_op(name: str, n: int, x, out_len: int) -> np.ndarray:
    x = _f64(x)
    out = np.empty(out_len, dtype=np.float64)
    _check(getattr(load(), name)(n, _ptr(x), _ptr(out)), name)
    return out


def b1(n, f):
    return _img_op("orc_b1", n, f, 2 * n * n)


def b2(n, f):
    return _img_op("orc_b2", n, f, 4 * n * n)


def b1t(n, p):
    return _img_op("orc_b1t", n, p, n * n)


def b2t(n, q):
    return _img_op("orc_b2t", n, q, n * n)


def s_eps(x, eps) -> float:
    x = _f64(x)
    return float(load().orc_s_eps(_ptr(x), len(x), eps))


def reg_value(n, lam1, lam2, eps, f) -> float:
    f = _f64(f)
    out = np.zeros(1)
    _check(load().orc_reg_value(n, lam1, lam2, eps, _ptr(f), _ptr(out)), "reg_value")
    return float(out[0])


def grad_reg(n, lam1, lam2, eps, f) -> np.ndarray:
    f = _f64(f)
    out = np.empty(n * n)
    _check(load().orc_grad_reg(n, lam1, lam2, eps, _ptr(f), _ptr(out)), "grad_reg")
    return out


def grad_fidelity(A, g, gamma, x):
    """(grad F(x), number of floored bins)."""
    rp, col, val = _csr(A)
    g, gamma, x = _f64(g), _f64(gamma), _f64(x)
    out = np.empty(A.n_cols)
    cl = np.zeros(1, dtype=np.int64)
    _check(load().orc_grad_fidelity(A.n_rows, A.n_cols, _ptr(rp), _ptr(col), _ptr(val), _ptr(g),
                                    _ptr(gamma), _ptr(x), _ptr(out), _ptr(cl)), "grad_fidelity")
    return out, int(cl[0])


def objective(A, n, g, gamma, lam1, lam2, eps, x) -> float:
    rp, col, val = _csr(A)
    g, gamma, x = _f64(g), _f64(gamma), _f64(x)
    out = np.zeros(1)
    _check(load().orc_objective(n, A.n_rows, _ptr(rp), _ptr(col), _ptr(val), _ptr(g), _ptr(gamma),
                                lam1, lam2, eps, _ptr(x), _ptr(out)), "objective")
    return float(out[0])


def em_lambda(A) -> np.ndarray:
    rp, col, val = _csr(A)
    out = np.empty(A.n_cols)
    _check(load().orc_em_lambda(A.n_rows, A.n_cols, _ptr(rp), _ptr(col), _ptr(val), _ptr(out)),
           "em_lambda")
    return out


def init_image(n, n_angles, g, gamma) -> np.ndarray:
    g, gamma = _f64(g), _f64(gamma)
    out = np.empty(n * n)
    _check(load().orc_init_image(n, len(g), n_angles, _ptr(g), _ptr(gamma), _ptr(out)),
           "init_image")
    return out


def theta(k, a=0.125, b=1.0, omega=1.0) -> float:
    return float(load().orc_theta(k, a, b, omega))


def appga(A, n, n_angles, g, gamma, lam1, lam2, eps, omega, iterations, a=0.125, b=1.0, beta=1.0,
          momentum=MOMENTUM_GN, precond=PRECOND_EM, precond_freeze_iter=0, fixed_p=None,
          fixed_p_scalar=0.0, f_init=None, history=False, iterates=False, round_f32=False):
    """Run APPGA in FP64.

    Returns dict(f=f^{K+1}, obj=[Phi(f^1..f^{K+1})] or None, re=[RE(2..K+1)] or None,
    iterates=(K+1, d) array f^1..f^{K+1} or None, clamps=number of floored bins).
    round_f32 is a diagnostic (not the method): f~, A f~, e, grad F, grad R and f are
    rounded to FP32 every iteration, to measure how much a problem amplifies
    FP32-size perturbations (its sensitivity floor).
    """
    rp, col, val = _csr(A)
    g, gamma = _f64(g), _f64(gamma)
    f_out = np.empty(n * n)
    fi = None if f_init is None else _f64(f_init)
    fp = None if fixed_p is None else _f64(fixed_p)
    obj = np.empty(iterations + 1) if history else None
    re = np.empty(iterations) if history else None
    fh = np.empty((iterations + 1, n * n)) if iterates else None
    cl = np.zeros(1, dtype=np.int64)
    st = load().orc_appga(n, A.n_rows, _ptr(rp), _ptr(col), _ptr(val), n_angles, _ptr(g),
                          _ptr(gamma), lam1, lam2, eps, omega, a, b, beta, iterations, momentum,
                          precond, precond_freeze_iter, _ptr(fp), fixed_p_scalar, _ptr(fi),
                          _ptr(f_out), _ptr(obj), _ptr(re), _ptr(fh), _ptr(cl), int(bool(round_f32)))
    _check(st, "appga")
    return dict(f=f_out, obj=obj, re=re, iterates=fh, clamps=int(cl[0]))


def t_nesterov(k: int) -> float:
    """Nesterov's sequence t_k (t_0 = 1), Section 4.3."""
    return load().orc_t_nesterov(k)


def theta_nesterov(k: int) -> float:
    return load().orc_theta_nesterov(k)


def hoitv_value(n, lam1, lam2, f) -> float:
    """lambda1 sum ||(B1 f)_i|| + lambda2 sum ||(B2 f)_i|| (model HOTV)."""
    out = np.zeros(1)
    _check(load().orc_hoitv_value(n, lam1, lam2, _ptr(_f64(f)), _ptr(out)), "hoitv_value")
    return float(out[0])


def objective_hoitv(A, n, g, gamma, lam1, lam2, f) -> float:
    rp, col, val = _csr(A)
    out = np.zeros(1)
    _check(load().orc_objective_hoitv(n, A.n_rows, _ptr(rp), _ptr(col), _ptr(val), _ptr(_f64(g)),
                                      _ptr(_f64(gamma)), lam1, lam2, _ptr(_f64(f)), _ptr(out)),
           "objective_hoitv")
    return float(out[0])


def afppa(A, n, n_angles, g, gamma, lam1, lam2, omega, iterations, a=0.125, b=1.0, beta=1.0,
          momentum=MOMENTUM_GN, precond=PRECOND_EM, fixed_p_scalar=0.0, f_init=None, history=False,
          duals=False, round_f32=False):
    """Run AFPPA (FPPA with momentum NONE, AFPPA-N with NESTEROV) in FP64 on the nonsmooth HOITV model.

    Returns dict(f=f^{K+1}, b, c (duals when asked), obj=[Phi_HOITV(f^1..f^{K+1})] or None,
    re=[RE(2..K+1)] or None, rho=(K, 2) array of (rho1, rho2) or None, clamps).
    """
    rp, col, val = _csr(A)
    g, gamma = _f64(g), _f64(gamma)
    d = n * n
    f_out = np.empty(d)
    b_out = np.empty(2 * d) if duals else None
    c_out = np.empty(4 * d) if duals else None
    obj = np.empty(iterations + 1) if history else None
    re = np.empty(iterations) if history else None
    rho = np.empty(2 * iterations) if history else None
    fi = None if f_init is None else _f64(f_init)
    cl = np.zeros(1, dtype=np.int64)
    st = load().orc_afppa(n, A.n_rows, _ptr(rp), _ptr(col), _ptr(val), n_angles, _ptr(g), _ptr(gamma),
                          lam1, lam2, omega, a, b, beta, iterations, momentum, precond, fixed_p_scalar,
                          _ptr(fi), _ptr(f_out), _ptr(b_out), _ptr(c_out), _ptr(obj), _ptr(re), _ptr(rho),
                          _ptr(cl), int(bool(round_f32)))
    _check(st, "afppa")
    return dict(f=f_out, b=b_out, c=c_out, obj=obj, re=re,
                rho=None if rho is None else rho.reshape(iterations, 2), clamps=int(cl[0]))


# ------------------------------------------------------------- factored model ---

def psf_radius(fwhm: float) -> int:
    """Half-width R of the truncated Gaussian PSF: ceil(3 sigma), sigma = FWHM / (2 sqrt(2 ln 2))."""
    import math
    return int(math.ceil(3.0 * fwhm / (2.0 * math.sqrt(2.0 * math.log(2.0)))))


def psf_taps(fwhm: float, R: Optional[int] = None) -> np.ndarray:
    """The 2R + 1 normalised Gaussian taps (Section 4.1's space-invariant PSF)."""
    R = psf_radius(fwhm) if R is None else R
    w = np.empty(2 * R + 1)
    _check(load().orc_psf_taps(fwhm, R, _ptr(w)), "psf_taps")
    return w


def psf_apply(n: int, fwhm: float, x, R: Optional[int] = None) -> np.ndarray:
    """H x: the 2-D Gaussian blur of the n x n image x (zero outside the image)."""
    w = psf_taps(fwhm, R)
    x = _f64(x)
    out = np.empty(n * n)
    _check(load().orc_psf_apply(n, (len(w) - 1) // 2, _ptr(w), _ptr(x), _ptr(out)), "psf_apply")
    return out


def attenuation(A, mu) -> np.ndarray:
    """Per-ray attenuation factors exp(-(A mu)_i)."""
    rp, col, val = _csr(A)
    mu = _f64(mu)
    out = np.empty(A.n_rows)
    _check(load().orc_attenuation(A.n_rows, _ptr(rp), _ptr(col), _ptr(val), _ptr(mu), _ptr(out)),
           "attenuation")
    return out


def factored_matrix(G, n: int, fwhm: float, factors=None):
    """The explicit A = diag(factors) G H (a SparseMatrix) for small images: H is formed
    column by column with psf_apply on unit vectors, then multiplied out with scipy."""
    import scipy.sparse as sp
    d = n * n
    cols = []
    for j in range(d):
        e = np.zeros(d)
        e[j] = 1.0
        cols.append(sp.csc_matrix(psf_apply(n, fwhm, e).reshape(d, 1)))
    H = sp.hstack(cols).tocsr()
    Gs = sp.csr_matrix((G.val, G.col, G.row_ptr), shape=(G.n_rows, G.n_cols))
    if factors is not None:
        Gs = sp.diags(_f64(factors)) @ Gs
    A = (Gs @ H).tocsr()
    A.eliminate_zeros()
    A.sort_indices()
    return type(G)(A.shape[0], A.shape[1], A.indptr.astype(np.int64), A.indices.astype(np.int32),
                   A.data.astype(np.float64))
