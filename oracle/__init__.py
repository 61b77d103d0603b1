"""CPU oracle for the randomized PNE/HPNE least-squares path -- TEST INFRASTRUCTURE.

Plain FP64 C (``pne_oracle.c``) wrapped with ctypes.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package; the GPU library never does, and the two share no code.

All matrices cross this boundary as numpy float64 arrays in column-major
(Fortran) order.  Precision codes: 0 AUTO, 1 FP64, 2 FP32, 3 FP16, 4 BF16,
5 FP8 (OCP e4m3).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pne_oracle.c")
_LIB = os.path.join(_HERE, "libpne_oracle.so")

PREC = {"auto": 0, "fp64": 1, "fp32": 2, "fp16": 3, "bf16": 4, "fp8": 5}

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no threads)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fno-fast-math",
                               "-ffp-contract=off", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        i64, u64, u32, i32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        P = ctypes.c_void_p
        sig = {
            "oracle_philox4x32_10": (None, [P, P, P]),
            "oracle_omega_entry": (ctypes.c_double, [u64, u32, i64, i64]),
            "oracle_omega": (None, [u64, u32, i64, i64, P]),
            "oracle_round_fp32": (ctypes.c_double, [ctypes.c_double]),
            "oracle_round_bf16": (ctypes.c_double, [ctypes.c_double]),
            "oracle_round_fp16": (ctypes.c_double, [ctypes.c_double]),
            "oracle_round_e4m3": (ctypes.c_double, [ctypes.c_double]),
            "oracle_sketch": (i32, [i64, i64, P, i64, i64, u64, u32, i32, i64, P, i64, P]),
            "oracle_householder_r": (i32, [i64, i64, P, i64, P, i64]),
            "oracle_qr_ls": (i32, [i64, i64, P, i64, P, P]),
            "oracle_precondition": (i32, [i64, i64, P, i64, P, i64, P, i64]),
            "oracle_gram": (None, [i64, i64, P, i64, P, i64, P, P, i64, P]),
            "oracle_cholesky": (i32, [i64, P, i64]),
            "oracle_lu": (i32, [i64, P, i64, P]),
            "oracle_cholesky_solve": (i32, [i64, P, i64, P, P]),
            "oracle_lu_solve": (i32, [i64, P, i64, P, P, P]),
            "oracle_upper_solve": (i32, [i64, P, i64, P, P]),
            "oracle_cond_est": (i32, [i64, i64, P, i64, ctypes.c_double, P, P, P]),
            "oracle_sketch_entries": (i32, [i64, P, i64, i64, u64, u32, i32, i64, i64, P, P, P, P]),
            "oracle_fp16_qr_scale": (ctypes.c_double, [i64, i64, P, i64]),
            "oracle_solve": (i32, [i32, i64, i64, P, i64, P, i64, u64, u32, i32, i32, i64, i32,
                                   ctypes.c_double, i32, P, P, P, P]),
            "oracle_next_smooth": (i64, [i64]),
            "oracle_srft_sign": (i32, [u64, u32, i64]),
            "oracle_srft_index": (i64, [u64, u32, i64, i64]),
            "oracle_srft_sketch": (i32, [i64, i64, P, i64, i64, u64, u32, i32, P, i64]),
            "oracle_srft_entries": (i32, [i64, P, i64, i64, u64, u32, i32, i64, P, P, P]),
            "oracle_nne": (i32, [i64, i64, P, i64, P, i64, P, i32, P]),
            "oracle_cond_est_qr": (i32, [i64, i64, P, i64, i64, u64, u32, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _f64(a) -> np.ndarray:
    return np.asfortranarray(np.asarray(a, dtype=np.float64))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def omega(seed: int, s: int, m: int, pid: int = 0) -> np.ndarray:
    """The unscaled s x m Gaussian sketch (N(0,1) entries)."""
    out = np.zeros((s, m), dtype=np.float64, order="F")
    lib().oracle_omega(seed, pid, s, m, _ptr(out))
    return out


def round_to(x, prec: str) -> np.ndarray:
    f = {"fp32": lib().oracle_round_fp32, "bf16": lib().oracle_round_bf16,
         "fp16": lib().oracle_round_fp16, "fp8": lib().oracle_round_e4m3}[prec]
    x = np.asarray(x, dtype=np.float64)
    return np.array([f(float(v)) for v in x.ravel()]).reshape(x.shape)


def sketch(A, s: int, seed: int, prec: str = "fp64", pid: int = 0, block_rows: int = 128,
           want_abs: bool = False):
    A = _f64(A)
    m, n = A.shape
    As = np.zeros((s, n), order="F")
    Aabs = np.zeros((s, n), order="F") if want_abs else None
    rc = lib().oracle_sketch(m, n, _ptr(A), m, s, seed, pid, PREC[prec], block_rows, _ptr(As), s,
                             _ptr(Aabs) if want_abs else None)
    if rc:
        raise ValueError(f"oracle_sketch failed: {rc}")
    return (As, Aabs) if want_abs else As


def sketch_entries(A, s: int, seed: int, rows, cols, prec: str = "fp64", pid: int = 0,
                   block_rows: int = 128):
    """Entries (rows[t], cols[t]) of the sketch and of its absolute product."""
    A = _f64(A)
    m = A.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(rows.size)
    out_abs = np.zeros(rows.size)
    rc = lib().oracle_sketch_entries(m, _ptr(A), m, s, seed, pid, PREC[prec], block_rows, rows.size,
                                     _ptr(rows), _ptr(cols), _ptr(out), _ptr(out_abs))
    if rc:
        raise ValueError(f"oracle_sketch_entries failed: {rc}")
    return out, out_abs


def fp16_qr_scale(As) -> float:
    """Power-of-two factor applied to a sketch before its FP16 QR."""
    As = _f64(As)
    s, n = As.shape
    return float(lib().oracle_fp16_qr_scale(s, n, _ptr(As), s))


def householder_r(W) -> np.ndarray:
    W = _f64(W).copy(order="F")
    s, n = W.shape
    R = np.zeros((n, n), order="F")
    rc = lib().oracle_householder_r(s, n, _ptr(W), s, _ptr(R), n)
    if rc:
        raise ValueError(f"oracle_householder_r failed: {rc}")
    return R


def qr_ls(A, b) -> np.ndarray:
    A = _f64(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    m, n = A.shape
    x = np.zeros(n)
    rc = lib().oracle_qr_ls(m, n, _ptr(A), m, _ptr(b), _ptr(x))
    if rc:
        raise ValueError(f"oracle_qr_ls failed: {rc}")
    return x


def precondition(A, R):
    A = _f64(A)
    R = _f64(R)
    m, n = A.shape
    Ap = np.zeros((m, n), order="F")
    rc = lib().oracle_precondition(m, n, _ptr(A), m, _ptr(R), n, _ptr(Ap), m)
    return Ap, rc


def gram(X, Y, b=None):
    X, Y = _f64(X), _f64(Y)
    m, n = X.shape
    C = np.zeros((n, n), order="F")
    c = np.zeros(n)
    bb = None if b is None else np.ascontiguousarray(b, dtype=np.float64)
    lib().oracle_gram(m, n, _ptr(X), m, _ptr(Y), m, _ptr(bb) if bb is not None else None,
                      _ptr(C), n, _ptr(c) if bb is not None else None)
    return (C, c) if b is not None else C


def cholesky(C):
    L = _f64(C).copy(order="F")
    n = L.shape[0]
    info = lib().oracle_cholesky(n, _ptr(L), n)
    return L, info


def lu(C):
    LU = _f64(C).copy(order="F")
    n = LU.shape[0]
    piv = np.zeros(n, dtype=np.int32)
    info = lib().oracle_lu(n, _ptr(LU), n, _ptr(piv))
    return LU, piv, info


def cholesky_solve(L, c):
    L = _f64(L)
    c = np.ascontiguousarray(c, dtype=np.float64)
    y = np.zeros_like(c)
    lib().oracle_cholesky_solve(L.shape[0], _ptr(L), L.shape[0], _ptr(c), _ptr(y))
    return y


def lu_solve(LU, piv, c):
    LU = _f64(LU)
    c = np.ascontiguousarray(c, dtype=np.float64)
    piv = np.ascontiguousarray(piv, dtype=np.int32)
    x = np.zeros_like(c)
    lib().oracle_lu_solve(LU.shape[0], _ptr(LU), LU.shape[0], _ptr(piv), _ptr(c), _ptr(x))
    return x


def upper_solve(R, y):
    R = _f64(R)
    y = np.ascontiguousarray(y, dtype=np.float64)
    x = np.zeros_like(y)
    info = lib().oracle_upper_solve(R.shape[0], _ptr(R), R.shape[0], _ptr(y), _ptr(x))
    return x, info


def cond_est(A, known_kappa: float = 0.0):
    """Returns (kappa0, kappa0_with_factor_n, precision code)."""
    A = _f64(A)
    m, n = A.shape
    k0 = ctypes.c_float()
    k0n = ctypes.c_float()
    ch = ctypes.c_int32()
    lib().oracle_cond_est(m, n, _ptr(A), m, known_kappa, ctypes.byref(k0), ctypes.byref(k0n),
                          ctypes.byref(ch))
    return float(k0.value), float(k0n.value), int(ch.value)


SKETCH_KIND = {"gaussian": 0, "srft": 1}


def solve(A, b, *, hpne: bool = False, s: int | None = None, seed: int = 0, pid: int = 0,
          sketch_prec: str = "fp64", qr_prec: str | None = None, block_rows: int = 128,
          refine_steps: int = 0, known_kappa: float = 0.0, sketch_kind: str = "gaussian"):
    """Algorithm 1 (PNE or HPNE).  Returns dict(x, R, info, prec_used, kappa0)."""
    A = _f64(A)
    b = np.ascontiguousarray(b, dtype=np.float64)
    m, n = A.shape
    s = 3 * n if s is None else s
    qr_prec = sketch_prec if qr_prec is None else qr_prec
    x = np.zeros(n)
    R = np.zeros((n, n), order="F")
    used = np.zeros(2, dtype=np.int32)
    k0 = ctypes.c_float()
    info = lib().oracle_solve(int(hpne), m, n, _ptr(A), m, _ptr(b), s, seed, pid, PREC[sketch_prec],
                              PREC[qr_prec], block_rows, refine_steps, known_kappa, SKETCH_KIND[sketch_kind],
                              _ptr(x), _ptr(R),
                              _ptr(used), ctypes.byref(k0))
    return {"x": x, "R": R, "info": int(info), "prec_used": (int(used[0]), int(used[1])),
            "kappa0": float(k0.value)}


def nne(A, B, b, refine_steps: int = 0):
    """Not-normal equations B^T A x = B^T b (Section 5.2).  Returns (x, info)."""
    A, B = _f64(A), _f64(B)
    b = np.ascontiguousarray(b, dtype=np.float64)
    m, n = A.shape
    if B.shape != (m, n):
        raise ValueError("B must have the shape of A")
    x = np.zeros(n)
    info = lib().oracle_nne(m, n, _ptr(A), m, _ptr(B), m, _ptr(b), refine_steps, _ptr(x))
    return x, int(info)


def cond_est_qr(A, s: int | None = None, seed: int = 0, pid: int = 0):
    """Condition estimate from the FP32 QR of the FP32 sketch.  Returns
    (kappa0, precision code)."""
    A = _f64(A)
    m, n = A.shape
    s = 3 * n if s is None else s
    k0 = ctypes.c_float()
    ch = ctypes.c_int32()
    rc = lib().oracle_cond_est_qr(m, n, _ptr(A), m, s, seed, pid, ctypes.byref(k0), ctypes.byref(ch))
    if rc:
        raise ValueError(f"oracle_cond_est_qr failed: {rc}")
    return float(k0.value), int(ch.value)


def next_smooth(m: int) -> int:
    """Smallest 7-smooth integer >= m (the padded length of the SRFT)."""
    return int(lib().oracle_next_smooth(m))


def srft_signs(seed: int, m: int, pid: int = 0) -> np.ndarray:
    return np.array([lib().oracle_srft_sign(seed, pid, j) for j in range(m)], dtype=np.float64)


def srft_indices(seed: int, s: int, mp: int, pid: int = 0) -> np.ndarray:
    return np.array([lib().oracle_srft_index(seed, pid, i, mp) for i in range(s)], dtype=np.int64)


def srft_sketch(A, s: int, seed: int, prec: str = "fp64", pid: int = 0) -> np.ndarray:
    """A_s = (1/sqrt(s)) S H D A with the Hartley transform (Section 6.2)."""
    A = _f64(A)
    m, n = A.shape
    As = np.zeros((s, n), order="F")
    rc = lib().oracle_srft_sketch(m, n, _ptr(A), m, s, seed, pid, PREC[prec], _ptr(As), s)
    if rc:
        raise ValueError(f"oracle_srft_sketch failed: {rc}")
    return As


def srft_entries(A, s: int, seed: int, rows, cols, prec: str = "fp64", pid: int = 0) -> np.ndarray:
    """Entries (rows[t], cols[t]) of the SRFT sketch, one by one."""
    A = _f64(A)
    m = A.shape[0]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(rows.size)
    rc = lib().oracle_srft_entries(m, _ptr(A), m, s, seed, pid, PREC[prec], rows.size, _ptr(rows), _ptr(cols),
                                   _ptr(out))
    if rc:
        raise ValueError(f"oracle_srft_entries failed: {rc}")
    return out
