"""ctypes binding of libpne.so (include/pne.h).  Argument marshalling only:
every step of the solve runs in the library's HIP kernels.  torch supplies
device memory (inputs, outputs, workspace) and the stream.

Matrices are column-major: pass A as an (m, n) float64 CUDA tensor with
strides (1, lda), e.g. ``At.t()`` for an (n, m) contiguous tensor ``At``.
The library must be built (``python -m paper_2603_16644_amd.build``); there
is no fallback path.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpne.so")

PREC = {"auto": 0, "fp64": 1, "fp32": 2, "fp16": 3, "bf16": 4, "fp8": 5}
PREC_NAME = {v: k for k, v in PREC.items()}
STATUS = {0: "ok", -1: "invalid argument", -2: "out of host memory", -3: "HIP runtime error",
          -4: "workspace too small", -5: "unsupported size or option"}

EXPORTS = ["pne_default_opts", "pne_workspace_size", "pne_solve", "hpne_solve",
           "sketch_precond_workspace_size", "sketch_precond", "cond_est_workspace_size", "cond_est",
           "pne_sketch_workspace_size", "pne_sketch", "pne_batched_workspace_size",
           "pne_solve_batched", "pne_gram_workspace_size", "pne_gram", "pne_status_string",
           "pne_profile_enable", "pne_profile_read", "pne_profile_phase_name",
           "pne_noalloc_max_bytes", "pne_solve_noalloc", "cond_est_qr_workspace_size", "cond_est_qr",
           "nne_workspace_size", "nne_solve", "pne_batch_plan_create", "pne_batch_plan_execute",
           "pne_batch_plan_execute_graph", "pne_batch_plan_destroy", "pne_autotune_batched_workspace_size",
           "pne_autotune_batched", "pne_sketch_srft_workspace_size", "pne_sketch_srft", "qr_ls_workspace_size",
           "qr_ls_solve"]


class PneError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn}: {STATUS.get(status, status)} ({status})")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("s", ctypes.c_int64), ("seed", ctypes.c_uint64), ("problem_id", ctypes.c_uint32),
                ("sketch_prec", ctypes.c_int32), ("qr_prec", ctypes.c_int32),
                ("known_kappa", ctypes.c_double), ("refine_steps", ctypes.c_int32),
                ("block_rows", ctypes.c_int32), ("cond_method", ctypes.c_int32),
                ("sketch_kind", ctypes.c_int32), ("check_finite", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("sketch_prec_used", ctypes.c_int32), ("qr_prec_used", ctypes.c_int32),
                ("kappa0", ctypes.c_float), ("refine_steps_run", ctypes.c_int32)]


class TuneResult(ctypes.Structure):
    _fields_ = [("batch_kchunk", ctypes.c_int64), ("shortk_tile", ctypes.c_int32),
                ("lower_small_n", ctypes.c_int32), ("ms", ctypes.c_double), ("stored", ctypes.c_int32),
                ("persistent", ctypes.c_int32)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("a_offset", ctypes.c_int64), ("b_offset", ctypes.c_int64),
                ("x_offset", ctypes.c_int64), ("problem_id", ctypes.c_int64)]


_lib = None


def lib():
    """Load libpne.so; raises if it is not built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2603_16644_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        i64, P, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
        OP = ctypes.POINTER(Opts)
        sigs = {
            "pne_default_opts": (None, [OP]),
            "pne_workspace_size": (sz, [i64, i64, OP, ctypes.c_int]),
            "pne_solve": (ctypes.c_int, [i64, i64, P, i64, P, P, OP, P, sz, P, P, P]),
            "hpne_solve": (ctypes.c_int, [i64, i64, P, i64, P, P, OP, P, sz, P, P, P]),
            "sketch_precond_workspace_size": (sz, [i64, i64, OP]),
            "sketch_precond": (ctypes.c_int, [i64, i64, P, i64, OP, P, i64, P, sz, P, P, P]),
            "cond_est_workspace_size": (sz, [i64, i64]),
            "cond_est": (ctypes.c_int, [i64, i64, P, i64, P, P, P, sz, P]),
            "pne_sketch_workspace_size": (sz, [i64, i64, i64, ctypes.c_int32]),
            "pne_sketch": (ctypes.c_int, [i64, i64, P, i64, i64, ctypes.c_uint64, ctypes.c_uint32,
                                          ctypes.c_int32, ctypes.c_int32, P, i64, P, sz, P]),
            "pne_batched_workspace_size": (sz, [i64, P, OP, ctypes.c_int]),
            "pne_solve_batched": (ctypes.c_int, [i64, P, P, P, P, OP, ctypes.c_int, P, sz, P, P]),
            "pne_gram_workspace_size": (sz, [i64, i64, ctypes.c_int]),
            "pne_gram": (ctypes.c_int, [i64, i64, P, i64, P, P, i64, ctypes.c_int, ctypes.c_int, P, i64, P, P,
                                        P, sz, P, P]),
            "pne_status_string": (ctypes.c_char_p, [ctypes.c_int]),
            "pne_profile_enable": (ctypes.c_int, [ctypes.c_int]),
            "pne_profile_read": (ctypes.c_int, [P, ctypes.c_int]),
            "pne_profile_phase_name": (ctypes.c_char_p, [ctypes.c_int]),
            "pne_noalloc_max_bytes": (sz, []),
            "cond_est_qr_workspace_size": (sz, [i64, i64, i64]),
            "cond_est_qr": (ctypes.c_int, [i64, i64, P, i64, i64, ctypes.c_uint64, P, P, P, sz, P]),
            "nne_workspace_size": (sz, [i64, i64]),
            "qr_ls_workspace_size": (sz, [i64, i64]),
            "qr_ls_solve": (ctypes.c_int, [i64, i64, P, i64, P, P, P, sz, P, P]),
            "pne_sketch_srft_workspace_size": (sz, [i64, i64, ctypes.c_int32]),
            "pne_sketch_srft": (ctypes.c_int, [i64, i64, P, i64, i64, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int32,
                                               P, i64, P, sz, P]),
            "pne_batch_plan_create": (ctypes.c_int, [i64, P, P, P, P, OP, ctypes.c_int, P, sz, P, P,
                                                     ctypes.POINTER(ctypes.c_void_p)]),
            "pne_batch_plan_execute": (ctypes.c_int, [P, P]),
            "pne_batch_plan_execute_graph": (ctypes.c_int, [P, P]),
            "pne_batch_plan_destroy": (None, [P]),
            "pne_autotune_batched_workspace_size": (sz, [i64, P, OP, ctypes.c_int]),
            "pne_autotune_batched": (ctypes.c_int, [i64, P, P, P, P, OP, ctypes.c_int, P, sz, P, P,
                                                    ctypes.POINTER(TuneResult)]),
            "nne_solve": (ctypes.c_int, [i64, i64, P, i64, P, i64, P, P, ctypes.c_int32, P, sz, P, P]),
            "pne_solve_noalloc": (ctypes.c_int, [i64, i64, P, i64, P, P, OP, ctypes.c_int, P, P, P]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def make_opts(s: int = 0, seed: int = 0, problem_id: int = 0, sketch_prec="auto", qr_prec=None,
              known_kappa: float = 0.0, refine_steps: int = 1, block_rows: int = 128,
              cond_method: int = 0, sketch_kind="gaussian", check_finite: bool = False) -> Opts:
    o = Opts()
    lib().pne_default_opts(ctypes.byref(o))
    o.s = int(s)
    o.seed = int(seed)
    o.problem_id = int(problem_id)
    o.sketch_prec = PREC[sketch_prec] if isinstance(sketch_prec, str) else int(sketch_prec)
    qp = sketch_prec if qr_prec is None else qr_prec
    o.qr_prec = PREC[qp] if isinstance(qp, str) else int(qp)
    o.known_kappa = float(known_kappa)
    o.refine_steps = int(refine_steps)
    o.block_rows = int(block_rows)
    o.cond_method = int(cond_method)
    o.sketch_kind = {"gaussian": 0, "srft": 1}[sketch_kind] if isinstance(sketch_kind, str) else int(sketch_kind)
    o.check_finite = int(bool(check_finite))
    return o


def _stream_ptr(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _colmajor(A: torch.Tensor):
    if A.dim() != 2 or A.dtype != torch.float64 or not A.is_cuda:
        raise ValueError("A must be a 2-D float64 CUDA tensor")
    m, n = A.shape
    if A.stride(0) != 1 or A.stride(1) < max(m, 1):
        raise ValueError("A must be column-major: strides (1, lda) with lda >= m (use At.t())")
    return m, n, A.stride(1)


class Workspace:
    """Grow-only device workspace (one per device/stream user)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


_ws = Workspace()


def _check(fn: str, rc: int):
    if rc != 0:
        raise PneError(fn, rc)


def _solve(hpne: bool, A, b, x=None, opts: Opts | None = None, stream=None, workspace=None):
    m, n, lda = _colmajor(A)
    if b.dtype != torch.float64 or not b.is_contiguous() or b.numel() != m:
        raise ValueError("b must be a contiguous float64 vector of length m")
    opts = opts or make_opts()
    x = torch.empty(n, dtype=torch.float64, device=A.device) if x is None else x
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    need = lib().pne_workspace_size(m, n, ctypes.byref(opts), int(hpne))
    if need == 0:
        raise PneError("pne_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    hinfo = Info()
    fn = lib().hpne_solve if hpne else lib().pne_solve
    rc = fn(m, n, A.data_ptr(), lda, b.data_ptr(), x.data_ptr(), ctypes.byref(opts), ws.data_ptr(),
            ws.numel(), info.data_ptr(), ctypes.byref(hinfo), _stream_ptr(stream))
    _check("hpne_solve" if hpne else "pne_solve", rc)
    meta = {"sketch_prec": PREC_NAME.get(hinfo.sketch_prec_used), "qr_prec": PREC_NAME.get(hinfo.qr_prec_used),
            "kappa0": hinfo.kappa0, "refine_steps": hinfo.refine_steps_run}
    return x, info, meta


def pne_solve(A, b, x=None, opts: Opts | None = None, stream=None, workspace=None):
    """PNE solve (include/pne.h pne_solve).  Returns (x, info tensor, meta dict)."""
    return _solve(False, A, b, x, opts, stream, workspace)


def hpne_solve(A, b, x=None, opts: Opts | None = None, stream=None, workspace=None):
    """HPNE solve (include/pne.h hpne_solve).  Returns (x, info tensor, meta dict)."""
    return _solve(True, A, b, x, opts, stream, workspace)


def pne_solve_noalloc(A, b, x=None, opts: Opts | None = None, hpne: bool = False, stream=None):
    """PNE/HPNE solve without a workspace (include/pne.h pne_solve_noalloc):
    the library's per-GPU static scratch array replaces dwork.  Returns
    (x, info tensor, meta dict)."""
    m, n, lda = _colmajor(A)
    if b.dtype != torch.float64 or not b.is_contiguous() or b.numel() != m:
        raise ValueError("b must be a contiguous float64 vector of length m")
    opts = opts or make_opts()
    x = torch.empty(n, dtype=torch.float64, device=A.device) if x is None else x
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    hinfo = Info()
    rc = lib().pne_solve_noalloc(m, n, A.data_ptr(), lda, b.data_ptr(), x.data_ptr(), ctypes.byref(opts),
                                 int(hpne), info.data_ptr(), ctypes.byref(hinfo), _stream_ptr(stream))
    _check("pne_solve_noalloc", rc)
    meta = {"sketch_prec": PREC_NAME.get(hinfo.sketch_prec_used), "qr_prec": PREC_NAME.get(hinfo.qr_prec_used),
            "kappa0": hinfo.kappa0, "refine_steps": hinfo.refine_steps_run}
    return x, info, meta


def sketch_precond(A, opts: Opts | None = None, stream=None, workspace=None):
    """R_s (n x n FP64, upper, column-major) of the sketch; returns (R, info, meta)."""
    m, n, lda = _colmajor(A)
    opts = opts or make_opts()
    Rt = torch.empty(n, n, dtype=torch.float64, device=A.device)  # Rt.t() is column-major R
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    need = lib().sketch_precond_workspace_size(m, n, ctypes.byref(opts))
    if need == 0:
        raise PneError("sketch_precond_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    hinfo = Info()
    rc = lib().sketch_precond(m, n, A.data_ptr(), lda, ctypes.byref(opts), Rt.data_ptr(), n, ws.data_ptr(),
                              ws.numel(), info.data_ptr(), ctypes.byref(hinfo), _stream_ptr(stream))
    _check("sketch_precond", rc)
    return Rt.t(), info, {"sketch_prec": PREC_NAME.get(hinfo.sketch_prec_used),
                          "qr_prec": PREC_NAME.get(hinfo.qr_prec_used)}


def cond_est(A, stream=None, workspace=None):
    """(kappa0 float tensor, precision-code int tensor) on the device."""
    m, n, lda = _colmajor(A)
    k0 = torch.empty(1, dtype=torch.float32, device=A.device)
    ch = torch.empty(1, dtype=torch.int32, device=A.device)
    need = lib().cond_est_workspace_size(m, n)
    if need == 0:
        raise PneError("cond_est_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    rc = lib().cond_est(m, n, A.data_ptr(), lda, k0.data_ptr(), ch.data_ptr(), ws.data_ptr(), ws.numel(),
                        _stream_ptr(stream))
    _check("cond_est", rc)
    return k0, ch


def cond_est_qr(A, s: int = 0, seed: int = 0, stream=None, workspace=None):
    """(kappa0, precision code) device tensors from the FP32 QR of the FP32
    sketch (include/pne.h cond_est_qr)."""
    m, n, lda = _colmajor(A)
    k0 = torch.empty(1, dtype=torch.float32, device=A.device)
    ch = torch.empty(1, dtype=torch.int32, device=A.device)
    need = lib().cond_est_qr_workspace_size(m, n, s)
    if need == 0:
        raise PneError("cond_est_qr_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    rc = lib().cond_est_qr(m, n, A.data_ptr(), lda, s, seed, k0.data_ptr(), ch.data_ptr(), ws.data_ptr(),
                           ws.numel(), _stream_ptr(stream))
    _check("cond_est_qr", rc)
    return k0, ch


def nne_solve(A, B, b, x=None, refine_steps: int = 0, stream=None, workspace=None):
    """Not-normal equations B^T A x = B^T b (include/pne.h nne_solve).
    A and B column-major (m, n) float64 CUDA tensors.  Returns (x, info)."""
    m, n, lda = _colmajor(A)
    mb, nb, ldb = _colmajor(B)
    if (mb, nb) != (m, n):
        raise ValueError("B must have the shape of A")
    if b.dtype != torch.float64 or not b.is_contiguous() or b.numel() != m:
        raise ValueError("b must be a contiguous float64 vector of length m")
    x = torch.empty(n, dtype=torch.float64, device=A.device) if x is None else x
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    need = lib().nne_workspace_size(m, n)
    if need == 0:
        raise PneError("nne_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    rc = lib().nne_solve(m, n, A.data_ptr(), lda, B.data_ptr(), ldb, b.data_ptr(), x.data_ptr(), refine_steps,
                         ws.data_ptr(), ws.numel(), info.data_ptr(), _stream_ptr(stream))
    _check("nne_solve", rc)
    return x, info


def pne_sketch(A, s: int, seed: int = 0, problem_id: int = 0, prec="fp64", block_rows: int = 128,
               stream=None, workspace=None):
    """A_s = Omega A (s x n FP64 column-major view)."""
    m, n, lda = _colmajor(A)
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    Ast = torch.empty(n, s, dtype=torch.float64, device=A.device)
    need = lib().pne_sketch_workspace_size(m, n, s, p)
    if need == 0:
        raise PneError("pne_sketch_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    rc = lib().pne_sketch(m, n, A.data_ptr(), lda, s, seed, problem_id, p, block_rows, Ast.data_ptr(), s,
                          ws.data_ptr(), ws.numel(), _stream_ptr(stream))
    _check("pne_sketch", rc)
    return Ast.t()


def qr_ls_solve(A, b, x=None, stream=None, workspace=None):
    """FP64 Householder-QR least-squares solve (include/pne.h qr_ls_solve).
    Returns (x, info)."""
    m, n, lda = _colmajor(A)
    if b.dtype != torch.float64 or not b.is_contiguous() or b.numel() != m:
        raise ValueError("b must be a contiguous float64 vector of length m")
    x = torch.empty(n, dtype=torch.float64, device=A.device) if x is None else x
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    need = lib().qr_ls_workspace_size(m, n)
    if need == 0:
        raise PneError("qr_ls_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    rc = lib().qr_ls_solve(m, n, A.data_ptr(), lda, b.data_ptr(), x.data_ptr(), ws.data_ptr(), ws.numel(),
                           info.data_ptr(), _stream_ptr(stream))
    _check("qr_ls_solve", rc)
    return x, info


def pne_sketch_srft(A, s: int, seed: int = 0, problem_id: int = 0, prec="fp64", stream=None, workspace=None):
    """SRFT sketch A_s = (1/sqrt(s)) S H D A (s x n FP64 column-major view)."""
    m, n, lda = _colmajor(A)
    p = PREC[prec] if isinstance(prec, str) else int(prec)
    Ast = torch.empty(n, s, dtype=torch.float64, device=A.device)
    need = lib().pne_sketch_srft_workspace_size(m, n, p)
    if need == 0:
        raise PneError("pne_sketch_srft_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    rc = lib().pne_sketch_srft(m, n, A.data_ptr(), lda, s, seed, problem_id, p, Ast.data_ptr(), s, ws.data_ptr(),
                               ws.numel(), _stream_ptr(stream))
    _check("pne_sketch_srft", rc)
    return Ast.t()


def pne_solve_batched(A_base, b_base, x_base, descs, opts: Opts | None = None, hpne: bool = False,
                      stream=None, workspace=None):
    """Batched solve over problems described by `descs` (list of dicts with m, n,
    lda, a_offset, b_offset, x_offset in float64 elements and an optional
    problem_id, the sketch counter word, default the list index).  Returns
    info (batch,)."""
    opts = opts or make_opts()
    batch = len(descs)
    arr = (ProblemDesc * batch)()
    for i, d in enumerate(descs):
        arr[i] = ProblemDesc(d["m"], d["n"], d["lda"], d["a_offset"], d["b_offset"], d["x_offset"],
                             d.get("problem_id", i))
    info = torch.zeros(batch, dtype=torch.int32, device=A_base.device)
    need = lib().pne_batched_workspace_size(batch, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(opts),
                                            int(hpne))
    if need == 0:
        raise PneError("pne_batched_workspace_size", -1)
    ws = (workspace or _ws).get(need, A_base.device)
    rc = lib().pne_solve_batched(batch, ctypes.cast(arr, ctypes.c_void_p), A_base.data_ptr(), b_base.data_ptr(),
                                 x_base.data_ptr(), ctypes.byref(opts), int(hpne), ws.data_ptr(), ws.numel(),
                                 info.data_ptr(), _stream_ptr(stream))
    _check("pne_solve_batched", rc)
    return info


def pne_gram(A, b, R, hpne: bool = False, factor: bool = False, stream=None, workspace=None):
    """Normal-equation matrix for a given preconditioner R (include/pne.h
    pne_gram).  Returns (C (n x n column-major view), c, piv or None, info)."""
    m, n, lda = _colmajor(A)
    if R.shape != (n, n) or R.dtype != torch.float64 or R.stride(0) != 1:
        raise ValueError("R must be an n x n column-major float64 CUDA tensor")
    Ct = torch.empty(n, n, dtype=torch.float64, device=A.device)
    c = torch.empty(n, dtype=torch.float64, device=A.device)
    piv = torch.empty(n, dtype=torch.int32, device=A.device) if (hpne and factor) else None
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    need = lib().pne_gram_workspace_size(m, n, int(hpne))
    if need == 0:
        raise PneError("pne_gram_workspace_size", -1)
    ws = (workspace or _ws).get(need, A.device)
    rc = lib().pne_gram(m, n, A.data_ptr(), lda, b.data_ptr(), R.data_ptr(), R.stride(1), int(hpne), int(factor),
                        Ct.data_ptr(), n, c.data_ptr(), piv.data_ptr() if piv is not None else None,
                        ws.data_ptr(), ws.numel(), info.data_ptr(), _stream_ptr(stream))
    _check("pne_gram", rc)
    return Ct.t(), c, piv, info


def _desc_array(descs):
    arr = (ProblemDesc * len(descs))()
    for i, d in enumerate(descs):
        arr[i] = ProblemDesc(d["m"], d["n"], d["lda"], d["a_offset"], d["b_offset"], d["x_offset"],
                             d.get("problem_id", i))
    return arr


class BatchPlan:
    """A batched solve prepared once (include/pne.h pne_batch_plan_create) and
    executed many times.  Owns its workspace tensor; A, b, x must stay alive
    and in place while the plan is used."""

    def __init__(self, A_base, b_base, x_base, descs, opts: Opts | None = None, hpne: bool = False, stream=None):
        self.opts = opts or make_opts()
        self.arr = _desc_array(descs)
        batch = len(descs)
        self.info = torch.zeros(batch, dtype=torch.int32, device=A_base.device)
        need = lib().pne_batched_workspace_size(batch, ctypes.cast(self.arr, ctypes.c_void_p),
                                                ctypes.byref(self.opts), int(hpne))
        if need == 0:
            raise PneError("pne_batched_workspace_size", -1)
        self.ws = torch.empty(need, dtype=torch.uint8, device=A_base.device)
        self._keep = (A_base, b_base, x_base)
        h = ctypes.c_void_p()
        rc = lib().pne_batch_plan_create(batch, ctypes.cast(self.arr, ctypes.c_void_p), A_base.data_ptr(),
                                         b_base.data_ptr(), x_base.data_ptr(), ctypes.byref(self.opts), int(hpne),
                                         self.ws.data_ptr(), self.ws.numel(), self.info.data_ptr(),
                                         _stream_ptr(stream), ctypes.byref(h))
        _check("pne_batch_plan_create", rc)
        self.handle = h

    def execute(self, stream=None):
        _check("pne_batch_plan_execute", lib().pne_batch_plan_execute(self.handle, _stream_ptr(stream)))
        return self.info

    def execute_graph(self, stream):
        """Capture on the first call, then launch the instantiated hipGraph
        (stream: a non-default torch.cuda.Stream)."""
        _check("pne_batch_plan_execute_graph", lib().pne_batch_plan_execute_graph(self.handle, _stream_ptr(stream)))
        return self.info

    def close(self):
        if getattr(self, "handle", None):
            lib().pne_batch_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_batched(A_base, b_base, x_base, descs, opts: Opts | None = None, hpne: bool = False, stream=None):
    """Autotuner of the batched path (include/pne.h pne_autotune_batched).
    Returns a dict with the chosen parameters, their time and whether they
    were stored in $PNE_TUNE_CACHE."""
    opts = opts or make_opts()
    arr = _desc_array(descs)
    batch = len(descs)
    need = lib().pne_autotune_batched_workspace_size(batch, ctypes.cast(arr, ctypes.c_void_p), ctypes.byref(opts),
                                                     int(hpne))
    if need == 0:
        raise PneError("pne_autotune_batched_workspace_size", -1)
    ws = torch.empty(need, dtype=torch.uint8, device=A_base.device)
    info = torch.zeros(batch, dtype=torch.int32, device=A_base.device)
    res = TuneResult()
    rc = lib().pne_autotune_batched(batch, ctypes.cast(arr, ctypes.c_void_p), A_base.data_ptr(), b_base.data_ptr(),
                                    x_base.data_ptr(), ctypes.byref(opts), int(hpne), ws.data_ptr(), ws.numel(),
                                    info.data_ptr(), _stream_ptr(stream), ctypes.byref(res))
    _check("pne_autotune_batched", rc)
    return {"batch_kchunk": res.batch_kchunk, "shortk_tile": res.shortk_tile, "lower_small_n": res.lower_small_n,
            "ms": res.ms, "stored": bool(res.stored), "persistent": bool(res.persistent)}
