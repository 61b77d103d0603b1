"""The C-ABI library loads and exports every function include/pne.h declares,
and its host-side argument checks run without a GPU (they return before any
device call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pne.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\*?(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def pne():
    import paper_2603_16644_amd as p
    if not os.path.exists(p._lib.LIB_PATH):
        from paper_2603_16644_amd.build import build
        build()
    return p


def test_header_lists_the_boundary():
    names = declared_functions()
    for must in ["pne_solve", "hpne_solve", "sketch_precond", "cond_est", "pne_solve_batched",
                 "pne_workspace_size", "pne_sketch"]:
        assert must in names


def test_library_exports_every_declared_symbol(pne):
    L = pne.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(declared_functions()) <= set(pne._lib.EXPORTS) | {"pne_profile_enable", "pne_profile_read",
                                                                  "pne_profile_phase_name"}


def test_host_argument_checks(pne):
    L = pne.lib()
    o = pne.make_opts(sketch_prec="bf16", qr_prec="fp32")
    by = ctypes.byref
    # sizes
    assert L.pne_workspace_size(100, 200, by(o), 0) == 0          # m < n
    assert L.pne_workspace_size(1000, 100, by(o), 0) > 0
    bad = pne.make_opts(s=50)
    assert L.pne_workspace_size(1000, 100, by(bad), 0) == 0        # s < n
    fp8qr = pne.make_opts(sketch_prec="fp8", qr_prec="fp8")
    assert L.pne_workspace_size(1000, 100, by(fp8qr), 0) == 0      # FP8 QR not allowed
    br = pne.make_opts(sketch_prec="fp8", qr_prec="fp32", block_rows=100)
    assert L.pne_workspace_size(1000, 100, by(br), 0) == 0         # block rows not a multiple of 64
    # solve entry points reject bad arguments before touching a device
    one = ctypes.c_void_p(256)
    assert L.pne_solve(1000, 100, None, 1000, one, one, by(o), one, 1 << 30, one, None, None) == -1
    assert L.pne_solve(1000, 100, one, 999, one, one, by(o), one, 1 << 30, one, None, None) == -1
    assert L.hpne_solve(1000, 100, one, 1000, one, one, by(o), one, 16, one, None, None) == -4
    assert L.pne_solve(10**6, 5000, one, 10**6, one, one, by(o), one, 1 << 40, one, None, None) == -5
    assert L.cond_est(10, 20, one, 10, one, one, one, 1 << 20, None) == -1
    assert L.pne_status_string(-4) == b"workspace too small"
    # the no-allocation entry point checks sizes against its static array first
    assert L.pne_noalloc_max_bytes() == 64 << 20
    assert L.pne_solve_noalloc(20000, 1000, one, 20000, one, one, by(o), 0, one, None, None) == -4
    assert L.pne_solve_noalloc(1000, 100, None, 1000, one, one, by(o), 0, one, None, None) == -1
    assert L.pne_solve_noalloc(1000, 100, one, 1000, one, one, by(o), 2, one, None, None) == -1
    assert L.pne_solve_noalloc(100, 200, one, 100, one, one, by(o), 1, one, None, None) == -1


def test_workspace_grows_with_problem(pne):
    L = pne.lib()
    o = pne.make_opts(sketch_prec="bf16", qr_prec="fp32")
    a = L.pne_workspace_size(10_000, 100, ctypes.byref(o), 0)
    b = L.pne_workspace_size(100_000, 100, ctypes.byref(o), 0)
    assert b > a >= 10_000 * 100 * 8   # at least A_p


def test_batched_workspace_sizing_runs_on_host(pne):
    """The batched workspace query records the whole launch sequence of every
    member on the host (no device call) and bounds its group tables."""
    from paper_2603_16644_amd._lib import ProblemDesc
    L = pne.lib()
    shapes = [(2000, 64), (3100, 100), (2500, 33)]
    arr = (ProblemDesc * 3)()
    ao = bo = xo = 0
    for i, (m, n) in enumerate(shapes):
        arr[i] = ProblemDesc(m, n, m, ao, bo, xo)
        ao += m * n
        bo += m
        xo += n
    o = pne.make_opts(sketch_prec="bf16", qr_prec="fp32")
    p = ctypes.cast(arr, ctypes.c_void_p)
    total = L.pne_batched_workspace_size(3, p, ctypes.byref(o), 0)
    singles = sum(L.pne_workspace_size(m, n, ctypes.byref(o), 0) for m, n in shapes)
    assert total > 0 and total >= 0.5 * singles
    assert L.pne_batched_workspace_size(3, p, ctypes.byref(o), 1) > 0     # HPNE
    auto = pne.make_opts()
    assert L.pne_batched_workspace_size(3, p, ctypes.byref(auto), 0) > total
    arr[1] = ProblemDesc(50, 100, 50, 0, 0, 0)                           # m < n
    assert L.pne_batched_workspace_size(3, p, ctypes.byref(o), 0) == 0
    one = ctypes.c_void_p(256)
    assert L.pne_solve_batched(3, p, one, one, one, ctypes.byref(o), 0, one, 1 << 30, one, None) == -1


def test_no_cpu_fallback():
    """Without the built library the binding raises, and CPU tensors are
    refused: nothing computes the solve outside the HIP library."""
    import subprocess
    import sys
    code = (
        "import paper_2603_16644_amd._lib as l\n"
        "l.LIB_PATH = '/nonexistent/libpne.so'\n"
        "import paper_2603_16644_amd as p, torch\n"
        "try:\n"
        "    p.lib()\n"
        "    raise SystemExit('library call did not raise')\n"
        "except RuntimeError:\n"
        "    pass\n"
        "A = torch.randn(50, 5, dtype=torch.float64)\n"
        "b = torch.randn(50, dtype=torch.float64)\n"
        "for fn in (p.pne_solve, p.hpne_solve):\n"
        "    try:\n"
        "        fn(A, b)\n"
        "        raise SystemExit('CPU tensors were accepted')\n"
        "    except ValueError:\n"
        "        pass\n"
        "print('ok')\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
