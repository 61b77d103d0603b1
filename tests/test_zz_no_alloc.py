"""The no-allocation entry point (pne_solve_noalloc) against pne_solve /
hpne_solve with a caller workspace: same kernels on the same inputs, so x
and info agree bit for bit.  Two calls in a row on the shared static scratch
array, the second with a smaller problem, check that nothing of the first
call leaks into the second.  Needs an MI355X; run with -m gpu."""
import numpy as np
import pytest
import torch

from workloads import make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pne():
    import paper_2603_16644_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


def dev(A_np):
    return torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()


def solve_both(pne, p, hpne, opts):
    A, b = dev(p.numpy_A()), torch.from_numpy(p.numpy_b()).cuda()
    fn = pne.hpne_solve if hpne else pne.pne_solve
    x_ws, info_ws, _ = fn(A, b, opts=opts)
    x_na, info_na, meta = pne.pne_solve_noalloc(A, b, opts=opts, hpne=hpne)
    torch.cuda.synchronize()
    return (x_ws.cpu().numpy(), int(info_ws.item())), (x_na.cpu().numpy(), int(info_na.item())), meta


@pytest.mark.parametrize("hpne", [False, True])
def test_noalloc_matches_workspace_entry_point_twice(pne, hpne):
    from paper_2603_16644_amd import _lib
    big = make_problem(3000, 257, 1e6, 1e-4, seed=7001)
    small = make_problem(777, 65, 1e4, 1e-6, seed=7002)
    opts = pne.make_opts(seed=3, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    need_big = _lib.lib().pne_workspace_size(3000, 257, _lib.ctypes.byref(opts), int(hpne))
    assert 0 < need_big <= _lib.lib().pne_noalloc_max_bytes()
    for p in (big, small):                  # second call smaller than the first
        (xw, iw), (xn, inn), meta = solve_both(pne, p, hpne, opts)
        assert iw == 0 and inn == 0
        assert np.array_equal(xw, xn), np.max(np.abs(xw - xn))
        err = np.linalg.norm(xn - p.numpy_x_star()) / np.linalg.norm(p.numpy_x_star())
        assert err < 1e-6
        assert meta["sketch_prec"] == "bf16" and meta["qr_prec"] == "fp32"


def test_noalloc_auto_precision_matches(pne):
    p = make_problem(2000, 100, 1e2, 1e-6, seed=7003)
    opts = pne.make_opts(seed=4, sketch_prec="auto", refine_steps=1)
    (xw, iw), (xn, inn), meta = solve_both(pne, p, False, opts)
    assert iw == 0 and inn == 0 and meta["qr_prec"] in ("fp16", "fp32", "fp64")
    assert np.array_equal(xw, xn)


def test_noalloc_rejects_oversized_problem(pne):
    from paper_2603_16644_amd import _lib
    m, n = 20_000, 1000                     # A_p alone (160 MB) exceeds the static array
    A = torch.zeros(n, m, dtype=torch.float64, device="cuda").t()
    b = torch.zeros(m, dtype=torch.float64, device="cuda")
    with pytest.raises(pne.PneError) as e:
        pne.pne_solve_noalloc(A, b, opts=pne.make_opts(sketch_prec="fp32"))
    assert e.value.status == -4
