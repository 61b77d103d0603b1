"""GPU FP64 Householder-QR least-squares solver (qr_ls_solve, the direct
method of Section 7.4) against the CPU oracle's Householder QR solve.
Needs an MI355X; run with -m gpu."""
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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(y))


@pytest.mark.parametrize("m,n,kappa,rho", [(3000, 100, 1e8, 1e-6), (20000, 257, 1e6, 1e-4), (64, 64, 1e3, 0.0),
                                           (777, 65, 1e10, 1e-2), (13000, 33, 1e2, 1e-10)])
def test_qr_ls_matches_oracle(pne, orc, m, n, kappa, rho):
    """One to three tree levels, a square system (one padded block), a
    consistent right-hand side (rho = 0: zero residual diagonal is fine)."""
    p = make_problem(m, n, kappa, rho, seed=m + 7 * n)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    x, info = pne.qr_ls_solve(dev(A), torch.from_numpy(b).cuda())
    assert int(host(info)[0]) == 0
    xo = orc.qr_ls(A, b)
    err_qr = relerr(xo, xs)
    xg = host(x)
    assert relerr(xg, xs) <= 10 * max(err_qr, 1e-15)
    # both are backward-stable Householder solves of the same problem
    assert relerr(xg, xo) <= 10 * max(err_qr, 1e-15)


def test_qr_ls_full_size_and_rank_deficiency(pne, orc):
    import os
    p = make_problem(100_000, 1000, 1e6, 1e-4, seed=1002, device="cpu")
    path = os.path.join(os.path.dirname(__file__), "golden", "err_qr_full_size.txt")
    err_qr = [float(l.split()[6]) for l in open(path) if l.startswith("ls_100000x1000_k1e6")][0]
    x, info = pne.qr_ls_solve(p.At.cuda().t(), p.b.cuda())
    assert int(host(info)[0]) == 0
    assert relerr(host(x), p.numpy_x_star()) <= 10 * err_qr
    # a zero column: R_A has a zero diagonal entry -> 1000 + k, x NaN
    q = make_problem(2000, 40, 1e2, 1e-6, seed=5)
    A = q.numpy_A().copy(order="F")
    A[:, 11] = 0.0
    x, info = pne.qr_ls_solve(dev(A), torch.from_numpy(q.numpy_b()).cuda())
    code = int(host(info)[0])
    assert 1001 <= code <= 1040
    assert np.all(np.isnan(host(x)))
