"""GPU parity of the not-normal equations solve (nne_solve) and of the
condition estimate from the FP32 QR of the sketch (cond_est_qr, AUTO with
cond_method = 1) against the CPU oracle, through the C ABI.  Needs an
MI355X; run with -m gpu."""
import math

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


def relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(y))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------ not-normal equations

@pytest.mark.parametrize("m,n,kappa,rho,refine", [(3000, 257, 1e4, 1e-6, 0), (2048, 64, 1e2, 1e-2, 1),
                                                  (777, 65, 1e6, 1e-8, 1)])
def test_nne_orthonormal_b_matches_oracle(pne, orc, m, n, kappa, rho, refine):
    """B = an orthonormal basis of range(A): B^T A is as well conditioned as A,
    so the solve reaches the QR solver's accuracy; the GPU and the oracle
    solve the same system."""
    p = make_problem(m, n, kappa, rho, seed=m + n)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    Q = np.asfortranarray(np.linalg.qr(A)[0])
    x, info = pne.nne_solve(dev(A), dev(Q), torch.from_numpy(b).cuda(), refine_steps=refine)
    assert int(host(info)[0]) == 0
    xo, io = orc.nne(A, Q, b, refine_steps=refine)
    assert io == 0
    err_qr = relerr(orc.qr_ls(A, b), xs)
    xg = host(x)
    assert relerr(xg, xs) <= 10 * err_qr
    assert relerr(xg, xo) <= 10 * err_qr
    if kappa <= 1e3:
        assert relerr(xg, xs) <= 1e-12


def test_nne_general_b_matches_oracle(pne, orc):
    """B = A M with a random well-conditioned M: the same least-squares
    solution (Section 5.2); the conditioning of B^T A is that of A^T A, so
    the check is against the oracle's solve of the same equations."""
    p = make_problem(4000, 130, 1e3, 1e-4, seed=91)
    A, b = p.numpy_A(), p.numpy_b()
    rng = np.random.default_rng(91)
    B = np.asfortranarray(A @ (np.eye(130) + 0.2 * rng.standard_normal((130, 130))))
    x, info = pne.nne_solve(dev(A), dev(B), torch.from_numpy(b).cuda(), refine_steps=1)
    xo, io = orc.nne(A, B, b, refine_steps=1)
    assert int(host(info)[0]) == 0 and io == 0
    BtA = B.T @ A
    # both solve B^T A x = B^T b; they differ by rounding amplified by kappa(B^T A)
    assert relerr(host(x), xo) <= 100 * np.linalg.cond(BtA) * 2.0 ** -53


def test_nne_with_preconditioned_b_is_hpne_accurate(pne, orc):
    """B = A_p = A R_s^{-1} with the GPU preconditioner: the HPNE system."""
    p = make_problem(5000, 200, 1e6, 1e-6, seed=92)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    Ad = dev(A)
    R, info, _ = pne.sketch_precond(Ad, opts=pne.make_opts(seed=3, sketch_prec="fp32", qr_prec="fp32"))
    Ap = np.asfortranarray(A @ np.linalg.inv(host(R)))
    x, info = pne.nne_solve(Ad, dev(Ap), torch.from_numpy(b).cuda(), refine_steps=1)
    assert int(host(info)[0]) == 0
    assert relerr(host(x), xs) <= 10 * relerr(orc.qr_ls(A, b), xs)


def test_nne_singular_reports_pivot(pne):
    p = make_problem(500, 40, 1e2, 1e-6, seed=93)
    A = p.numpy_A()
    B = A.copy(order="F")
    B[:, 7] = 0.0                      # B^T A has a zero row 7
    x, info = pne.nne_solve(dev(A), dev(B), torch.from_numpy(p.numpy_b()).cuda())
    code = int(host(info)[0])
    assert 3001 <= code <= 3040
    assert np.all(np.isnan(host(x)))


# ------------------------------------------------------------------ QR-based condition estimate

@pytest.mark.parametrize("kappa", [1e2, 1e5, 1e6, 1e10])
def test_cond_est_qr_matches_oracle(pne, orc, kappa):
    p = make_problem(4000, 100, kappa, 1e-6, seed=94)
    A = p.numpy_A()
    k0o, cho = orc.cond_est_qr(A, seed=4)
    k0, ch = pne.cond_est_qr(dev(A), seed=4)
    k0g, chg = float(host(k0)[0]), int(host(ch)[0])
    assert chg == cho
    if kappa <= 1e6:
        # FP32 QR and Hager solves on both sides, different summation orders:
        # kappa0 agrees to a few units of u_32 kappa in relative terms
        assert abs(k0g - k0o) < 0.05 + math.log10(1 + 2 ** -22 * kappa), (k0g, k0o)
    else:
        assert chg == 1


def test_auto_with_qr_estimate_reuses_fp32_preconditioner(pne, orc):
    """kappa = 1e6: the QR estimate picks single precision (the Gram estimate
    cannot, its Cholesky breaks down); the solve reuses the estimate's FP32
    sketch and QR, so x equals the explicit FP32/FP32 solve bit for bit."""
    p = make_problem(6000, 150, 1e6, 1e-6, seed=95)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    Ad, bd = dev(A), torch.from_numpy(b).cuda()
    o = pne.make_opts(seed=5, sketch_prec="auto", qr_prec="auto", refine_steps=1, cond_method=1)
    x, info, meta = pne.pne_solve(Ad, bd, opts=o)
    assert meta["sketch_prec"] == "fp32" and meta["qr_prec"] == "fp32"
    assert 4.0 <= meta["kappa0"] <= 8.0
    assert int(host(info)[0]) == 0
    o32 = pne.make_opts(seed=5, sketch_prec="fp32", qr_prec="fp32", refine_steps=1)
    x32, info32, _ = pne.pne_solve(Ad, bd, opts=o32)
    assert np.array_equal(host(x), host(x32))
    assert relerr(host(x), xs) <= 10 * relerr(orc.qr_ls(A, b), xs)
    # the Gram estimate picks double on the same input
    _, _, meta_g = pne.pne_solve(Ad, bd, opts=pne.make_opts(seed=5, sketch_prec="auto", refine_steps=1))
    assert meta_g["qr_prec"] == "fp64"


@pytest.mark.parametrize("hpne", [False, True])
def test_auto_qr_estimate_half_and_double(pne, orc, hpne):
    for kappa, want in [(1e2, "fp16"), (1e10, "fp64")]:
        p = make_problem(3000, 100, kappa, 1e-6, seed=96)
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        o = pne.make_opts(seed=6, sketch_prec="auto", qr_prec="auto", refine_steps=1, cond_method=1)
        fn = pne.hpne_solve if hpne else pne.pne_solve
        x, info, meta = fn(dev(A), torch.from_numpy(b).cuda(), opts=o)
        assert meta["qr_prec"] == want
        assert int(host(info)[0]) == 0
        assert relerr(host(x), xs) <= 10 * relerr(orc.qr_ls(A, b), xs)


def test_batched_auto_with_qr_estimate(pne, orc):
    from workloads import pack_batch
    shapes = [(3000, 100, 1e2, 1e-6), (4000, 120, 1e6, 1e-6), (2500, 64, 1e10, 1e-8)]
    probs = [make_problem(m, n, k, r, seed=970 + i) for i, (m, n, k, r) in enumerate(shapes)]
    A, b, x, descs = pack_batch(probs)
    o = pne.make_opts(seed=7, sketch_prec="auto", qr_prec="auto", refine_steps=1, cond_method=1)
    info = pne.pne_solve_batched(A, b, x, descs, opts=o)
    assert np.all(host(info) == 0)
    xh = host(x)
    for p, d in zip(probs, descs):
        xg = xh[d["x_offset"]:d["x_offset"] + p.n]
        A_, b_, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        assert relerr(xg, xs) <= 10 * relerr(orc.qr_ls(A_, b_), xs)
