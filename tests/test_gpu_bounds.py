"""The paper's accuracy experiments on the GPU path (Sections 7.2-7.4,
Figures 1-5 and 7, qualitatively): errors of the HIP PNE/HPNE against the
perturbation bounds evaluated by oracle/bounds.py and against the oracle's
QR solver on the same seeded inputs.  Needs an MI355X; run with -m gpu."""
import numpy as np
import pytest
import torch

from oracle import bounds as B
from workloads import make_problem

pytestmark = pytest.mark.gpu
U2 = 2.0 ** -52


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


def gpu_sweep(pne, orc, kappa, prec, hpne, n, rhos, m=6000):
    rows = []
    for rho in rhos:
        p = make_problem(m, n, kappa, rho, seed=200 + n + int(-np.log10(rho)))
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        Ad = dev(A)
        o = pne.make_opts(s=3 * n, seed=1, sketch_prec=prec, qr_prec=prec, refine_steps=0)
        fn = pne.hpne_solve if hpne else pne.pne_solve
        x, info, _ = fn(Ad, torch.from_numpy(b).cuda(), opts=o)
        R, _, _ = pne.sketch_precond(Ad, opts=o)            # the same R_s (same seed and precision)
        assert int(host(info)[0]) == 0
        xg, Rg = host(x), host(R)
        u1 = U2 if prec == "fp64" else B.U_SINGLE
        q, bd = B.all_bounds(A, b, Rg, xg, u1, U2)
        err = float(np.linalg.norm(xg - xs) / np.linalg.norm(xg))
        err_qr = float(np.linalg.norm(orc.qr_ls(A, b) - xs) / np.linalg.norm(xs))
        rows.append((rho, err, err_qr, q, bd))
    return rows


@pytest.mark.parametrize("hpne", [False, True])
def test_double_precision_figures_1_2(pne, orc, hpne):
    for rho, err, err_qr, q, bd in gpu_sweep(pne, orc, 1e4, "fp64", hpne, 100, [1e-12, 1e-6, 1e-3, 1e-1]):
        assert err <= (bd["eq32"] if hpne else bd["eq41"]), (rho, err, bd)
        if not hpne:
            assert bd["eq31"] <= bd["eq41"]
        else:
            assert 0.9 <= bd["eq42"] / bd["eq32"] <= 1.1
        if rho > 1e-4:
            assert err <= 10 * err_qr


@pytest.mark.parametrize("hpne,n", [(False, 100), (True, 100), (False, 1000), (True, 1000)])
def test_mixed_precision_figures_3_4(pne, orc, hpne, n):
    """kappa = 1e8, FP32 preconditioner: the new bound holds, the old one is a
    severe overestimate; error at most ~100x the QR solver's for small
    residuals, as accurate for large ones."""
    new, old = ("eq32", "eq42") if hpne else ("eq41", "eq31")
    rhos = [1e-10, 1e-6, 1e-2] if n == 1000 else [1e-12, 1e-8, 1e-4, 1e-1]
    for rho, err, err_qr, q, bd in gpu_sweep(pne, orc, 1e8, "fp32", hpne, n, rhos):
        assert err <= bd[new], (rho, err, bd[new])
        assert bd[old] >= 1e2 * bd[new], (rho, bd)
        assert err <= (100 if rho < 1e-6 else 10) * err_qr, (rho, err, err_qr)


@pytest.mark.parametrize("kappa,want", [(1e2, "fp16"), (1e10, "fp64")])
def test_automatic_precision_figure_7(pne, orc, kappa, want):
    """Section 7.4, Figure 7, with m = 2^15 rows standing in for 2^17 (the
    oracle QR solve stays within seconds) and n = 400: AUTO picks half
    precision at kappa = 1e2 (almost as accurate as the QR solver) and double
    at kappa = 1e10 (as accurate)."""
    for n in (400,):
        p = make_problem(1 << 15, n, kappa, 1e-6, seed=300 + n)
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        o = pne.make_opts(seed=2, sketch_prec="auto", qr_prec="auto", refine_steps=0)
        x, info, meta = pne.pne_solve(dev(A), torch.from_numpy(b).cuda(), opts=o)
        assert meta["qr_prec"] == want and int(host(info)[0]) == 0
        err = float(np.linalg.norm(host(x) - xs) / np.linalg.norm(xs))
        err_qr = float(np.linalg.norm(orc.qr_ls(A, b) - xs) / np.linalg.norm(xs))
        assert err <= (100 if want == "fp16" else 10) * err_qr, (n, err, err_qr)
