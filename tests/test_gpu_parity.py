"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Needs an MI355X; run with -m gpu."""
import math

import numpy as np
import pytest
import torch

from workloads import make_problem

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def pne():
    import paper_2603_16644_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


def dev(A_np):
    """Column-major float64 CUDA view of a host matrix."""
    return torch.from_numpy(np.ascontiguousarray(A_np.T)).cuda().t()


def relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(y))


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


# ------------------------------------------------------------------ sketch generator

@pytest.mark.parametrize("pid", [0, 3])
def test_sketch_of_identity_reproduces_generator(pne, orc, pid):
    m, s = 200, 300
    eye = dev(np.eye(m))
    As = host(pne.pne_sketch(eye, s, seed=11, problem_id=pid, prec="fp64")) * math.sqrt(s)
    Om = orc.omega(11, s, m, pid=pid)
    # FP32 Box-Muller on the GPU against FP64 in the oracle
    np.testing.assert_allclose(As, Om, rtol=2e-6, atol=2e-6)


@pytest.mark.parametrize("prec,ulp", [("bf16", 2.0 ** -7), ("fp16", 2.0 ** -10), ("fp8", 2.0 ** -3)])
def test_sketch_of_identity_rounds_like_oracle(pne, orc, prec, ulp):
    m, s = 256, 300
    As = host(pne.pne_sketch(dev(np.eye(m)), s, seed=5, prec=prec)) * math.sqrt(s)
    ref = orc.round_to(orc.omega(5, s, m), prec)
    same = np.isclose(As, ref, rtol=1e-6, atol=0)
    assert same.mean() > 0.98                       # identical codes except at rounding ties
    np.testing.assert_allclose(As, ref, rtol=ulp * 1.01, atol=1e-30)


# ------------------------------------------------------------------ sketch product

SKETCH_TOL = {"fp64": 1e-5, "fp32": 1e-4, "bf16": 2.0 ** -7 + 1e-4, "fp16": 2.0 ** -10 + 1e-4,
              "fp8": 2.0 ** -3 + 1e-4}
SKETCH_MEAN = {"fp64": 1e-6, "fp32": 1e-5, "bf16": 3e-4, "fp16": 3e-5, "fp8": 3e-3}


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16", "fp8"])
@pytest.mark.parametrize("shape", [(1000, 100, 300), (5000, 300, 900)])
def test_sketch_parity(pne, orc, prec, shape):
    m, n, s = shape
    p = make_problem(m, n, 1e4, 1e-6, seed=7)
    A = p.numpy_A()
    got = host(pne.pne_sketch(dev(A), s, seed=21, prec=prec))
    ref, ab = orc.sketch(A, s, seed=21, prec=prec, want_abs=True)
    err = np.abs(got - ref)
    assert np.all(err <= SKETCH_TOL[prec] * ab + 1e-300)
    assert float(np.mean(err / ab)) <= SKETCH_MEAN[prec]


# ------------------------------------------------------------------ preconditioner

@pytest.mark.parametrize("qr_prec", ["fp64", "fp32"])
def test_sketch_precond_parity(pne, orc, qr_prec):
    m, n, s = 3000, 200, 600
    p = make_problem(m, n, 1e2, 1e-6, seed=8)
    A = p.numpy_A()
    o = pne.make_opts(s=s, seed=4, sketch_prec=qr_prec, qr_prec=qr_prec)
    R, info, meta = pne.sketch_precond(dev(A), o)
    Rg = host(R)
    assert int(host(info)[0]) == 0
    assert np.all(np.tril(Rg, -1) == 0)
    Ro = orc.solve(A, p.numpy_b(), s=s, seed=4, sketch_prec=qr_prec, qr_prec=qr_prec)["R"]
    # R^T R = A_s^T A_s: the Gram matrices agree to the sketch/QR rounding level
    scale = np.linalg.norm(Ro, 2) ** 2
    tol = 1e-5 if qr_prec == "fp64" else 1e-4
    assert np.abs(Rg.T @ Rg - Ro.T @ Ro).max() <= tol * scale
    # the diagonal agrees in magnitude (row signs are a convention)
    np.testing.assert_allclose(np.abs(np.diag(Rg)), np.abs(np.diag(Ro)), rtol=1e-3)


# ------------------------------------------------------------------ end to end

CASES = [  # (sketch, qr, refine, kappa)
    ("fp64", "fp64", 0, 1e8),
    ("fp32", "fp32", 0, 1e8),
    ("fp32", "fp32", 1, 1e8),
    ("bf16", "fp32", 2, 1e6),
    ("fp16", "fp16", 2, 1e3),
    ("fp8", "fp32", 4, 1e6),
]


@pytest.mark.parametrize("hpne", [False, True])
@pytest.mark.parametrize("sk,qr,refine,kappa", CASES)
def test_solve_parity_small(pne, orc, hpne, sk, qr, refine, kappa):
    """m = 1000, n = 100, s = 300, relative residual 1e-6: the GPU solution is
    within 10x the QR solver's error and agrees with the oracle's solve."""
    m, n, s = 1000, 100, 300
    p = make_problem(m, n, kappa, 1e-6, seed=1001)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    err_qr = relerr(orc.qr_ls(A, b), xs)
    o = pne.make_opts(s=s, seed=1, sketch_prec=sk, qr_prec=qr, refine_steps=refine)
    fn = pne.hpne_solve if hpne else pne.pne_solve
    x, info, meta = fn(dev(A), torch.from_numpy(b).cuda(), opts=o)
    xg = host(x)
    assert int(host(info)[0]) == 0
    err = relerr(xg, xs)
    xo = orc.solve(A, b, hpne=hpne, s=s, seed=1, sketch_prec=sk, qr_prec=qr, refine_steps=refine)["x"]
    assert err <= 10 * err_qr
    assert relerr(xg, xo) * 1.0 <= 10 * err_qr + 10 * relerr(xo, xs)


@pytest.mark.parametrize("m,n", [(777, 65), (3000, 257), (2048, 64)])
def test_solve_ragged_shapes(pne, orc, m, n):
    p = make_problem(m, n, 1e5, 1e-4, seed=m + n)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    err_qr = relerr(orc.qr_ls(A, b), xs)
    for hpne in (False, True):
        o = pne.make_opts(seed=2, sketch_prec="bf16", qr_prec="fp32", refine_steps=2)
        fn = pne.hpne_solve if hpne else pne.pne_solve
        x, info, _ = fn(dev(A), torch.from_numpy(b).cuda(), opts=o)
        assert int(host(info)[0]) == 0
        assert relerr(host(x), xs) <= 10 * err_qr


def test_zero_column_reports_singular_preconditioner(pne):
    p = make_problem(800, 40, 1e3, 1e-4, seed=3)
    A = p.numpy_A().copy(order="F")
    A[:, 5] = 0.0
    for fn in (pne.pne_solve, pne.hpne_solve):
        o = pne.make_opts(seed=1, sketch_prec="fp64", qr_prec="fp64", refine_steps=1)
        x, info, _ = fn(dev(A), torch.from_numpy(p.numpy_b()).cuda(), opts=o)
        assert int(host(info)[0]) == 1006
        assert np.all(np.isnan(host(x)))


def test_deterministic(pne):
    p = make_problem(4000, 200, 1e6, 1e-4, seed=9)
    A, b = dev(p.numpy_A()), torch.from_numpy(p.numpy_b()).cuda()
    o = pne.make_opts(seed=3, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    x1 = host(pne.pne_solve(A, b, opts=o)[0]).copy()
    x2 = host(pne.pne_solve(A, b, opts=o)[0]).copy()
    assert np.array_equal(x1, x2)


# ------------------------------------------------------------------ condition estimate

@pytest.mark.parametrize("kappa,code", [(1e2, 3), (1e10, 1)])
def test_cond_est_pick_matches_paper_and_oracle(pne, orc, kappa, code):
    n, m = 400, 4000
    p = make_problem(m, n, kappa, 1e-6, seed=30)
    A = p.numpy_A()
    k0, ch = pne.cond_est(dev(A))
    k0g, chg = float(host(k0)[0]), int(host(ch)[0])
    k0o, _, cho = orc.cond_est(A)
    assert chg == code == cho
    if math.isfinite(k0o):
        assert abs(k0g - k0o) < 0.05
    else:
        assert not math.isfinite(k0g)


def test_auto_precision_solve(pne, orc):
    p = make_problem(4000, 400, 1e2, 1e-6, seed=31)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    o = pne.make_opts(seed=1, sketch_prec="auto", qr_prec="auto", refine_steps=1)
    x, info, meta = pne.pne_solve(dev(A), torch.from_numpy(b).cuda(), opts=o)
    assert meta["sketch_prec"] == "fp16" and meta["qr_prec"] == "fp16"
    assert int(host(info)[0]) == 0
    assert relerr(host(x), xs) <= 10 * relerr(orc.qr_ls(A, b), xs)


def test_known_kappa_skips_estimate(pne):
    p = make_problem(2000, 100, 1e5, 1e-6, seed=32)
    o = pne.make_opts(seed=1, sketch_prec="auto", qr_prec="auto", known_kappa=1e5)
    _, info, meta = pne.pne_solve(dev(p.numpy_A()), torch.from_numpy(p.numpy_b()).cuda(), opts=o)
    assert meta["sketch_prec"] == "fp32" and abs(meta["kappa0"] - 5.0) < 1e-6


# ------------------------------------------------------------------ full size (m = 1e5, n = 1e3)

@pytest.fixture(scope="module")
def big():
    return make_problem(100_000, 1000, 1e6, 1e-4, seed=1002, device="cuda")


def test_full_size_sketch_sampled_entries(pne, orc, big):
    s = 3000
    As = host(pne.pne_sketch(big.A, s, seed=2, prec="bf16"))
    rng = np.random.default_rng(0)
    rows = rng.integers(0, s, 12)
    cols = rng.integers(0, 1000, 12)
    A = big.numpy_A()
    ref, ab = orc.sketch_entries(A, s, 2, rows, cols, prec="bf16")
    assert np.all(np.abs(As[rows, cols] - ref) <= SKETCH_TOL["bf16"] * ab)


@pytest.mark.parametrize("sk,qr,refine", [("bf16", "fp32", 1), ("fp32", "fp32", 0), ("fp64", "fp64", 0)])
def test_full_size_accuracy(pne, big, sk, qr, refine):
    """Known solution: error within 10x the first-order least-squares bound
    kappa u (1 + kappa rho) of Lemma 1.1 (the QR solver sits at or below it)."""
    o = pne.make_opts(s=3000, seed=2, sketch_prec=sk, qr_prec=qr, refine_steps=refine)
    x, info, _ = pne.pne_solve(big.A, big.b, opts=o)
    assert int(host(info)[0]) == 0
    err = relerr(host(x), host(big.x_star))
    bound = big.kappa * U64 * (1 + big.kappa * big.rho)
    assert err <= 10 * bound


def test_profile_phases(pne, big):
    import ctypes
    L = pne.lib()
    L.pne_profile_enable(1)
    try:
        o = pne.make_opts(s=3000, seed=2, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
        pne.pne_solve(big.A, big.b, opts=o)
        ms = (ctypes.c_double * 16)()
        cnt = L.pne_profile_read(ms, 16)
        names = [L.pne_profile_phase_name(i).decode() for i in range(cnt)]
        t = dict(zip(names, list(ms)[:cnt]))
        for ph in ["sketch_gemm", "qr", "trsm", "gram_gemm", "factor", "solve", "refine"]:
            assert t[ph] > 0.0, (ph, t)
    finally:
        L.pne_profile_enable(0)
