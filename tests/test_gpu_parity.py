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


def padded(A_np, extra=37):
    """Column-major CUDA view with lda = m + extra (odd padding: unaligned columns)."""
    m, n = A_np.shape
    buf = torch.full((n, m + extra), float("nan"), dtype=torch.float64)
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A_np.T))
    return buf.cuda()[:, :m].t()


def test_padded_leading_dimension(pne, orc):
    """lda > m (odd padding, NaN in the pad rows): every entry point reads only
    the m rows of each column and gives the results of the unpadded call."""
    m, n = 1500, 90
    p = make_problem(m, n, 1e4, 1e-5, seed=1010)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    Ap, Au = padded(A), dev(A)
    assert Ap.stride(1) == m + 37
    bd = torch.from_numpy(b).cuda()
    err_qr = relerr(orc.qr_ls(A, b), xs)
    for prec in ("fp32", "bf16", "fp8"):
        s1 = host(pne.pne_sketch(Ap, 270, seed=3, prec=prec))
        s2 = host(pne.pne_sketch(Au, 270, seed=3, prec=prec))
        np.testing.assert_array_equal(s1, s2)
    k1, c1 = pne.cond_est(Ap)
    k2, c2 = pne.cond_est(Au)
    assert float(host(k1)[0]) == float(host(k2)[0]) and int(host(c1)[0]) == int(host(c2)[0])
    for fn in (pne.pne_solve, pne.hpne_solve):
        o = pne.make_opts(seed=4, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
        x1, i1, _ = fn(Ap, bd, opts=o)
        x2, i2, _ = fn(Au, bd, opts=o)
        assert int(host(i1)[0]) == 0 and int(host(i2)[0]) == 0
        assert relerr(host(x1), xs) <= 10 * err_qr
        assert relerr(host(x1), host(x2)) <= 1e-12


@pytest.mark.parametrize("hpne", [False, True])
def test_check_finite_rejects_non_finite_inputs(pne, hpne):
    """pne_opts.check_finite: a NaN in b or an infinity in A (also one in a
    padded A's m rows, but not NaN in its pad rows) makes the call return
    PNE_EINVAL before solving; finite inputs give the same x, bit for bit, as
    the call without the check."""
    m, n = 1500, 90
    p = make_problem(m, n, 1e4, 1e-5, seed=1032)
    A, b = p.numpy_A(), p.numpy_b()
    fn = pne.hpne_solve if hpne else pne.pne_solve
    o = pne.make_opts(seed=4, sketch_prec="bf16", qr_prec="fp32", refine_steps=1, check_finite=True)
    o0 = pne.make_opts(seed=4, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    bd = torch.from_numpy(b).cuda()
    x0, i0, _ = fn(dev(A), bd, opts=o0)
    x1, i1, _ = fn(padded(A), bd, opts=o)   # NaN pad rows are not part of A
    assert int(host(i0)[0]) == 0 and int(host(i1)[0]) == 0
    assert np.array_equal(host(x0), host(x1))
    bb = b.copy()
    bb[m - 1] = np.nan
    with pytest.raises(pne.PneError) as e:
        fn(dev(A), torch.from_numpy(bb).cuda(), opts=o)
    assert e.value.status == -1
    Ab = A.copy()
    Ab[17, n - 1] = np.inf
    with pytest.raises(pne.PneError) as e:
        fn(padded(Ab), bd, opts=o)
    assert e.value.status == -1


def test_bf16_qr_precision_end_to_end(pne, orc):
    m, n, s = 2000, 80, 240
    p = make_problem(m, n, 1e3, 1e-5, seed=1011)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    err_qr = relerr(orc.qr_ls(A, b), xs)
    o = pne.make_opts(s=s, seed=6, sketch_prec="bf16", qr_prec="bf16", refine_steps=2)
    R, info, _ = pne.sketch_precond(dev(A), o)
    assert int(host(info)[0]) == 0
    Rg = host(R)
    Ro = orc.solve(A, b, s=s, seed=6, sketch_prec="bf16", qr_prec="bf16")["R"]
    # R_s entries are BF16 numbers; GPU and oracle factor the same rounded
    # sketch up to FP32-vs-FP64 rounding, so they agree to one BF16 ulp
    np.testing.assert_array_equal(Rg, Rg.astype(np.float32).astype(np.float64))
    assert np.abs(Rg.T @ Rg - Ro.T @ Ro).max() <= 2.0 ** -6 * np.linalg.norm(Ro, 2) ** 2
    for hpne in (False, True):
        fn = pne.hpne_solve if hpne else pne.pne_solve
        x, info, meta = fn(dev(A), torch.from_numpy(b).cuda(), opts=o)
        assert int(host(info)[0]) == 0 and meta["qr_prec"] == "bf16"
        assert relerr(host(x), xs) <= 10 * err_qr


@pytest.mark.parametrize("hpne", [False, True])
def test_gram_and_factors_elementwise(pne, orc, hpne):
    """The normal-equation matrix, its right-hand side, the Cholesky factor
    (PNE) and the LU factors with their pivots (HPNE) against the oracle for
    the same preconditioner R (kernel-level parity of steps 4-6)."""
    m, n = 1000, 100
    # kappa(R) = 1e3 keeps the two substitution orders for A_p within ~1e-12
    p = make_problem(m, n, 1e3, 1e-6, seed=1001)
    A, b = p.numpy_A(), p.numpy_b()
    R = orc.solve(A, b, s=300, seed=1, sketch_prec="fp32", qr_prec="fp32")["R"]
    Ap, _ = orc.precondition(A, R)
    Co, co = orc.gram(Ap, A if hpne else Ap, b)
    Cg, cg, _, info = pne.pne_gram(dev(A), torch.from_numpy(b).cuda(), dev(R), hpne=hpne, factor=False)
    Cg, cg = host(Cg), host(cg)
    mag = np.abs(Ap).T @ np.abs(A if hpne else Ap)
    sel = np.ones((n, n), bool) if hpne else np.tril(np.ones((n, n), bool))
    # FP64 sums of m products in another order, plus the A_p rounding (kappa(R) u |A_p|)
    assert np.all(np.abs(Cg - Co)[sel] <= 1e-10 * mag[sel] + 1e-13 * np.abs(Co).max())
    np.testing.assert_allclose(cg, co, rtol=1e-10, atol=1e-13 * np.abs(co).max())
    Fg, _, piv, info = pne.pne_gram(dev(A), torch.from_numpy(b).cuda(), dev(R), hpne=hpne, factor=True)
    assert int(host(info)[0]) == 0
    Fg = host(Fg)
    if hpne:
        LUo, pivo, io = orc.lu(Co)
        assert io == 0
        np.testing.assert_array_equal(host(piv), pivo)
        np.testing.assert_allclose(Fg, LUo, rtol=0, atol=1e-8 * np.abs(LUo).max())
    else:
        Lo, io = orc.cholesky(Co)
        assert io == 0
        Lg = np.tril(Fg)
        np.testing.assert_allclose(Lg, Lo, rtol=0, atol=1e-8 * np.abs(Lo).max())


_GRAMS = {}   # (m, n) -> (A, b, oracle C, oracle c), shared by the PNE and HPNE cases


@pytest.mark.parametrize("hpne", [False, True])
@pytest.mark.parametrize("m,n", [(6000, 700), (5999, 700), (6001, 300)])
def test_gram_split_k_tiles_elementwise(pne, orc, hpne, m, n):
    """Split-K Gram products with K above 4096: order 700 in 128 x 128 tiles,
    order 300 in 64 x 64 tiles.  A_p's leading dimension is m rounded up to
    even, so its K tiles take the 16-byte loads of the Gram loop; HPNE's
    second operand A keeps the caller's leading dimension, and an odd one
    takes the general loop (as does a ragged last K chunk).  For PNE in
    128 x 128 tiles the diagonal tiles split their lower triangles between
    the four wavefronts and cut K apart from the others.  Both orders leave
    a partial last tile.  R = I makes A_p = A exactly, so only the summation
    order differs from the oracle's product (bound m u sum |a_ki| |a_kj|)."""
    if (m, n) not in _GRAMS:
        rng = np.random.default_rng(1021 + m)
        A = rng.standard_normal((m, n))
        b = rng.standard_normal(m)
        _GRAMS[(m, n)] = (A, b) + orc.gram(A, A, b)
    A, b, Co, co = _GRAMS[(m, n)]
    Cg, cg, _, info = pne.pne_gram(dev(A), torch.from_numpy(b).cuda(), dev(np.eye(n)), hpne=hpne, factor=False)
    assert int(host(info)[0]) == 0
    Cg, cg = host(Cg), host(cg)
    mag = np.abs(A).T @ np.abs(A)
    sel = np.ones((n, n), bool) if hpne else np.tril(np.ones((n, n), bool))
    assert np.all(np.abs(Cg - Co)[sel] <= m * 1.2e-16 * mag[sel])
    magc = np.abs(A).T @ np.abs(b)
    assert np.all(np.abs(cg - co) <= m * 1.2e-16 * magc)


@pytest.mark.parametrize("hpne", [False, True])
@pytest.mark.parametrize("col", [0, 21, 70, 99])
def test_factor_breakdown_reports_column(pne, orc, hpne, col):
    """A zero column j of A_p (A with column j zero, R = I) makes C singular
    at column j: the Cholesky reports 2000 + j + 1 and the LU 3000 + j + 1,
    as the oracle's factorizations do (columns in the first and in the
    second, partial, 64-column block, and inside a 16-column step)."""
    m, n = 1000, 100
    p = make_problem(m, n, 1e2, 1e-6, seed=1013)
    A = p.numpy_A().copy(order="F")
    A[:, col] = 0.0
    b = p.numpy_b()
    R = np.eye(n)
    Co, _ = orc.gram(A, A, b)
    if hpne:
        _, _, io = orc.lu(Co)
    else:
        _, io = orc.cholesky(Co)
    assert io == (3000 if hpne else 2000) + col + 1
    _, _, _, info = pne.pne_gram(dev(A), torch.from_numpy(b).cuda(), dev(R), hpne=hpne, factor=True)
    assert int(host(info)[0]) == io


def test_nan_entry_reports_breakdown(pne):
    """A non-finite entry in A: both solvers report a numerical failure and
    return NaN instead of a wrong x with info 0."""
    p = make_problem(900, 50, 1e3, 1e-4, seed=1012)
    A = p.numpy_A().copy(order="F")
    A[17, 9] = np.nan
    for fn in (pne.pne_solve, pne.hpne_solve):
        o = pne.make_opts(seed=1, sketch_prec="fp32", qr_prec="fp32", refine_steps=1)
        x, info, _ = fn(dev(A), torch.from_numpy(p.numpy_b()).cuda(), opts=o)
        assert int(host(info)[0]) != 0
        assert np.all(np.isnan(host(x)))


@pytest.mark.parametrize("scale", [1e6, 1e-6])
def test_fp16_preconditioner_any_scale(pne, orc, scale):
    """AUTO picks FP16 for kappa = 1e2 whatever the scale of A; the FP16 QR
    keeps R_s in range, so huge or tiny entries solve as accurately."""
    p = make_problem(3000, 100, 1e2, 1e-6, seed=1013)
    A, b, xs = p.numpy_A() * scale, p.numpy_b(), p.numpy_x_star() / scale
    err_qr = relerr(orc.qr_ls(A, b), xs)
    o = pne.make_opts(seed=2, sketch_prec="auto", qr_prec="auto", refine_steps=1)
    x, info, meta = pne.pne_solve(dev(A), torch.from_numpy(b).cuda(), opts=o)
    assert meta["qr_prec"] == "fp16"
    assert int(host(info)[0]) == 0
    assert relerr(host(x), xs) <= 10 * err_qr
    o16 = pne.make_opts(seed=2, sketch_prec="fp16", qr_prec="fp16", refine_steps=1)
    x, info, _ = pne.hpne_solve(dev(A), torch.from_numpy(b).cuda(), opts=o16)
    assert int(host(info)[0]) == 0
    assert relerr(host(x), xs) <= 10 * err_qr


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


def test_auto_picks_single_precision(pne, orc):
    """kappa = 3.5e3, n = 400: the estimate lands in the single-precision
    band (4 <= kappa0 <= 8), on the GPU as in the oracle.  The band is
    narrow for an FP32 Gram (its Cholesky breaks down from kappa ~ 4e3 on,
    which selects double), so the case sits just inside it.  There
    kappa(A)^2 u_32 is about 0.7: the rounding error of the FP32 Gram is of
    the size of its smallest eigenvalue, so the estimate depends on the
    summation order (MFMA blocks on the GPU, sequential sums in the oracle)
    by a few tenths in log10.  The pick is what must agree."""
    p = make_problem(4000, 400, 3.5e3, 1e-6, seed=1014)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    k0o, _, cho = orc.cond_est(A)
    assert cho == 2 and 4.2 < k0o < 7.8
    o = pne.make_opts(seed=1, sketch_prec="auto", qr_prec="auto", refine_steps=1)
    x, info, meta = pne.pne_solve(dev(A), torch.from_numpy(b).cuda(), opts=o)
    assert meta["sketch_prec"] == "fp32" and meta["qr_prec"] == "fp32"
    assert 4.0 <= meta["kappa0"] <= 8.0 and abs(meta["kappa0"] - k0o) < 0.6
    assert int(host(info)[0]) == 0
    assert relerr(host(x), xs) <= 10 * relerr(orc.qr_ls(A, b), xs)


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

def golden_err_qr():
    """name -> (m, n, kappa, rho, seed, err_qr) from tests/golden/err_qr_full_size.txt,
    written by tests/golden/make_err_qr.py (oracle QR solve on the CPU-generated problem)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "err_qr_full_size.txt")
    out = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            t = line.split()
            out[t[0]] = (int(t[1]), int(t[2]), float(t[3]), float(t[4]), int(t[5]), float(t[6]))
    return out


@pytest.fixture(scope="module")
def big():
    # generated on the CPU (as the stored oracle QR error was), then moved to the GPU
    p = make_problem(100_000, 1000, 1e6, 1e-4, seed=1002, device="cpu")
    p.At, p.b, p.x_star = p.At.cuda(), p.b.cuda(), p.x_star.cuda()
    return p


def test_full_size_sketch_sampled_entries(pne, orc, big):
    s = 3000
    As = host(pne.pne_sketch(big.A, s, seed=2, prec="bf16"))
    rng = np.random.default_rng(0)
    rows = rng.integers(0, s, 12)
    cols = rng.integers(0, 1000, 12)
    A = big.numpy_A()
    ref, ab = orc.sketch_entries(A, s, 2, rows, cols, prec="bf16")
    assert np.all(np.abs(As[rows, cols] - ref) <= SKETCH_TOL["bf16"] * ab)


@pytest.mark.parametrize("hpne,sk,qr,refine", [(False, "bf16", "fp32", 1), (False, "fp32", "fp32", 0),
                                                (False, "fp64", "fp64", 0), (True, "bf16", "fp32", 1),
                                                (True, "fp64", "fp64", 0)])
def test_full_size_accuracy(pne, big, hpne, sk, qr, refine):
    """m = 1e5, n = 1e3, kappa = 1e6, rho = 1e-4: error within 10x the oracle
    QR solver's own error on the same (CPU-generated) problem."""
    m, n, kappa, rho, seed, err_qr = golden_err_qr()["ls_100000x1000_k1e6"]
    assert (m, n, seed) == (big.m, big.n, big.seed)
    o = pne.make_opts(s=3000, seed=2, sketch_prec=sk, qr_prec=qr, refine_steps=refine)
    fn = pne.hpne_solve if hpne else pne.pne_solve
    x, info, _ = fn(big.A, big.b, opts=o)
    assert int(host(info)[0]) == 0
    err = relerr(host(x), host(big.x_star))
    assert err <= 10 * err_qr, (err, err_qr)


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
