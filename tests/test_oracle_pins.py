"""Pins for the CPU oracle: each check ties an oracle function to something other
than itself -- published known-answer vectors, library routines, exact rational
arithmetic, closed forms, the paper's worked outcomes and bounds.  CPU only."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.stats as sst
import torch

from workloads import make_problem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U64 = 2.0 ** -53


def relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(y))


# ---------------------------------------------------------------- generator

def test_philox_known_answers(orc):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = orc.philox4x32_10(v[0:4], v[4:6])
        assert [int(o) for o in out] == v[6:10]


def test_omega_is_standard_normal(orc):
    Om = orc.omega(seed=12345, s=16, m=8192)
    z = Om.ravel()
    assert abs(z.mean()) < 4.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 0.03
    assert sst.kstest(z, "norm").pvalue > 1e-3
    # rows produced by different counter words must be uncorrelated
    c = np.corrcoef(Om)
    off = c[~np.eye(c.shape[0], dtype=bool)]
    assert np.max(np.abs(off)) < 0.06


def test_omega_counter_layout(orc):
    # every entry depends on (seed, pid, i, j); changing any of them changes it
    base = orc.lib().oracle_omega_entry(7, 0, 5, 11)
    assert base == orc.lib().oracle_omega_entry(7, 0, 5, 11)
    for args in [(8, 0, 5, 11), (7, 1, 5, 11), (7, 0, 6, 11), (7, 0, 5, 12), (7 + (1 << 32), 0, 5, 11)]:
        assert orc.lib().oracle_omega_entry(*args) != base


# ---------------------------------------------------------------- rounding

def test_rounding_matches_library_conversions(orc):
    rng = np.random.default_rng(3)
    x32 = np.concatenate([rng.standard_normal(4000) * 10.0 ** rng.uniform(-6, 4, 4000),
                          [0.0, 1.0, -1.0, 2.0 ** -130, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9]]
                         ).astype(np.float32)
    xd = x32.astype(np.float64)
    ref_bf16 = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.round_to(xd, "bf16"), ref_bf16)
    ref_fp16 = x32.astype(np.float16).astype(np.float64)
    np.testing.assert_array_equal(orc.round_to(xd, "fp16"), ref_fp16)
    small = xd[np.abs(xd) <= 448.0]
    ref_e4m3 = torch.tensor(small.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    np.testing.assert_array_equal(orc.round_to(small, "fp8"), ref_e4m3)
    # e4m3 saturates instead of overflowing
    np.testing.assert_array_equal(orc.round_to(np.array([500.0, -1e6, 470.0]), "fp8"),
                                  [448.0, -448.0, 448.0])
    np.testing.assert_array_equal(orc.round_to(np.array([1e10]), "fp16"), [np.inf])


# ---------------------------------------------------------------- sketch

@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_sketch_elementwise_precisions(orc, prec):
    rng = np.random.default_rng(5)
    m, n, s = 300, 7, 13
    A = np.asfortranarray(rng.standard_normal((m, n)))
    Om = orc.omega(seed=99, s=s, m=m)
    if prec == "fp64":
        Oq, Aq = Om, A
    else:
        tdt = torch.float32 if prec == "fp32" else torch.bfloat16
        cv = lambda M: torch.tensor(M.astype(np.float32)).to(tdt).to(torch.float64).numpy()
        Oq, Aq = cv(Om), cv(A)
    ref = (Oq @ Aq) / math.sqrt(s)
    got = orc.sketch(A, s, seed=99, prec=prec)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * float((np.abs(Oq) @ np.abs(Aq)).max()))


@pytest.mark.parametrize("prec", ["fp16", "fp8"])
def test_sketch_block_scaled(orc, prec):
    rng = np.random.default_rng(6)
    m, n, s, br = 300, 5, 9, 128     # 300 rows: two full blocks and a ragged one
    A = rng.standard_normal((m, n)) * np.array([1.0, 1e-6, 1e3, 2.0 ** -20, 7.0])
    A[130:256, 3] = 0.0               # an all-zero block
    A = np.asfortranarray(A)
    Om = orc.omega(seed=4, s=s, m=m)
    A32 = torch.tensor(A.astype(np.float32))
    if prec == "fp16":
        Oq = torch.tensor(Om.astype(np.float32)).to(torch.float16).to(torch.float64)
    else:
        Oq = torch.tensor(Om.astype(np.float32)).clamp(-448, 448).to(torch.float8_e4m3fn).to(torch.float64)
    ref = torch.zeros(s, n, dtype=torch.float64)
    for k0 in range(0, m, br):
        blk = A32[k0:k0 + br]
        amax = blk.abs().max(dim=0).values
        if prec == "fp16":
            e = torch.floor(torch.log2(amax.double()))
            scale = torch.where(amax > 0, 2.0 ** (e - 14), torch.zeros_like(e)).float()
        else:
            scale = torch.where(amax > 0, amax / 448.0, torch.zeros_like(amax))
        safe = torch.where(scale > 0, scale, torch.ones_like(scale))
        t = blk / safe
        if prec == "fp16":
            q = t.to(torch.float16).to(torch.float64)
        else:
            q = t.clamp(-448, 448).to(torch.float8_e4m3fn).to(torch.float64)
        q = torch.where(scale > 0, q, torch.zeros_like(q))
        ref += (Oq[:, k0:k0 + br] @ q) * scale.double()
    ref = ref.numpy() / math.sqrt(s)
    got = orc.sketch(A, s, seed=4, prec=prec, block_rows=br)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-300)


def _lib_round(M, prec):
    """Library conversion of float64 values through FP32 to the operand format."""
    t = torch.tensor(np.asarray(M, dtype=np.float64).astype(np.float32))
    if prec == "fp64":
        return torch.tensor(np.asarray(M, dtype=np.float64))
    if prec == "fp32":
        return t.to(torch.float64)
    if prec == "bf16":
        return t.to(torch.bfloat16).to(torch.float64)
    if prec == "fp16":
        return t.to(torch.float16).to(torch.float64)
    return t.clamp(-448, 448).to(torch.float8_e4m3fn).to(torch.float64)


def _explicit_sketch(orc, A, s, seed, prec, br=128):
    """Omega A / sqrt(s) and |Omega_q| |A_q| scale / sqrt(s) with the oracle's
    Omega, operands rounded by the torch conversions and the per-block scales
    of the FP16/FP8 formats formed here."""
    m, n = A.shape
    Om = orc.omega(seed=seed, s=s, m=m)
    Oq = _lib_round(Om, prec)
    if prec not in ("fp16", "fp8"):
        Aq = _lib_round(A, prec)
        return ((Oq @ Aq) / math.sqrt(s)).numpy(), ((Oq.abs() @ Aq.abs()) / math.sqrt(s)).numpy()
    A32 = torch.tensor(A.astype(np.float32))
    ref = torch.zeros(s, n, dtype=torch.float64)
    ab = torch.zeros(s, n, dtype=torch.float64)
    for k0 in range(0, m, br):
        blk = A32[k0:k0 + br]
        amax = blk.abs().max(dim=0).values
        if prec == "fp16":
            e = torch.floor(torch.log2(amax.double()))
            scale = torch.where(amax > 0, 2.0 ** (e - 14), torch.zeros_like(e)).float()
        else:
            scale = torch.where(amax > 0, amax / 448.0, torch.zeros_like(amax))
        safe = torch.where(scale > 0, scale, torch.ones_like(scale))
        t = blk / safe
        q = t.to(torch.float16) if prec == "fp16" else t.clamp(-448, 448).to(torch.float8_e4m3fn)
        q = torch.where(scale > 0, q.to(torch.float64), torch.zeros(q.shape, dtype=torch.float64))
        ref += (Oq[:, k0:k0 + br] @ q) * scale.double()
        ab += (Oq[:, k0:k0 + br].abs() @ q.abs()) * scale.double()
    return ref.numpy() / math.sqrt(s), ab.numpy() / math.sqrt(s)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16", "fp16", "fp8"])
def test_sketch_entries_match_explicit_product(orc, prec):
    """The entry-by-entry sketch (used at full size, where the whole product is
    too slow on the CPU) against the explicit product with library-rounded
    operands: 300 rows (two full 128-row blocks and a ragged one), columns of
    very different scales and an all-zero block."""
    rng = np.random.default_rng(55)
    m, n, s, br = 300, 5, 9, 128
    A = rng.standard_normal((m, n)) * np.array([1.0, 1e-6, 1e3, 2.0 ** -20, 7.0])
    A[130:256, 3] = 0.0
    A[256:, 1] = 0.0                  # the ragged block of column 1 is zero too
    A = np.asfortranarray(A)
    ref, ab = _explicit_sketch(orc, A, s, 17, prec, br)
    rows, cols = np.meshgrid(np.arange(s), np.arange(n), indexing="ij")
    got, got_abs = orc.sketch_entries(A, s, 17, rows.ravel(), cols.ravel(), prec=prec, block_rows=br)
    np.testing.assert_allclose(got, ref.ravel(), rtol=0, atol=1e-12 * ab.ravel().max())
    assert np.all(np.abs(got - ref.ravel()) <= 1e-11 * np.abs(ref.ravel()) + 1e-13 * ab.ravel())
    np.testing.assert_allclose(got_abs, ab.ravel(), rtol=1e-12, atol=0)


def test_sketch_subspace_embedding(orc):
    # For orthonormal U the sketch Omega U / sqrt(s) has singular values in
    # [1 - sqrt(n/s), 1 + sqrt(n/s)] up to fluctuations (Marchenko-Pastur).
    rng = np.random.default_rng(8)
    m, n, s = 4000, 40, 120
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    sv = np.linalg.svd(orc.sketch(np.asfortranarray(U), s, seed=3), compute_uv=False)
    lo, hi = 1 - math.sqrt(n / s), 1 + math.sqrt(n / s)
    assert 0.75 * lo < sv.min() and sv.max() < 1.15 * hi


# ---------------------------------------------------------------- QR pieces

def test_householder_r_matches_lapack(orc):
    rng = np.random.default_rng(9)
    W = rng.standard_normal((60, 25)) @ np.diag(np.logspace(0, -6, 25))
    R = orc.householder_r(W)
    Rl = np.linalg.qr(W, mode="r")
    sg = np.sign(np.diag(Rl)) * np.sign(np.diag(R))
    np.testing.assert_allclose(R, sg[:, None] * Rl, rtol=0, atol=1e-13)
    assert np.all(np.tril(R, -1) == 0)
    # LAPACK sign convention: beta = -sign(alpha) ||x||
    W2 = np.array([[3.0, 1.0], [4.0, 2.0], [0.0, 5.0]])
    R2 = orc.householder_r(W2)
    assert R2[0, 0] == pytest.approx(-5.0)


def _exact_ls(A, b):
    """Least squares by exact rational arithmetic on A^T A x = A^T b."""
    m, n = len(A), len(A[0])
    M = [[sum(Fraction(A[k][i]) * Fraction(A[k][j]) for k in range(m)) for j in range(n)]
         + [sum(Fraction(A[k][i]) * Fraction(b[k]) for k in range(m))] for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] / M[i][i] for i in range(n)]


def _tiny_cases():
    rng = np.random.default_rng(10)
    out = []
    while len(out) < 12:
        m = int(rng.integers(2, 7))
        n = int(rng.integers(1, min(m, 3) + 1))
        A = rng.integers(-5, 6, size=(m, n)).astype(float)
        if np.linalg.matrix_rank(A) < n:
            continue
        b = rng.integers(-9, 10, size=m).astype(float)
        out.append((A, b))
    return out


def test_qr_ls_exact_rational(orc):
    for A, b in _tiny_cases():
        xe = np.array([float(v) for v in _exact_ls(A.tolist(), b.tolist())])
        x = orc.qr_ls(A, b)
        assert np.allclose(x, xe, rtol=1e-13, atol=1e-13 * np.abs(xe).max())


@pytest.mark.parametrize("hpne", [False, True])
def test_pne_hpne_exact_rational(orc, hpne):
    # In exact arithmetic PNE and HPNE give the least-squares solution for any
    # nonsingular R_s; with FP64 throughout they must agree to rounding.
    for A, b in _tiny_cases():
        m, n = A.shape
        xe = np.array([float(v) for v in _exact_ls(A.tolist(), b.tolist())])
        r = orc.solve(A, b, hpne=hpne, s=max(3 * n, m), seed=2)
        assert r["info"] == 0
        assert np.allclose(r["x"], xe, rtol=1e-11, atol=1e-11 * np.abs(xe).max())


def test_qr_ls_error_obeys_lemma(orc):
    # Lemma 1.1: error <= kappa eps (1 + kappa * residual), eps ~ rounding of A
    for kappa, rho in [(1e2, 1e-2), (1e4, 1e-6), (1e6, 1e-3)]:
        p = make_problem(800, 40, kappa, rho, seed=11)
        x = orc.qr_ls(p.numpy_A(), p.numpy_b())
        err = relerr(x, p.numpy_x_star())
        bound = kappa * U64 * (1 + kappa * rho)
        assert err <= 50 * math.sqrt(800 * 40) * bound
        assert err >= 1e-3 * bound or err < 1e-14


def test_qr_ls_matches_lstsq(orc):
    p = make_problem(2000, 60, 1e5, 1e-5, seed=12)
    A, b = p.numpy_A(), p.numpy_b()
    x = orc.qr_ls(A, b)
    xl = np.linalg.lstsq(A, b, rcond=None)[0]
    assert relerr(x, xl) < 1e5 * 1e-14


# ---------------------------------------------------------------- A_p, Gram, factorizations

def test_precondition_matches_triangular_solve(orc):
    rng = np.random.default_rng(13)
    A = np.asfortranarray(rng.standard_normal((200, 30)))
    R = np.triu(rng.standard_normal((30, 30))) + 5 * np.eye(30)
    Ap, info = orc.precondition(A, R)
    assert info == 0
    ref = sla.solve_triangular(R, A.T, trans="T", lower=False).T  # A R^{-1}
    np.testing.assert_allclose(Ap, ref, rtol=1e-12, atol=1e-13)
    R[7, 7] = 0.0
    assert orc.precondition(A, R)[1] == 1008


def test_gram_matches_matmul(orc):
    rng = np.random.default_rng(14)
    X, Y = rng.standard_normal((150, 12)), rng.standard_normal((150, 12))
    b = rng.standard_normal(150)
    C, c = orc.gram(X, Y, b)
    np.testing.assert_allclose(C, X.T @ Y, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(c, X.T @ b, rtol=1e-13, atol=1e-12)


def test_cholesky_matches_lapack_and_breakdown(orc):
    rng = np.random.default_rng(15)
    M = rng.standard_normal((40, 20))
    C = M.T @ M
    L, info = orc.cholesky(C)
    assert info == 0
    np.testing.assert_allclose(L, np.linalg.cholesky(C), rtol=1e-12, atol=1e-12)
    D = np.diag([4.0, 1.0, -1.0, 2.0])
    assert orc.cholesky(D)[1] == 2003
    y = orc.cholesky_solve(L, np.arange(20.0))
    np.testing.assert_allclose(y, np.linalg.solve(C, np.arange(20.0)), rtol=1e-10)


def test_lu_matches_lapack(orc):
    rng = np.random.default_rng(16)
    C = rng.standard_normal((25, 25))
    LU, piv, info = orc.lu(C)
    assert info == 0
    lu_ref, piv_ref = sla.lu_factor(C)
    np.testing.assert_array_equal(piv, piv_ref)
    np.testing.assert_allclose(LU, lu_ref, rtol=1e-12, atol=1e-12)
    c = rng.standard_normal(25)
    np.testing.assert_allclose(orc.lu_solve(LU, piv, c), np.linalg.solve(C, c), rtol=1e-10)
    # ties: the first row of largest magnitude is the pivot (LAPACK i?amax)
    T = np.array([[1.0, 2.0, 0.0], [-1.0, 1.0, 1.0], [1.0, 0.0, 3.0]])
    _, pt, _ = orc.lu(T)
    assert pt[0] == 0
    _, pz, iz = orc.lu(np.array([[0.0, 1.0], [0.0, 2.0]]))
    assert iz == 3001


def test_upper_solve(orc):
    rng = np.random.default_rng(17)
    R = np.triu(rng.standard_normal((15, 15))) + 3 * np.eye(15)
    y = rng.standard_normal(15)
    x, info = orc.upper_solve(R, y)
    assert info == 0
    np.testing.assert_allclose(x, sla.solve_triangular(R, y), rtol=1e-12)
    R[4, 4] = 0.0
    x, info = orc.upper_solve(R, y)
    assert info == 1005 and np.all(np.isnan(x))


# ---------------------------------------------------------------- Algorithm 1 end to end

def test_pne_hpne_agree_with_qr_solver(orc):
    # Section 7.2: in double precision PNE/HPNE are as accurate as the QR
    # solver once the relative residual exceeds 1e-4 (m = 6000, n = 100,
    # kappa = 1e4).
    for rho in [1e-3, 1e-1]:
        p = make_problem(6000, 100, 1e4, rho, seed=20)
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        eq = relerr(orc.qr_ls(A, b), xs)
        for hpne in (False, True):
            r = orc.solve(A, b, hpne=hpne, s=300, seed=1)
            assert r["info"] == 0
            assert relerr(r["x"], xs) <= 3 * eq + 1e-15


def test_mixed_fp32_preconditioner_accuracy(orc):
    # Section 7.3: with a single precision preconditioner at kappa = 1e8 the
    # error is within about a factor 100 of the QR solver for small residuals
    # and as accurate for large ones.
    for rho, factor in [(1e-8, 300.0), (1e-2, 5.0)]:
        p = make_problem(6000, 100, 1e8, rho, seed=21)
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        eq = relerr(orc.qr_ls(A, b), xs)
        for hpne in (False, True):
            r = orc.solve(A, b, hpne=hpne, s=300, seed=1, sketch_prec="fp32", qr_prec="fp32")
            assert r["info"] == 0
            assert relerr(r["x"], xs) <= factor * eq


def test_kappa_Ap_closed_form(orc):
    # Gaussian sketch, s = 3n, exact preconditioner: kappa(A_p) = kappa(Omega U),
    # asymptotically (1 + sqrt(1/3)) / (1 - sqrt(1/3)) = 3.73.
    p = make_problem(3000, 60, 1e6, 1e-6, seed=22)
    A = p.numpy_A()
    r = orc.solve(A, p.numpy_b(), s=180, seed=5)
    Ap, info = orc.precondition(A, r["R"])
    sv = np.linalg.svd(Ap, compute_uv=False)
    assert 2.0 < sv[0] / sv[-1] < 6.0


def test_rscond_lemma_for_fp32_preconditioner(orc):
    # Lemma 5.1: kappa(A R1^{-1}) <= kappa(A_p) (1 + e k(R_s)) / (1 - e k(R_s))
    p = make_problem(3000, 60, 1e5, 1e-6, seed=23)
    A, b = p.numpy_A(), p.numpy_b()
    R64 = orc.solve(A, b, s=180, seed=5)["R"]
    R32 = orc.solve(A, b, s=180, seed=5, sketch_prec="fp32", qr_prec="fp32")["R"]
    kap = lambda M: (lambda sv: sv[0] / sv[-1])(np.linalg.svd(M, compute_uv=False))
    k_ap = kap(orc.precondition(A, R64)[0])
    k_a1 = kap(orc.precondition(A, R32)[0])
    eps = np.linalg.norm(R32 - R64, 2) / np.linalg.norm(R64, 2)
    ek = eps * kap(R64)
    assert ek < 1
    assert k_a1 <= k_ap * (1 + ek) / (1 - ek) * 1.0001


def test_refinement_restores_accuracy(orc):
    p = make_problem(3000, 50, 1e6, 1e-4, seed=24)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    eq = relerr(orc.qr_ls(A, b), xs)
    r0 = orc.solve(A, b, s=150, seed=1, sketch_prec="bf16", qr_prec="fp32", refine_steps=0)
    r2 = orc.solve(A, b, s=150, seed=1, sketch_prec="bf16", qr_prec="fp32", refine_steps=2)
    assert relerr(r0["x"], xs) > 10 * eq       # the BF16 preconditioner alone is not enough
    assert relerr(r2["x"], xs) <= 10 * eq      # two FP64 corrections are


def test_hpne_refinement_restores_accuracy(orc):
    """HPNE branch of the refinement: the correction solves the HPNE system
    with right-hand side A_p^T r (LU factors reused)."""
    p = make_problem(3000, 50, 1e6, 1e-4, seed=24)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    eq = relerr(orc.qr_ls(A, b), xs)
    r0 = orc.solve(A, b, hpne=True, s=150, seed=1, sketch_prec="bf16", qr_prec="fp32", refine_steps=0)
    r2 = orc.solve(A, b, hpne=True, s=150, seed=1, sketch_prec="bf16", qr_prec="fp32", refine_steps=2)
    assert r0["info"] == 0 and r2["info"] == 0
    assert relerr(r0["x"], xs) > 10 * eq
    assert relerr(r2["x"], xs) <= 10 * eq
    # one refinement step is one step of the stationary iteration x += M^{-1} A_p^T (b - A x)
    # with M = A_p^T A: check the first step against that definition done with LAPACK
    Ap, _ = orc.precondition(A, r0["R"])
    M = Ap.T @ A
    x1 = orc.solve(A, b, hpne=True, s=150, seed=1, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)["x"]
    x1_ref = r0["x"] + np.linalg.solve(M, Ap.T @ (b - A @ r0["x"]))
    assert relerr(x1, x1_ref) <= 1e-3 * relerr(r0["x"], xs)


def _r_up_to_signs(R, Rref, ulp):
    sg = np.sign(np.diag(R)) * np.sign(np.diag(Rref))
    d = np.abs(R - sg[:, None] * Rref)
    # equal except where the two factorizations' rounding straddles a tie of the narrow format
    assert np.mean(d == 0) > 0.95
    assert np.all(d <= ulp * np.abs(Rref) + 1e-300)


@pytest.mark.parametrize("prec,ulp", [("bf16", 2.0 ** -7), ("fp16", 2.0 ** -10)])
def test_low_precision_qr_path(orc, prec, ulp):
    """qr_prec = BF16/FP16: A_s is rounded to the format (FP16 after an exact
    power-of-two scaling), factorized, R_s rounded to the format and the
    scale divided out.  Reference: LAPACK's QR of the library-rounded
    sketch."""
    p = make_problem(600, 20, 1e2, 1e-6, seed=25)
    A, b = p.numpy_A(), p.numpy_b()
    s = 60
    As = orc.sketch(A, s, seed=3, prec=prec)
    c = orc.fp16_qr_scale(As) if prec == "fp16" else 1.0
    Aq = _lib_round(As * c, prec).numpy() if prec == "bf16" else \
        torch.tensor((As.astype(np.float32).astype(np.float64) * c).astype(np.float32)).to(torch.float16).double().numpy()
    Rl = np.linalg.qr(Aq, mode="r")
    Rref = _lib_round(Rl, prec).numpy() / c
    R = orc.solve(A, b, s=s, seed=3, sketch_prec=prec, qr_prec=prec)["R"]
    _r_up_to_signs(R, Rref, ulp)


def test_fp16_qr_scale_properties(orc):
    """The FP16 QR scale is a power of two that brings max |A_s| into
    [2^(k-1), 2^k) with k = 14 - ceil(log4 s), so every column norm of the
    scaled sketch (and every entry of R_s) stays below 2^14 < 65504."""
    rng = np.random.default_rng(26)
    for s, n, mag in [(60, 20, 1.0), (3000, 40, 1e9), (300, 100, 1e-9), (257, 3, 3.0)]:
        As = rng.standard_normal((s, n)) * mag
        c = orc.fp16_qr_scale(As)
        m, e = math.frexp(c)
        assert m == 0.5                                  # a power of two
        k = 14 - math.ceil(math.log(s, 4) - 1e-12)
        amax = np.abs(As.astype(np.float32)).max() * c
        assert 2.0 ** (k - 1) <= amax < 2.0 ** k
        assert np.linalg.norm(As * c, axis=0).max() < 2.0 ** 14
        assert orc.fp16_qr_scale(As * 2.0 ** 20) == c * 2.0 ** -20
    assert orc.fp16_qr_scale(np.zeros((10, 2))) == 1.0


def test_fp16_preconditioner_is_scale_invariant(orc):
    """Algorithm 1 picks u_p from kappa alone: a well-conditioned problem with
    huge or tiny entries solves with the FP16 preconditioner as accurately as
    the unscaled one (x scales with 1/c for A -> c A)."""
    p = make_problem(2000, 40, 1e2, 1e-6, seed=27)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    for c in (1.0, 1e6, 1e-6):
        eq = relerr(orc.qr_ls(c * A, b), xs / c)
        r = orc.solve(c * A, b, s=120, seed=1, sketch_prec="fp16", qr_prec="fp16", refine_steps=2)
        assert r["info"] == 0
        assert np.all(np.isfinite(r["R"]))
        assert relerr(r["x"], xs / c) <= 10 * eq


def test_lu_nan_pivot_reports_breakdown(orc):
    C = np.array([[2.0, 1.0, 0.0], [1.0, np.nan, 1.0], [0.0, 1.0, 3.0]])
    _, piv, info = orc.lu(C)
    assert info == 3002
    assert np.all((piv >= 0) & (piv < 3))
    C2 = np.array([[np.nan, 1.0], [5.0, 2.0]])
    assert orc.lu(C2)[2] == 3001


# ---------------------------------------------------------------- condition estimate

def _golden_selection():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "precision_selection.txt"))
            if l.strip() and not l.startswith("#")]
    return [(float(k), int(n), int(c)) for k, n, c in rows]


@pytest.mark.parametrize("kappa,n,code", _golden_selection())
def test_precision_pick_worked_cases(orc, kappa, n, code):
    p = make_problem(10 * n, n, kappa, 1e-6, seed=30)
    k0, k0n, ch = orc.cond_est(p.numpy_A())
    assert ch == code


def test_cond_est_is_a_good_lower_estimate(orc):
    # Hager's estimate never exceeds the 1-norm of the inverse (in exact
    # arithmetic; the FP32 solves perturb it by about u32 kappa(G), so the
    # strict check uses kappa(A) <= 3e2) and is within a factor 10 of it.
    for kappa in [1e1, 1e2, 3e2, 3e3]:
        p = make_problem(2000, 50, kappa, 1e-6, seed=31)
        A32 = p.numpy_A().astype(np.float32).astype(np.float64)
        G = A32.T @ A32
        exact = 0.5 * math.log10(np.abs(G).sum(0).max() * np.abs(np.linalg.inv(G)).sum(0).max())
        k0, k0n, ch = orc.cond_est(p.numpy_A())
        slack = 1e-3 if kappa <= 3e2 else 0.5 * math.log10(1 + 2 ** -23 * kappa ** 2)
        assert k0 <= exact + slack
        assert k0 >= exact - 0.5
        assert k0n == pytest.approx(k0 + 0.5 * math.log10(50), abs=1e-4)
        # the 2-norm condition number sits below the 1-norm bound with factor n
        assert math.log10(kappa) <= k0n + 0.05


@pytest.mark.parametrize("kind", ["diagonal", "laplacian"])
def test_cond_est_exact_where_hager_is_exact(orc, kind):
    """Hager's 1-norm estimate is exact when the inverse has no sign changes
    it could miss: for a diagonal G it returns max 1 / G_ii, and for an
    inverse-positive G (the 1D Laplacian tridiag(-1, 2, -1), an M-matrix)
    the first sign vector is all ones, so the next iterate picks the largest
    column sum of G^{-1} exactly.  A is built so that G = fl32(A)^T fl32(A)
    is that matrix (up to the FP32 rounding of A), and kappa0 must equal
    (1/2) log10(||G||_1 ||G^{-1}||_1) to FP32 accuracy."""
    n, m = 40, 120
    if kind == "diagonal":
        d = np.geomspace(1.0, 1e-3, n)
        A = np.zeros((m, n))
        A[:n, :n] = np.diag(d)
    else:
        T = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
        A = np.zeros((m, n))
        A[:n, :n] = np.linalg.cholesky(T).T
    A32 = A.astype(np.float32).astype(np.float64)
    G = A32.T @ A32
    Gi = np.linalg.inv(G)
    if kind == "laplacian":
        assert np.all(Gi > 0)
    exact = 0.5 * math.log10(np.abs(G).sum(0).max() * np.abs(Gi).sum(0).max())
    k0, _, _ = orc.cond_est(A)
    assert k0 == pytest.approx(exact, abs=2e-4)


def test_known_kappa_thresholds(orc):
    A = np.eye(3)
    assert orc.cond_est(A, known_kappa=1e2)[2] == 3
    assert orc.cond_est(A, known_kappa=1e4)[2] == 2      # kappa0 = 4 is not < 4
    assert orc.cond_est(A, known_kappa=1e8)[2] == 2      # kappa0 = 8 is <= 8
    assert orc.cond_est(A, known_kappa=1.1e8)[2] == 1


def test_invalid_arguments(orc):
    A = np.ones((3, 4))
    with pytest.raises(ValueError):
        orc.qr_ls(A, np.ones(3))
    assert orc.solve(np.eye(4), np.ones(4), s=2)["info"] == -1


# ---------------------------------------------------------------- not-normal equations (Section 5.2)

def _exact_nne(A, B, b):
    """B^T A x = B^T b solved in exact rational arithmetic (Gauss-Jordan)."""
    m, n = len(A), len(A[0])
    M = [[sum(Fraction(B[k][i]) * Fraction(A[k][j]) for k in range(m)) for j in range(n)]
         + [sum(Fraction(B[k][i]) * Fraction(b[k]) for k in range(m))] for i in range(n)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        M[c] = [v / M[c][c] for v in M[c]]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c]
                M[r] = [a - f * bb for a, bb in zip(M[r], M[c])]
    return [M[i][n] for i in range(n)]


def test_nne_exact_rational_equals_least_squares(orc):
    # For B = A C' with C' nonsingular the not-normal equations have the
    # least-squares solution (Section 5.2, proof of the theorem: A = B C).
    rng = np.random.default_rng(77)
    for A, b in _tiny_cases():
        m, n = A.shape
        Cp = np.triu(rng.integers(1, 4, size=(n, n))).astype(float)   # nonsingular upper triangle
        B = A @ Cp                        # integer B with the column space of A
        fe = _exact_nne(A.tolist(), B.tolist(), b.tolist())
        assert fe == list(_exact_ls(A.tolist(), b.tolist()))             # exactly x_LS
        xe = np.array([float(v) for v in fe])
        x, info = orc.nne(A, B, b)
        assert info == 0
        assert np.allclose(x, xe, rtol=1e-11, atol=1e-11 * np.abs(xe).max())


def test_nne_with_preconditioned_b_is_the_hpne(orc):
    # Remark in Section 5.2: B = A_p gives the HPNE; the oracle takes the same
    # arithmetic steps, so the results agree bit for bit.
    p = make_problem(600, 40, 1e5, 1e-6, seed=78)
    A, b = p.numpy_A(), p.numpy_b()
    r = orc.solve(A, b, hpne=True, s=120, seed=3, sketch_prec="fp64", refine_steps=0)
    Ap, rc = orc.precondition(A, r["R"])
    assert rc == 0
    x, info = orc.nne(A, Ap, b)
    assert info == 0 and np.array_equal(x, r["x"])
    # and one refinement step of each is the same correction
    r1 = orc.solve(A, b, hpne=True, s=120, seed=3, sketch_prec="fp64", refine_steps=1)
    x1, _ = orc.nne(A, Ap, b, refine_steps=1)
    assert np.array_equal(x1, r1["x"])


def test_nne_obeys_perturbation_theorem(orc):
    # Theorem (Section 5.2): ||x^ - x*|| / ||x^|| <= kappa(B^T A) nu (eps_B res + (1 + eps_B) eps_A)
    # with nu = ||B|| ||A|| / ||B^T A||.  The computed B^T A and B^T b have
    # backward errors of order m u in A and B; the check takes eps = 4 m u.
    rng = np.random.default_rng(79)
    for kappa, rho in [(1e3, 1e-8), (1e5, 1e-4), (1e6, 1e-2)]:
        p = make_problem(800, 30, kappa, rho, seed=int(kappa) % 1000 + 80)
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        B = A @ (np.eye(30) + 0.3 * rng.standard_normal((30, 30)))
        x, info = orc.nne(A, B, b)
        assert info == 0
        BtA = B.T @ A
        nu = np.linalg.norm(B, 2) * np.linalg.norm(A, 2) / np.linalg.norm(BtA, 2)
        res = np.linalg.norm(A @ x - b) / (np.linalg.norm(A, 2) * np.linalg.norm(x))
        eps = 4 * 800 * U64
        bound = np.linalg.cond(BtA) * nu * (eps * res + (1 + eps) * eps)
        err = np.linalg.norm(x - xs) / np.linalg.norm(x)
        assert err <= bound, (kappa, err, bound)


def test_nne_detects_wrong_operand_order(orc):
    # A^T B x = A^T b (operands swapped) is a different system when B is not
    # a multiple of A: the oracle must not be symmetric in A and B.
    p = make_problem(300, 12, 1e2, 1e-2, seed=81)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    rng = np.random.default_rng(81)
    B = A @ (np.eye(12) + 0.5 * rng.standard_normal((12, 12)))
    x, _ = orc.nne(A, B, b)
    xw = np.linalg.solve(A.T @ B, A.T @ b)
    assert relerr(x, xs) < 1e-10 * 1e2
    assert relerr(x, xw) > 1e-6


def test_nne_zero_pivot(orc):
    A = np.array([[1.0, 0.0], [0.0, 1.0], [0.0, 0.0]])
    B = np.array([[1.0, 0.0], [0.0, 0.0], [0.0, 0.0]])       # B^T A singular
    x, info = orc.nne(A, B, np.ones(3))
    assert info == 3002 and np.all(np.isnan(x))


# ---------------------------------------------------------------- QR-based condition estimate

@pytest.mark.parametrize("kappa,code", [(1e2, 3), (1e5, 2), (1e6, 2), (1e10, 1)])
def test_cond_est_qr_picks(orc, kappa, code):
    # kappa = 1e2 -> half and 1e10 -> double (Section 7.4, Figure 7), and the
    # single-precision band of Algorithm 1 is reached for kappa well above the
    # ~4e3 where the FP32 Gram estimate breaks down.
    p = make_problem(4000, 100, kappa, 1e-6, seed=82)
    k0, ch = orc.cond_est_qr(p.numpy_A(), seed=4)
    assert ch == code, (kappa, k0)
    if kappa >= 1e5:
        assert orc.cond_est(p.numpy_A())[2] == 1     # the Gram estimate cannot see it


def test_cond_est_qr_is_a_good_lower_estimate(orc):
    # Hager's estimate never exceeds ||R^{-1}||_1 (FP32 solves perturb it by
    # about u32 kappa) and is within a factor 10 of it; R is recomputed here
    # from the same FP32 sketch by LAPACK in FP64.
    for kappa in [1e1, 1e3, 1e5]:
        p = make_problem(3000, 60, kappa, 1e-6, seed=83)
        A = p.numpy_A()
        As = orc.sketch(A, 180, 5, prec="fp32").astype(np.float32).astype(np.float64)
        R = np.linalg.qr(As, mode="r")
        exact = math.log10(np.abs(R).sum(0).max() * np.abs(np.linalg.inv(R)).sum(0).max())
        k0, _ = orc.cond_est_qr(A, s=180, seed=5)
        assert exact - 1.0 <= k0 <= exact + math.log10(1 + 2 ** -22 * kappa * 60)
        # and kappa_1(R) brackets kappa_2(A) up to the sketch distortion and the
        # 1-norm / 2-norm factor n
        assert math.log10(kappa) - 0.6 <= exact <= math.log10(kappa) + 0.6 + math.log10(60)


def test_cond_est_qr_overflow_is_double(orc):
    A = np.zeros((50, 5))
    A[:, :4] = np.random.default_rng(84).standard_normal((50, 4))   # rank 4
    k0, ch = orc.cond_est_qr(A, seed=1)
    assert ch == 1 and (not math.isfinite(k0) or k0 > 8)


# ---------------------------------------------------------------- SRFT sketch (Section 6.2, eq. e_sketch)

def test_next_smooth_is_minimal_7_smooth(orc):
    def smooth(x):
        for p in (2, 3, 5, 7):
            while x % p == 0:
                x //= p
        return x == 1
    for m in list(range(1, 600)) + [1999, 4097, 100003, 999983]:
        mp = orc.next_smooth(m)
        assert mp >= m and smooth(mp)
        assert all(not smooth(x) for x in range(m, mp))


@pytest.mark.parametrize("m,prec", [(60, "fp64"), (97, "fp64"), (250, "fp32"), (131, "bf16")])
def test_srft_matches_dense_hartley_product(orc, m, prec):
    """The oracle's SRFT equals (1/sqrt(s)) S H D A with H = Re(F) - Im(F)
    formed from numpy's FFT of the identity (F_kj = exp(-2 pi i k j / m')),
    the zero-padded rows dropped, and A rounded by torch's conversions."""
    rng = np.random.default_rng(m)
    A = rng.standard_normal((m, 7)) * 10.0 ** rng.uniform(-3, 3, size=7)
    s = 40
    mp = orc.next_smooth(m)
    D = orc.srft_signs(11, mp, pid=2)
    k = orc.srft_indices(11, s, mp, pid=2)
    F = np.fft.fft(np.eye(mp))
    H = F.real - F.imag
    Om = H[k][:, :m] * D[:m] / math.sqrt(s)
    Aq = A
    if prec == "fp32":
        Aq = A.astype(np.float32).astype(np.float64)
    elif prec == "bf16":
        Aq = torch.tensor(A, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    ref = Om @ Aq
    got = orc.srft_sketch(A, s, 11, prec=prec, pid=2)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    # H / sqrt(m') is orthogonal (the Hartley transform is an involution up to m')
    assert np.allclose(H @ H, mp * np.eye(mp), atol=1e-9 * mp)


def test_srft_sampling_and_signs(orc):
    mp = 997 * 1 + 3          # 1000 bins
    mp = orc.next_smooth(mp)
    k = orc.srft_indices(5, 40000, mp)
    assert k.min() >= 0 and k.max() < mp
    counts = np.bincount(k, minlength=mp)
    chi2 = ((counts - 40000 / mp) ** 2 / (40000 / mp)).sum()
    assert sst.chi2.sf(chi2, mp - 1) > 1e-3
    d = orc.srft_signs(5, 20000)
    assert set(np.unique(d)) == {-1.0, 1.0} and abs(d.mean()) < 4 / math.sqrt(20000)
    assert not np.array_equal(orc.srft_signs(5, 256, pid=1), orc.srft_signs(5, 256, pid=0))
    assert not np.array_equal(orc.srft_indices(6, 50, mp), orc.srft_indices(5, 50, mp))


def test_srft_subspace_embedding(orc):
    """Section 6.2: with d = 3n sampled rows the preconditioned matrix tends
    to have kappa(A_p) <~ 10; kappa(A_p) = kappa(Omega U) for the orthonormal
    basis U of range(A)."""
    rng = np.random.default_rng(33)
    for m, n in [(2000, 50), (3000, 100)]:
        U = np.linalg.qr(rng.standard_normal((m, n)))[0]
        Y = orc.srft_sketch(U, 3 * n, 9)
        sv = np.linalg.svd(Y, compute_uv=False)
        assert sv[0] / sv[-1] < 10.0, sv[0] / sv[-1]
        # a coherent basis (columns of the identity) is spread by H D as well
        E = np.eye(m)[:, :n]
        sv = np.linalg.svd(orc.srft_sketch(E, 3 * n, 9), compute_uv=False)
        assert sv[0] / sv[-1] < 10.0


@pytest.mark.parametrize("prec,refine", [("fp64", 0), ("fp32", 1), ("bf16", 1)])
def test_pne_hpne_with_srft_sketch(orc, prec, refine):
    p = make_problem(3000, 100, 1e6, 1e-6, seed=44)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    err_qr = relerr(orc.qr_ls(A, b), xs)
    qr_prec = "fp64" if prec == "fp64" else "fp32"
    for hpne in (False, True):
        r = orc.solve(A, b, hpne=hpne, s=300, seed=3, sketch_prec=prec, qr_prec=qr_prec, refine_steps=refine,
                      sketch_kind="srft")
        assert r["info"] == 0
        assert relerr(r["x"], xs) <= 10 * err_qr


def test_srft_entries_match_full_sketch(orc):
    A = np.random.default_rng(45).standard_normal((500, 6))
    for prec in ("fp64", "fp32", "bf16"):
        As = orc.srft_sketch(A, 30, 4, prec=prec, pid=1)
        r, c = np.array([0, 5, 29, 17]), np.array([0, 3, 5, 1])
        assert np.array_equal(orc.srft_entries(A, 30, 4, r, c, prec=prec, pid=1), As[r, c])
