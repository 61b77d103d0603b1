"""Pins of the bound evaluators (oracle/bounds.py) against the paper's
statements about them (Sections 7.2 and 7.3, Figures 1-4) and against the
closed forms they reduce to; the solves are the CPU oracle's.  CPU only."""
import numpy as np
import pytest

from oracle import bounds as B
from workloads import make_problem

U2 = 2.0 ** -52
RHOS = [1e-12, 1e-8, 1e-4, 1e-1]


def relerr_xhat(x, xs):
    return float(np.linalg.norm(x - xs) / np.linalg.norm(x))


def sweep(orc, kappa, prec, hpne, n=100, m=6000):
    out = []
    for rho in RHOS:
        p = make_problem(m, n, kappa, rho, seed=100 + int(-np.log10(rho)))
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        r = orc.solve(A, b, hpne=hpne, s=3 * n, seed=1, sketch_prec=prec, qr_prec=prec, refine_steps=0)
        assert r["info"] == 0
        u1 = U2 if prec == "fp64" else B.U_SINGLE
        q, bd = B.all_bounds(A, b, r["R"], r["x"], u1, U2)
        err_qr = float(np.linalg.norm(orc.qr_ls(A, b) - xs) / np.linalg.norm(xs))
        out.append((rho, relerr_xhat(r["x"], xs), err_qr, q, bd))
    return out


def test_double_precision_pne_bounds(orc):
    """Figure 1 (m = 6000, n = 100, kappa = 1e4, u1 = u2 = 2^-52): both PNE
    bounds hold, the old bound (31) is the tighter one (its factor
    ||R_s x^|| / (||R_s|| ||x^||) <= 1), and for residuals above 1e-4 the PNE
    solution is as accurate as the QR solver's."""
    for rho, err, err_qr, q, bd in sweep(orc, 1e4, "fp64", False):
        assert err <= bd["eq31"] <= bd["eq41"], (rho, err, bd)
        assert q["rx"] <= 1.0
        if rho > 1e-4:
            assert err <= 10 * err_qr


def test_double_precision_hpne_bounds(orc):
    """Figure 2: the old (42) and new (32) HPNE bounds are essentially the same
    in double precision, and both hold."""
    for rho, err, err_qr, q, bd in sweep(orc, 1e4, "fp64", True):
        assert err <= bd["eq32"] and err <= bd["eq42"]
        assert 0.9 <= bd["eq42"] / bd["eq32"] <= 1.1
        if rho > 1e-4:
            assert err <= 10 * err_qr


@pytest.mark.parametrize("hpne", [False, True])
def test_mixed_precision_bounds(orc, hpne):
    """Figures 3-4 (kappa = 1e8, single-precision preconditioner, u1 = 2^-23,
    u2 = 2^-52): the new bound holds and follows the error, the old bound is
    a severe overestimate; below rho ~ 1e-6 the error is at most about 100x
    the QR solver's, above it about as accurate."""
    new, old = ("eq32", "eq42") if hpne else ("eq41", "eq31")
    rows = sweep(orc, 1e8, "fp32", hpne)
    for rho, err, err_qr, q, bd in rows:
        assert err <= bd[new], (rho, err, bd[new])
        assert bd[old] >= 1e3 * bd[new] or rho < 1e-10, (rho, bd)
        assert q["kappa_R"] * B.U_SINGLE > 1.0          # the old bound's eta1 is O(1) here
        if rho < 1e-6:
            assert err <= 100 * err_qr
        else:
            assert err <= 10 * err_qr
    # the new bound grows with the residual as the error does
    assert rows[-1][4][new] / rows[0][4][new] > 1e4 and rows[-1][1] / rows[0][1] > 1e4


def test_bounds_with_exact_preconditioner_reduce_to_lemma(orc):
    """With R_s the R factor of A itself: A_p = Q has kappa 1, A_p^T A = R,
    nu = 1, so (41) and (32) become kappa u2 (kappa res + 1 + kappa u2), the
    least-squares bound of Lemma 1.1 with eps = u2 plus kappa^2 u2^2
    (Section 4: 'resembles the one in Lemma l_ls')."""
    p = make_problem(3000, 60, 1e5, 1e-6, seed=120)
    A, b = p.numpy_A(), p.numpy_b()
    R = np.linalg.qr(A, mode="r")
    x = orc.qr_ls(A, b)
    q, bd = B.all_bounds(A, b, R, x, U2, U2)
    assert abs(q["kappa_Ap"] - 1.0) < 1e-8 and abs(q["nu"] - 1.0) < 1e-8
    assert abs(q["kappa_ApTA"] / q["kappa_A"] - 1.0) < 1e-6
    k = q["kappa_A"]
    ref = B.lemma_ls(k, U2, q["res"]) + (k * U2) ** 2 * k
    for name in ("eq41", "eq32"):
        assert abs(bd[name] / ref - 1.0) < 1e-5, (name, bd[name], ref)


def test_eta1_definition():
    # |kappa u / (1 - kappa u)| stays positive when kappa u > 1 (Section 7.1)
    assert B.eta1(10.0, 0.01) == pytest.approx(0.1 / 0.9)
    assert B.eta1(1e8, 2.0 ** -23) == pytest.approx(abs(1e8 * 2.0 ** -23 / (1 - 1e8 * 2.0 ** -23)))
    assert B.eta1(1e8, 2.0 ** -23) > 0


def test_nne_first_order_bound_holds(orc):
    """Section 5.2, eq. (e_fonne), for B an orthonormal basis of range(A)."""
    for kappa, rho in [(1e3, 1e-8), (1e6, 1e-3)]:
        p = make_problem(2000, 40, kappa, rho, seed=121)
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        Q = np.linalg.qr(A)[0]
        x, info = orc.nne(A, Q, b)
        assert info == 0
        eps = 4 * 2000 * 2.0 ** -53
        assert relerr_xhat(x, xs) <= B.nne_first_order(A, Q, b, x, eps, eps)
