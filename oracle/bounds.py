"""Perturbation bounds of the paper as evaluators -- TEST INFRASTRUCTURE.

Plain numpy, every condition number from an SVD.  For a computed solution
x^ of min ||A x - b|| obtained with the preconditioner R_s (A_p = A R_s^{-1})
these functions evaluate the four bounds listed in Section 7.1 "Setup"
(u1: unit roundoff of the precision the preconditioner was computed in, u2:
the working precision of the rest):

  eq. (31)  old PNE bound (Theorem t_3):
      kappa(R_s) kappa(A_p) ||R_s x^|| / (||R_s|| ||x^||)
        * (u2 + kappa(A_p) eta1 (||A_p y^ - b|| / (||A_p|| ||y^||) + u2)),
      y^ = R_s x^,  eta1 = |kappa(R_s) u1 / (1 - kappa(R_s) u1)|
  eq. (41)  improved PNE bound (Theorem t_55):
      kappa(R_s) kappa(A_p) u2 (kappa(A_p) kappa(R_s) res + 1 + kappa(A) u2)
  eq. (42)  old HPNE bound (Theorem t_2):
      kappa(A_p^T A) nu (eta1 res + (1 + eta1) u2)
  eq. (32)  improved HPNE bound (Theorem t_22):
      kappa(A_p^T A) nu u2 (kappa(R_s) res + 1 + kappa(A) u2)

with res = ||A x^ - b|| / (||A|| ||x^||) and
nu = ||A_p|| ||A|| / ||A_p^T A||.  Also the least-squares bound of Lemma
1.1 (l_ls) and the first-order not-normal-equations bound of Section 5.2
(eq. e_fonne).  All bound the relative error ||x^ - x*|| / ||x^||.

Only tests/ may import this module; it shares nothing with the GPU library.
"""
from __future__ import annotations

import numpy as np

U_DOUBLE = 2.0 ** -52      # the paper's u for double precision (Section 7.2)
U_SINGLE = 2.0 ** -23      # and for single precision (Section 7.3)


def cond2(M) -> float:
    """Two-norm condition number w.r.t. left inversion, from the singular values."""
    s = np.linalg.svd(np.asarray(M, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1])


def norm2(M) -> float:
    return float(np.linalg.svd(np.asarray(M, dtype=np.float64), compute_uv=False)[0])


def quantities(A, b, R, x):
    """The SVD-based quantities every bound uses."""
    A = np.asarray(A, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    Ap = np.linalg.solve(R.T, A.T).T                # A R^{-1}
    nA, nAp, nR = norm2(A), norm2(Ap), norm2(R)
    ApTA = Ap.T @ A
    y = R @ x
    return {
        "kappa_A": cond2(A), "kappa_R": cond2(R), "kappa_Ap": cond2(Ap), "kappa_ApTA": cond2(ApTA),
        "nu": nAp * nA / norm2(ApTA),
        "res": float(np.linalg.norm(A @ x - b) / (nA * np.linalg.norm(x))),
        "res_p": float(np.linalg.norm(Ap @ y - b) / (nAp * np.linalg.norm(y))),
        "rx": float(np.linalg.norm(y) / (nR * np.linalg.norm(x))),
    }


def eta1(kappa_R: float, u1: float) -> float:
    """eta_1 = |kappa(R_s) u1 / (1 - kappa(R_s) u1)| (Section 7.1)."""
    return abs(kappa_R * u1 / (1.0 - kappa_R * u1))


def eq31(q, u1: float, u2: float) -> float:
    e = eta1(q["kappa_R"], u1)
    return q["kappa_R"] * q["kappa_Ap"] * q["rx"] * (u2 + q["kappa_Ap"] * e * (q["res_p"] + u2))


def eq41(q, u1: float, u2: float) -> float:
    return q["kappa_R"] * q["kappa_Ap"] * u2 * (q["kappa_Ap"] * q["kappa_R"] * q["res"] + 1.0 + q["kappa_A"] * u2)


def eq42(q, u1: float, u2: float) -> float:
    e = eta1(q["kappa_R"], u1)
    return q["kappa_ApTA"] * q["nu"] * (e * q["res"] + (1.0 + e) * u2)


def eq32(q, u1: float, u2: float) -> float:
    return q["kappa_ApTA"] * q["nu"] * u2 * (q["kappa_R"] * q["res"] + 1.0 + q["kappa_A"] * u2)


def lemma_ls(kappa_A: float, eps: float, res: float) -> float:
    """Lemma 1.1 (l_ls): kappa(A) eps (1 + kappa(A) res)."""
    return kappa_A * eps * (1.0 + kappa_A * res)


def nne_first_order(A, B, b, x, eps_A: float, eps_B: float) -> float:
    """First-order not-normal-equations bound (Section 5.2, eq. e_fonne):
    kappa(B^T A) (eps_B ||A x^ - b|| / (||A|| ||x^||) + eps_A)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    res = float(np.linalg.norm(A @ x - b) / (norm2(A) * np.linalg.norm(x)))
    return cond2(B.T @ A) * (eps_B * res + eps_A)


def all_bounds(A, b, R, x, u1: float, u2: float):
    q = quantities(A, b, R, x)
    return q, {"eq31": eq31(q, u1, u2), "eq41": eq41(q, u1, u2), "eq42": eq42(q, u1, u2),
               "eq32": eq32(q, u1, u2)}
