#!/usr/bin/env python3
"""Accuracy sweeps of the paper's experiments (Sections 7.2-7.4, Figures 1-5
and 7), printed as markdown tables: relative error of the solution against
the least-squares residual, beside the oracle QR solver's error and the
perturbation bounds (31)/(41) (PNE) or (42)/(32) (HPNE) evaluated with
SVD-based condition numbers (oracle/bounds.py).

  python tests/sweep_accuracy.py [--solver gpu|oracle] [--quick]

--solver gpu (default when a GPU is present) solves with the HIP library,
--solver oracle with the CPU oracle.  Inputs are the seeded synthetic
problems of workloads/ (Algorithm 2's construction with A = U diag(sigma) V^T).
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import bounds as B  # noqa: E402
from workloads import make_problem  # noqa: E402

U2 = 2.0 ** -52


def solve(args, A, b, hpne, prec, n, seed=1):
    if args.solver == "oracle":
        r = oracle.solve(A, b, hpne=hpne, s=3 * n, seed=seed, sketch_prec=prec, qr_prec=prec, refine_steps=0)
        return r["x"], r["R"], r["prec_used"]
    import torch
    import paper_2603_16644_amd as pne
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    o = pne.make_opts(s=3 * n, seed=seed, sketch_prec=prec, qr_prec=prec, refine_steps=0)
    fn = pne.hpne_solve if hpne else pne.pne_solve
    x, info, meta = fn(Ad, torch.from_numpy(b).cuda(), opts=o)
    o2 = pne.make_opts(s=3 * n, seed=seed, sketch_prec=meta["sketch_prec"], qr_prec=meta["qr_prec"])
    R, _, _ = pne.sketch_precond(Ad, opts=o2)
    torch.cuda.synchronize()
    return x.cpu().numpy(), R.cpu().numpy(), (meta["sketch_prec"], meta["qr_prec"])


def figure(args, title, m, n, kappa, prec, hpne, rhos):
    u1 = U2 if prec == "fp64" else B.U_SINGLE
    names = ("eq42", "eq32") if hpne else ("eq31", "eq41")
    print(f"\n### {title}\n")
    print(f"m = {m}, n = {n}, kappa = {kappa:.0e}, preconditioner {prec}, {'HPNE' if hpne else 'PNE'}, "
          f"solver {args.solver}\n")
    print(f"| rho | error | QR error | {names[0]} (old) | {names[1]} (new) | kappa(A_p) |")
    print("|---:|---:|---:|---:|---:|---:|")
    for rho in rhos:
        p = make_problem(m, n, kappa, rho, seed=500 + n + int(-np.log10(rho)))
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        x, R, _ = solve(args, A, b, hpne, prec, n)
        q, bd = B.all_bounds(A, b, R, x, u1, U2)
        err = np.linalg.norm(x - xs) / np.linalg.norm(x)
        eqr = np.linalg.norm(oracle.qr_ls(A, b) - xs) / np.linalg.norm(xs)
        print(f"| {rho:.0e} | {err:.2e} | {eqr:.2e} | {bd[names[0]]:.2e} | {bd[names[1]]:.2e} | "
              f"{q['kappa_Ap']:.2f} |", flush=True)


def figure7(args, kappa, ns, m):
    print(f"\n### Figure 7 (automatic precision), kappa = {kappa:.0e}, m = {m}\n")
    print("| n | picked | error | QR error |")
    print("|---:|---|---:|---:|")
    for n in ns:
        p = make_problem(m, n, kappa, 1e-6, seed=700 + n)
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        x, _, used = solve(args, A, b, False, "auto", n)
        err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
        eqr = np.linalg.norm(oracle.qr_ls(A, b) - xs) / np.linalg.norm(xs)
        print(f"| {n} | {used[1]} | {err:.2e} | {eqr:.2e} |", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--solver", choices=["gpu", "oracle"], default=None)
    ap.add_argument("--quick", action="store_true", help="fewer residuals, n = 1000 cases left out")
    args = ap.parse_args()
    if args.solver is None:
        try:
            import torch
            args.solver = "gpu" if torch.cuda.is_available() else "oracle"
        except Exception:
            args.solver = "oracle"
    rhos = [1e-14, 1e-10, 1e-6, 1e-3, 1e-1] if args.quick else list(10.0 ** np.arange(-14, 1, 2))
    figure(args, "Figure 1 (PNE, double)", 6000, 100, 1e4, "fp64", False, rhos)
    figure(args, "Figure 2 (HPNE, double)", 6000, 100, 1e4, "fp64", True, rhos)
    figure(args, "Figure 3a (PNE, single preconditioner)", 6000, 100, 1e8, "fp32", False, rhos)
    figure(args, "Figure 4a (HPNE, single preconditioner)", 6000, 100, 1e8, "fp32", True, rhos)
    if not args.quick:
        figure(args, "Figure 3b (PNE, single preconditioner)", 6000, 1000, 1e8, "fp32", False, rhos[::2])
        figure(args, "Figure 4b (HPNE, single preconditioner)", 6000, 1000, 1e8, "fp32", True, rhos[::2])
    figure7(args, 1e2, [400, 600], 1 << 15)
    figure7(args, 1e10, [400, 600], 1 << 15)


if __name__ == "__main__":
    main()
