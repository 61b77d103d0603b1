"""Writes err_qr_full_size.txt: the relative error ||x_QR - x_*|| / ||x_*|| of
the oracle's Householder least-squares solve (oracle.qr_ls) on seeded
full-size problems, generated on the CPU exactly as the GPU tests generate
them.  The GPU tests hold the library's solutions to 10 x these values.

Run from the repository root:  python tests/golden/make_err_qr.py
(plain single-threaded oracle; about ten minutes on one core)."""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import make_problem  # noqa: E402
from workloads.problems import draw_batch_shapes  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "err_qr_full_size.txt")

# members of the 512-problem batch (shapes drawn with seed 0) whose QR error is stored
BATCH_MEMBERS = sorted(int(i) for i in np.random.default_rng(7).choice(512, 16, replace=False))


def cases():
    yield "ls_100000x1000_k1e6", 100_000, 1000, 1e6, 1e-4, 1002
    shapes = draw_batch_shapes(512, 0)
    for i in BATCH_MEMBERS:
        m, n, k, r = shapes[i]
        yield f"batch512_member{i}", m, n, k, r, 40000 + i


def main():
    lines = ["# name m n kappa rho seed err_qr   (oracle.qr_ls on the CPU-generated problem)"]
    for name, m, n, k, r, seed in cases():
        t0 = time.time()
        p = make_problem(m, n, k, r, seed=seed, device="cpu")
        x = oracle.qr_ls(p.numpy_A(), p.numpy_b())
        xs = p.numpy_x_star()
        err = float(np.linalg.norm(x - xs) / np.linalg.norm(xs))
        lines.append(f"{name} {m} {n} {k!r} {r!r} {seed} {err:.6e}")
        print(lines[-1], f"({time.time() - t0:.1f} s)", flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
