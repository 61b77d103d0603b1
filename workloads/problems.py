"""Exact least-squares problems A = U diag(sigma) V^T, b = A x_* + r.

The construction follows the paper's recipe for "exact" least-squares
problems (Section 7, Algorithm 2): an orthonormal basis U of range(A), a
prescribed condition number, a known solution x_* and a residual r that is
orthogonal to range(A) and has a prescribed relative size

    rho = ||r|| / (||A|| ||x_*||),   ||A||_2 = sigma_1 = 1.

Differences from Algorithm 2, all deliberate: the triangular factor is
replaced by the SVD form diag(sigma) V^T (V a random orthogonal matrix),
x_* ~ N(0, I) is not normalised, and U is the thin orthonormal factor of a
Gaussian matrix rather than the first columns of a full m x m orthogonal
matrix.  For very tall problems U is assembled from k independent orthonormal
blocks, U = [Q_1; ...; Q_k] / sqrt(k), which keeps U^T U = I.

Storage: A is column-major (the LAPACK convention of the library); it is held
as a torch tensor ``At`` of shape (n, m), row-major, so ``At.data_ptr()`` is a
column-major m x n matrix with leading dimension m.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch


# Workloads (m, n, kappa, rho, sigma profile, sketch rows).  The second entry
# is the single-GPU throughput workload.
CONFIGS = {
    "ls_1000x100_k1e8": dict(m=1000, n=100, kappa=1e8, rho=1e-6, sigma="geometric", s=300),
    "ls_100000x1000_k1e6": dict(m=100_000, n=1000, kappa=1e6, rho=1e-4, sigma="geometric", s=3000),
    "ls_1000000x2000_k1e10": dict(m=1_000_000, n=2000, kappa=1e10, rho=1e-8, sigma="half_ones",
                                  s=6000),
    "batch512": dict(batch=512),
    "ls_4000000x1000_k1e8": dict(m=4_000_000, n=1000, kappa=1e8, rho=1e-6, sigma="geometric",
                                 s=4000),
}


def sigma_geometric(n: int, kappa: float) -> np.ndarray:
    """sigma_i = kappa^(-(i-1)/(n-1)): 1 down to 1/kappa."""
    if n == 1:
        return np.ones(1)
    return kappa ** (-np.arange(n, dtype=np.float64) / (n - 1))


def sigma_half_ones_loguniform(n: int, kappa: float, rng: np.random.Generator) -> np.ndarray:
    """First n/2 values 1, the last exactly 1/kappa, the rest 10^U(-log10 kappa, 0),
    sorted in decreasing order."""
    h = n // 2
    lk = math.log10(kappa)
    mid = 10.0 ** rng.uniform(-lk, 0.0, size=n - h - 1)
    sig = np.concatenate([np.ones(h), np.sort(mid)[::-1], [1.0 / kappa]])
    return sig


@dataclasses.dataclass
class Problem:
    At: torch.Tensor        # (n, m) row-major == A column-major, lda = m
    b: torch.Tensor         # (m,)
    x_star: torch.Tensor    # (n,)
    sigma: np.ndarray
    m: int
    n: int
    kappa: float
    rho: float
    seed: int

    @property
    def A(self) -> torch.Tensor:
        """m x n view with column-major strides."""
        return self.At.t()

    def numpy_A(self) -> np.ndarray:
        """Column-major float64 numpy copy of A (host)."""
        return np.asfortranarray(self.At.detach().cpu().numpy().T)

    def numpy_b(self) -> np.ndarray:
        return self.b.detach().cpu().numpy().astype(np.float64)

    def numpy_x_star(self) -> np.ndarray:
        return self.x_star.detach().cpu().numpy().astype(np.float64)


def _orthonormal_columns(m: int, n: int, gen: torch.Generator, device) -> torch.Tensor:
    """m x n matrix with orthonormal columns (thin QR factor of Gaussian blocks)."""
    max_rows = 200_000
    k = max(1, math.ceil(m / max_rows))
    while k > 1 and m // k < n:
        k -= 1
    sizes = [m // k + (1 if i < m % k else 0) for i in range(k)]
    blocks = []
    for rows in sizes:
        G = torch.randn(rows, n, generator=gen, device=device, dtype=torch.float64)
        Q, _ = torch.linalg.qr(G, mode="reduced")
        blocks.append(Q)
        del G
    U = torch.cat(blocks, dim=0) if k > 1 else blocks[0]
    if k > 1:
        U /= math.sqrt(k)
    return U


def make_problem(m: int, n: int, kappa: float, rho: float, seed: int, sigma="geometric",
                 device="cpu") -> Problem:
    """Seeded problem with kappa(A) = kappa, ||A|| = 1, relative residual rho.

    `sigma` is "geometric", "half_ones" or an explicit array of n values
    (sigma_1 >= ... >= sigma_n > 0)."""
    if m < n:
        raise ValueError("need m >= n")
    device = torch.device(device)
    rng = np.random.default_rng(seed)
    if isinstance(sigma, str):
        if sigma == "geometric":
            sig = sigma_geometric(n, kappa)
        elif sigma == "half_ones":
            sig = sigma_half_ones_loguniform(n, kappa, rng)
        else:
            raise ValueError(sigma)
    else:
        sig = np.asarray(sigma, dtype=np.float64)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    U = _orthonormal_columns(m, n, gen, device)
    Gv = torch.randn(n, n, generator=gen, device=device, dtype=torch.float64)
    V, _ = torch.linalg.qr(Gv)
    sig_t = torch.as_tensor(sig, device=device, dtype=torch.float64)
    # A^T = V diag(sigma) U^T, stored (n, m) row-major == A column-major
    At = (V * sig_t) @ U.t()
    At = At.contiguous()
    x_star = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
    g = torch.randn(m, generator=gen, device=device, dtype=torch.float64)
    # two projection sweeps keep U^T r at rounding level
    for _ in range(2):
        g = g - U @ (U.t() @ g)
    r = g * (rho * float(sig[0]) * float(torch.linalg.norm(x_star)) / float(torch.linalg.norm(g)))
    b = At.t() @ x_star + r
    del U
    return Problem(At=At, b=b.contiguous(), x_star=x_star, sigma=sig, m=m, n=n, kappa=float(kappa),
                   rho=float(rho), seed=int(seed))


def draw_batch_shapes(batch: int = 512, seed: int = 0):
    """Independent draws: n ~ U{32..512}, m ~ U{2000..50000} with m >= 20 n
    (redrawn otherwise), log10 kappa ~ U(2, 8), log10 rho ~ U(-10, -2)."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < batch:
        n = int(rng.integers(32, 513))
        m = int(rng.integers(2000, 50001))
        if m < 20 * n:
            continue
        kappa = 10.0 ** rng.uniform(2.0, 8.0)
        rho = 10.0 ** rng.uniform(-10.0, -2.0)
        out.append((m, n, kappa, rho))
    return out


def make_batch(batch: int = 512, seed: int = 0, device="cpu", shapes=None):
    """A list of problems; member i is seeded with 40000 + i."""
    shapes = draw_batch_shapes(batch, seed) if shapes is None else shapes
    return [make_problem(m, n, kappa, rho, 40000 + i, device=device)
            for i, (m, n, kappa, rho) in enumerate(shapes)]


def pack_batch(probs, device="cuda", release=False):
    """Concatenate the members' A (column-major), b and x slots into flat
    device buffers.  Returns (A, b, x, descs), descs in the batched solver's
    format.  With release=True each member's A is dropped once copied."""
    descs, ao, bo, xo = [], 0, 0, 0
    for p in probs:
        descs.append(dict(m=p.m, n=p.n, lda=p.m, a_offset=ao, b_offset=bo, x_offset=xo))
        ao += p.m * p.n
        bo += p.m
        xo += p.n
    A = torch.empty(ao, dtype=torch.float64, device=device)
    b = torch.empty(bo, dtype=torch.float64, device=device)
    for p, d in zip(probs, descs):
        # At (n, m) row-major is A column-major
        A[d["a_offset"]:d["a_offset"] + p.m * p.n] = p.At.reshape(-1).to(device)
        b[d["b_offset"]:d["b_offset"] + p.m] = p.b.to(device)
        if release:
            p.At = None
    x = torch.zeros(xo, dtype=torch.float64, device=device)
    return A, b, x, descs
