"""GPU checks at the two largest single-problem workloads, where the oracle can
only check sampled entries one by one and the solution is checked against
its known value:

  m = 10^6, n = 2000, kappa = 1e10 (half the singular values 1, the rest
  log-uniform down to 1e-10), relative residual 1e-8, s = 6000, AUTO precision
  with one refinement step;

  m = 4*10^6, n = 1000, kappa = 1e8 (geometric), relative residual 1e-6,
  s = 4000, HPNE with an FP8 e4m3 sketch (per-128-row-block scales) and an
  FP32 QR, against the all-FP64 HPNE.

Each needs tens of GB of device memory; the problems are generated on the
device and freed at the end of the module."""
import gc

import numpy as np
import pytest
import torch

from workloads import make_problem

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53
SAMPLE_TOL = {"fp64": 1e-5, "fp8": 2.0 ** -3 + 1e-4}


@pytest.fixture(scope="module")
def pne():
    import paper_2603_16644_amd as p
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    p.lib()
    return p


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(y))


def sampled_sketch_check(pne, orc, prob, s, seed, prec, n_samples=8):
    """Entries of the GPU sketch against the oracle's, computed one by one on
    the sampled columns only (the sketch of a column depends on that column
    alone, FP8 block scales included)."""
    As = pne.pne_sketch(prob.A, s, seed=seed, prec=prec)
    rng = np.random.default_rng(11)
    rows = rng.integers(0, s, n_samples)
    cols = rng.integers(0, prob.n, n_samples)
    got = host(As)[rows, cols]
    del As
    sub = np.asfortranarray(prob.At[torch.as_tensor(cols, device=prob.At.device)].cpu().numpy().T)
    ref, ab = orc.sketch_entries(sub, s, seed, rows, np.arange(n_samples), prec=prec)
    assert np.all(np.abs(got - ref) <= SAMPLE_TOL[prec] * ab), (got, ref, ab)


def release(prob):
    """Drop the problem's device tensors (the fixture object itself lives on
    until the end of the module)."""
    prob.At = prob.b = prob.x_star = None
    gc.collect()
    torch.cuda.empty_cache()


# ------------------------------------------------------------------ m = 1e6, n = 2000

@pytest.fixture(scope="module")
def p3():
    p = make_problem(1_000_000, 2000, 1e10, 1e-8, seed=1003, sigma="half_ones", device="cuda")
    torch.cuda.synchronize()
    yield p
    release(p)


def test_1e6x2000_sampled_sketch_fp64(pne, orc, p3):
    sampled_sketch_check(pne, orc, p3, 6000, 3, "fp64")


def test_1e6x2000_auto_picks_double_and_is_accurate(pne, p3):
    """kappa = 1e10: the FP32 Gram of the estimate breaks down, so the pick is
    double (Section 7.4); the solution then meets the least-squares bound."""
    o = pne.make_opts(s=6000, seed=3, sketch_prec="auto", qr_prec="auto", refine_steps=1)
    x, info, meta = pne.pne_solve(p3.A, p3.b, opts=o)
    assert int(host(info)[0]) == 0
    assert meta["sketch_prec"] == "fp64" and meta["qr_prec"] == "fp64"
    err = relerr(host(x), host(p3.x_star))
    bound = p3.kappa * U64 * (1 + p3.kappa * p3.rho)
    assert err <= 10 * bound, (err, bound)


def test_1e6x2000_forced_fp32_preconditioner_runs(pne, p3):
    """The forced FP32 sketch and QR at kappa = 1e10 (u_32 kappa >> 1): the
    preconditioner is poor, the solve must still finish without breakdown and
    one FP64 refinement step must not increase the error."""
    errs = []
    for k in (0, 1):
        o = pne.make_opts(s=6000, seed=3, sketch_prec="fp32", qr_prec="fp32", refine_steps=k)
        x, info, _ = pne.pne_solve(p3.A, p3.b, opts=o)
        assert int(host(info)[0]) == 0
        errs.append(relerr(host(x), host(p3.x_star)))
    assert np.all(np.isfinite(errs)) and errs[1] <= errs[0] * 1.01, errs


# ------------------------------------------------------------------ m = 4e6, n = 1000

@pytest.fixture(scope="module")
def p5(p3):
    release(p3)
    p = make_problem(4_000_000, 1000, 1e8, 1e-6, seed=1005, device="cuda")
    torch.cuda.synchronize()
    yield p
    release(p)


def test_4e6x1000_sampled_sketch_fp8(pne, orc, p5):
    sampled_sketch_check(pne, orc, p5, 4000, 5, "fp8")


def test_4e6x1000_fp8_hpne_matches_fp64_hpne(pne, p5):
    bound = p5.kappa * U64 * (1 + p5.kappa * p5.rho)
    xs = host(p5.x_star)
    o64 = pne.make_opts(s=4000, seed=5, sketch_prec="fp64", qr_prec="fp64", refine_steps=0)
    x, info, _ = pne.hpne_solve(p5.A, p5.b, opts=o64)
    assert int(host(info)[0]) == 0
    e64 = relerr(host(x), xs)
    assert e64 <= 10 * bound, (e64, bound)
    o8 = pne.make_opts(s=4000, seed=5, sketch_prec="fp8", qr_prec="fp32", refine_steps=3)
    x, info, _ = pne.hpne_solve(p5.A, p5.b, opts=o8)
    assert int(host(info)[0]) == 0
    e8 = relerr(host(x), xs)
    assert e8 <= 10 * bound and e8 <= 10 * e64, (e8, e64, bound)
