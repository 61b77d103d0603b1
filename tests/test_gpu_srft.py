"""GPU parity of the SRFT sketch (Section 6.2, eq. e_sketch, with the real
Hartley transform) against the CPU oracle's definition, and of the solves
that use it.  Needs an MI355X; run with -m gpu."""
import math

import numpy as np
import pytest
import torch

from workloads import make_problem

pytestmark = pytest.mark.gpu


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


def relerr(x, y):
    return float(np.linalg.norm(np.asarray(x) - np.asarray(y)) / np.linalg.norm(y))


# FFT rounding error per entry: a few units of the arithmetic's roundoff
# times log2 m', relative to ||z|| / sqrt(s) with z = a_2c + i a_2c+1 the
# complex column the pair of columns is transformed as (an FFT is accurate
# normwise: the smaller column of a pair inherits the error of the larger);
# both sides round A identically
TOL = {"fp64": 1e-14, "fp32": 2e-6, "bf16": 2e-6}


def pair_scale(A, cols, s, mp):
    """||(a_2c, a_2c+1)|| / sqrt(s) * log2 m' for every column in cols."""
    nrm = np.linalg.norm(A, axis=0)
    n = A.shape[1]
    out = []
    for c in cols:
        c0 = c - (c % 2)
        pair = nrm[c0] ** 2 + (nrm[c0 + 1] ** 2 if c0 + 1 < n else 0.0)
        out.append(math.sqrt(pair))
    return np.array(out) / math.sqrt(s) * max(1.0, math.log2(mp))


@pytest.mark.parametrize("m,n,s", [(777, 65, 200), (3000, 257, 771), (32, 3, 20), (1, 1, 4), (6007, 10, 30),
                                   (50000, 8, 24)])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_srft_sketch_matches_oracle(pne, orc, m, n, s, prec):
    """Ragged shapes: odd n (a column pair with one column), a length that is
    a single radix (32), m = 1, a prime m (padded to the next 7-smooth
    length), and a long column."""
    rng = np.random.default_rng(m + n)
    A = rng.standard_normal((m, n)) * 10.0 ** rng.uniform(-2, 2, size=n)
    As = host(pne.pne_sketch_srft(dev(A), s, seed=9, problem_id=3, prec=prec))
    ref = orc.srft_sketch(A, s, 9, prec=prec, pid=3)
    mp = orc.next_smooth(m)
    scale = pair_scale(A, range(n), s, mp)
    assert np.all(np.abs(As - ref) <= TOL[prec] * scale[None, :]), np.max(np.abs(As - ref) / scale[None, :])


def test_srft_sketch_padded_lda(pne, orc):
    m, n, lda = 1000, 20, 1100
    A = np.random.default_rng(5).standard_normal((lda, n))
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()[:m]
    As = host(pne.pne_sketch_srft(Ad, 60, seed=2, prec="fp64"))
    ref = orc.srft_sketch(A[:m], 60, 2, prec="fp64")
    assert np.allclose(As, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("hpne", [False, True])
@pytest.mark.parametrize("prec,qr,refine", [("fp64", "fp64", 0), ("fp32", "fp32", 1), ("bf16", "fp32", 1)])
def test_solve_with_srft_matches_oracle(pne, orc, hpne, prec, qr, refine):
    p = make_problem(3000, 100, 1e6, 1e-6, seed=401)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    o = pne.make_opts(s=300, seed=3, sketch_prec=prec, qr_prec=qr, refine_steps=refine, sketch_kind="srft")
    fn = pne.hpne_solve if hpne else pne.pne_solve
    x, info, _ = fn(dev(A), torch.from_numpy(b).cuda(), opts=o)
    assert int(host(info)[0]) == 0
    err_qr = relerr(orc.qr_ls(A, b), xs)
    xo = orc.solve(A, b, hpne=hpne, s=300, seed=3, sketch_prec=prec, qr_prec=qr, refine_steps=refine,
                   sketch_kind="srft")
    assert xo["info"] == 0
    assert relerr(host(x), xs) <= 10 * err_qr
    assert relerr(host(x), xo["x"]) <= 10 * err_qr


def test_srft_auto_and_batched(pne, orc):
    """AUTO with the SRFT (an FP16 pick sketches in FP32), and a batch of
    uneven members with SRFT sketches."""
    from workloads import pack_batch
    shapes = [(3000, 100, 1e2, 1e-6), (2500, 64, 1e5, 1e-8), (4001, 130, 1e10, 1e-6)]
    probs = [make_problem(m, n, k, r, seed=410 + i) for i, (m, n, k, r) in enumerate(shapes)]
    o = pne.make_opts(seed=4, sketch_prec="auto", qr_prec="auto", refine_steps=1, sketch_kind="srft")
    for p in probs:
        A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
        x, info, meta = pne.pne_solve(dev(A), torch.from_numpy(b).cuda(), opts=o)
        assert int(host(info)[0]) == 0
        assert relerr(host(x), xs) <= 10 * relerr(orc.qr_ls(A, b), xs)
    A, b, x, descs = pack_batch(probs)
    ob = pne.make_opts(seed=4, sketch_prec="bf16", qr_prec="fp32", refine_steps=2, sketch_kind="srft")
    info = pne.pne_solve_batched(A, b, x, descs, opts=ob)
    assert np.all(host(info) == 0)
    xb = host(x)
    for p, d in zip(probs, descs):
        xs = p.numpy_x_star()
        assert relerr(xb[d["x_offset"]:d["x_offset"] + p.n], xs) <= 10 * relerr(
            orc.qr_ls(p.numpy_A(), p.numpy_b()), xs)


def test_srft_full_size(pne, orc):
    """m = 1e5, n = 1e3 (m' = 100 000 is 7-smooth): sampled sketch entries
    against the oracle one by one, and the mixed PNE with an SRFT sketch
    within 10x the stored oracle QR error."""
    import os
    p = make_problem(100_000, 1000, 1e6, 1e-4, seed=1002, device="cpu")
    A = p.numpy_A()
    Ad = p.At.cuda().t()
    As = host(pne.pne_sketch_srft(Ad, 3000, seed=2, prec="fp32"))
    rng = np.random.default_rng(1)
    rows, cols = rng.integers(0, 3000, 8), rng.integers(0, 1000, 8)
    ref = orc.srft_entries(A, 3000, 2, rows, cols, prec="fp32")
    scale = pair_scale(A, cols, 3000, 100_000)
    assert np.all(np.abs(As[rows, cols] - ref) <= TOL["fp32"] * scale)
    path = os.path.join(os.path.dirname(__file__), "golden", "err_qr_full_size.txt")
    err_qr = [float(l.split()[6]) for l in open(path) if l.startswith("ls_100000x1000_k1e6")][0]
    o = pne.make_opts(s=3000, seed=2, sketch_prec="bf16", qr_prec="fp32", refine_steps=1, sketch_kind="srft")
    x, info, _ = pne.pne_solve(Ad, p.b.cuda(), opts=o)
    assert int(host(info)[0]) == 0
    assert relerr(host(x), p.numpy_x_star()) <= 10 * err_qr
