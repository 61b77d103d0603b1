"""GPU checks of the batched solver (pne_solve_batched): many independent
problems of uneven m, n and kappa solved by grouped launches, one per step of
the pipeline.  Each member is checked against its known solution and the
CPU oracle's QR solve, and against the single-problem solver."""
import numpy as np
import pytest
import torch

from workloads import make_problem
from workloads.problems import draw_batch_shapes, pack_batch

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


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


def pack(probs, device="cuda"):
    return pack_batch(probs, device)


SHAPES = [(2000, 64, 1e3, 1e-4), (3100, 100, 1e5, 1e-8), (2500, 33, 1e2, 1e-2), (6000, 300, 1e6, 1e-6),
          (1999, 96, 1e4, 1e-3), (4097, 129, 1e7, 1e-10)]


@pytest.fixture(scope="module")
def small_batch(orc):
    probs = [make_problem(m, n, k, r, seed=40000 + i) for i, (m, n, k, r) in enumerate(SHAPES)]
    err_qr = [relerr(orc.qr_ls(p.numpy_A(), p.numpy_b()), p.numpy_x_star()) for p in probs]
    return probs, err_qr


@pytest.mark.parametrize("hpne", [False, True])
def test_batched_members_accurate_and_match_single(pne, small_batch, hpne):
    probs, err_qr = small_batch
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=5, sketch_prec="bf16", qr_prec="fp32", refine_steps=3)
    info = pne.pne_solve_batched(A, b, x, descs, opts=o, hpne=hpne)
    assert np.all(host(info) == 0)
    xb = host(x)
    fn = pne.hpne_solve if hpne else pne.pne_solve
    for i, (p, d) in enumerate(zip(probs, descs)):
        xi = xb[d["x_offset"]:d["x_offset"] + p.n]
        xs = p.numpy_x_star()
        assert relerr(xi, xs) <= 10 * err_qr[i], (i, relerr(xi, xs), err_qr[i])
        oi = pne.make_opts(seed=5, problem_id=i, sketch_prec="bf16", qr_prec="fp32", refine_steps=3)
        x1, _, _ = fn(p.A.cuda(), p.b.cuda(), opts=oi)
        assert relerr(xi, host(x1)) <= 10 * err_qr[i] + relerr(host(x1), xs)


def test_batched_deterministic(pne, small_batch):
    probs, _ = small_batch
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=9, sketch_prec="fp16", qr_prec="fp16", refine_steps=2)
    pne.pne_solve_batched(A, b, x, descs, opts=o)
    x0 = host(x).copy()
    x.zero_()
    pne.pne_solve_batched(A, b, x, descs, opts=o)
    assert np.array_equal(x0, host(x))


@pytest.mark.parametrize("hpne", [False, True])
def test_batched_member_independent_of_batch(pne, small_batch, hpne):
    """A member's x does not depend on the other members: solved inside the
    full batch and alone (same problem id, so the same sketch), the results
    are bitwise equal.  Members share every grouped launch, so a race or an
    indexing slip between members would show up here."""
    probs, _ = small_batch
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=11, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    info = pne.pne_solve_batched(A, b, x, descs, opts=o, hpne=hpne)
    assert np.all(host(info) == 0)
    xb = host(x)
    for i in (1, 3, 5):
        p = probs[i]
        A1, b1, x1, d1 = pack([p])
        d1[0]["problem_id"] = i
        info1 = pne.pne_solve_batched(A1, b1, x1, d1, opts=o, hpne=hpne)
        assert int(host(info1)[0]) == 0
        d = descs[i]
        assert np.array_equal(host(x1)[:p.n], xb[d["x_offset"]:d["x_offset"] + p.n]), i


def test_batched_auto_mixes_precisions(pne, orc):
    """AUTO picks per member (kappa 1e2 -> half, 3e3 -> single, 1e10 -> double);
    members of different precisions run in the same batched call."""
    shapes = [(3000, 100, 1e2, 1e-6), (3000, 100, 3e3, 1e-6), (3000, 100, 1e10, 1e-6), (2500, 70, 1e2, 1e-3)]
    probs = [make_problem(m, n, k, r, seed=41000 + i) for i, (m, n, k, r) in enumerate(shapes)]
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=3, sketch_prec="auto", qr_prec="auto", refine_steps=2)
    info = pne.pne_solve_batched(A, b, x, descs, opts=o)
    assert np.all(host(info) == 0)
    xb = host(x)
    picks = []
    for i, (p, d) in enumerate(zip(probs, descs)):
        xi = xb[d["x_offset"]:d["x_offset"] + p.n]
        err_qr = relerr(orc.qr_ls(p.numpy_A(), p.numpy_b()), p.numpy_x_star())
        assert relerr(xi, p.numpy_x_star()) <= 10 * err_qr
        picks.append(orc.cond_est(p.numpy_A())[2])
    assert picks[0] == 3 and picks[2] == 1   # FP16, FP64


def test_batched_singular_member_is_isolated(pne):
    probs = [make_problem(m, n, k, r, seed=42000 + i)
             for i, (m, n, k, r) in enumerate([(2000, 50, 1e3, 1e-6), (2200, 40, 1e3, 1e-6)])]
    probs[1].At[7].zero_()          # column 8 of member 1 is zero
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=1, sketch_prec="fp32", qr_prec="fp32", refine_steps=1)
    info = host(pne.pne_solve_batched(A, b, x, descs, opts=o))
    assert info[0] == 0 and 1000 < info[1] <= 1000 + 40
    xb = host(x)
    assert np.all(np.isfinite(xb[:50])) and np.all(np.isnan(xb[50:90]))


# ------------------------------------------------------------------ plans, graphs, autotuner

def test_plan_executions_match_one_shot_call(pne, small_batch):
    """A plan executed twice gives the one-shot batched call's x bit for bit
    (same grouped launches; the info words and flags are cleared by kernels
    at every execution)."""
    probs, _ = small_batch
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=5, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    pne.pne_solve_batched(A, b, x, descs, opts=o)
    ref = host(x).copy()
    plan = pne.BatchPlan(A, b, x, descs, opts=o)
    for _ in range(2):
        x.zero_()
        info = plan.execute()
        assert np.all(host(info) == 0)
        assert np.array_equal(host(x), ref)
    plan.close()


@pytest.mark.parametrize("auto", [False, True])
def test_plan_graph_replays_match_uncaptured(pne, small_batch, auto):
    """The plan captured into a hipGraph and replayed three times, with other
    eager work and host synchronisations between the replays: every replay
    matches the uncaptured execution bit for bit."""
    probs, _ = small_batch
    A, b, x, descs = pack(probs)
    if auto:
        o = pne.make_opts(seed=6, sketch_prec="auto", qr_prec="auto", refine_steps=1, cond_method=1)
    else:
        o = pne.make_opts(seed=6, sketch_prec="fp16", qr_prec="fp16", refine_steps=2)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan = pne.BatchPlan(A, b, x, descs, opts=o, stream=st)
        plan.execute(stream=st)
        st.synchronize()
        ref = host(x).copy()
        for k in range(3):
            x.fill_(float("nan"))
            junk = torch.randn(1 << 20, device="cuda").sum()        # unrelated eager work
            info = plan.execute_graph(st)
            st.synchronize()
            assert float(junk) == float(junk)
            assert np.all(host(info) == 0)
            assert np.array_equal(host(x), ref), k
    plan.close()


def test_persistent_launches_match_ordinary(pne, small_batch, tmp_path, monkeypatch):
    """The grouped MFMA products run as persistent launches (as many
    work-groups as fit, taking their tiles from a counter in the group
    table) give bitwise the results of the ordinary grouped launches, in a
    one-shot call and in a plan replayed three times from a hipGraph (the
    counters must be back at zero after every launch)."""
    import json
    probs, _ = small_batch
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PNE_TUNE_CACHE", str(cache))
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=13, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    pne.autotune_batched(A, b, x, descs, opts=o)
    (key, entry), = json.loads(cache.read_text()).items()
    outs = {}
    for pe in (0, 1):
        # a different file size, so that the library reads the file again
        cache.write_text(json.dumps({key: dict(entry, persistent=pe)}, indent=1 + 3 * pe))
        x.zero_()
        info = pne.pne_solve_batched(A, b, x, descs, opts=o)
        assert np.all(host(info) == 0)
        outs[pe] = host(x).copy()
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            plan = pne.BatchPlan(A, b, x, descs, opts=o, stream=st)
            for k in range(3):
                x.fill_(float("nan"))
                info = plan.execute_graph(st)
                st.synchronize()
                assert np.all(host(info) == 0)
                assert np.array_equal(host(x), outs[pe]), (pe, k)
        plan.close()
    assert np.array_equal(outs[0], outs[1])


def test_autotuner_stores_and_reuses_parameters(pne, small_batch, tmp_path, monkeypatch):
    """The autotuner times its candidates on the batch, stores the fastest in
    $PNE_TUNE_CACHE; later batched calls of the same workload read it back
    (their results equal a plan built with the stored parameters) and stay
    accurate."""
    import json
    probs, err_qr = small_batch
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("PNE_TUNE_CACHE", str(cache))
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=7, sketch_prec="bf16", qr_prec="fp32", refine_steps=2)
    res = pne.autotune_batched(A, b, x, descs, opts=o)
    assert res["stored"] and res["ms"] > 0
    assert res["batch_kchunk"] in (4096, 8192, 16384) and res["shortk_tile"] in (64, 128)
    assert res["persistent"] in (False, True)
    data = json.loads(cache.read_text())
    assert len(data) == 1
    (key, entry), = data.items()
    assert key.startswith("batched/pne/sk4/qr2/") and entry["batch_kchunk"] == res["batch_kchunk"]
    assert entry["persistent"] == int(res["persistent"])
    x.zero_()
    info = pne.pne_solve_batched(A, b, x, descs, opts=o)
    assert np.all(host(info) == 0)
    xb = host(x).copy()
    plan = pne.BatchPlan(A, b, x, descs, opts=o)
    x.zero_()
    plan.execute()
    assert np.array_equal(host(x), xb)
    plan.close()
    for i, (p, d) in enumerate(zip(probs, descs)):
        assert relerr(xb[d["x_offset"]:d["x_offset"] + p.n], p.numpy_x_star()) <= 10 * err_qr[i]


# ------------------------------------------------------------------ 512 problems

def test_batch512_known_solutions(pne):
    """512 problems, m ~ U[2000, 50000], n ~ U[32, 512] with m >= 20 n,
    kappa log-uniform in [1e2, 1e8], residual log-uniform in [1e-10, 1e-2],
    BF16 sketches (s = 3n), FP32 QR, three FP64 refinement steps: every member
    within 10x the first-order least-squares bound kappa u (1 + kappa rho)."""
    shapes = draw_batch_shapes(512, 0)
    probs = [make_problem(m, n, k, r, seed=40000 + i, device="cuda") for i, (m, n, k, r) in enumerate(shapes)]
    A, b, x, descs = pack(probs)
    xs = [host(p.x_star) for p in probs]
    for p in probs:
        p.At = None
    torch.cuda.empty_cache()
    o = pne.make_opts(seed=0, sketch_prec="bf16", qr_prec="fp32", refine_steps=3)
    info = host(pne.pne_solve_batched(A, b, x, descs, opts=o))
    assert np.all(info == 0), np.nonzero(info)
    xb = host(x)
    bad = []
    for i, (p, d) in enumerate(zip(probs, descs)):
        e = relerr(xb[d["x_offset"]:d["x_offset"] + p.n], xs[i])
        bound = p.kappa * U64 * (1 + p.kappa * p.rho)
        if not e <= 10 * bound:
            bad.append((i, p.m, p.n, p.kappa, p.rho, e, bound))
    assert not bad, bad[:10]
    # the same batch as a plan captured into a hipGraph: two replays match
    # the uncaptured call bit for bit
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan = pne.BatchPlan(A, b, x, descs, opts=o, stream=st)
        for k in range(2):
            x.fill_(float("nan"))
            info = plan.execute_graph(st)
            st.synchronize()
            assert np.all(host(info) == 0)
            assert np.array_equal(host(x), xb), k
        plan.close()


def test_batch512_sampled_members_within_qr_error(pne):
    """Sixteen members of the 512-problem batch, generated on the CPU as the
    stored oracle QR errors were (tests/golden/err_qr_full_size.txt, written by
    tests/golden/make_err_qr.py) and solved together in one batched call with
    their member indices as problem ids: members never interact and every
    member's products are cut into the same fixed row chunks in any batch, so
    each result is the one the member gets inside the full batch.  Each is
    within 10x the oracle QR solver's own error."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "err_qr_full_size.txt")
    rows = [l.split() for l in open(path) if l.startswith("batch512_member")]
    assert len(rows) == 16
    shapes = draw_batch_shapes(512, 0)
    probs, errs, ids = [], [], []
    for t in rows:
        i = int(t[0][len("batch512_member"):])
        m, n, k, r = shapes[i]
        assert (m, n, int(t[5])) == (int(t[1]), int(t[2]), 40000 + i)
        probs.append(make_problem(m, n, k, r, seed=40000 + i, device="cpu"))
        errs.append(float(t[6]))
        ids.append(i)
    A, b, x, descs = pack(probs)
    for d, i in zip(descs, ids):
        d["problem_id"] = i
    o = pne.make_opts(seed=0, sketch_prec="bf16", qr_prec="fp32", refine_steps=3)
    info = host(pne.pne_solve_batched(A, b, x, descs, opts=o))
    assert np.all(info == 0)
    xb = host(x)
    bad = []
    for p, d, e_qr, i in zip(probs, descs, errs, ids):
        e = relerr(xb[d["x_offset"]:d["x_offset"] + p.n], p.numpy_x_star())
        if not e <= 10 * e_qr:
            bad.append((i, p.m, p.n, p.kappa, p.rho, e, e_qr))
    assert not bad, bad


def test_batch_repeatable_bitwise(pne):
    """128 members of the batch distribution (m up to 50000, n up to 512:
    tens of thousands of work-groups per grouped launch), solved four times
    into the same output: every run gives the same x bit for bit and no info
    code.  The sums of the library run in a fixed order, so a difference can
    only come from a race between work-groups."""
    shapes = draw_batch_shapes(128, 3)
    probs = [make_problem(m, n, k, r, seed=50000 + i, device="cuda") for i, (m, n, k, r) in enumerate(shapes)]
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=0, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    x0 = None
    for _ in range(4):
        x.fill_(float("nan"))
        info = host(pne.pne_solve_batched(A, b, x, descs, opts=o))
        assert np.all(info == 0)
        xr = host(x).copy()
        if x0 is None:
            x0 = xr
        else:
            assert np.array_equal(xr, x0)


def test_batched_check_finite(pne, small_batch):
    """check_finite in a batched call: a NaN in one member's b makes the call
    return PNE_EINVAL; with finite inputs the result equals the unchecked
    call's bit for bit."""
    probs, _ = small_batch
    A, b, x, descs = pack(probs)
    o = pne.make_opts(seed=9, sketch_prec="bf16", qr_prec="fp32", refine_steps=1, check_finite=True)
    o0 = pne.make_opts(seed=9, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    pne.pne_solve_batched(A, b, x, descs, opts=o0)
    x0 = host(x).copy()
    x.zero_()
    info = host(pne.pne_solve_batched(A, b, x, descs, opts=o))
    assert np.all(info == 0) and np.array_equal(x0, host(x))
    d = descs[3]
    b[d["b_offset"] + 5] = float("nan")
    with pytest.raises(pne.PneError) as e:
        pne.pne_solve_batched(A, b, x, descs, opts=o)
    assert e.value.status == -1
