#!/usr/bin/env python3
"""Throughput of the randomized PNE least-squares solve on one MI355X.

Workload (single problem): m = 100,000, n = 1,000, kappa(A) = 1e6 (geometric
singular values), relative residual 1e-4, Gaussian sketch s = 3,000.  One
step = one complete pne_solve (sketch, sketch QR, A R_s^{-1}, Gram, Cholesky,
triangular solves, FP64 refinement) on inputs already resident in HBM.

The headline is the mixed-precision path (BF16 sketch with FP32
accumulation, FP32 QR, one FP64 refinement step); the all-FP64 path and the
FP32 preconditioner are timed beside it on the same input, with their
errors against the known solution.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

M, N, KAPPA, RHO, S = 100_000, 1000, 1e6, 1e-4, 3000
WORKLOAD = "ls_100000x1000_k1e6_rho1e-4_s3000"
METRIC = "LS solves/sec + MFMA roofline %, mixed vs FP64 PNE/HPNE at equal rel. error"
PEAK_FP64 = 78.6e12      # dense FP64 MFMA, FLOP/s
PEAK_BF16 = 2.5e15       # dense BF16 MFMA, FLOP/s
PEAK_HBM = 8.0e12        # B/s
U64 = 2.0 ** -53
COPY_PROBE_BYTES = 512 << 20   # read once and written once by the copy probe


# --only: name -> (solver, options of make_opts); solver "qr" is qr_ls_solve
ONLY_CASES = {
    "mixed_pne": ("pne", dict(sketch_prec="bf16", qr_prec="fp32", refine_steps=1)),
    "mixed_hpne": ("hpne", dict(sketch_prec="bf16", qr_prec="fp32", refine_steps=1)),
    "fp64_pne": ("pne", dict(sketch_prec="fp64", qr_prec="fp64", refine_steps=0)),
    "fp64_hpne": ("hpne", dict(sketch_prec="fp64", qr_prec="fp64", refine_steps=0)),
    "srft_fp32_pne": ("pne", dict(sketch_prec="fp32", qr_prec="fp32", refine_steps=0, sketch_kind="srft")),
    "qr_solver": ("qr", None),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="mixed path only (profiling runs)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 512-problem batched measurement")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the m = 1e6 (AUTO) and m = 4e6 (FP8 HPNE) single-problem measurements")
    ap.add_argument("--batch-only", action="store_true",
                    help="only the 512-problem batched measurement (profiling runs); prints its JSON object")
    ap.add_argument("--only", choices=sorted(ONLY_CASES),
                    help="time one solver configuration on the single-problem workload and print "
                         "its JSON object (profiling runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="run one plain elementwise copy (torch.neg) of 512 MiB first, so that "
                         "hardware byte counters can be scaled against a kernel of known traffic")
    return ap.parse_args()


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2603_16644_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def time_solver(pne, prob, opts, steps, warmup, hpne=False, profile=False):
    import torch
    fn = pne.hpne_solve if hpne else pne.pne_solve
    x = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    L = pne.lib()
    for _ in range(warmup):
        fn(prob.A, prob.b, x=x, opts=opts)
    torch.cuda.synchronize()
    phases = []
    if profile:
        L.pne_profile_enable(1)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, info, _ = fn(prob.A, prob.b, x=x, opts=opts)
            if profile:
                ms = (ctypes.c_double * 16)()
                cnt = L.pne_profile_read(ms, 16)
                phases.append({L.pne_profile_phase_name(i).decode(): ms[i] for i in range(cnt)})
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    finally:
        if profile:
            L.pne_profile_enable(0)
    assert int(info.item()) == 0, f"solver info {int(info.item())}"
    xs = prob.x_star
    err = float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs))
    return (t1 - t0) / steps, err, phases


def time_qr_solver(pne, prob, steps, warmup):
    """The FP64 Householder-QR least-squares solver (qr_ls_solve) on the
    same problem: seconds per solve and relative error."""
    import torch
    x = torch.empty(prob.n, dtype=torch.float64, device="cuda")
    for _ in range(warmup):
        pne.qr_ls_solve(prob.A, prob.b, x=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, info = pne.qr_ls_solve(prob.A, prob.b, x=x)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert int(info.item()) == 0, f"qr solver info {int(info.item())}"
    err = float(torch.linalg.norm(x - prob.x_star) / torch.linalg.norm(prob.x_star))
    return (t1 - t0) / steps, err


def mean_phases(phases):
    keys = phases[0].keys()
    out = {}
    for k in keys:
        v = [p[k] for p in phases if p[k] >= 0]
        if v:
            out[k] = sum(v) / len(v)
    return out


def roofline(ph):
    """Dominant single-kernel phase against its MFMA peak (algorithmic flops)."""
    cands = {
        # C = A_p^T A_p (lower triangle incl. diagonal) and c = A_p^T b
        "gram_gemm": (M * N * (N + 1) + 2 * M * N, PEAK_FP64, "GemmCm<double,double,double,128,128,true>"),
        # A_s = Omega A, BF16 operands
        "sketch_gemm": (2 * S * M * N, PEAK_BF16, "GemmLp<bf16,false>"),
    }
    best = max(cands, key=lambda k: ph.get(k, 0.0))
    flops, peak, kname = cands[best]
    t = ph[best] * 1e-3
    achieved = flops / t
    traffic = None
    tf = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tf):
        try:
            rec = json.load(open(tf)).get(best)
            if rec and rec.get("source_hash") == source_hash(*rec.get("source_files", ["?"])):
                traffic = rec["bytes_per_launch"]
        except (ValueError, OSError):
            traffic = None
    return {"kernel": kname, "phase": best, "bound": "mfma", "achieved": achieved / 1e12,
            "peak": peak / 1e12, "unit": "TFLOP/s", "frac": achieved / peak, "traffic": traffic,
            "ms_per_launch": ph[best], "algorithmic_flops": flops}


def time_batched(pne, steps, warmup):
    """512 independent problems (m ~ U[2000, 50000], n ~ U[32, 512], m >= 20 n,
    kappa log-uniform in [1e2, 1e8], residual log-uniform in [1e-10, 1e-2]),
    BF16 sketches with s = 3n, FP32 QR, one FP64 refinement step, solved by
    pne_solve_batched (grouped launches).  Returns solves/s and, per member,
    whether the error is within 10x kappa u (1 + kappa rho)."""
    import torch

    from workloads import draw_batch_shapes, make_problem, pack_batch
    shapes = draw_batch_shapes(512, 0)
    probs = [make_problem(m, n, k, r, seed=40000 + i, device="cuda") for i, (m, n, k, r) in enumerate(shapes)]
    A, b, x, descs = pack_batch(probs, release=True)
    xs = [p.x_star for p in probs]
    torch.cuda.empty_cache()
    L = pne.lib()
    out = {"workload": "batch512_m2000-50000_n32-512_k1e2-1e8", "problems": len(probs),
           "sum_mn": int(sum(p.m * p.n for p in probs))}
    for refine in (1, 3):
        o = pne.make_opts(seed=0, sketch_prec="bf16", qr_prec="fp32", refine_steps=refine)
        for _ in range(warmup):
            pne.pne_solve_batched(A, b, x, descs, opts=o)
        torch.cuda.synchronize()
        L.pne_profile_enable(1)
        t0 = time.perf_counter()
        for _ in range(steps):
            info = pne.pne_solve_batched(A, b, x, descs, opts=o)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms = (ctypes.c_double * 16)()
        cnt = L.pne_profile_read(ms, 16)
        L.pne_profile_enable(0)
        phases = {L.pne_profile_phase_name(i).decode(): round(ms[i], 4) for i in range(cnt) if ms[i] >= 0}
        ok = 0
        for p, d, xstar in zip(probs, descs, xs):
            xi = x[d["x_offset"]:d["x_offset"] + p.n]
            e = float(torch.linalg.norm(xi - xstar) / torch.linalg.norm(xstar))
            ok += e <= 10 * p.kappa * U64 * (1 + p.kappa * p.rho)
        dt = (t1 - t0) / steps
        out[f"refine{refine}"] = {"solves_per_s": len(probs) / dt, "ms": dt * 1e3,
                                  "members_within_bound": int(ok), "info_nonzero": int((info != 0).sum()),
                                  "phases_ms": phases}
    # the same batch as a plan (tables uploaded once) replayed as a hipGraph
    o = pne.make_opts(seed=0, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        plan = pne.BatchPlan(A, b, x, descs, opts=o, stream=st)
        plan.execute_graph(st)
        st.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = plan.execute_graph(st)
        st.synchronize()
        t1 = time.perf_counter()
        plan.close()
    dt = (t1 - t0) / steps
    out["refine1_plan_graph"] = {"solves_per_s": len(probs) / dt, "ms": dt * 1e3,
                                 "info_nonzero": int((info != 0).sum())}
    return out


def host_cpu():
    """Core count and CPU model of the host the oracle runs on."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": model}


def oracle_config1():
    """The oracle's whole solve of the m = 1000, n = 100 problem (kappa 1e8,
    rho 1e-6, s = 300, FP32 preconditioner, one refinement step), and its QR
    solver on the same problem: wall seconds and errors."""
    import numpy as np

    import oracle
    from workloads import make_problem
    p = make_problem(1000, 100, 1e8, 1e-6, seed=1001)
    A, b, xs = p.numpy_A(), p.numpy_b(), p.numpy_x_star()
    t0 = time.perf_counter()
    r = oracle.solve(A, b, s=300, seed=1, sketch_prec="fp32", qr_prec="fp32", refine_steps=1)
    t1 = time.perf_counter()
    xq = oracle.qr_ls(A, b)
    t2 = time.perf_counter()
    rel = lambda x: float(np.linalg.norm(x - xs) / np.linalg.norm(xs))
    return {"pne_s": round(t1 - t0, 4), "pne_rel_err": rel(r["x"]), "qr_ls_s": round(t2 - t1, 4),
            "qr_ls_rel_err": rel(xq)}


def cpu_baseline(prob, ms_rows=5000):
    """Oracle (plain single-threaded C, FP64 with BF16 operand emulation) timed
    per step on the first `ms_rows` rows of the same A; the row-proportional
    steps are scaled by M / ms_rows, the rest (QR, Cholesky, solves) taken as
    measured."""
    import numpy as np

    import oracle
    A = prob.numpy_A()[:ms_rows]
    A = np.asfortranarray(A)
    b = prob.numpy_b()[:ms_rows]
    oracle.lib()
    t = {}
    t0 = time.perf_counter()
    As = oracle.sketch(A, S, seed=2, prec="bf16")
    t["sketch"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    R = oracle.householder_r(As.astype(np.float32).astype(np.float64))
    t["qr"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    Ap, _ = oracle.precondition(A, R)
    t["trsm"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    C, c = oracle.gram(Ap, Ap, b)
    t["gram"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    L, info = oracle.cholesky(C)
    y = oracle.cholesky_solve(L, c)
    x, _ = oracle.upper_solve(R, y)
    t["factor_solve"] = time.perf_counter() - t0
    scale = M / ms_rows
    # the refinement's two matrix-vector passes (4mn flops) are below 0.1% of
    # the sketch and are not timed
    per_solve = scale * (t["sketch"] + t["trsm"] + t["gram"]) + t["qr"] + 2 * t["factor_solve"]
    sample_s = sum(t.values())
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": 1, "kind": "oracle", "host": host_cpu(),
            "config1_whole_solve": oracle_config1(),
            "sample": (f"oracle steps on the first {ms_rows} of {M} rows (n={N}, s={S}, BF16 operand "
                       f"emulation, single thread, {sample_s:.1f} s of CPU work); row-proportional steps "
                       f"(sketch, A R^-1, Gram) scaled by {scale:.0f}x, QR/Cholesky/"
                       f"solves as measured"),
            "phase_seconds": {k: round(v, 3) for k, v in t.items()}}


def time_large(pne, steps, warmup):
    """The two largest single-problem workloads (generated on the device):
    m = 1e6, n = 2000, kappa = 1e10 (half the singular values 1), rho = 1e-8,
    s = 6000: AUTO precision with one refinement step, and the forced FP32
    preconditioner with one step; m = 4e6, n = 1000, kappa = 1e8, rho = 1e-6,
    s = 4000: HPNE with an FP8 e4m3 sketch (per-128-row-block scales), FP32
    QR and two refinement steps, against the all-FP64 HPNE."""
    import gc

    import torch

    from workloads import make_problem
    out = {}
    p3 = make_problem(1_000_000, 2000, 1e10, 1e-8, seed=1003, sigma="half_ones", device="cuda")
    torch.cuda.synchronize()
    b3 = 1e10 * U64 * (1 + 1e10 * 1e-8)
    rows = {}
    for name, o, hp in [("auto_pne_refine1", pne.make_opts(s=6000, seed=3, sketch_prec="auto", qr_prec="auto",
                                                            refine_steps=1), False),
                        ("fp32_pne_refine1", pne.make_opts(s=6000, seed=3, sketch_prec="fp32", qr_prec="fp32",
                                                           refine_steps=1), False)]:
        print(f"[bench] timing m=1e6 n=2000 {name}", file=sys.stderr, flush=True)
        t, e, _ = time_solver(pne, p3, o, steps, warmup, hpne=hp)
        _, _, meta = pne.pne_solve(p3.A, p3.b, opts=o)
        rows[name] = {"solves_per_s": 1.0 / t, "ms": t * 1e3, "rel_err": e, "precision": meta["qr_prec"]}
    out["ls_1000000x2000_k1e10"] = dict(rows, lemma_bound=b3)
    p3.At = p3.b = p3.x_star = None
    del p3
    gc.collect()
    torch.cuda.empty_cache()
    p5 = make_problem(4_000_000, 1000, 1e8, 1e-6, seed=1005, device="cuda")
    torch.cuda.synchronize()
    b5 = 1e8 * U64 * (1 + 1e8 * 1e-6)
    rows = {}
    for name, o in [("fp8_hpne_refine2", pne.make_opts(s=4000, seed=5, sketch_prec="fp8", qr_prec="fp32",
                                                       refine_steps=2)),
                    ("fp64_hpne", pne.make_opts(s=4000, seed=5, sketch_prec="fp64", qr_prec="fp64",
                                                refine_steps=0))]:
        print(f"[bench] timing m=4e6 n=1000 {name}", file=sys.stderr, flush=True)
        t, e, _ = time_solver(pne, p5, o, steps, warmup, hpne=True)
        rows[name] = {"solves_per_s": 1.0 / t, "ms": t * 1e3, "rel_err": e}
    out["ls_4000000x1000_k1e8"] = dict(rows, lemma_bound=b5)
    p5.At = p5.b = p5.x_star = None
    del p5
    gc.collect()
    torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                                   "(how the solve would shard over GPUs is a design note only; no multi-GPU path is built)"}))
        sys.exit(2)
    import torch

    import paper_2603_16644_amd as pne
    from workloads import make_problem
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.batch_only:
        print("[bench] timing the 512-problem batch", file=sys.stderr, flush=True)
        print(json.dumps(time_batched(pne, args.steps, args.warmup)))
        return
    print(f"[bench] generating m={M} n={N} kappa={KAPPA:g} rho={RHO:g}", file=sys.stderr, flush=True)
    prob = make_problem(M, N, KAPPA, RHO, seed=1002, device="cuda")
    torch.cuda.synchronize()
    if args.only:
        solver, kw = ONLY_CASES[args.only]
        print(f"[bench] timing {args.only}", file=sys.stderr, flush=True)
        if solver == "qr":
            t, e = time_qr_solver(pne, prob, args.steps, args.warmup)
        else:
            t, e, _ = time_solver(pne, prob, pne.make_opts(s=S, seed=2, **kw), args.steps, args.warmup,
                                  hpne=solver == "hpne")
        print(json.dumps({"case": args.only, "workload": WORKLOAD, "ms": t * 1e3, "rel_err": e,
                          "steps": args.steps, "warmup": args.warmup}))
        return
    if args.copy_probe:
        src = torch.zeros(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst
    bound = KAPPA * U64 * (1 + KAPPA * RHO)

    mixed = pne.make_opts(s=S, seed=2, sketch_prec="bf16", qr_prec="fp32", refine_steps=1)
    print("[bench] timing mixed PNE", file=sys.stderr, flush=True)
    t_mix, e_mix, ph = time_solver(pne, prob, mixed, args.steps, args.warmup, profile=True)
    phases = mean_phases(ph)
    out_extra = {}
    if not args.quick:
        fp64 = pne.make_opts(s=S, seed=2, sketch_prec="fp64", qr_prec="fp64", refine_steps=0)
        fp32 = pne.make_opts(s=S, seed=2, sketch_prec="fp32", qr_prec="fp32", refine_steps=0)
        print("[bench] timing FP64 PNE", file=sys.stderr, flush=True)
        t64, e64, ph64 = time_solver(pne, prob, fp64, args.steps, args.warmup, profile=True)
        print("[bench] timing FP32-preconditioner PNE", file=sys.stderr, flush=True)
        t32, e32, _ = time_solver(pne, prob, fp32, args.steps, args.warmup)
        print("[bench] timing mixed HPNE", file=sys.stderr, flush=True)
        th, eh, phh = time_solver(pne, prob, mixed, args.steps, args.warmup, hpne=True, profile=True)
        print("[bench] timing FP64 HPNE", file=sys.stderr, flush=True)
        th64, eh64, phh64 = time_solver(pne, prob, fp64, args.steps, args.warmup, hpne=True, profile=True)
        # the paper's GPU setting (Section 7.4): SRFT sketch, FP32 preconditioner
        srft32 = pne.make_opts(s=S, seed=2, sketch_prec="fp32", qr_prec="fp32", refine_steps=0, sketch_kind="srft")
        srftbf = pne.make_opts(s=S, seed=2, sketch_prec="bf16", qr_prec="fp32", refine_steps=1, sketch_kind="srft")
        print("[bench] timing SRFT PNE", file=sys.stderr, flush=True)
        ts32, es32, phs32 = time_solver(pne, prob, srft32, args.steps, args.warmup, profile=True)
        tsbf, esbf, _ = time_solver(pne, prob, srftbf, args.steps, args.warmup)
        print("[bench] timing the FP64 QR solver", file=sys.stderr, flush=True)
        tq, eq = time_qr_solver(pne, prob, args.steps, args.warmup)
        out_extra = {
            "fp64_pne": {"solves_per_s": 1.0 / t64, "ms": t64 * 1e3, "rel_err": e64,
                         "phases_ms": {k: round(v, 4) for k, v in mean_phases(ph64).items()}},
            "fp32_precond_pne": {"solves_per_s": 1.0 / t32, "ms": t32 * 1e3, "rel_err": e32},
            "mixed_hpne": {"solves_per_s": 1.0 / th, "ms": th * 1e3, "rel_err": eh,
                           "phases_ms": {k: round(v, 4) for k, v in mean_phases(phh).items()}},
            "fp64_hpne": {"solves_per_s": 1.0 / th64, "ms": th64 * 1e3, "rel_err": eh64,
                          "phases_ms": {k: round(v, 4) for k, v in mean_phases(phh64).items()}},
            "srft_fp32_precond_pne": {"solves_per_s": 1.0 / ts32, "ms": ts32 * 1e3, "rel_err": es32,
                                      "phases_ms": {k: round(v, 4) for k, v in mean_phases(phs32).items()}},
            "srft_bf16_pne_refine1": {"solves_per_s": 1.0 / tsbf, "ms": tsbf * 1e3, "rel_err": esbf},
            "qr_solver": {"solves_per_s": 1.0 / tq, "ms": tq * 1e3, "rel_err": eq,
                          "kind": "FP64 Householder QR of [A b] (TSQR tree), Q never formed"},
            "speedup_vs_qr_solver": tq / t_mix,
            "speedup_vs_fp64": t64 / t_mix,
            "hpne_speedup_vs_fp64": th64 / th,
            "equal_error": bool(e_mix <= 10 * max(e64, bound * 1e-3) and e_mix <= 10 * bound),
        }
    line = {
        "metric": METRIC, "value": 1.0 / t_mix, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": t_mix * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f32+f64", "data": "synthetic",
        "config": {"workload": WORKLOAD, "m": M, "n": N, "kappa": KAPPA, "rho": RHO, "s": S,
                   "solver": "pne", "sketch_prec": "bf16", "qr_prec": "fp32", "refine_steps": 1,
                   "parallelism": "single"},
        "rel_err": e_mix, "lemma_bound": bound,
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "roofline": roofline(phases),
    }
    line.update(out_extra)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(prob)
    else:
        line["cpu_baseline"] = None
    if not args.quick and not args.no_batch:
        print("[bench] timing the 512-problem batch", file=sys.stderr, flush=True)
        del prob
        torch.cuda.empty_cache()
        line["batch512"] = time_batched(pne, max(2, args.steps // 2), 1)
    if not args.quick and not args.no_large:
        line["large"] = time_large(pne, 2, 1)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
