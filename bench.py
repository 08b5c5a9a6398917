"""Benchmark: one step = one full sketch-and-precondition solve (Alg. 1:
sketch generation, sketch apply, Householder QR of the sketch, x0, LSQR to
tolerance) of the FP64 workload m = 2^20, n = 1000, d = 4000, zeta = 8 on one
MI355X, with A and b resident in HBM before the timed region.

Prints ONE JSON line.  `value` is solves per second of that workload;
`roofline` reports the dominant kernel (the fused LSQR pass over A) from
HIP-event timings taken on its own stream inside the timed region;
`cpu_baseline` times the CPU oracle on a bounded row sample of the same
workload and projects it to the full size.  `forms` adds the other three
forms, each against the plain FP64 form on the same problems at the same
accuracy (the FP64 form's loosest LSQR tolerance whose results are as close
to the FP64 reference as the mixed form's):
  * mixed   - one large solve, m = 2^22, n = 4096, d = 2n, A stored in FP32 (FP64
              arithmetic; FP32 refinement; BF16-input sketch with refinement);
  * batched - 512 uneven FP32 problems in one sap_solve_batch call, refinement
              form against the FP64 batched form and FP64 single solves;
  * served  - a Poisson request stream (200 req/s for 10 s) through
              sap_submit/poll, refinement form against the FP64 form served
              the same way, with p50/p99 latency.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time & SA/GEMV GB/s, mixed vs FP64 at rel-err 1e-8; p50/p99 solve latency"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_GFLOPS = 78600.0  # MI355X dense FP64 (vector and matrix)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=1 << 16)
    ap.add_argument("--m", type=int, default=1 << 20)
    ap.add_argument("--n", type=int, default=1000)
    ap.add_argument("--d", type=int, default=4000)
    ap.add_argument("--zeta", type=int, default=8)
    ap.add_argument("--fig5-m", type=int, default=600000)
    ap.add_argument("--fig5-n", default="300,600,1000,1300")
    ap.add_argument("--forms", default="mixed,batched,served,fig5,sparse,hbm",
                    help="comma list of extra forms to run (mixed, batched, served, fig5, sparse, hbm; empty for none)")
    ap.add_argument("--hbm-m", type=int, default=1 << 19)
    ap.add_argument("--hbm-n", type=int, default=500)
    ap.add_argument("--sparse-m", type=int, default=500000)
    ap.add_argument("--sparse-n", type=int, default=500)
    ap.add_argument("--sparse-reps", type=int, default=5)
    ap.add_argument("--mixed-m", type=int, default=1 << 22)
    ap.add_argument("--mixed-n", type=int, default=4096)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-duration", type=float, default=10.0)
    ap.add_argument("--serve-pool", type=int, default=256,
                    help="distinct problems in the served stream's device-resident pool")
    ap.add_argument("--no-adaptive-d", action="store_true",
                    help="skip the solve at the embedding dimension of eq. (4.2)")
    ap.add_argument("--gaussian-input", action="store_true",
                    help="column-scaled Gaussian A of the same shape instead of the SVD-built one (cheap to "
                         "generate; for counter runs, where the kernels move the same bytes)")
    ap.add_argument("--kernel", choices=["apply", "qr", "batch"], default=None,
                    help="time one kernel alone instead of the solve (for profiler runs): 'apply' times "
                         "sps_apply (Y = S [A b]) on an --m x --n matrix of --a-dtype into a --y-dtype Y; "
                         "'qr' times sap_qr on a --d x (--n + 1) FP64 matrix; 'batch' times the batched "
                         "refinement form on the --batch-count problems of the batched form")
    ap.add_argument("--a-dtype", choices=["f64", "f32", "bf16"], default="f64")
    ap.add_argument("--y-dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--copy-ref-mib", type=int, default=2048,
                    help="size of the plain device-to-device copy timed as the achievable-bandwidth reference")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(A, b, m, d, zeta, seed, tol, iters_gpu):
    """Oracle (plain C, one thread) on the first rows of the workload (A, b:
    host arrays of that sample); per-phase times projected to the full m
    (generation, apply and each LSQR iteration scale with m; the QR of the
    d x (n+1) sketch does not), using the GPU's iteration count."""
    import oracle
    rows = A.shape[0]
    t0 = time.perf_counter()
    x, info = oracle.solve(A, b, d, zeta, seed, tol=tol, maxiter=200)
    wall = time.perf_counter() - t0
    scale = m / rows
    per_iter = info["t_iterate"] / max(1, info["iters"])
    t_full = (info["t_generate"] + info["t_apply"]) * scale + info["t_qr"] + per_iter * scale * iters_gpu
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle solve on the first {rows} of {m} rows (n={A.shape[1]}, d={d}, zeta={zeta}): "
                       f"{wall:.1f} s wall, generate {info['t_generate']:.2f} s, apply {info['t_apply']:.2f} s, "
                       f"QR {info['t_qr']:.2f} s, {info['iters']} LSQR iterations {info['t_iterate']:.2f} s; "
                       f"projected to m={m} with {iters_gpu} iterations: {t_full:.1f} s per solve")}


def rel(a, b):
    import torch
    return (torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b)).item()


def widen(A32):
    """FP64 copy of an FP32 matrix (exact), built in row chunks."""
    import torch
    A64 = torch.empty(A32.shape, dtype=torch.float64, device=A32.device)
    step = 1 << 18
    for r0 in range(0, A32.shape[0], step):
        A64[r0:r0 + step] = A32[r0:r0 + step].to(torch.float64)
    return A64


def copy_reference(torch, mib):
    """Plain device-to-device copy of `mib` MiB (torch's copy_ between
    same-typed tensors, which the HIP runtime runs as its blit copy kernel),
    timed with HIP events: the streaming bandwidth a plain copy reaches on
    this GPU, and the known-size kernel that calibrates the HBM byte
    counters."""
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_moved": 2 * (mib << 20), "avg_ms": ms, "gbs": 2 * (mib << 20) / (ms * 1e-3) / 1e9}


TRAFFIC_PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles",
                               "lsqr_pass_fp64_m1048576_n1000_counters.md")
# the fused pass's own code: (file, first marker, last marker)
PASS_SOURCES = (("lsqr.hip", "[fused-pass-begin]", "[fused-pass-end]"),
                ("common.h", "[wave-helpers-begin]", "[wave-helpers-end]"))


def pass_sources_sha256():
    """Hash of the fused pass kernel's code (the marked regions), so that the
    committed HBM counters are reported only while they describe it."""
    import hashlib
    h = hashlib.sha256()
    for f, b, e in PASS_SOURCES:
        with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2506_03070_amd", "csrc", f),
                  encoding="utf-8") as fh:
            text = fh.read()
        i, j = text.index(b), text.index(e)
        h.update(text[i:j].encode("utf-8"))
    return h.hexdigest()


def measured_traffic(m, n):
    """HBM bytes per full pass launch from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated against a copy of known size), or
    None when the workload differs or the pass kernel's sources changed since
    the counters were taken."""
    if (m, n) != (1 << 20, 1000) or not os.path.exists(TRAFFIC_PROFILE):
        return None
    fields = {}
    with open(TRAFFIC_PROFILE) as fh:
        for line in fh:
            mt = re.match(r"^\s*(traffic_bytes_per_launch|sources_sha256):\s*(\S+)", line)
            if mt:
                fields[mt.group(1)] = mt.group(2)
    if fields.get("sources_sha256") != pass_sources_sha256() or "traffic_bytes_per_launch" not in fields:
        return None
    return int(fields["traffic_bytes_per_launch"])


def pass_bytes(m, n, esize):
    # the fused pass reads A once and u once and writes u once (p, the
    # per-workgroup partials and the state are < 0.3%)
    return m * n * esize + 2 * m * 8


def qr_flops(d, nc):
    # Householder QR of a d x nc matrix: 2 d nc^2 - 2 nc^3 / 3
    return 2.0 * d * nc * nc - 2.0 * nc ** 3 / 3.0


def apply_bytes(m, n, d, zeta, esize, ysize):
    # A and b once, the sketch (zeta int32 + one 64-bit sign word per row), Y once
    return m * n * esize + m * 8 + m * (zeta * 4 + 8) + d * (n + 1) * ysize


# Target relative error of the mixed-precision forms, and the LSQR tolerances
# tried for the FP64 form when matching that accuracy (the loosest one whose
# results are as accurate is the comparison point).
TARGET_REL_ERR = 1e-8
FP64_MATCH_TOLS = (1e-8, 1e-10)


def pick_matching(runs, bound):
    """The first run (loosest tolerance first) whose max relative error is
    within `bound`, else the last (tightest) one."""
    for r in runs:
        if r["rel_err_max"] <= bound:
            return r
    return runs[-1]


def form_mixed(args, sap, torch, inputs):
    """Mixed forms on one large matrix (A stored FP32) against the FP64 form
    on its exact FP64 copy.  Accuracy of every result is measured against the
    FP64 form at tol 1e-12; the FP64 form is also run at looser tolerances and
    the loosest one that is as accurate as the refinement form is the
    same-accuracy comparison."""
    m, n = args.mixed_m, args.mixed_n
    log(f"bench[mixed]: generating m={m} n={n} FP32 A")
    A32, b, _, meta = inputs.config2_torch("cuda", m=m, n=n)
    d, zeta, seed, tol, maxiter = meta["d"], meta["zeta"], meta["sketch_seed"], meta["tol"], meta["maxiter"]
    ctx = sap.default_context(0)

    def timed(A, mode, tol_, warm=True):
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        mx = maxiter if mode not in (sap.SAP_MODE_MIXED_FP32_REFINE, sap.SAP_MODE_MIXED_BF16SA) else 4 * maxiter
        if warm:
            sap.sap_solve(A, b, d, zeta, seed, tol=tol_, maxiter=mx, x=x, mode=mode)
            torch.cuda.synchronize()
        ctx.profile(True)
        ctx.profile_read(sap.PROF_PASS, reset=True)
        ctx.profile_read(sap.PROF_APPLY, reset=True)
        t0 = time.perf_counter()
        r = sap.sap_solve(A, b, d, zeta, seed, tol=tol_, maxiter=mx, x=x, mode=mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ctx.profile(False)
        npass, mspass = ctx.profile_read(sap.PROF_PASS)
        nap, msap = ctx.profile_read(sap.PROF_APPLY)
        es = A.element_size()
        pb = pass_bytes(m, n, es)
        ab = apply_bytes(m, n, d, zeta, 2 if mode == sap.SAP_MODE_MIXED_BF16SA else es, 8)
        return x, dict(solve_ms=dt * 1e3, status=r.info["status_name"], iters=r.info["iters"],
                       refinements=r.info["refinements"], tol=tol_,
                       phases_ms={"generate": r.info["t_generate_ms"], "apply": r.info["t_apply_ms"],
                                  "qr": r.info["t_qr_ms"], "iterate": r.info["t_iterate_ms"]},
                       pass_gbs=pb / (mspass / max(1, min(npass, r.info["iters"] + max(1, r.info["refinements"])))
                                      * 1e-3) / 1e9,
                       sa_gbs=ab / (msap / max(1, nap) * 1e-3) / 1e9)

    log("bench[mixed]: FP32-storage solve (FP64 arithmetic)")
    xm, rm = timed(A32, sap.SAP_MODE_MIXED_FP32, tol)
    log(f"bench[mixed]: {rm}")
    log("bench[mixed]: FP32 refinement form to a 1e-8 relative correction")
    xr, rr = timed(A32, sap.SAP_MODE_MIXED_FP32_REFINE, TARGET_REL_ERR)
    log(f"bench[mixed]: refine {rr}")
    log("bench[mixed]: BF16-input sketch with the refinement form")
    xb, rb = timed(A32, sap.SAP_MODE_MIXED_BF16SA, TARGET_REL_ERR)
    log(f"bench[mixed]: bf16sa {rb}")
    log("bench[mixed]: widening A to FP64 for the FP64 form")
    A64 = widen(A32)
    del A32
    torch.cuda.empty_cache()
    x64, r64 = timed(A64, sap.SAP_MODE_FP64, tol)
    log(f"bench[mixed]: fp64 tol {tol:g} {r64}")
    fp64_runs = []
    for t in FP64_MATCH_TOLS:
        xt, rt = timed(A64, sap.SAP_MODE_FP64, t, warm=False)
        rt["rel_err_max"] = rel(xt, x64)
        fp64_runs.append(rt)
        log(f"bench[mixed]: fp64 tol {t:g} {rt}")
    del A64
    torch.cuda.empty_cache()
    for r_, x_ in ((rm, xm), (rr, xr), (rb, xb)):
        r_["rel_err_vs_fp64"] = rel(x_, x64)
    match = pick_matching(fp64_runs, max(TARGET_REL_ERR, rr["rel_err_vs_fp64"]))
    return {"workload": f"m={m} n={n} d={d} zeta={zeta}, A_ij = g_ij 10^(-6 j/(n-1)) stored FP32, "
                        f"b = A x + 1e-8 noise; errors relative to the FP64 form at tol {tol:g}",
            "mixed": rm, "refine": rr, "bf16sa": rb, "fp64": r64, "fp64_looser": fp64_runs,
            "fp64_same_accuracy": {"tol": match["tol"], "solve_ms": match["solve_ms"],
                                   "rel_err": match["rel_err_max"]},
            "speedup_mixed_vs_fp64_same_tol": r64["solve_ms"] / rm["solve_ms"],
            "refine_speedup_same_accuracy": match["solve_ms"] / rr["solve_ms"],
            "bf16sa_speedup_same_accuracy": match["solve_ms"] / rb["solve_ms"]}


def _batch_errs(xs, xref):
    e = sorted(rel(a, b) for a, b in zip(xs, xref))
    return {"rel_err_median": e[len(e) // 2], "rel_err_max": e[-1]}


def form_batched(args, sap, torch, inputs):
    """Batched form over uneven FP32 problems: the refinement form (FP32 inner
    passes, FP64 residual, to a 1e-8 relative correction) against the FP64
    form (FP64 copies of the matrices, FP64 arithmetic) in the same batched
    machinery and as one-at-a-time single solves, at the same accuracy.
    Errors are relative to the FP64 batched form at tol 1e-12."""
    shapes = inputs.batch_shapes(count=args.batch_count)
    log(f"bench[batched]: generating {len(shapes)} problems")
    As, bs = [], []
    for s in shapes:
        A, b, _ = inputs.make_problem_torch(s["m"], s["n"], kind="colscale", cond=s["cond"], noise=1e-8,
                                            seed=s["seed"], device="cuda", dtype=torch.float32)
        As.append(A)
        bs.append(b)
    ds = [s["d"] for s in shapes]
    seeds = [s["seed"] + 1 for s in shapes]
    tot_bytes = sum(A.numel() * 4 for A in As)
    A64s = [A.to(torch.float64) for A in As]
    torch.cuda.synchronize()

    def run_batch(Alist, mode, tol, maxiter):
        sap.sap_solve_batch(Alist, bs, ds, 8, seeds, tol=tol, maxiter=maxiter, mode=mode, max_refine=12)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xs, st, infos = sap.sap_solve_batch(Alist, bs, ds, 8, seeds, tol=tol, maxiter=maxiter, mode=mode,
                                            max_refine=12)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = sum(1 for i in infos if i["status"] == sap.SAP_OK)
        its = sorted(i["iters"] for i in infos)
        return xs, {"ms": dt * 1e3, "solves_per_s": len(Alist) / dt, "converged": ok, "tol": tol,
                    "iters_median": its[len(its) // 2]}

    log("bench[batched]: FP64 reference (FP64 batched form, tol 1e-12)")
    xref, rref = run_batch(A64s, sap.SAP_MODE_FP64, 1e-12, 300)
    log("bench[batched]: refinement form")
    xmix, rmix = run_batch(As, sap.SAP_MODE_MIXED_FP32_REFINE, TARGET_REL_ERR, 1000)
    rmix.update(_batch_errs(xmix, xref))
    log(f"bench[batched]: refine {rmix}")
    fp64_runs = []
    for t in FP64_MATCH_TOLS:
        xt, rt = run_batch(A64s, sap.SAP_MODE_FP64, t, 300)
        rt.update(_batch_errs(xt, xref))
        fp64_runs.append(rt)
        log(f"bench[batched]: fp64 tol {t:g} {rt}")
    match = pick_matching(fp64_runs, max(TARGET_REL_ERR, rmix["rel_err_max"]))
    # the FP64 form one solve after another, at the matching tolerance
    x64s = [torch.empty(A.shape[1], dtype=torch.float64, device="cuda") for A in As]
    sap.sap_solve(A64s[0], bs[0], ds[0], 8, seeds[0], tol=match["tol"], maxiter=300, x=x64s[0])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(len(As)):
        sap.sap_solve(A64s[k], bs[k], ds[k], 8, seeds[k], tol=match["tol"], maxiter=300, x=x64s[k])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t0
    seq = {"ms": t_seq * 1e3, "solves_per_s": len(As) / t_seq, "tol": match["tol"]}
    seq.update(_batch_errs(x64s, xref))
    del A64s, As
    torch.cuda.empty_cache()
    return {"workload": f"{len(shapes)} problems, m ~ U[5000, 200000], n ~ U{{32..256}}, d = 4n, zeta = 8, "
                        "FP32 A (column scales, cond log-uniform in [1e2, 1e8]), b = A x + 1e-8 noise; "
                        "errors relative to the FP64 batched form at tol 1e-12",
            "a_bytes": tot_bytes, "refine": rmix, "fp64_reference": rref, "fp64_batched": fp64_runs,
            "fp64_sequential_same_accuracy": seq,
            "speedup_vs_fp64_batched_same_accuracy": match["ms"] / rmix["ms"],
            "speedup_vs_fp64_sequential_same_accuracy": seq["ms"] / rmix["ms"]}


def served_run(sap, torch, reqs, probs, bs_req, mode, tol, maxiter, tag):
    """Submit the stream at its arrival times through sap_submit on a fresh
    context; latency = submit to finished (the library's own clock)."""
    import numpy as np
    ctx = sap.Context(0)
    A0, _ = probs[reqs[0]["pool"]]
    t = sap.sap_submit(A0, bs_req[0], reqs[0]["d"], 8, 1, tol=tol, maxiter=maxiter, mode=mode, max_refine=12,
                       ctx=ctx)
    sap.sap_poll(t, wait=True, ctx=ctx)  # warm-up request (not counted)
    tickets = []
    t_start = time.perf_counter()
    for k, r in enumerate(reqs):
        delay = t_start + r["t"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        A, _ = probs[r["pool"]]
        tickets.append(sap.sap_submit(A, bs_req[k], r["d"], 8, 101 + k, tol=tol, maxiter=maxiter, mode=mode,
                                      max_refine=12, ctx=ctx))
    lat, xs, ok = [], [], 0
    for t in tickets:
        st, info, x = sap.sap_poll(t, wait=True, ctx=ctx)
        lat.append(info["t_total_ms"])
        xs.append(x)
        ok += st == sap.SAP_OK
    t_end = time.perf_counter()
    stats = sap.sap_serve_stats(ctx)
    ctx.close()
    lat = np.asarray(lat)
    log(f"bench[served]: {tag}: {len(reqs)} requests in {t_end - t_start:.2f} s")
    return xs, {"tol": tol, "ok": int(ok), "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()),
                "solves_per_s": len(reqs) / (t_end - t_start), "wall_s": t_end - t_start, "serve_stats": stats}


def form_served(args, sap, torch, inputs):
    """Served form: a Poisson request stream over a device-resident pool of
    problems (each request one pool matrix with its own right-hand side),
    submitted at the arrival times.  The refinement form (FP32 A) and the FP64
    form (FP64 copies of the pool, FP64 arithmetic, served the same way at
    the tolerance that matches the refinement form's accuracy on a sample)
    serve the same stream; accuracy is measured on a sample of requests
    against single FP64 solves at tol 1e-12."""
    import numpy as np
    reqs = inputs.served_stream(rate=args.serve_rate, duration=args.serve_duration)
    pool_shapes = inputs.served_stream(rate=1.0, duration=float(args.serve_pool) * 1.5,
                                       seed=inputs.config_seed(4) + 1)[:args.serve_pool]
    log(f"bench[served]: {len(reqs)} requests over a pool of {len(pool_shapes)} problems")
    probs = []
    for k, r in enumerate(pool_shapes):
        A, _, _ = inputs.make_problem_torch(r["m"], r["n"], kind="colscale", cond=1e6, noise=1e-8,
                                            seed=inputs.config_seed(4) + 13 * k, device="cuda", dtype=torch.float32)
        probs.append((A, r["n"]))
    probs64 = [(A.to(torch.float64), n) for A, n in probs]
    rng = np.random.default_rng(inputs.config_seed(4) + 2)
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.config_seed(4) + 3)
    bs_req = []
    for r in reqs:  # b = A x_true + 1e-8 noise, one x_true per request
        r["pool"] = int(rng.integers(len(probs)))
        A64, n = probs64[r["pool"]]
        r["d"] = 4 * n
        xt = torch.randn(n, generator=g, device="cuda", dtype=torch.float64)
        bb = A64 @ xt
        bb += 1e-8 * (bb.norm() / np.sqrt(A64.shape[0])) * torch.randn(A64.shape[0], generator=g, device="cuda",
                                                                        dtype=torch.float64)
        bs_req.append(bb)
    torch.cuda.synchronize()
    # accuracy sample: single FP64 solves at tol 1e-12 of the first requests
    ns = min(48, len(reqs))
    xref = []
    for k in range(ns):
        r = reqs[k]
        xref.append(sap.sap_solve(probs64[r["pool"]][0], bs_req[k], r["d"], 8, 101 + k, tol=1e-12,
                                  maxiter=300).x.clone())
    # the FP64 tolerance matching the refinement form on the sample (batched solves of the sample)
    sA = [probs[reqs[k]["pool"]][0] for k in range(ns)]
    sA64 = [probs64[reqs[k]["pool"]][0] for k in range(ns)]
    sds = [reqs[k]["d"] for k in range(ns)]
    sseeds = [101 + k for k in range(ns)]
    xs_r, _, _ = sap.sap_solve_batch(sA, bs_req[:ns], sds, 8, sseeds, tol=TARGET_REL_ERR, maxiter=1000,
                                     mode=sap.SAP_MODE_MIXED_FP32_REFINE, max_refine=12)
    err_r = max(rel(a, b) for a, b in zip(xs_r, xref))
    tol64 = FP64_MATCH_TOLS[-1]
    for t in FP64_MATCH_TOLS:
        xs_t, _, _ = sap.sap_solve_batch(sA64, bs_req[:ns], sds, 8, sseeds, tol=t, maxiter=300)
        if max(rel(a, b) for a, b in zip(xs_t, xref)) <= max(TARGET_REL_ERR, err_r):
            tol64 = t
            break
    torch.cuda.synchronize()
    log(f"bench[served]: FP64 tolerance matching the refinement form's accuracy: {tol64:g}")
    xm, rm = served_run(sap, torch, reqs, probs, bs_req, sap.SAP_MODE_MIXED_FP32_REFINE, TARGET_REL_ERR, 1000,
                        "refine")
    rm.update(_batch_errs(xm[:ns], xref))
    x64, r64 = served_run(sap, torch, reqs, probs64, bs_req, sap.SAP_MODE_FP64, tol64, 300, "fp64")
    r64.update(_batch_errs(x64[:ns], xref))
    del probs64, probs, bs_req
    torch.cuda.empty_cache()
    return {"workload": f"{len(reqs)} requests, Poisson {args.serve_rate:g} req/s for {args.serve_duration:g} s, "
                        f"each one of a pool of {len(pool_shapes)} problems with its own b: m ~ lognormal(median "
                        "1e5, sigma 1) clamped to [8n, 2^21], n in {64,128,256,512}, d = 4n, zeta = 8, FP32 A "
                        f"(column scales, cond 1e6); accuracy on the first {ns} requests against FP64 solves at "
                        "tol 1e-12",
            "requests": len(reqs), "refine": rm, "fp64": r64,
            "p99_speedup": r64["p99_ms"] / rm["p99_ms"], "p50_speedup": r64["p50_ms"] / rm["p50_ms"]}


def adaptive_d(sap, torch, A, b, x, m, n, d, zeta, seed, tol, maxiter, pass_ms, qr_ms, fixed_ms, fixed_iters):
    """The same problem at other embedding dimensions (Sec. 4.3): a sweep of
    d = k n, eq. (4.2)'s d (paper form, and with this run's measured cost
    ratio), and the machine-aware pick of sap_choose_d (its one-time
    calibration timed separately).  The headline value stays the fixed d."""
    def solve_ms(dd, reps=3):
        sap.sap_solve(A, b, dd, zeta, seed, tol=tol, maxiter=maxiter, x=x)  # warm-up
        torch.cuda.synchronize()
        times, infos = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = sap.sap_solve(A, b, dd, zeta, seed, tol=tol, maxiter=maxiter, x=x)
            torch.cuda.synchronize()
            times.append((time.perf_counter() - t0) * 1e3)
            infos.append(r.info)
        k = sorted(range(len(times)), key=times.__getitem__)[len(times) // 2]
        return times[k], infos[k]

    ratio = (pass_ms / (m * n)) / (qr_ms / (d * n * n))
    d_ratio = sap.sap_embedding_dim(m, n, tol, ratio)
    d_paper = sap.sap_embedding_dim(m, n, tol)
    t0 = time.perf_counter()
    d_pick = sap.sap_choose_d(A, b, zeta, tol)
    torch.cuda.synchronize()
    calib_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    sap.sap_choose_d(A, b, zeta, tol)
    cached_ms = (time.perf_counter() - t0) * 1e3
    log(f"bench: sap_choose_d picks d = {d_pick} ({calib_ms:.0f} ms calibration, {cached_ms:.2f} ms cached); "
        f"eq. (4.2) paper form {d_paper}, measured ratio {ratio:.3f} -> {d_ratio}")
    sweep = []
    for dk in sorted({min(f * n, m, 16384) for f in (2, 3, 4, 6, 8, 12)} | {d_pick}):
        ms, i = solve_ms(dk, reps=1 if dk != d_pick else 3)
        sweep.append({"d": dk, "iters": i["iters"], "iters_estimate": sap.sap_iteration_estimate(n, dk, tol),
                      "solve_ms": ms, "apply_ms": i["t_apply_ms"], "qr_ms": i["t_qr_ms"],
                      "iterate_ms": i["t_iterate_ms"]})
        log(f"bench: d = {dk}: {ms:.1f} ms, {i['iters']} iterations")
    best = min(sweep, key=lambda r: r["solve_ms"])
    pick = next(r for r in sweep if r["d"] == d_pick)
    ms_paper, i_paper = solve_ms(min(d_paper, 16384))
    return {"sweep": sweep, "chosen": {"rule": "sap_choose_d (every phase timed on this GPU)", "d": d_pick,
                                       "solve_ms": pick["solve_ms"], "iters": pick["iters"],
                                       "calibration_ms": calib_ms, "cached_call_ms": cached_ms,
                                       "vs_sweep_best": pick["solve_ms"] / best["solve_ms"],
                                       "sweep_best_d": best["d"]},
            "eq42_paper_form": {"d": d_paper, "solve_ms": ms_paper, "iters": i_paper["iters"]},
            "eq42_measured_ratio": {"cost_ratio": ratio, "d": d_ratio},
            "fixed_d": d, "fixed_iters": fixed_iters, "fixed_iters_estimate": sap.sap_iteration_estimate(n, d, tol),
            "fixed_solve_ms": fixed_ms, "chosen_speedup_vs_fixed": fixed_ms / pick["solve_ms"]}


def form_fig5(args, sap, torch, inputs):
    """Sec. 4.3's experiment (Fig. 5): m = 6e5, several n, tol 1e-5, ||b|| = 1
    and ||b - A x*|| = 1/2, the fixed d = 12 n against eq. (4.2)'s d and the
    machine-aware pick.  A = U diag(sigma) V^T (sigma log-spaced 1..1e-6) with
    U, V orthonormal factors of seeded Gaussians; b = (sqrt(3)/2) A y / ||A y||
    + (1/2) r / ||r||, r the part of a Gaussian orthogonal to range(U).  The
    solver's d <= 16384 keeps 12 n <= 16384 (n <= 1365)."""
    import numpy as np
    m, tol, zeta = args.fig5_m, 1e-5, 8
    rows = []
    g = torch.Generator(device="cuda")
    for n in [int(v) for v in args.fig5_n.split(",") if v]:
        g.manual_seed(inputs.config_seed(5) + n)
        U, _ = torch.linalg.qr(torch.randn(m, n, generator=g, device="cuda", dtype=torch.float64))
        V, _ = torch.linalg.qr(torch.randn(n, n, generator=g, device="cuda", dtype=torch.float64))
        sig = torch.logspace(0.0, -6.0, n, device="cuda", dtype=torch.float64)
        A = (U * sig[None, :]) @ V.T
        Ay = U @ (sig * (V.T @ torch.randn(n, generator=g, device="cuda", dtype=torch.float64)))
        r = torch.randn(m, generator=g, device="cuda", dtype=torch.float64)
        r -= U @ (U.T @ r)
        b = (np.sqrt(3.0) / 2.0) * Ay / Ay.norm() + 0.5 * r / r.norm()
        del U, V, r, Ay
        x = torch.empty(n, dtype=torch.float64, device="cuda")

        def run(dd):
            sap.sap_solve(A, b, dd, zeta, 11, tol=tol, maxiter=500, x=x)
            torch.cuda.synchronize()
            ts = []
            for _ in range(3):
                t0 = time.perf_counter()
                res = sap.sap_solve(A, b, dd, zeta, 11, tol=tol, maxiter=500, x=x)
                torch.cuda.synchronize()
                ts.append((time.perf_counter() - t0) * 1e3)
            return float(np.median(ts)), res.info

        row = {"n": n}
        for tag, dd in (("fixed_12n", min(12 * n, 16384)), ("eq42", min(sap.sap_embedding_dim(m, n, tol), 16384))):
            ms, info = run(dd)
            row[tag] = {"d": dd, "solve_ms": ms, "iters": info["iters"], "status": info["status_name"]}
        t0 = time.perf_counter()
        dp = sap.sap_choose_d(A, b, zeta, tol)
        torch.cuda.synchronize()
        calib = (time.perf_counter() - t0) * 1e3
        ms, info = run(dp)
        row["chosen"] = {"d": dp, "solve_ms": ms, "iters": info["iters"], "status": info["status_name"],
                         "calibration_ms": calib}
        row["residual_norm"] = float((b - A @ x).norm())
        log(f"bench[fig5]: {row}")
        rows.append(row)
        del A, b, x
        torch.cuda.empty_cache()
    return {"workload": f"Sec. 4.3 / Fig. 5: m = {m}, tol {tol:g}, ||b|| = 1, ||b - A x*|| = 1/2, zeta = {zeta}, "
                        "A = U diag(sigma) V^T with sigma log-spaced 1..1e-6; median of 3 solves",
            "rows": rows}


def _event_ms(torch, fn, reps):
    """Median of reps event-timed calls of fn on the current stream."""
    import numpy as np
    fn()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def form_sparse(args, sap, torch, inputs):
    """Sec. 4.1's sparse recipe at Table 1's size (m = 5e5, n = 500, +-1
    entries at density 0.01): the sketch apply on the stored entries against
    the dense apply of the same matrix held densely (Fig. 2's comparison,
    over d and zeta), and Alg. 1 with the sparse LSQR pass against the dense
    solve of the same matrix.  Rates on the stored-entry bytes: indptr
    (8 (m + 1)), column indices (4 nnz) and values (8 nnz)."""
    import numpy as np
    m, n, dens = args.sparse_m, args.sparse_n, 0.01
    A, b_np, _ = inputs.make_sparse_problem(m, n, dens, values="sign", noise=1e-6, seed=inputs.config_seed(6))
    ip = torch.from_numpy(A.indptr.astype(np.int64)).cuda()
    ix = torch.from_numpy(A.indices.astype(np.int32)).cuda()
    v = torch.from_numpy(A.data.astype(np.float64)).cuda()
    b = torch.from_numpy(b_np).cuda()
    rows = torch.repeat_interleave(torch.arange(m, device="cuda"), ip[1:] - ip[:-1])
    Ad = torch.zeros(m, n, dtype=torch.float64, device="cuda")
    Ad[rows, ix.long()] = v
    del rows
    nnz = int(A.nnz)
    nnz_bytes = 8 * (m + 1) + 12 * nnz
    seed = inputs.config_seed(6) + 1
    ctx = sap.default_context(0)
    apply_rows = []
    for zeta in (8, 12, 24):
        for d in (2 * n, 4 * n, 8 * n):
            idx, sign = sap.sps_generate(m, d, zeta, seed)
            Ys = torch.empty(n + 1, d, dtype=torch.float64, device="cuda")
            Yd = torch.empty(n + 1, d, dtype=torch.float64, device="cuda")
            ms_s = _event_ms(torch, lambda: sap.sps_apply_csr(idx, sign, d, zeta, ip, ix, v, (m, n), b, Y=Ys), 5)
            ms_d = _event_ms(torch, lambda: sap.sps_apply(idx, sign, d, zeta, Ad, b, Y=Yd), 5)
            err = float((Ys - Yd).norm() / Yd.norm())
            apply_rows.append({"zeta": zeta, "d": d, "sparse_ms": ms_s, "dense_ms": ms_d,
                               "dense_over_sparse": ms_d / ms_s, "sparse_nnz_gbs": nnz_bytes / (ms_s * 1e-3) / 1e9,
                               "rel_diff": err})
            log(f"bench[sparse]: apply zeta={zeta} d={d}: sparse {ms_s:.3f} ms, dense {ms_d:.3f} ms, diff {err:.1e}")
            del idx, sign, Ys, Yd
    d, zeta, tol = 4 * n, 8, 1e-12
    xs = torch.empty(n, dtype=torch.float64, device="cuda")
    xd = torch.empty(n, dtype=torch.float64, device="cuda")
    sap.sap_solve_csr(ip, ix, v, (m, n), b, d, zeta, seed, tol=tol, maxiter=300, x=xs)
    ctx.profile(True)
    ctx.profile_read(sap.PROF_PASS, reset=True)
    ts, infos = [], []
    for _ in range(args.sparse_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = sap.sap_solve_csr(ip, ix, v, (m, n), b, d, zeta, seed, tol=tol, maxiter=300, x=xs)
        ts.append((time.perf_counter() - t0) * 1e3)
        infos.append(r.info)
    ctx.profile(False)
    n_pass, ms_pass = ctx.profile_read(sap.PROF_PASS)
    n_full = sum(i["iters"] + 1 for i in infos)
    pass_ms = ms_pass / max(1, min(n_pass, n_full))
    pass_bytes_s = nnz_bytes + 16 * m  # + u read and written
    sap.sap_solve(Ad, b, d, zeta, seed, tol=tol, maxiter=300, x=xd)
    td = []
    for _ in range(args.sparse_reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rd = sap.sap_solve(Ad, b, d, zeta, seed, tol=tol, maxiter=300, x=xd)
        td.append((time.perf_counter() - t0) * 1e3)
    res_s = float((b - Ad @ xs).norm())
    res_d = float((b - Ad @ xd).norm())
    i0 = infos[-1]
    out = {"workload": f"Sec. 4.1 sparse recipe: m = {m}, n = {n}, +-1 at density {dens} (nnz {nnz}), "
                       f"b = A x + 1e-6 noise; solve d = {d}, zeta = {zeta}, tol {tol:g}",
           "apply": apply_rows,
           "solve": {"sparse_ms": float(np.median(ts)), "dense_ms": float(np.median(td)),
                     "dense_over_sparse": float(np.median(td) / np.median(ts)),
                     "iters": i0["iters"], "dense_iters": rd.info["iters"],
                     "phases_ms": {k: i0[k] for k in ("t_generate_ms", "t_apply_ms", "t_qr_ms", "t_iterate_ms")},
                     "pass_avg_ms": pass_ms, "pass_bytes": pass_bytes_s,
                     "pass_gbs": pass_bytes_s / (pass_ms * 1e-3) / 1e9,
                     "residual_sparse": res_s, "residual_dense": res_d,
                     "x_rel_diff": float((xs - xd).norm() / xd.norm())}}
    log(f"bench[sparse]: solve {out['solve']}")
    del Ad
    torch.cuda.empty_cache()
    return out


def form_hbm(args, sap, torch, inputs):
    """App. D.3's comparison (Fig. 6): LSQR, heavy-ball momentum with
    eta = sqrt(n/d) and with the safer sqrt(1.1) sqrt(n/d), and gradient
    descent, on a leverage-skewed dense problem and on the hard case of
    Sec. 4.1 (the first n columns of the identity, where sqrt(n/d)
    underestimates the distortion), to tol 1e-10 (maxiter 400); beside them
    the s-step form of App. D.4.2 with blocks of 4 and 8 steps (s + 1 passes
    over A per block).  Reports time, steps, passes over A and
    ||A(x - x_ref)|| / ||b|| with x_ref LSQR's solution."""
    m, n, d, zeta, tol = args.hbm_m, args.hbm_n, 4 * args.hbm_n, 8, 1e-10
    rows = []
    for kind in ("svd", "identity"):
        if kind == "svd":
            A, b, _ = inputs.make_problem_torch(m, n, kind="svd", cond=1e8, noise=1e-6, seed=inputs.config_seed(7),
                                                row_scale=True, device="cuda")
        else:
            A = torch.zeros(m, n, dtype=torch.float64, device="cuda")
            A[torch.arange(n, device="cuda"), torch.arange(n, device="cuda")] = 1.0
            g = torch.Generator(device="cuda")
            g.manual_seed(inputs.config_seed(7) + 1)
            b = torch.randn(m, generator=g, device="cuda", dtype=torch.float64)
        x = torch.empty(n, dtype=torch.float64, device="cuda")
        nb = float(b.norm())

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            return (time.perf_counter() - t0) * 1e3, r

        ms, r = timed(lambda: sap.sap_solve(A, b, d, zeta, 13, tol=tol, maxiter=400, x=x))
        xref = x.clone()
        row = {"problem": kind, "lsqr": {"ms": ms, "iters": r.info["iters"], "status": r.info["status_name"]}}
        for tag, kw in (("hbm", {}), ("hbm_safe", {"eta_scale": 1.1 ** 0.5}), ("gd", {"gradient_descent": True})):
            ms, r = timed(lambda: sap.sap_solve_hbm(A, b, d, zeta, 13, tol=tol, maxiter=400, x=x, **kw))
            err = float((A @ (x - xref)).norm()) / nb
            row[tag] = {"ms": ms, "iters": r.info["iters"], "status": r.info["status_name"], "err_vs_lsqr": err}
        for s in (4, 8):
            ms, r = timed(lambda: sap.sap_solve_sstep(A, b, d, zeta, 13, tol=tol, maxiter=400, x=x, s=s))
            err = float((A @ (x - xref)).norm()) / nb
            steps = r.info["iters"]
            row[f"sstep{s}"] = {"ms": ms, "iters": steps, "passes": steps + steps // s + 1,
                                "status": r.info["status_name"], "err_vs_lsqr": err}
        log(f"bench[hbm]: {row}")
        rows.append(row)
        del A, b, x, xref
        torch.cuda.empty_cache()
    return {"workload": f"App. D.3 / Fig. 6: m = {m}, n = {n}, d = 4n, zeta = {zeta}, tol {tol:g}; "
                        "leverage-skewed U diag(sigma) V^T (sigma 1..1e-8) and the first n columns of the identity",
            "rows": rows}


def kernel_apply(args, sap, torch, inputs):
    """sps_apply alone: warm-up, then --steps applies timed with events on
    the current stream (the stream the library launches on).  One JSON line."""
    m, n, d, zeta = args.m, args.n, args.d, args.zeta
    ta = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[args.a_dtype]
    ty = {"f64": torch.float64, "f32": torch.float32}[args.y_dtype]
    log(f"bench[apply]: m={m} n={n} d={d} zeta={zeta} A {args.a_dtype} Y {args.y_dtype}")
    # a copy of known size in the same process calibrates the HBM byte counters
    copy_ref = copy_reference(torch, args.copy_ref_mib) if args.copy_ref_mib > 0 else None
    A, b, _ = inputs.make_problem_torch(m, n, kind="colscale", cond=1e6, noise=1e-6, seed=inputs.config_seed(1),
                                        device="cuda", dtype=ta)
    idx, sign = sap.sps_generate(m, d, zeta, inputs.config_seed(1) + 1)
    Y = sap.sps_apply(idx, sign, d, zeta, A, b, y_dtype=ty)
    for _ in range(args.warmup):
        sap.sps_apply(idx, sign, d, zeta, A, b, y_dtype=ty, Y=Y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        sap.sps_apply(idx, sign, d, zeta, A, b, y_dtype=ty, Y=Y)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    ab = apply_bytes(m, n, d, zeta, A.element_size(), Y.element_size())
    print(json.dumps({"kernel": "apply", "m": m, "n": n, "d": d, "zeta": zeta, "a_dtype": args.a_dtype,
                      "y_dtype": args.y_dtype, "steps": args.steps, "avg_ms": ms, "bytes": ab,
                      "gbs": ab / (ms * 1e-3) / 1e9, "frac": ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "a_only_gbs": m * n * A.element_size() / (ms * 1e-3) / 1e9, "copy_reference": copy_ref}),
          flush=True)


def kernel_qr(args, sap, torch, inputs):
    """sap_qr alone on a seeded Gaussian d x (n+1) FP64 matrix (the shape of
    the sketch [SA Sb]): warm-up, then --steps factorisations of a fresh copy
    timed with events.  One JSON line with the rate against the FP64 peak."""
    d, nc = args.d, args.n + 1
    g = torch.Generator(device="cuda")
    g.manual_seed(inputs.config_seed(8))
    Y0 = torch.randn(nc, d, generator=g, dtype=torch.float64, device="cuda")
    Y = Y0.clone()
    for _ in range(max(1, args.warmup)):
        Y.copy_(Y0)
        sap.sap_qr(Y)
    torch.cuda.synchronize()
    ts = []
    for _ in range(args.steps):
        Y.copy_(Y0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        sap.sap_qr(Y)
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    import numpy as np
    ms = float(np.median(ts))
    fl = qr_flops(d, nc)
    print(json.dumps({"kernel": "qr", "d": d, "ncols": nc, "steps": args.steps, "median_ms": ms, "flops": fl,
                      "tflops": fl / (ms * 1e-3) / 1e12, "frac_fp64": fl / (ms * 1e-3) / 1e9 / FP64_PEAK_GFLOPS}),
          flush=True)


def kernel_batch(args, sap, torch, inputs):
    """The batched form's refinement-form solve alone (the problems of
    form_batched, FP32 A, target 1e-8): a warm-up, then --steps timed
    batches.  One JSON line."""
    shapes = inputs.batch_shapes(count=args.batch_count)
    As, bs = [], []
    for s in shapes:
        A, b, _ = inputs.make_problem_torch(s["m"], s["n"], kind="colscale", cond=s["cond"], noise=1e-8,
                                            seed=s["seed"], device="cuda", dtype=torch.float32)
        As.append(A)
        bs.append(b)
    ds = [s["d"] for s in shapes]
    seeds = [s["seed"] + 1 for s in shapes]
    mode = sap.SAP_MODE_MIXED_FP32_REFINE

    def run():
        return sap.sap_solve_batch(As, bs, ds, 8, seeds, tol=1e-8, maxiter=1000, mode=mode, max_refine=12)
    for _ in range(max(1, args.warmup)):
        run()
    torch.cuda.synchronize()
    ts = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        _, _, infos = run()
        torch.cuda.synchronize()
        ts.append((time.perf_counter() - t0) * 1e3)
    import numpy as np
    print(json.dumps({"kernel": "batch", "problems": len(As), "a_bytes": sum(A.numel() * 4 for A in As),
                      "steps": args.steps, "median_ms": float(np.median(ts)),
                      "converged": sum(1 for i in infos if i["status"] == sap.SAP_OK)}), flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}); "
              "the library runs on one GPU and has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    import paper_2506_03070_amd as sap

    torch.cuda.set_device(0)
    if args.kernel == "apply":
        kernel_apply(args, sap, torch, inputs)
        return
    if args.kernel == "qr":
        kernel_qr(args, sap, torch, inputs)
        return
    if args.kernel == "batch":
        kernel_batch(args, sap, torch, inputs)
        return
    copy_ref = copy_reference(torch, args.copy_ref_mib) if args.copy_ref_mib > 0 else None
    if copy_ref:
        log(f"bench: copy reference {copy_ref['gbs']:.0f} GB/s")
    m, n, d, zeta = args.m, args.n, args.d, args.zeta
    log(f"bench: generating workload m={m} n={n} d={d} zeta={zeta} (FP64) on the GPU")
    t0 = time.perf_counter()
    if args.gaussian_input:
        A, b, x_true = inputs.make_problem_torch(m, n, kind="colscale", cond=1e4, noise=1e-6,
                                                 seed=inputs.config_seed(1), device="cuda")
        meta = dict(sketch_seed=inputs.config_seed(1) + 1, tol=1e-12, maxiter=200)
    elif (m, n) == (1 << 20, 1000):
        A, b, x_true, meta = inputs.config1_torch("cuda")
    else:
        A, b, x_true = inputs.make_problem_torch(m, n, kind="svd", cond=1e8, noise=1e-6,
                                                 seed=inputs.config_seed(1), row_scale=True, device="cuda")
        meta = dict(sketch_seed=inputs.config_seed(1) + 1, tol=1e-12, maxiter=200)
    torch.cuda.synchronize()
    log(f"bench: workload ready in {time.perf_counter() - t0:.1f} s")
    seed, tol, maxiter = meta["sketch_seed"], meta["tol"], meta["maxiter"]

    ctx = sap.default_context(0)
    x = torch.empty(n, dtype=torch.float64, device="cuda")
    for w in range(args.warmup):
        r = sap.sap_solve(A, b, d, zeta, seed, tol=tol, maxiter=maxiter, x=x)
        log(f"bench: warmup {w}: {r.info['status_name']} iters={r.info['iters']} "
            f"phases(ms) gen={r.info['t_generate_ms']:.2f} apply={r.info['t_apply_ms']:.2f} "
            f"qr={r.info['t_qr_ms']:.2f} iter={r.info['t_iterate_ms']:.2f}")
    torch.cuda.synchronize()

    ctx.profile(True)
    ctx.profile_read(sap.PROF_PASS, reset=True)
    ctx.profile_read(sap.PROF_APPLY, reset=True)
    infos = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    step_ms = []
    for k in range(args.steps):
        t_k = time.perf_counter()
        r = sap.sap_solve(A, b, d, zeta, seed, tol=tol, maxiter=maxiter, x=x)  # returns when x is final
        step_ms.append((time.perf_counter() - t_k) * 1e3)
        infos.append(r.info)
        log(f"bench: step {k}: {r.info['status_name']} iters={r.info['iters']}")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ctx.profile(False)
    n_pass, ms_pass = ctx.profile_read(sap.PROF_PASS)
    n_apply, ms_apply = ctx.profile_read(sap.PROF_APPLY)

    ms_per_step = 1e3 * elapsed / args.steps
    iters = int(np.median([i["iters"] for i in infos]))
    pb = pass_bytes(m, n, 8)
    ab = apply_bytes(m, n, d, zeta, 8, 8)
    # launches that did a full pass: the initialisation pass plus one per
    # iteration; the few launches after convergence return at once (they
    # come from launching iterations in batches of eight) and are excluded
    # from the average (their few microseconds stay in the total)
    n_full = sum(i["iters"] + 1 for i in infos)
    pass_avg_ms = ms_pass / max(1, min(n_pass, n_full))
    apply_avg_ms = ms_apply / max(1, n_apply)
    pass_gbs = pb / (pass_avg_ms * 1e-3) / 1e9
    apply_gbs = ab / (apply_avg_ms * 1e-3) / 1e9

    # Accuracy of the last solve in the paper's metric, via the normal equations
    # residual computed with plain torch (checker only)
    r_vec = b - A @ x
    ne = torch.linalg.vector_norm(A.T @ r_vec).item()
    rel_ne = ne / (torch.linalg.matrix_norm(A, ord="fro").item() * torch.linalg.vector_norm(r_vec).item())

    def med(key):
        return float(np.median([i[key] for i in infos]))

    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "plain FP64 sketch-and-precondition solve, m=2^20 n=1000 d=4000 zeta=8, "
                               "A = U diag(sigma) V^T (sigma 1..1e-8, leverage-skewed U), b = A x + 1e-6 noise, "
                               "LSQR tol 1e-12",
                   "m": m, "n": n, "d": d, "zeta": zeta, "tol": tol, "precision": "fp64"},
        "roofline": {"bound": "hbm", "kernel": "lsqr_pass_kernel (fused A p / A^T u pass)",
                     "achieved": pass_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": pass_gbs / HBM_PEAK_GBS,
                     "traffic": measured_traffic(m, n), "bytes_per_launch": pb, "avg_launch_ms": pass_avg_ms,
                     "launches": n_pass, "full_launches": n_full},
        "sa": {"kernel": "apply_strip_kernel", "achieved_gbs": apply_gbs, "frac": apply_gbs / HBM_PEAK_GBS,
               "bytes_per_launch": ab, "avg_launch_ms": apply_avg_ms, "launches": n_apply,
               "a_only_gbs": m * n * 8 / (apply_avg_ms * 1e-3) / 1e9},
        "qr": {"flops": qr_flops(d, n + 1), "ms": med("t_qr_ms"),
               "gflops": qr_flops(d, n + 1) / (med("t_qr_ms") * 1e-3) / 1e9,
               "frac_fp64": qr_flops(d, n + 1) / (med("t_qr_ms") * 1e-3) / 1e9 / FP64_PEAK_GFLOPS},
        "phases_ms": {"generate": med("t_generate_ms"), "apply": med("t_apply_ms"), "qr": med("t_qr_ms"),
                      "iterate": med("t_iterate_ms")},
        "iters": iters,
        # per-solve statistics in the paper's form (median, 5-95% range), over the timed steps
        "solve_ms": {"runs": len(step_ms), "median": float(np.median(step_ms)),
                     "p5": float(np.percentile(step_ms, 5)), "p95": float(np.percentile(step_ms, 95))},
        "normal_eq_residual_rel": rel_ne,
        "copy_reference": copy_ref,
        "cpu_baseline": None,
        "forms": {},
    }
    if not args.no_adaptive_d:
        out["embedding_dim"] = adaptive_d(sap, torch, A, b, x, m, n, d, zeta, seed, tol, maxiter,
                                          pass_avg_ms, med("t_qr_ms"), ms_per_step, iters)
    rows = min(args.cpu_sample_rows, m)
    A_sample, b_sample = A[:rows].cpu().numpy(), b[:rows].cpu().numpy()
    del A, r_vec
    torch.cuda.empty_cache()
    for f in [f for f in args.forms.split(",") if f]:
        fn = {"mixed": form_mixed, "batched": form_batched, "served": form_served, "fig5": form_fig5,
              "sparse": form_sparse, "hbm": form_hbm}.get(f)
        if fn is None:
            log(f"bench: unknown form {f}")
            continue
        t0 = time.perf_counter()
        out["forms"][f] = fn(args, sap, torch, inputs)
        log(f"bench: form {f} done in {time.perf_counter() - t0:.1f} s")
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a row sample")
        out["cpu_baseline"] = cpu_baseline(A_sample, b_sample, m, d, zeta, seed, tol, iters)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
