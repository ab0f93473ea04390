"""Benchmark: penalty-gradient evaluations per second of the batched solve.

Workload: one UBQP instance, n = 2500, symmetric integer Q at 10% density with
nonzeros uniform over +-{1..100}, b = 0, and 256 random starts uniform in
[0,1)^n, all solved together (Algorithm 3 with projected alternating BB
subproblems). One step = one whole batched solve: Q preparation, every sweep
of Q.X products (subproblem and lambda_min / CG products), the per-column
state machine, and the exact int64 objectives. Inputs are resident in device
memory before the timed region starts.

The default operand type is I8: exact integer products on int8 MFMA (an
iterate rounded to the grid 2^-27, eigen/CG vectors to 55 bits of their
scale; see include/psdp.h). Its only error is that rounding of x, below the
rounding error of an FP32 GEMM. The same line also reports the FP32-GEMM solve
of the same workload (`fp32_gemm`).

value = penalty-gradient evaluations (one column of Q.X plus its gradient
epilogue) per second over the timed steps. The JSON line also reports the
roofline of the dominant kernel (the per-column step kernel, HBM-bound, timed
with HIP events on the library's solve stream around every launch of one
more solve of the same workload), the roofline of the Q.X product kernels, a
plain single-instance comparison at equal objective on a subset of starts,
and the FP64 oracle's rate on a bounded sample of the same workload on the
host cores.

With I8 operands the line also carries `sparse`: a sparse Max-Cut workload
(n = 8000, G(n, 0.005) with +-1 weights, b = -We, 16 starts, diagonal
perturbation) solved with the sparse-row products (the automatic choice at
that size and density) and with the dense digit products, at equal
objectives, with the sparse product kernel's average launch time and rate.

`python bench.py --calibrate-copy` only copies 1 GiB between two device
buffers (the reference kernel for the HBM byte counters).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0       # MI355X HBM3E, GB/s
PEAK_INT8_TOPS = 5000.0     # MI355X dense int8 MFMA, TOPS
PEAK_FP32_TFLOPS = 157.3    # MI355X dense FP32 MFMA
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 MFMA
STEP_BYTES_PER_COLUMN = 80  # about 10 FP64 vectors of n per column update
START_SEED = 3              # start set of the first timed step (the workload generator's default)
STEP_SOURCES = ("paper_2408_04875_amd/csrc/solver.hip", "paper_2408_04875_amd/csrc/common.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_n2500_b256_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=2500)
    ap.add_argument("--starts", type=int, default=256)
    ap.add_argument("--plain-starts", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-gemv", action="store_true")
    ap.add_argument("--no-group", action="store_true")
    ap.add_argument("--group-only", action="store_true", help="only the uneven-batch group leg")
    ap.add_argument("--gemv-only", action="store_true", help="only the large single-instance GEMV leg")
    ap.add_argument("--qx", default="i8", choices=["i8", "f32", "f64"])
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--gemm-yardstick", action="store_true",
                    help="time the library's digit product next to hipBLASLt's int8 GEMM of the same shape")
    return ap.parse_args()


def code_only(text: str) -> str:
    """Source text without // comments and blank lines (comments do not change
    the kernel the traffic counters measured)."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            out.append(code)
    return "\n".join(out)


def step_source_hash():
    h = hashlib.sha256()
    for rel in STEP_SOURCES:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    runs, or None when they are missing or the kernel source changed since."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256") != step_source_hash():
        return None
    return t.get("bytes_per_launch")


def calibrate_copy():
    import torch
    nbytes = 1 << 30
    src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}), flush=True)


def gemm_yardstick(n=2500, counts=(16, 64, 256), reps=10):
    """The subproblem product of B columns (4 B digit rows of length ldq
    against the int8 Q) through the library's stand-alone digit product,
    next to hipBLASLt's int8 GEMM (torch._int_mm, int32 result) of the same
    [4 B x ldq] x [ldq x ldq] shape. The stand-alone call also validates its
    inputs on the host, so only a kernel trace (rocprofv3 --kernel-trace
    --stats) compares the two kernels; the HIP events here time the GEMM."""
    import numpy as np
    import torch
    import paper_2408_04875_amd as P
    from workloads import gen

    P.load()
    ld = (n + 63) // 64 * 64
    Q, _, X = gen.sparse_2500_starts(n=n, B=max(counts))
    Qd = torch.from_numpy(Q).cuda()
    del Q
    out = []
    for B in counts:
        Xd = torch.from_numpy(np.ascontiguousarray(X[:B])).cuda()
        for _ in range(reps):
            P.qx_digits(Qd, Xd, digits=4)
        g = torch.Generator(device="cuda").manual_seed(B)
        A8 = torch.randint(-64, 65, (4 * B, ld), dtype=torch.int8, device="cuda", generator=g)
        B8 = torch.randint(-127, 128, (ld, ld), dtype=torch.int8, device="cuda", generator=g)
        torch._int_mm(A8, B8)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            torch._int_mm(A8, B8)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out.append({"columns": B, "digit_rows": 4 * B, "k": ld, "q_rows": ld,
                    "int_mm_us_events": us, "int8_tops": 2.0 * 4 * B * ld * ld / us * 1e-6})
    print(json.dumps({"gemm_yardstick": out, "n": n}), flush=True)


def cpu_baseline(Q, b, X0, budget_s=20.0):
    """FP64 oracle (as it stands) on a bounded sample: one start, until the
    subproblem evaluations of whole penalty updates exceed ~budget_s."""
    from oracle import psdp as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count()
    t0 = time.perf_counter()
    evals = outer = 0
    wall = 1.0
    for mo in (1, 2, 4):
        t = time.perf_counter()
        r = O.solve(Q, b, O.Params(max_outer=mo), x0=X0[0])
        wall = time.perf_counter() - t
        evals, outer = r.inner_iters, r.outer_iters
        if time.perf_counter() - t0 > budget_s:
            break
    return {"value": evals / wall, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"start 0 of the n=2500 workload, {outer} penalty updates, {evals} evaluations "
                      f"(dense eigensolver and BLAS matvecs included), {wall:.1f} s"}


def sparse_leg(P, gen, torch, dev, n=8000, p_edge=0.005, B=16):
    """Sparse-row products against digit products on a sparse Max-Cut graph."""
    import numpy as np
    W = gen.maxcut_graph(n, 9, p_edge)
    bw = (-W.sum(axis=1)).astype(np.int32)
    X0 = gen.random_box_points(n, B, 5)
    nnz = int(np.count_nonzero(W))
    Wd, bd, Xd = (torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (W, bw, X0))
    kw = dict(qx_dtype="i8", perturb="diag", sigma=0.5, seed=3)

    def run(sparse, timing=0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = P.solve(Wd, bd, X0=Xd, sparse=sparse, timing=timing, **kw)
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    run(-1)
    auto, wa = run(-1)
    dense, wd = run(0)
    ev = sum(s["inner_iters"] for s in auto.stats)
    same = int((auto.obj.cpu().numpy() == dense.obj.cpu().numpy()).sum())
    timed_run, _ = run(-1, timing=1)
    s0 = timed_run.stats[0]
    halves = sum(s["inner_iters"] + 2 * s["aux_matvecs"] for s in timed_run.stats)
    # per column half: the gathered operand words (4 B per nonzero), a share
    # of the packed nonzeros (4 B per nonzero per group of 4 halves) and the
    # int64 outputs
    per_half = 4 * nnz + nnz + 8 * n
    qs = s0["qx_seconds"] + s0["aux_seconds"]
    return {"workload": f"maxcut n={n} G(n,{p_edge}) +-1 weights, b=-We, diag perturbation sigma 0.5, "
                        f"{B} random starts, Q.X i8",
            "nnz": nnz, "evals_per_s_sparse": ev / wa, "evals_per_s_dense": ev / wd,
            "speedup_sparse_vs_dense": wd / wa, "equal_objective": same, "starts": B,
            "sparse_sweeps": int(auto.stats[0]["sparse_sweeps"]), "sweeps": int(auto.stats[0]["sweeps"]),
            "sparse_kernel": {"kernel": "sparse_kernel (CSR rows, int64 exact)", "launches": s0["qx_launches"],
                              "avg_launch_us": qs / max(s0["qx_launches"], 1) * 1e6,
                              "bytes_per_column_half": per_half,
                              "achieved": halves * per_half / qs / 1e9 if qs > 0 else 0.0,
                              "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": halves * per_half / qs / 1e9 / PEAK_HBM_GBS if qs > 0 else 0.0}}


def gemv_leg(P, gen, torch, dev, n=16384, outer=3):
    """Single-instance solves (one start) on a Q too large for the caches
    (n = 16384: 1.07 GB in FP32, 0.54 GB in BF16 against 256 MB of Infinity
    Cache), a few penalty updates each: the product is the GEMV kernel
    reading all of Q once per evaluation or lambda_min matvec."""
    import numpy as np
    Q, b = gen.sparse_int(n, 5)
    Qd, bd = torch.from_numpy(Q).to(dev), torch.from_numpy(b).to(dev)
    del Q
    x0 = torch.from_numpy(gen.random_box_points(n, 1, 6)).to(dev)
    ld = (n + 15) // 16 * 16
    out = {"workload": f"one start, n={n}, 10% density ints +-[1,100], b=0, {outer} penalty updates"}
    for qx, eb in (("f32", 4), ("bf16", 2)):
        r = P.solve(Qd, bd, X0=x0, qx_dtype=qx, max_outer=outer, timing=1)
        s0 = r.stats[0]
        products = s0["inner_iters"] + s0["aux_matvecs"]
        secs = s0["qx_seconds"] + s0["aux_seconds"]
        launches = s0["qx_launches"]
        per = n * ld * eb  # Q bytes per product (x, 8n bytes, stays in cache)
        out[qx] = {"kernel": f"gemv_kernel<{'float' if qx == 'f32' else '__hip_bfloat16'}, 4>",
                   "bound": "hbm", "products": int(products), "launches": int(launches),
                   "avg_launch_us": secs / max(launches, 1) * 1e6, "bytes_per_product": per,
                   "achieved": products * per / secs / 1e9 if secs > 0 else 0.0, "peak": PEAK_HBM_GBS,
                   "unit": "GB/s", "frac": products * per / secs / 1e9 / PEAK_HBM_GBS if secs > 0 else 0.0,
                   "note": "bytes of the launches that had a live column over the time of all launches"}
    return out


def group_leg(P, gen, torch, dev, count=512):
    """The uneven batch: 512 instances with n uniform in [100, 3000], half
    Max-Cut graphs (p = 0.05, weights +-1), half dense integer Q of density
    0.1-0.8, BF16 operands, diagonal perturbation sigma = 1e-3 max|Q_ij|,
    one start each, all advanced in one group launch per sweep."""
    import numpy as np
    insts = gen.uneven_group(seed=4, count=count, nmin=100, nmax=3000)
    sigma = max(1e-3 * float(np.abs(d["Q"]).max()) for d in insts)
    Qs = [torch.from_numpy(d["Q"]).to(dev) for d in insts]
    bs = [torch.from_numpy(d["b"]).to(dev) for d in insts]
    ns = [d["n"] for d in insts]
    seeds = [d["seed"] for d in insts]
    kw = dict(qx_dtype="bf16", perturb="diag", sigma=sigma)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xh, obj, st = P.solve_group(Qs, bs, seeds=seeds, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evals = sum(s["inner_iters"] for s in st)
    # the same solve with HIP events around every product launch
    _, obj2, st2 = P.solve_group(Qs, bs, seeds=seeds, timing=1, **kw)
    qs = st2[0]["qx_seconds"]
    ld = [(n + 15) // 16 * 16 for n in ns]
    qbytes = sum((s["inner_iters"] + s["aux_matvecs"]) * n * l * 2 for s, n, l in zip(st2, ns, ld))
    return {"workload": f"{count} instances, n uniform in [100, 3000], half Max-Cut G(n, 0.05) +-1, half dense "
                        f"density 0.1-0.8 ints +-[1,100]; BF16 Q.X, diag perturbation sigma {sigma:g}, one start each",
            "sum_n2": int(sum(n * n for n in ns)), "evals": int(evals),
            "aux_matvecs": int(sum(s["aux_matvecs"] for s in st)), "sweeps": int(st[0]["sweeps"]),
            "wall_s": wall, "evals_per_s": evals / wall,
            "same_objectives_timed_run": bool((obj.cpu() == obj2.cpu()).all()),
            "exit_reasons": {k: int((np.array([s["exit_reason"] for s in st]) == v).sum())
                             for k, v in (("converged", 0), ("outer_cap", 1), ("stall", 2))},
            "gemv_group_kernel": {"launches": int(st2[0]["qx_launches"]), "seconds": qs,
                                  "bytes": int(qbytes), "achieved": qbytes / qs / 1e9 if qs > 0 else 0.0,
                                  "peak": PEAK_HBM_GBS, "unit": "GB/s",
                                  "frac": qbytes / qs / 1e9 / PEAK_HBM_GBS if qs > 0 else 0.0,
                                  "note": "BF16 Q bytes of every product over the product launches' event time"}}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described in the design notes but not part of this build.", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gemm_yardstick:
        gemm_yardstick(n=args.n)
        gemm_yardstick(n=16384, counts=(256,))
        return
    import numpy as np
    import torch
    import paper_2408_04875_amd as P
    from workloads import gen

    dev = torch.device("cuda:0")
    P.load()
    if args.gemv_only:
        print(json.dumps({"gemv": gemv_leg(P, gen, torch, dev)}), flush=True)
        return
    if args.group_only:
        print(json.dumps({"group": group_leg(P, gen, torch, dev)}), flush=True)
        return
    n, B = args.n, args.starts
    # Timed step j solves start set START_SEED + j on the same Q: the length
    # of a solve is set by its slowest start, which moves a lot between start
    # sets (and with any ulp-level change of the arithmetic), so the value
    # averages over several sets instead of riding on one.
    Q, b, X0 = gen.sparse_2500_starts(n=n, B=B, seed_x=START_SEED)
    Qd = torch.from_numpy(Q).to(dev)
    bd = torch.from_numpy(b).to(dev)
    X0d = torch.from_numpy(X0).to(dev)
    X0s = [X0d] + [torch.from_numpy(gen.sparse_2500_starts(n=n, B=B, seed_x=START_SEED + j)[2]).to(dev)
                   for j in range(1, max(args.steps, 1))]
    torch.cuda.synchronize()

    def step(qx, timing=False, X=None):
        return P.solve(Qd, bd, X0=X0d if X is None else X, qx_dtype=qx, timing=1 if timing else 0)

    def timed(qx, steps, warmup):
        for _ in range(warmup):
            step(qx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = [step(qx, X=X0s[j]) for j in range(steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        evals = sum(sum(s["inner_iters"] for s in r.stats) for r in res)
        return res, wall, evals

    results, wall, evals = timed(args.qx, args.steps, args.warmup)
    print(f"bench: {args.qx} {args.steps} timed steps in {wall:.2f} s", file=sys.stderr, flush=True)
    aux = sum(sum(s["aux_matvecs"] for s in r.stats) for r in results)
    # one more solve of the first start set with HIP events around every launch
    # (library solve stream): per-kernel average durations and algorithmic work
    s0 = step(args.qx, timing=True).stats[0]
    step_s, step_l, colsteps = s0["step_seconds"], s0["step_launches"], s0["column_steps"]
    step_bytes = STEP_BYTES_PER_COLUMN * n * colsteps
    qx_s = s0["qx_seconds"] + s0["aux_seconds"]
    qx_f = s0["qx_flops"] + s0["aux_flops"]
    qx_l = s0["qx_launches"]
    step_rl = {"bound": "hbm", "achieved": step_bytes / step_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "frac": step_bytes / step_s / 1e9 / PEAK_HBM_GBS, "traffic": measured_traffic(),
               "kernel": "solver_step_kernel (per-column subproblem / LOBPCG / CG step, one block per column)",
               "launches": step_l, "avg_launch_us": step_s / max(step_l, 1) * 1e6,
               "bytes_per_launch": step_bytes / max(step_l, 1),
               "bytes_per_unit": f"{STEP_BYTES_PER_COLUMN} n per column update", "column_updates": colsteps,
               "share_of_gpu_time": step_s / (step_s + qx_s) if step_s + qx_s > 0 else None}
    if args.qx == "i8":
        qx_peak, qx_unit, qx_name = PEAK_INT8_TOPS, "TOPS", "digit_kernel (int8 MFMA, exact int32/int64)"
    elif args.qx == "f32":
        qx_peak, qx_unit, qx_name = PEAK_FP32_TFLOPS, "TFLOP/s", "stream/gemm kernels (FP32 MFMA; FP64 aux)"
    else:
        qx_peak, qx_unit, qx_name = PEAK_FP64_TFLOPS, "TFLOP/s", "stream/gemm kernels (FP64 MFMA)"
    qx_rl = {"bound": "mfma", "achieved": qx_f / qx_s / 1e12 if qx_s > 0 else 0.0, "peak": qx_peak,
             "unit": qx_unit, "frac": (qx_f / qx_s / 1e12 / qx_peak) if qx_s > 0 else 0.0,
             "kernel": qx_name, "launches": qx_l, "seconds": qx_s,
             "work": "2 n^2 multiply-adds per column product (algorithmic; the int8 path executes 4 or 8 "
                     "digit products per column)"}
    dominant, other = (step_rl, qx_rl) if step_s >= qx_s else (qx_rl, step_rl)
    first = results[0]
    objs = first.obj.cpu().numpy()
    out = {
        "metric": "penalty-grad evals/s & roofline frac, batched vs plain, n=2500 at equal objective",
        "value": evals / wall,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"i8": "i8 digits, exact i32/i64 Q.X; f64 state", "f32": "f32 Q.X; f64 state",
                  "f64": "f64"}[args.qx],
        "data": "synthetic",
        "config": {"workload": f"ubqp n={n} 10% density ints +-[1,100] b=0, {B} random starts in [0,1)^n "
                               f"(one start set per step, seeds {START_SEED}..{START_SEED + args.steps - 1}), "
                               f"batched PABB, Q.X {args.qx}",
                   "n": n, "starts": B, "global_batch": B, "parallelism": "single gpu"},
        "roofline": dominant,
        "roofline_other": other,
        "solve": {"evals": evals // args.steps, "aux_matvecs": aux // args.steps,
                  "sweeps": int(first.stats[0]["sweeps"]),
                  "best_obj": int(objs.min()), "best_start": first.best,
                  "exit_reasons": {k: int((np.array([s["exit_reason"] for s in first.stats]) == v).sum())
                                   for k, v in (("converged", 0), ("outer_cap", 1), ("stall", 2))},
                  "note": f"first timed step (start set {START_SEED})"},
        "steps_detail": [{"start_seed": START_SEED + j,
                          "evals": int(sum(s["inner_iters"] for s in r.stats)),
                          "aux_matvecs": int(sum(s["aux_matvecs"] for s in r.stats)),
                          "sweeps": int(r.stats[0]["sweeps"]), "best_obj": int(r.obj.min()),
                          "mean_obj": float(r.obj.double().mean())} for j, r in enumerate(results)],
    }
    if not args.no_fp32 and args.qx != "f32":
        fres, fwall, fevals = timed("f32", 1, 0)
        out["fp32_gemm"] = {"value": fevals / fwall, "unit": "evals/s", "steps": 1,
                            "best_obj": int(fres[-1].obj.min()),
                            "note": "same workload with FP32-MFMA Q.X (FP64 lambda_min/CG products)"}
    if not args.no_plain and args.plain_starts > 0:
        # the same starts one by one through the single-instance path (same operand type)
        ks = list(range(args.plain_starts))
        torch.cuda.synchronize()
        t = time.perf_counter()
        plain = [P.solve(Qd, bd, X0=X0d[k].contiguous(), qx_dtype=args.qx) for k in ks]
        torch.cuda.synchronize()
        pw = time.perf_counter() - t
        pe = [p.stats[0]["inner_iters"] for p in plain]
        po = [int(p.obj[0]) for p in plain]
        same = [k for k in ks if po[k] == int(objs[k])]
        plain_rate = sum(pe) / pw
        be = np.array([s["inner_iters"] for s in first.stats])
        out["plain"] = {"starts": len(ks), "evals_per_s": plain_rate, "wall_s": pw,
                        "equal_objective": len(same),
                        "speedup_batched_vs_plain": (evals / wall) / plain_rate,
                        "batched_evals_matching": int(be[same].sum()) if same else 0,
                        "plain_evals_matching": int(sum(pe[k] for k in same))}
    if not args.no_sparse and args.qx == "i8":
        out["sparse"] = sparse_leg(P, gen, torch, dev)
    if not args.no_gemv:
        out["gemv"] = gemv_leg(P, gen, torch, dev)
    if not args.no_group:
        out["group"] = group_leg(P, gen, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Q, b, X0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
