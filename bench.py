"""Benchmark: penalty-gradient evaluations per second of the batched solve.

Workload: one UBQP instance, n = 2500, symmetric integer Q at 10% density with
nonzeros uniform over +-{1..100}, b = 0, and 256 random starts uniform in
[0,1)^n per step, all solved batched (Algorithm 3 with projected alternating
BB subproblems). One step = one start set of 256 starts solved to the end:
every sweep of Q.X products (subproblem and lambda_min products), the
per-column state machine, and the exact int64 objectives. By default the
timed steps' start sets run as one queued launch of 1024 columns (--slots):
a column whose start ends takes the next queued start, so the launch stays
full instead of idling while each set's slowest start finishes; every start
performs exactly the arithmetic of its own-column solve (tested bit for
bit). The same sets solved one launch per set are reported beside it
(`per_set_launches`). Inputs are resident in device memory before the timed
region starts.

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
DIGIT_SOURCES = ("paper_2408_04875_amd/csrc/qx8.hip", "paper_2408_04875_amd/csrc/launch.hpp",
                 "paper_2408_04875_amd/csrc/common.hpp")
# the kernels whose rocprofv3 records (kernel trace, HBM counters) the bench line cites, by the
# name fragment that selects their dispatches, with the sources each record is keyed to
RECORDED_KERNELS = {"psdp::solver_step_kernel<": STEP_SOURCES, "psdp::digit_kernel<": DIGIT_SOURCES}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kernels_n2500_b256_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=2500)
    ap.add_argument("--starts", type=int, default=256)
    ap.add_argument("--plain-starts", type=int, default=32)
    ap.add_argument("--slots", type=int, default=1024,
                    help="solve the timed steps' start sets as one queued launch with this many columns "
                         "(0: one launch per start set)")
    ap.add_argument("--lanes", type=int, default=0,
                    help="lanes of the queued integer-product solve (psdp_params.lanes; 0: the library's choice)")
    ap.add_argument("--no-per-set", action="store_true",
                    help="skip the comparison with one launch per start set")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-replay", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--record-trace", nargs=1, metavar="STATS_CSV",
                    help="write the step and digit kernels' rocprofv3 kernel-trace record from a kernel_stats.csv")
    ap.add_argument("--record-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write the step and digit kernels' HBM traffic record from four rocprofv3 "
                         "counter_collection.csv")
    ap.add_argument("--no-sparse", action="store_true")
    ap.add_argument("--no-gemv", action="store_true")
    ap.add_argument("--no-group", action="store_true")
    ap.add_argument("--group-only", action="store_true", help="only the uneven-batch group leg")
    ap.add_argument("--gemv-only", action="store_true", help="only the large single-instance GEMV leg")
    ap.add_argument("--sparse-only", action="store_true", help="only the sparse Max-Cut leg")
    ap.add_argument("--qx", default="i8", choices=["i8", "f32", "f64"])
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--yardstick-counts", default="16,64,256",
                    help="column counts of the n=2500 yardstick (comma separated)")
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


def source_hash(sources=STEP_SOURCES):
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()


def step_source_hash():
    return source_hash(STEP_SOURCES)


TRACE_FILE = os.path.join(ROOT, "profiles", "kernels_n2500_b256_trace.json")
# the bench command the kernel records are taken from: the default configuration (queued launch
# of 1024 columns) over twenty start sets, without the side legs
PROFILE_ARGS = ("--steps 20 --warmup 0 --no-cpu-baseline --no-plain --no-fp32 --no-sparse --no-gemv --no-group "
                "--no-replay --no-adjoint --no-per-set")
STEP_KERNEL_PREFIX = "psdp::solver_step_kernel<"
DIGIT_KERNEL_PREFIX = "psdp::digit_kernel<"


def _csv_rows(path):
    import csv
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def record_trace(stats_csv):
    """Writes TRACE_FILE from a rocprofv3 --kernel-trace --stats summary
    (kernel_stats.csv): calls and average duration of each recorded kernel
    (all its instantiations), keyed to that kernel's sources."""
    rows = _csv_rows(stats_csv)
    recs = {}
    for frag, sources in RECORDED_KERNELS.items():
        sel = [r for r in rows if frag in r["Name"]]
        calls = sum(int(r["Calls"]) for r in sel)
        total = sum(float(r["TotalDurationNs"]) for r in sel)
        recs[frag] = {"kernel": [r["Name"] for r in sel], "source_sha256": source_hash(sources), "calls": calls,
                      "avg_ns": total / max(calls, 1)}
    rec = {"records": recs,
           "command": "cd /tmp && rocprofv3 --kernel-trace --stats -d <out> -o run -- python -u <repo>/bench.py "
                      + PROFILE_ARGS,
           "note": "both queued solves of the run (the timed one and the one with HIP events around every launch); "
                   "the two lanes run concurrently, so launch durations include time shared with the other lane"}
    with open(TRACE_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def record_traffic(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """Writes TRAFFIC_FILE from four rocprofv3 --pmc counter runs: FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch) over the bench command and over
    --calibrate-copy (1 GiB copied three times); each counter is scaled so
    that it reads 1 GiB for the 1 GiB copy."""
    def per_dispatch(path, counter, frag):
        vals = [float(r["Counter_Value"]) for r in _csv_rows(path)
                if r["Counter_Name"] == counter and frag in r["Kernel_Name"]]
        return sum(vals) / max(len(vals), 1), len(vals)
    # the copy run launches one kind of large kernel: take every dispatch above 1 MiB
    cf = [float(r["Counter_Value"]) for r in _csv_rows(copy_fetch_csv) if r["Counter_Name"] == "FETCH_SIZE"]
    cw = [float(r["Counter_Value"]) for r in _csv_rows(copy_write_csv) if r["Counter_Name"] == "WRITE_SIZE"]
    cf = [v for v in cf if v > 1024.0]
    cw = [v for v in cw if v > 1024.0]
    gib_kib = (1 << 30) / 1024.0
    fs, ws = gib_kib / (sum(cf) / len(cf)), gib_kib / (sum(cw) / len(cw))
    recs = {}
    for frag, sources in RECORDED_KERNELS.items():
        f_kib, nd = per_dispatch(fetch_csv, "FETCH_SIZE", frag)
        w_kib, _ = per_dispatch(write_csv, "WRITE_SIZE", frag)
        fb, wb = f_kib * 1024.0 * fs, w_kib * 1024.0 * ws
        recs[frag] = {"source_sha256": source_hash(sources), "bytes_per_launch": fb + wb,
                      "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb, "dispatches": nd,
                      "fetch_size_kib_avg": f_kib, "write_size_kib_avg": w_kib}
    rec = {"workload": "n = 2500, 20 sets of 256 starts through 1024 columns in two lanes, I8 operands",
           "records": recs,
           "copy_calibration": {"bytes": 1 << 30, "fetch_size_kib": sum(cf) / len(cf),
                                "write_size_kib": sum(cw) / len(cw), "fetch_scale": fs, "write_scale": ws},
           "commands": [f"cd /tmp && rocprofv3 --pmc {c} --output-format csv -d <out> -o run -- python -u "
                        f"<repo>/bench.py {a}" for c in ("FETCH_SIZE", "WRITE_SIZE")
                        for a in (PROFILE_ARGS, "--calibrate-copy")],
           "note": "bytes = FETCH_SIZE KiB x 1024 x fetch_scale + WRITE_SIZE KiB x 1024 x write_scale, averaged "
                   "over the kernel's dispatches of both solves of the run (timed and instrumented)"}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def _record(path, frag, key):
    """One field of a kernel's committed record, or None when the record is
    missing or the kernel's sources changed since it was taken."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    r = t.get("records", {}).get(frag)
    if not r or r.get("source_sha256") != source_hash(RECORDED_KERNELS[frag]):
        return None
    return r.get(key)


def measured_avg_ns(frag=STEP_KERNEL_PREFIX):
    """Average launch duration from the committed rocprofv3 kernel trace."""
    return _record(TRACE_FILE, frag, "avg_ns")


def measured_traffic(frag=STEP_KERNEL_PREFIX):
    """HBM bytes per launch from the committed rocprofv3 counter runs."""
    return _record(TRAFFIC_FILE, frag, "bytes_per_launch")


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
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), model)
    except OSError:
        pass
    return {"value": evals / wall, "unit": "evals/s", "cores": cores, "kind": "oracle", "cpu_model": model,
            "sample": f"start 0 of the n=2500 workload, {outer} penalty updates, {evals} evaluations "
                      f"(dense eigensolver and BLAS matvecs included), {wall:.1f} s"}


def cpu_eval_rate(shapes=((1000, 1), (2500, 1), (2500, 256), (4096, 64)), budget_s=4.0):
    """FP64 penalty-gradient evaluations on the host: NumPy U = Q X and the
    epilogue g = 2 (U - p o X) + (b + p) at the configurations' shapes, with
    all BLAS threads and with one, median over repetitions (at most 50, about
    budget_s per shape and thread count)."""
    import numpy as np
    from threadpoolctl import threadpool_limits, threadpool_info
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    threads_all = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    out = {"cpu_model": model, "os_cpu_count": os.cpu_count(), "blas_threads_all": threads_all, "rates": []}
    rng = np.random.default_rng(0)
    for n, B in shapes:
        Q = rng.standard_normal((n, n))
        X = rng.random((n, B))
        b, p = rng.standard_normal(n), rng.random(n)
        row = {"n": n, "B": B}
        for label, nt in (("all", threads_all), ("one", 1)):
            with threadpool_limits(nt):
                times = []
                t_end = time.perf_counter() + budget_s
                while len(times) < 50 and (len(times) < 3 or time.perf_counter() < t_end):
                    t = time.perf_counter()
                    U = Q @ X
                    G = 2.0 * (U - p[:, None] * X) + (b + p)[:, None]
                    times.append(time.perf_counter() - t)
                del U, G
            med = float(np.median(times))
            row[f"evals_per_s_{label}_threads"] = B / med
            row[f"reps_{label}"] = len(times)
        out["rates"].append(row)
    return out


def adjoint_leg(P, gen, torch, reps=20):
    """The differentiation configuration: n = 4096 FP32 Q ~ N(0,1), 64 points:
    the forward evaluation (h, grad h) and the adjoint's dQ = X Diag(w) X^T,
    each timed alone with events on torch's current stream (the stream the
    library's stream-ordered entry points run on), median of reps."""
    import numpy as np
    Q, b, X, p, w = gen.dense_normal_batch()
    n, B = X.shape[1], X.shape[0]
    Qd, bd, Xd, pd, wd = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (Q, b, X, p, w))
    _, G = P.eval_penalty_grad(Qd, bd, pd, Xd)

    def med(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.median(ts))

    tf = med(lambda: P.eval_penalty_grad(Qd, bd, pd, Xd))
    tq = med(lambda: P.penalty_adjoint(Xd, G, wd, want=("dQ",)))
    fl = 2.0 * n * n * B
    return {"workload": f"n={n} dense Q ~ N(0,1) FP32, {B} points, FP32 operands and vectors",
            "forward": {"seconds": tf, "tflops": fl / tf / 1e12, "gbs_q": 4.0 * n * n / tf / 1e9,
                        "frac_fp32_mfma": fl / tf / 1e12 / PEAK_FP32_TFLOPS,
                        "note": "h and grad h: Q X on FP32 MFMA (2 n^2 B flops, Q read once) plus the epilogue"},
            "dQ": {"seconds": tq, "tflops": fl / tq / 1e12, "gbs_written": 4.0 * n * n / tq / 1e9,
                   "frac_fp32_mfma": fl / tq / 1e12 / PEAK_FP32_TFLOPS,
                   "frac_hbm_write": 4.0 * n * n / tq / 1e9 / PEAK_HBM_GBS,
                   "note": "dQ = X Diag(w) X^T (2 n^2 B flops, n^2 FP32 outputs written)"}}


def replay_records(prefix):
    """Stored oracle solves (tests/golden/oracle_replay.jsonl) whose names
    start with prefix, in file order."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_replay.jsonl")
    out = []
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            r = json.loads(line)
            if r.get("name", "").startswith(prefix):
                out.append(r)
    return out


def replay_leg(P, torch, Qd, bd, X0d):
    """Batched against plain at equal objectives by construction: the first
    16 starts of start set 3 replaying the stored oracle solves' penalty
    steps (the oracle's alpha per update), through the batched launch (I8
    and F64 operands, 16 columns) and one by one through the single-instance
    FP32-GEMV path; every result is compared with the oracle's objective."""
    import numpy as np
    out = {}
    for mode in ("fp64", "i8"):
        recs = replay_records(f"n2500_start")
        recs = [r for r in recs if r["product"] == mode]
        if len(recs) < 16:
            return {"note": "no stored oracle solves"}
        cap = max(len(r["alpha"]) for r in recs)
        A = np.ones((16, cap))
        for c, r in enumerate(recs[:16]):
            A[c, :len(r["alpha"])] = r["alpha"]
        ref = [r["obj"] for r in recs[:16]]
        qx = "f64" if mode == "fp64" else "i8"
        torch.cuda.synchronize()
        t = time.perf_counter()
        rb = P.solve(Qd, bd, X0=X0d[:16].contiguous(), qx_dtype=qx, alpha=A)
        torch.cuda.synchronize()
        wb = time.perf_counter() - t
        ob = [int(v) for v in rb.obj.cpu().numpy()]
        eb = sum(s["inner_iters"] for s in rb.stats)
        entry = {"batched": {"qx": qx, "evals_per_s": eb / wb, "wall_s": wb,
                             "equal_to_oracle": sum(int(a == c) for a, c in zip(ob, ref)), "best_obj": min(ob)},
                 "oracle_best_obj": min(ref)}
        if mode == "fp64":
            torch.cuda.synchronize()
            t = time.perf_counter()
            rp = [P.solve(Qd, bd, X0=X0d[c].contiguous(), qx_dtype="f32", alpha=A[c:c + 1]) for c in range(16)]
            torch.cuda.synchronize()
            wp = time.perf_counter() - t
            op = [int(r.obj[0]) for r in rp]
            ep = sum(r.stats[0]["inner_iters"] for r in rp)
            entry["plain_f32_gemv"] = {"evals_per_s": ep / wp, "wall_s": wp,
                                       "equal_to_oracle": sum(int(a == c) for a, c in zip(op, ref)),
                                       "best_obj": min(op)}
            entry["speedup_batched_vs_plain"] = (eb / wb) / (ep / wp)
        out[mode] = entry
    out["note"] = ("16 starts replaying the oracle's penalty steps; a batch of 16 columns, so its rate is far "
                   "below the 256-start launch")
    return out


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
    # of the packed nonzeros (4 B per nonzero, read once per pass of 16
    # halves) and the int64 outputs
    per_half = 4 * nnz + nnz // 4 + 8 * n
    qs = s0["qx_seconds"] + s0["aux_seconds"]
    return {"workload": f"maxcut n={n} G(n,{p_edge}) +-1 weights, b=-We, diag perturbation sigma 0.5, "
                        f"{B} random starts, Q.X i8",
            "nnz": nnz, "evals_per_s_sparse": ev / wa, "evals_per_s_dense": ev / wd,
            "speedup_sparse_vs_dense": wd / wa, "equal_objective": same, "starts": B,
            "sparse_sweeps": int(auto.stats[0]["sparse_sweeps"]), "sweeps": int(auto.stats[0]["sweeps"]),
            "sparse_kernel": {"kernel": "sparse_stage_kernel + sparse_kernel (CSR rows, int64 exact)", "launches": s0["qx_launches"],
                              "avg_launch_us": qs / max(s0["qx_launches"], 1) * 1e6,
                              "bytes_per_column_half": per_half,
                              "achieved": halves * per_half / qs / 1e9 if qs > 0 else 0.0,
                              "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": halves * per_half / qs / 1e9 / PEAK_HBM_GBS if qs > 0 else 0.0}}


def gemv_leg(P, gen, torch, dev, n=16384, outer=3):
    """Single-instance solves (one start) on a Q too large for the caches
    (n = 16384: 1.07 GB in FP32, 0.54 GB in BF16 against 256 MB of Infinity
    Cache), a few penalty updates each, with the product reading Q's unique
    half from packed upper tiles (the default at this size) and with the
    row-by-row GEMV reading all of Q. Algorithmic bytes per product: the
    unique half, n (n + 1) / 2 entries of Q."""
    Q, b = gen.sparse_int(n, 5)
    Qd, bd = torch.from_numpy(Q).to(dev), torch.from_numpy(b).to(dev)
    del Q
    x0 = torch.from_numpy(gen.random_box_points(n, 1, 6)).to(dev)
    ld = (n + 31) // 32 * 32
    nb = (n + 127) // 128
    out = {"workload": f"one start, n={n}, 10% density ints +-[1,100], b=0, {outer} penalty updates"}
    for qx, eb in (("f32", 4), ("bf16", 2)):
        for sym in (1, 0):
            r = P.solve(Qd, bd, X0=x0, qx_dtype=qx, max_outer=outer, timing=1, gemv_sym=sym)
            s0 = r.stats[0]
            products = s0["inner_iters"] + s0["aux_matvecs"]
            secs = s0["qx_seconds"] + s0["aux_seconds"]
            launches = s0["qx_launches"]
            unique = n * (n + 1) // 2 * eb
            stored = (nb * (nb + 1) // 2 * 128 * 128 if sym else n * ld) * eb
            name = ("symv_tile_kernel + symv_reduce_kernel" if sym else "gemv_kernel") + \
                f"<{'float' if qx == 'f32' else '__hip_bfloat16'}>"
            out[f"{qx}_{'tiles' if sym else 'rows'}"] = {
                "kernel": name, "bound": "hbm", "products": int(products), "launches": int(launches),
                "avg_launch_us": secs / max(launches, 1) * 1e6, "bytes_per_product": unique,
                "stored_bytes_per_product": stored,
                "achieved": products * unique / secs / 1e9 if secs > 0 else 0.0, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": products * unique / secs / 1e9 / PEAK_HBM_GBS if secs > 0 else 0.0,
                "stored_gbs": products * stored / secs / 1e9 if secs > 0 else 0.0,
                "note": "unique-half bytes of the products with a live column over the time of all product launches"}
    # vendor yardstick: torch.mv (the vendor BLAS GEMV) on the same Q, full storage
    Qf = Qd.to(torch.float32)
    for qx, dt, eb in (("f32", torch.float32, 4), ("bf16", torch.bfloat16, 2)):
        A = Qf.to(dt)
        v = x0[0].to(dt)
        torch.mv(A, v)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 20
        e0.record()
        for _ in range(reps):
            torch.mv(A, v)
        e1.record()
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        out[f"vendor_mv_{qx}"] = {"us": us, "stored_gbs": n * n * eb / us * 1e-3,
                                  "unique_gbs": n * (n + 1) // 2 * eb / us * 1e-3,
                                  "note": "torch.mv on the full matrix (vendor BLAS), events over 20 calls"}
        del A
    del Qf
    return out


def group_leg(P, gen, torch, dev, count=512):
    """The uneven batch: 512 instances with n uniform in [100, 3000], half
    Max-Cut graphs (p = 0.05, weights +-1), half dense integer Q of density
    0.1-0.8, BF16 operands, diagonal perturbation with each instance's own
    sigma = 1e-3 max|Q_ij| and seed = its index, one start each, all
    advanced in one group launch per sweep. Solved with the product from the
    instances' packed upper tiles (the default at this size: 3.3 GB of
    stored BF16 matrices) and with the row-by-row group GEMV; algorithmic
    bytes per product n_i (n_i + 1) / 2 BF16 entries (the unique half)."""
    import numpy as np
    insts = gen.uneven_group(seed=4, count=count, nmin=100, nmax=3000)
    sigmas = [1e-3 * float(np.abs(d["Q"]).max()) for d in insts]
    Qs = [torch.from_numpy(d["Q"]).to(dev) for d in insts]
    bs = [torch.from_numpy(d["b"]).to(dev) for d in insts]
    ns = [d["n"] for d in insts]
    seeds = [d["seed"] for d in insts]
    out = {"workload": f"{count} instances, n uniform in [100, 3000], half Max-Cut G(n, 0.05) +-1, half dense "
                       f"off-diagonal density 0.1-0.8 (off-diagonal ints in [-50, 50], diagonal in [-100, 100]); "
                       f"BF16 Q.X, diagonal perturbation sigma_i = 1e-3 max|Q_i| per instance "
                       f"({min(sigmas):g} to {max(sigmas):g}), one start each",
           "sum_n2": int(sum(n * n for n in ns))}
    objs = {}
    for name, sym in (("tiles", 1), ("rows", 0)):
        kw = dict(qx_dtype="bf16", perturb="diag", sigmas=sigmas, gemv_sym=sym)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xh, obj, st = P.solve_group(Qs, bs, seeds=seeds, **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        evals = sum(s["inner_iters"] for s in st)
        # the same solve with HIP events around every product launch
        _, obj2, st2 = P.solve_group(Qs, bs, seeds=seeds, timing=1, **kw)
        qs = st2[0]["qx_seconds"]
        products = [s["inner_iters"] + s["aux_matvecs"] for s in st2]
        unique = sum(k * n * (n + 1) // 2 * 2 for k, n in zip(products, ns))
        if sym:
            stored = sum(k * ((n + 127) // 128) * ((n + 127) // 128 + 1) // 2 * 128 * 128 * 2
                         for k, n in zip(products, ns))
            kname = "symv_group_tile_kernel<__hip_bfloat16> + symv_group_reduce_kernel"
        else:
            stored = sum(k * n * ((n + 31) // 32 * 32) * 2 for k, n in zip(products, ns))
            kname = "gemv_group_kernel<__hip_bfloat16>"
        objs[name] = obj.cpu()
        out[name] = {"evals": int(evals), "aux_matvecs": int(sum(s["aux_matvecs"] for s in st)),
                     "sweeps": int(st[0]["sweeps"]), "wall_s": wall, "evals_per_s": evals / wall,
                     "same_objectives_timed_run": bool((obj.cpu() == obj2.cpu()).all()),
                     "exit_reasons": {k: int((np.array([s["exit_reason"] for s in st]) == v).sum())
                                      for k, v in (("converged", 0), ("outer_cap", 1), ("stall", 2))},
                     "product": {"kernel": kname, "launches": int(st2[0]["qx_launches"]), "seconds": qs,
                                 "bytes": int(unique), "stored_bytes": int(stored),
                                 "achieved": unique / qs / 1e9 if qs > 0 else 0.0, "peak": PEAK_HBM_GBS,
                                 "unit": "GB/s", "frac": unique / qs / 1e9 / PEAK_HBM_GBS if qs > 0 else 0.0,
                                 "stored_gbs": stored / qs / 1e9 if qs > 0 else 0.0,
                                 "note": "unique-half BF16 bytes of every product over the product launches' "
                                         "event time (stored_gbs: the bytes each kernel reads)"}}
    out["equal_objectives_tiles_rows"] = int((objs["tiles"] == objs["rows"]).sum())
    out["evals_per_s"] = out["tiles"]["evals_per_s"]
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described in the design notes but not part of this build.", file=sys.stderr)
        sys.exit(2)
    if args.record_trace:
        record_trace(*args.record_trace)
        return
    if args.record_traffic:
        record_traffic(*args.record_traffic)
        return
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gemm_yardstick:
        gemm_yardstick(n=args.n, counts=tuple(int(c) for c in args.yardstick_counts.split(",")))
        if args.yardstick_counts == "16,64,256":
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
    if args.sparse_only:
        print(json.dumps({"sparse": sparse_leg(P, gen, torch, dev)}), flush=True)
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

    def step(qx, timing=False, X=None, slots=0):
        return P.solve(Qd, bd, X0=X0d if X is None else X, qx_dtype=qx, timing=1 if timing else 0, slots=slots,
                       lanes=args.lanes)

    class SetView:
        """One start set's share of a queued launch (the fields used below)."""
        def __init__(self, r, j):
            self.obj = r.obj[j * B:(j + 1) * B]
            self.stats = r.stats[j * B:(j + 1) * B]
            self.best = int(np.argmin(self.obj.cpu().numpy()))

    def timed(qx, steps, warmup, slots=0):
        for _ in range(warmup):
            step(qx)
        torch.cuda.synchronize()
        if slots:
            # every set's starts in one launch of `slots` columns: a column whose
            # start ends takes the next start, so the launch stays full
            Xall = torch.cat(X0s[:steps], dim=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = step(qx, X=Xall, slots=slots)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            res = [SetView(r, j) for j in range(steps)]
            for v in res:
                v.sweeps = int(r.stats[0]["sweeps"])
        else:
            t0 = time.perf_counter()
            res = [step(qx, X=X0s[j]) for j in range(steps)]
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            for v in res:
                v.sweeps = int(v.stats[0]["sweeps"])
        evals = sum(sum(s["inner_iters"] for s in r.stats) for r in res)
        return res, wall, evals

    results, wall, evals = timed(args.qx, args.steps, args.warmup, args.slots)
    print(f"bench: {args.qx} {args.steps} timed steps in {wall:.2f} s", file=sys.stderr, flush=True)
    aux = sum(sum(s["aux_matvecs"] for s in r.stats) for r in results)
    # one more solve with HIP events around every launch (library solve
    # stream): per-kernel average durations and algorithmic work. Per-set
    # launches: the first start set; queued: the timed sets' starts through
    # the same number of columns (the timed workload, launched eagerly)
    if args.slots:
        inst = step(args.qx, timing=True, X=torch.cat(X0s[:args.steps], dim=0), slots=args.slots)
    else:
        inst = step(args.qx, timing=True)
    s0 = inst.stats[0]
    inst_evals = sum(s["inner_iters"] for s in inst.stats)
    inst_aux = sum(s["aux_matvecs"] for s in inst.stats)
    step_s, step_l, colsteps = s0["step_seconds"], s0["step_launches"], s0["column_steps"]
    step_bytes = STEP_BYTES_PER_COLUMN * n * colsteps
    qx_s = s0["qx_seconds"] + s0["aux_seconds"]
    qx_f = s0["qx_flops"] + s0["aux_flops"]
    qx_l = s0["qx_launches"]
    rp_ns = measured_avg_ns(STEP_KERNEL_PREFIX)
    step_rl = {"bound": "hbm", "achieved": step_bytes / step_s / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
               "frac": step_bytes / step_s / 1e9 / PEAK_HBM_GBS, "traffic": measured_traffic(STEP_KERNEL_PREFIX),
               "frac_rocprof": (step_bytes / max(step_l, 1) / (rp_ns * 1e-9) / 1e9 / PEAK_HBM_GBS
                                if rp_ns else None),
               "avg_launch_us_rocprof": rp_ns * 1e-3 if rp_ns else None,
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
             "traffic": measured_traffic(DIGIT_KERNEL_PREFIX) if args.qx == "i8" else None,
             "kernel": qx_name, "launches": qx_l, "seconds": qx_s,
             "avg_launch_us": qx_s / max(qx_l, 1) * 1e6,
             "work": "2 n^2 multiply-adds per column product (algorithmic; the int8 path executes 4 or 8 "
                     "digit products per column)"}
    if args.qx == "i8":
        # the int8 MFMA work the digit kernel executes: 4 digit rows per subproblem column and 8 per
        # lambda_min column, each against the whole padded Q (ldq x ldq)
        ldq = (n + 63) // 64 * 64
        ex = 2.0 * ldq * ldq * (4.0 * inst_evals + 8.0 * inst_aux)
        dk_ns = measured_avg_ns(DIGIT_KERNEL_PREFIX)
        qx_rl.update({"executed_tops": ex / qx_s / 1e12 if qx_s > 0 else 0.0,
                      "executed_frac": ex / qx_s / 1e12 / qx_peak if qx_s > 0 else 0.0,
                      "avg_launch_us_rocprof": dk_ns * 1e-3 if dk_ns else None,
                      "frac_rocprof": (qx_f / max(qx_l, 1) / (dk_ns * 1e-9) / 1e12 / qx_peak if dk_ns else None)})
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
                               f"batched PABB, Q.X {args.qx}" +
                               (f", the steps' sets as one queued launch of {args.slots} columns"
                                if args.slots else ", one launch per set"),
                   "n": n, "starts": B, "global_batch": B, "slots": args.slots or B,
                   "parallelism": "single gpu"},
        "roofline": dominant,
        "roofline_other": other,
        "solve": {"evals": evals // args.steps, "aux_matvecs": aux // args.steps,
                  "sweeps": first.sweeps,
                  "best_obj": int(objs.min()), "best_start": first.best,
                  "exit_reasons": {k: int((np.array([s["exit_reason"] for s in first.stats]) == v).sum())
                                   for k, v in (("converged", 0), ("outer_cap", 1), ("stall", 2))},
                  "note": f"first timed step (start set {START_SEED})"},
        "steps_detail": [{"start_seed": START_SEED + j,
                          "evals": int(sum(s["inner_iters"] for s in r.stats)),
                          "aux_matvecs": int(sum(s["aux_matvecs"] for s in r.stats)),
                          "sweeps": r.sweeps, "best_obj": int(r.obj.min()),
                          "mean_obj": float(r.obj.double().mean())} for j, r in enumerate(results)],
    }
    if args.slots and not args.no_per_set:
        pres, pwall, pevals = timed(args.qx, args.steps, 0, 0)
        same = sum(int((a.obj.cpu() == b.obj.cpu()).all()) for a, b in zip(results, pres))
        out["per_set_launches"] = {"value": pevals / pwall, "unit": "evals/s", "ms_per_step": pwall / args.steps * 1e3,
                                   "sets_with_equal_objectives": same,
                                   "note": "the same start sets, one launch of 256 columns per set"}
    if not args.no_fp32 and args.qx != "f32":
        fres, fwall, fevals = timed("f32", args.steps, 0, args.slots)
        ft = (step("f32", timing=True, X=torch.cat(X0s[:args.steps], dim=0), slots=args.slots)
              if args.slots else step("f32", timing=True)).stats[0]
        out["fp32_gemm"] = {"value": fevals / fwall, "unit": "evals/s", "steps": args.steps,
                            "ms_per_step": fwall / args.steps * 1e3,
                            "best_obj": [int(r.obj.min()) for r in fres],
                            "mean_obj": [float(r.obj.double().mean()) for r in fres],
                            "fp32_products": {"tflops": ft["qx_flops"] / ft["qx_seconds"] / 1e12,
                                              "frac_fp32_mfma": ft["qx_flops"] / ft["qx_seconds"] / 1e12 /
                                              PEAK_FP32_TFLOPS, "launches": ft["qx_launches"],
                                              "avg_launch_us": ft["qx_seconds"] / max(ft["qx_launches"], 1) * 1e6},
                            "fp64_aux_products": {"tflops": ft["aux_flops"] / ft["aux_seconds"] / 1e12
                                                  if ft["aux_seconds"] > 0 else 0.0,
                                                  "frac_fp64_mfma": ft["aux_flops"] / ft["aux_seconds"] / 1e12 /
                                                  PEAK_FP64_TFLOPS if ft["aux_seconds"] > 0 else 0.0},
                            "note": "same start sets with FP32-MFMA subproblem products (FP64 lambda_min/CG "
                                    "products); the product fractions are algorithmic flops (2 n^2 per live column) "
                                    "over the event time of all product launches of one solve, tail included"}
    if not args.no_plain and args.plain_starts > 0:
        # the first starts of the first timed set one by one through the
        # single-instance path with FP32 storage and FP64 accumulation (the
        # plain method with an FP32 GEMV), and a few through the I8 path with
        # one column (the batched code path at B = 1)
        ks = list(range(args.plain_starts))
        torch.cuda.synchronize()
        t = time.perf_counter()
        plain = [P.solve(Qd, bd, X0=X0d[k].contiguous(), qx_dtype="f32") for k in ks]
        torch.cuda.synchronize()
        pw = time.perf_counter() - t
        pe = [p.stats[0]["inner_iters"] for p in plain]
        po = np.array([int(p.obj[0]) for p in plain])
        plain_rate = sum(pe) / pw
        bo = objs[:len(ks)]
        out["plain"] = {"path": "single-instance FP32 GEMV (FP64 accumulation), one start per solve",
                        "starts": len(ks), "evals_per_s": plain_rate, "wall_s": pw,
                        "speedup_batched_vs_plain": (evals / wall) / plain_rate,
                        "speedup_per_set_launches_vs_plain": (out["per_set_launches"]["value"] / plain_rate
                                                              if "per_set_launches" in out else None),
                        "equal_objective_vs_batched_i8": int((po == bo).sum()),
                        "mean_obj": float(po.mean()), "best_obj": int(po.min()),
                        "batched_same_starts_mean_obj": float(bo.mean()), "batched_same_starts_best_obj": int(bo.min()),
                        "note": "free-running trajectories of different product arithmetic part at this size, so "
                                "objectives are compared in distribution here and exactly in the replay leg"}
        k8 = ks[:8]
        torch.cuda.synchronize()
        t = time.perf_counter()
        pi8 = [P.solve(Qd, bd, X0=X0d[k].contiguous(), qx_dtype="i8") for k in k8]
        torch.cuda.synchronize()
        wi8 = time.perf_counter() - t
        oi8 = [int(p.obj[0]) for p in pi8]
        out["i8_batched_path_b1"] = {"starts": len(k8),
                                     "evals_per_s": sum(p.stats[0]["inner_iters"] for p in pi8) / wi8,
                                     "equal_objective_vs_batched": sum(int(a == int(c)) for a, c in zip(oi8, objs)),
                                     "note": "the I8 (batched) code path with one column per solve: the same "
                                             "per-column arithmetic as the 256-start launch"}
    if not args.no_replay and args.qx == "i8" and n == 2500 and B == 256:
        out["replay"] = replay_leg(P, torch, Qd, bd, X0d)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(P, gen, torch)
    if not args.no_sparse and args.qx == "i8":
        out["sparse"] = sparse_leg(P, gen, torch, dev)
    if not args.no_gemv:
        out["gemv"] = gemv_leg(P, gen, torch, dev)
    if not args.no_group:
        out["group"] = group_leg(P, gen, torch, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(Q, b, X0)
        out["cpu_eval_rate"] = cpu_eval_rate()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
