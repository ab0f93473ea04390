"""Real-valued instances (Section 2: Q real symmetric, b real) through
psdp_solve_f64, psdp_solve_host_* and psdp_round_objective_f64, against the
FP64 oracle. The objective of a rounded point is the exact sum of its terms
rounded once to FP64 on both sides (math.fsum in the oracle, an integer
superaccumulator on the GPU), so it is compared bit for bit.
"""
import numpy as np
import pytest

from oracle import psdp as O
from workloads import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    import paper_2408_04875_amd as P
    assert torch.cuda.is_available()
    P.load()
    return P


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _real_set():
    """Fifty real instances, n = 16..20 (ten each), Q and b ~ N(0,1)."""
    out = []
    seed = 700
    for n in range(16, 21):
        for _ in range(10):
            Q, b = gen.real_normal(n, seed)
            out.append((seed, Q, b))
            seed += 1
    return out


def test_real_solves_bit_exact_small_set(P):
    mism = []
    cases = _real_set()
    for seed, Q, b in cases:
        r = P.solve(_t(Q), _t(b))
        ref = O.solve(Q, b)
        got = float(r.obj[0].item())
        if got != ref.obj or not np.array_equal(r.xhat.cpu().numpy(), ref.xhat):
            mism.append((seed, got, ref.obj))
        assert r.stats[0]["exit_reason"] == ref.exit_reason
    print(f"real n=16..20: {len(cases) - len(mism)}/{len(cases)} bit-exact (x^ and FP64 objective); {mism}",
          flush=True)
    assert not mism


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_real_solve_n64_matches_oracle(P, seed):
    """n = 64 with Q ~ N(0,1): the rounded point and the FP64 objective equal
    the oracle's. Real data has no exact-product mode, so the products are
    FP64 sums in the kernels' order against the oracle's BLAS order; the
    per-update trace is compared up to its first divergence (reported) with
    the GPU replaying the oracle's x^0 and penalty steps, and the GPU's own
    lambda_min agrees with the dense eigenvalue while the traces agree."""
    Q, b = gen.real_normal(64, 900 + seed)
    ref = O.solve(Q, b)
    free = P.solve(_t(Q), _t(b))
    gam = O.reformation_gamma(Q, b)
    x0 = O.initial_point(Q + np.diag(gam), b - gam)
    alpha = np.array([[t["alpha"] for t in ref.trace]])
    r = P.solve(_t(Q), _t(b), X0=_t(x0), alpha=alpha, trace_cap=len(ref.trace) + 2)
    lam0 = abs(ref.trace[0]["lam"])
    first = None
    for s, t in enumerate(ref.trace):
        if r.trace[0, s, 1] != t["nI"] or r.trace[0, s, 4] != t["inner"]:
            first = s
            break
        floor = t["alpha"] / O.Params().eta
        if floor > t["lam"] * (1 + 1e-12):   # the floor decided alpha
            assert r.trace[0, s, 2] <= floor * (1 + 1e-9), s
        else:
            assert abs(r.trace[0, s, 2] - t["lam"]) <= 1e-5 * abs(t["lam"]) + 1e-9 * lam0, s
    print(f"real n=64 seed {seed}: free-running gpu {float(free.obj[0]):.17g} outer {free.stats[0]['outer_iters']} | "
          f"oracle {ref.obj:.17g} outer {ref.outer_iters} | replay {float(r.obj[0]):.17g}, first diverging update "
          f"{first}", flush=True)
    assert float(free.obj[0]) == ref.obj
    assert np.array_equal(free.xhat.cpu().numpy(), ref.xhat)


def test_real_path_on_integral_data_equals_integer_path(P):
    """Integer data given as doubles: psdp_solve_f64 performs the integer
    path's arithmetic (the FP64 objective is the exact integer)."""
    Q, b = gen.dense_int(64, 3)
    X0 = gen.random_box_points(64, 8, 11)
    for qdt in ("f64", "f32", "i8"):
        ri = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype=qdt)
        rf = P.solve(_t(Q.astype(np.float64)), _t(b.astype(np.float64)), X0=_t(X0), qx_dtype=qdt)
        assert np.array_equal(ri.xhat.cpu().numpy(), rf.xhat.cpu().numpy()), qdt
        assert np.array_equal(ri.obj.cpu().numpy().astype(np.float64), rf.obj.cpu().numpy()), qdt
        assert np.array_equal(ri.X.cpu().numpy(), rf.X.cpu().numpy()), qdt


def test_real_batched_f32_exact_data(P):
    """Float-valued real data (exact in FP32) on the batched FP32 path, and
    the best-of-batch index on FP64 objectives."""
    rng = np.random.default_rng(17)
    A = rng.standard_normal((96, 96)).astype(np.float32).astype(np.float64)
    Q = np.triu(A) + np.triu(A, 1).T
    b = rng.standard_normal(96).astype(np.float32).astype(np.float64)
    X0 = gen.random_box_points(96, 12, 5)
    r = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="f32")
    obj = r.obj.cpu().numpy()
    xh = r.xhat.cpu().numpy()
    for c in range(12):
        assert obj[c] == O.objective_real(Q, b, xh[c])
    assert r.best == int(np.argmin(obj))


def test_round_objective_f64_is_correctly_rounded_at_size(P):
    """psdp_round_objective_f64 on n = 2500 with entries spread over 120
    binary orders of magnitude and exact cancellations: every objective
    equals the correctly rounded sum (math.fsum)."""
    n, B = 2500, 6
    rng = np.random.default_rng(4)
    A = rng.standard_normal((n, n)) * np.exp2(rng.integers(-60, 60, size=(n, n)))
    Q = np.triu(A) + np.triu(A, 1).T
    Q[0, 1] = Q[1, 0] = 1e200
    Q[0, 2] = Q[2, 0] = -1e200
    b = rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, size=n))
    X = rng.random((B, n))
    X[:, :3] = 0.9
    xh, obj = P.round_objective(_t(Q), _t(b), _t(X))
    xh, obj = xh.cpu().numpy(), obj.cpu().numpy()
    for c in range(B):
        ref_x = (X[c] > 0.5).astype(np.uint8)
        assert np.array_equal(xh[c], ref_x)
        assert obj[c] == O.objective_real(Q, b, ref_x), c
    # the empty selection and a single entry
    X2 = np.zeros((2, n))
    X2[1, 7] = 1.0
    _, o2 = P.round_objective(_t(Q), _t(b), _t(X2))
    assert o2.cpu().numpy().tolist() == [0.0, float(Q[7, 7] + b[7])]


def test_host_pointer_entries_equal_device_entries(P):
    Q, b = gen.dense_int(50, 4)
    X0 = gen.random_box_points(50, 5, 2)
    d = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8")
    xh, obj, X, best, stats = P.solve_host(Q, b, X0=X0, qx_dtype="i8")
    assert np.array_equal(xh, d.xhat.cpu().numpy())
    assert np.array_equal(obj, d.obj.cpu().numpy())
    assert np.array_equal(X, d.X.cpu().numpy())
    assert best == d.best
    Qr, br = gen.real_normal(30, 3)
    d = P.solve(_t(Qr), _t(br))
    xh, obj, X, best, stats = P.solve_host(Qr, br)
    assert np.array_equal(xh[0], d.xhat.cpu().numpy()) and obj[0] == float(d.obj[0])


def test_real_input_checks(P):
    Q, b = gen.real_normal(40, 8)
    bad = Q.copy()
    bad[3, 5] = np.nan
    with pytest.raises(P.PSDPError, match="finite"):
        P.solve(_t(bad), _t(b))
    bb = b.copy()
    bb[2] = np.inf
    with pytest.raises(P.PSDPError, match="finite"):
        P.solve(_t(Q), _t(bb))
    bad = Q.copy()
    bad[3, 17] += 1e-9
    with pytest.raises(P.PSDPError, match=r"Q\[3\]\[17\] != Q\[17\]\[3\]"):
        P.solve(_t(bad), _t(b))
    for qdt in ("bf16", "f32", "i8"):
        with pytest.raises(P.PSDPError, match="unsupported"):
            P.solve(_t(Q), _t(b), qx_dtype=qdt)


def test_group_per_instance_sigmas_equal_single_solves(P):
    """Per-instance perturbation scales in the group launch: each instance
    equals its own single-instance solve with that scale and seed."""
    insts = gen.uneven_group(seed=4, count=6, nmin=20, nmax=90)
    sig = [1e-3 * float(np.abs(d["Q"]).max()) for d in insts]
    Qs = [_t(d["Q"]) for d in insts]
    bs = [_t(d["b"]) for d in insts]
    seeds = [d["seed"] for d in insts]
    xh, obj, stats = P.solve_group(Qs, bs, seeds=seeds, sigmas=sig, perturb="diag")
    for i, d in enumerate(insts):
        one = P.solve(Qs[i], bs[i], sigma=sig[i], perturb="diag", seed=seeds[i])
        assert int(one.obj[0]) == int(obj[i])
        assert np.array_equal(one.xhat.cpu().numpy(), xh[i].cpu().numpy())
