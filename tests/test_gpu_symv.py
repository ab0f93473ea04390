"""The single-instance product from the unique half of Q (packed 128 x 128
upper tiles, psdp_qx_single with sym = 1, psdp_params.gemv_sym) against
its FP64 definition Q_off x and against the row-by-row GEMV, whole
single-instance solves with it against the oracle, and the group product
from every instance's tiles against the single-instance one and the oracle.

Both products sum exact FP64 products (integer Q widened exactly) in FP64,
in different orders, so each lies within the accumulation bound
(n + 2) 2^-53 sum_j |Q_ij| |x_j| of the exact value (computed here by
math.fsum); the tile product is also reproducible run to run.
"""
import math

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


def _exact_rows(Q, x, rows):
    """Q_off x on the given rows as correctly rounded sums, with the bound."""
    out, bound = [], []
    n = len(x)
    for i in rows:
        q = Q[i].astype(np.float64)
        q[i] = 0.0
        out.append(math.fsum((q * x).tolist()) if n < 4096 else math.fsum(q[j] * x[j] for j in np.nonzero(q)[0]))
        bound.append((n + 2) * 2.0 ** -53 * float(np.abs(q) @ np.abs(x)))
    return np.array(out), np.array(bound)


@pytest.mark.parametrize("n", [1, 5, 127, 128, 129, 300, 1000, 2500])
@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16"])
def test_tile_product_within_fp64_bound(P, n, dtype):
    lim = 100 if dtype == "bf16" else 30000
    rng = np.random.default_rng(n)
    A = rng.integers(-lim, lim + 1, (n, n)) * (rng.random((n, n)) < 0.3)
    Q = (np.triu(A) + np.triu(A, 1).T).astype(np.int32)
    x = rng.random(n)
    rows = np.arange(n) if n <= 300 else np.sort(rng.choice(n, 200, replace=False))
    ref, bound = _exact_rows(Q, x, rows)
    ys = P.qx_single(_t(Q), _t(x), dtype=dtype, sym=True).cpu().numpy()
    yf = P.qx_single(_t(Q), _t(x), dtype=dtype, sym=False).cpu().numpy()
    assert (np.abs(ys[rows] - ref) <= bound).all()
    assert (np.abs(yf[rows] - ref) <= bound).all()
    ys2 = P.qx_single(_t(Q), _t(x), dtype=dtype, sym=True).cpu().numpy()
    assert np.array_equal(ys, ys2)
    print(f"n={n} {dtype}: max |tile - exact| / bound = {np.max(np.abs(ys[rows] - ref) / np.maximum(bound, 1e-300)):.2e}",
          flush=True)


def test_tile_product_full_size_sampled_rows(P):
    """n = 16384 (the single-instance GEMV workload, 10% density), FP32 and
    BF16 storage: 64 sampled rows against the exact sums."""
    n = 16384
    Q, _ = gen.sparse_int(n, 5)
    x = gen.random_box_points(n, 1, 6)[0]
    Qd, xd = _t(Q), _t(x)
    rows = np.sort(np.random.default_rng(3).choice(n, 64, replace=False))
    ref, bound = _exact_rows(Q, x, rows)
    for dtype in ("f32", "bf16"):
        y = P.qx_single(Qd, xd, dtype=dtype, sym=True).cpu().numpy()
        assert (np.abs(y[rows] - ref) <= bound).all(), dtype


def test_solves_with_tile_product_equal_the_oracle_small_set(P):
    """Single-instance solves (from x^0) reading Q from its unique half:
    the rounded point and the objective equal the oracle's on the n <= 20
    set and on the dense n = 64 instance, in FP32 and BF16 storage."""
    cases = gen.bruteforce_set()[::2] + [(0,) + gen.small_dense(0)]
    mism = []
    for seed, Q, b in cases:
        ref = O.solve(Q, b)
        for qdt in ("f32", "bf16"):
            r = P.solve(_t(Q), _t(b), qx_dtype=qdt, gemv_sym=1)
            if int(r.obj[0]) != ref.obj or not np.array_equal(r.xhat.cpu().numpy(), ref.xhat):
                mism.append((seed, qdt))
    print(f"tile-product solves: {2 * len(cases) - len(mism)}/{2 * len(cases)} equal to the oracle", flush=True)
    assert not mism


def test_auto_choice_and_solve_agreement_n4096(P):
    """From n = 4096 the default reads the tiles: a solve with the default
    equals one with gemv_sym = 1 bit for bit; the full-row solve is reported
    beside them (the summation orders differ, so the trajectories may
    part)."""
    n = 4096
    Q, b = gen.sparse_int(n, 9)
    x0 = gen.random_box_points(n, 1, 10)
    Qd, bd, xd = _t(Q), _t(b), _t(x0)
    a = P.solve(Qd, bd, X0=xd, qx_dtype="f32", max_outer=4)
    s = P.solve(Qd, bd, X0=xd, qx_dtype="f32", max_outer=4, gemv_sym=1)
    f = P.solve(Qd, bd, X0=xd, qx_dtype="f32", max_outer=4, gemv_sym=0)
    assert int(a.obj[0]) == int(s.obj[0])
    assert np.array_equal(a.X.cpu().numpy(), s.X.cpu().numpy())
    print(f"n=4096, 4 penalty updates: tiles {int(s.obj[0])} ({s.stats[0]['inner_iters']} evaluations), full rows "
          f"{int(f.obj[0])} ({f.stats[0]['inner_iters']} evaluations)", flush=True)


@pytest.mark.parametrize("qdt", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("poll", [64, 2])
def test_group_tiles_equal_single_instance_tiles(P, qdt, poll):
    """The group product from every instance's packed upper tiles (one work
    list over the live instances' tiles, rebuilt as instances finish: at
    polls every 2 sweeps many times) performs each instance's single-instance
    tile product bit for bit: rounded point, objective and counts equal the
    single-instance solves with gemv_sym = 1, for sizes around the 128-row
    tile edge."""
    insts = gen.uneven_group(seed=11, count=10, nmin=20, nmax=300)
    extra = [gen.sparse_int(n, 30 + n) for n in (127, 128, 129, 256, 257)]
    Qs = [_t(d["Q"]) for d in insts] + [_t(Q) for Q, _ in extra]
    bs = [_t(d["b"]) for d in insts] + [_t(b) for _, b in extra]
    sigma = max(1e-3 * float(np.abs(d["Q"]).max()) for d in insts)
    seeds = list(range(len(Qs)))
    xh, obj, stats = P.solve_group(Qs, bs, seeds=seeds, sigma=sigma, perturb="diag", qx_dtype=qdt, gemv_sym=1,
                                   poll_sweeps=poll)
    for i in range(len(Qs)):
        one = P.solve(Qs[i], bs[i], sigma=sigma, perturb="diag", seed=seeds[i], qx_dtype=qdt, gemv_sym=1)
        assert int(one.obj[0]) == int(obj[i]), i
        assert np.array_equal(one.xhat.cpu().numpy(), xh[i].cpu().numpy()), i
        for key in ("inner_iters", "aux_matvecs", "outer_iters", "exit_reason"):
            assert one.stats[0][key] == stats[i][key], (i, key)


def test_group_tiles_against_oracle_small_set(P):
    """Group solves of the n <= 20 brute-force set and the dense n = 64
    instance with the tile product (FP64 and BF16 storage): objectives and
    rounded points equal the oracle's."""
    cases = gen.bruteforce_set()[::2] + [(0,) + gen.small_dense(0)]
    mism = []
    for qdt in ("f64", "bf16"):
        xh, obj, _ = P.solve_group([_t(Q) for _, Q, _ in cases], [_t(b) for _, _, b in cases], qx_dtype=qdt,
                                   gemv_sym=1)
        for i, (seed, Q, b) in enumerate(cases):
            ref = O.solve(Q, b)
            if int(obj[i]) != ref.obj or not np.array_equal(xh[i].cpu().numpy(), ref.xhat):
                mism.append((seed, qdt))
    print(f"group tile-product solves: {2 * len(cases) - len(mism)}/{2 * len(cases)} equal to the oracle", flush=True)
    assert not mism
