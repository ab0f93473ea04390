"""Queued starts (psdp_params.slots): fewer columns than starts, a column
taking the next start when its own ends; and lanes (psdp_params.lanes):
the columns run as two to four concurrent launch sequences over shares of
the columns and starts. Every start performs the same
arithmetic as in a launch where it has its own column (the columns are
independent and every reduction has a fixed order), so the results of each
start must be identical bit for bit: final iterate, rounded point,
objective, evaluation and lambda_min product counts, penalty updates, exit
reason and the per-update trace."""
import numpy as np
import pytest

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


def _same(a, b):
    assert np.array_equal(a.X.cpu().numpy(), b.X.cpu().numpy())
    assert np.array_equal(a.xhat.cpu().numpy(), b.xhat.cpu().numpy())
    assert np.array_equal(a.obj.cpu().numpy(), b.obj.cpu().numpy())
    assert a.best == b.best
    for sa, sb in zip(a.stats, b.stats):
        for k in ("inner_iters", "aux_matvecs", "outer_iters", "exit_reason", "final_cret_rel", "final_binary_gap"):
            assert sa[k] == sb[k], k
    if a.trace is not None:
        assert np.array_equal(np.nan_to_num(a.trace, nan=-1.0), np.nan_to_num(b.trace, nan=-1.0))


@pytest.mark.parametrize("qdt,slots", [("i8", 5), ("i8", 16), ("f32", 8), ("f64", 7)])
def test_queued_starts_equal_own_columns(P, qdt, slots):
    Q, b, X0 = gen.sparse_2500_starts(n=300, B=24)
    full = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype=qdt, trace_cap=60)
    q = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype=qdt, trace_cap=60, slots=slots)
    print(f"{qdt} slots {slots}: sweeps {full.stats[0]['sweeps']} -> {q.stats[0]['sweeps']}", flush=True)
    _same(q, full)


def test_queued_starts_with_replayed_steps(P):
    Q, b, X0 = gen.sparse_2500_starts(n=200, B=12)
    A = np.random.default_rng(5).uniform(1.0, 50.0, size=(12, 3))
    full = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", alpha=A, trace_cap=40)
    q = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", alpha=A, trace_cap=40, slots=4)
    _same(q, full)
    assert np.array_equal(q.trace[:, :3, 3], A)


def test_queued_starts_full_size(P):
    """512 starts of the n = 2500 workload through 256 columns against the
    same starts in two launches of 256 (each start's own column)."""
    Q, b, X0 = gen.sparse_2500_starts(B=512)
    halves = [P.solve(_t(Q), _t(b), X0=_t(X0[h * 256:(h + 1) * 256]), qx_dtype="i8") for h in range(2)]
    q = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", slots=256)
    obj = np.concatenate([h.obj.cpu().numpy() for h in halves])
    X = np.concatenate([h.X.cpu().numpy() for h in halves])
    assert np.array_equal(q.obj.cpu().numpy(), obj)
    assert np.array_equal(q.X.cpu().numpy(), X)
    ev = [s["inner_iters"] for h in halves for s in h.stats]
    assert [s["inner_iters"] for s in q.stats] == ev
    sw = [h.stats[0]["sweeps"] for h in halves]
    print(f"512 starts: two launches of 256 take {sw} sweeps ({sum(sw)}), one queued launch of 256 columns "
          f"{q.stats[0]['sweeps']}", flush=True)


@pytest.mark.parametrize("lanes", [2, 3, 4])
@pytest.mark.parametrize("slots", [0, 6, 9])
def test_lanes_equal_one_lane(P, slots, lanes):
    """Two to four lanes (each with its share of the columns and of the
    starts, its own lists, queue and stream) against one, with and without
    queued starts: every start identical bit for bit."""
    Q, b, X0 = gen.sparse_2500_starts(n=300, B=24)
    one = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", trace_cap=60, slots=slots, lanes=1)
    many = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", trace_cap=60, slots=slots, lanes=lanes)
    _same(many, one)


@pytest.mark.parametrize("lanes", [2, 4])
def test_lanes_full_size_queued(P, lanes):
    """512 starts of the n = 2500 workload through 300 columns in two or four
    lanes against the same starts with a column each (two launches of 256)."""
    Q, b, X0 = gen.sparse_2500_starts(B=512)
    halves = [P.solve(_t(Q), _t(b), X0=_t(X0[h * 256:(h + 1) * 256]), qx_dtype="i8") for h in range(2)]
    q = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", slots=300, lanes=lanes)
    obj = np.concatenate([h.obj.cpu().numpy() for h in halves])
    assert np.array_equal(q.obj.cpu().numpy(), obj)
    assert np.array_equal(q.X.cpu().numpy(), np.concatenate([h.X.cpu().numpy() for h in halves]))
    assert [s["inner_iters"] for s in q.stats] == [s["inner_iters"] for h in halves for s in h.stats]
    print(f"512 starts, {lanes} lanes of {300 // lanes} columns: {q.stats[0]['sweeps']} sweeps", flush=True)
