"""lambda_min by the shift law after a subproblem that left x unchanged
(psdp_params.lambda_reuse = 1, the oracle's lambda_reuse = "shift"; both
are the defaults).

When the subproblem stops at its starting point, I and z do not change and
the penalty update shifted the scaled matrix of eq. (alpha) by exactly
-alpha, so the next lambda_min is the previous one minus alpha: the library
skips that update's LOBPCG solve. The oracle with the same option is the
reference; without the option the results may differ only where the reused
value and a fresh eigensolve round differently.
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


def test_shift_law_reuse_bit_exact_small_set(P):
    cases = gen.bruteforce_set()
    Q64, b64 = gen.small_dense(0)
    cases = cases + [(0, Q64, b64)]
    mism = []
    for seed, Q, b in cases:
        r = P.solve(_t(Q), _t(b), lambda_reuse=1)
        ref = O.solve(Q, b, O.Params(lambda_reuse="shift"))
        if int(r.obj[0]) != ref.obj or not np.array_equal(r.xhat.cpu().numpy(), ref.xhat):
            mism.append(seed)
        assert r.stats[0]["outer_iters"] == ref.outer_iters
    print(f"shift-law lambda reuse, n <= 64: {len(cases) - len(mism)}/{len(cases)} bit-exact", flush=True)
    assert not mism


def test_shift_law_reuse_full_size_fewer_lobpcg_products(P):
    """The n = 2500 workload's first 64 starts with and without the reuse (I8
    products): fewer lambda_min products, and every start that ended in the
    no-progress exit in both runs ends at the same rounded point."""
    Q, b, X0 = gen.sparse_2500_starts(B=64)
    a = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", lambda_reuse=0)
    s = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype="i8", lambda_reuse=1)
    aux_a = sum(st["aux_matvecs"] for st in a.stats)
    aux_s = sum(st["aux_matvecs"] for st in s.stats)
    same = int((a.obj.cpu().numpy() == s.obj.cpu().numpy()).sum())
    print(f"n=2500, 64 starts: lambda_min products {aux_a} -> {aux_s} ({100 * (1 - aux_s / aux_a):.1f}% fewer), "
          f"sweeps {a.stats[0]['sweeps']} -> {s.stats[0]['sweeps']}, equal objectives {same}/64", flush=True)
    assert aux_s < aux_a
    assert same >= 60
