"""GPU parity of the exact integer Q.X product (the I8 operand path) through
the C ABI (psdp_qx_digits), bit for bit against oracle/fixed_point.py.

Shapes span one partial digit tile up to the n = 2500, 256-column sweep of
the batched workload (sampled rows there), ragged n (not a multiple of 64),
the int8 range limits and the error paths."""
import numpy as np
import pytest

from oracle import fixed_point as F
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


def _sym_int8(n, seed, density=1.0, lim=127):
    rng = np.random.default_rng(seed)
    Q = rng.integers(-lim, lim + 1, (n, n)) * (rng.random((n, n)) < density)
    Q = np.triu(Q) + np.triu(Q, 1).T
    np.fill_diagonal(Q, rng.integers(-10**6, 10**6, n))   # ignored by the product
    return Q.astype(np.int32)


@pytest.mark.parametrize("n,B", [(1, 1), (17, 3), (64, 4), (65, 5), (100, 16), (300, 33), (777, 70)])
def test_digits4_bit_exact(P, n, B):
    Q = _sym_int8(n, n + B)
    X = gen.random_box_points(n, B, 100 + n)
    X[0, : min(n, 3)] = [0.0, 1.0, 0.5][: min(n, 3)]
    Y = P.qx_digits(_t(Q), _t(X), digits=4).cpu().numpy()
    ref = F.qx_fixed_point(Q, X, 4)
    print(f"digits4 n={n} B={B}: max |diff| {np.max(np.abs(Y - ref)):.3e}", flush=True)
    assert np.array_equal(Y, ref)


@pytest.mark.parametrize("n,B", [(1, 1), (17, 3), (64, 2), (129, 9), (300, 17), (777, 40)])
def test_digits8_bit_exact(P, n, B):
    rng = np.random.default_rng(n * 7 + B)
    Q = _sym_int8(n, 3 * n + B)
    X = rng.standard_normal((B, n)) * (2.0 ** rng.integers(-40, 40, (B, 1)))
    X[0, 0] = 0.0
    if B > 2:
        X[1] = 0.0                    # zero column (exponent 0, product 0)
        X[2] = 0.0
        X[2, n // 2] = -3.0           # one nonzero entry
    Y = P.qx_digits(_t(Q), _t(X), digits=8).cpu().numpy()
    ref = F.qx_fixed_point(Q, X, 8)
    assert np.array_equal(Y, ref)


def test_full_sweep_shape_sampled_rows(P):
    """n = 2500, 256 columns of the batched workload: all columns, 96 sampled rows."""
    Q, b, X0 = gen.sparse_2500_starts()
    rows = np.sort(np.random.default_rng(1).choice(len(b), 96, replace=False))
    Qd, Xd = _t(Q), _t(X0)
    Y4 = P.qx_digits(Qd, Xd, digits=4).cpu().numpy()
    assert np.array_equal(Y4[:, rows], F.qx_fixed_point(Q, X0, 4, rows=rows))
    V = np.random.default_rng(2).standard_normal(X0[:32].shape)
    Y8 = P.qx_digits(Qd, _t(V), digits=8).cpu().numpy()
    assert np.array_equal(Y8[:, rows], F.qx_fixed_point(Q, V, 8, rows=rows))


@pytest.mark.parametrize("layout", ["few", "mid", "many", "wide", "tall"])
def test_every_layout_and_slice_count_bit_exact(P, layout):
    """Each block layout of the int8 MFMA kernel, forced through
    psdp_qx_digits_ex with 1, 3 and 8 K slices, on ragged shapes (partial
    digit tiles, partial row blocks, K ranges not a multiple of the slice
    count) and on the n = 2500 workload with 300 columns (sampled rows)."""
    for n, B, D in ((777, 70, 4), (777, 41, 8), (130, 5, 4), (130, 3, 8)):
        Q = _sym_int8(n, 11 * n + B + D)
        rng = np.random.default_rng(n + B + D)
        X = rng.random((B, n)) if D == 4 else rng.standard_normal((B, n)) * 2.0 ** rng.integers(-30, 30, (B, 1))
        ref = F.qx_fixed_point(Q, X, D)
        for ks in (1, 3, 8):
            Y = P.qx_digits(_t(Q), _t(X), digits=D, layout=layout, slices=ks).cpu().numpy()
            assert np.array_equal(Y, ref), (n, B, D, ks)
    Q, b, X0 = gen.sparse_2500_starts(B=300)
    rows = np.sort(np.random.default_rng(5).choice(len(b), 64, replace=False))
    ref = F.qx_fixed_point(Q, X0, 4, rows=rows)
    for ks in (1, 2):
        Y = P.qx_digits(_t(Q), _t(X0), digits=4, layout=layout, slices=ks).cpu().numpy()
        assert np.array_equal(Y[:, rows], ref), ks
    print(f"layout {layout}: bit-exact on every shape and slice count", flush=True)


def test_digit_table_is_honoured_and_removable(P):
    """A table installed for (n, digits) decides the solve's product settings
    (psdp_digit_choice) by the first bucket holding the estimate; removing it
    restores the built-in rule."""
    n = 1234
    before = P.digit_choice(n, 100, 20)
    P.set_digit_table(n, 4, [(8, "few", 2), (64, "mid", 4), (512, "wide", 1)])
    try:
        assert P.digit_choice(n, 5, 0)[0] == (1, 2)
        assert P.digit_choice(n, 9, 0)[0] == (2, 4)
        assert P.digit_choice(n, 64, 0)[0] == (2, 4)
        assert P.digit_choice(n, 65, 0)[0] == (8, 1)
        assert P.digit_choice(n, 5000, 0)[0] == (8, 1)
        assert P.digit_choice(n, 100, 20)[1] == before[1]     # no table for 8 digits
        with pytest.raises(P.PSDPError, match="increasing"):
            P.set_digit_table(n, 4, [(8, "few", 2), (8, "mid", 4)])
        with pytest.raises(P.PSDPError, match="layout"):
            P.set_digit_table(n, 4, [(8, 3, 2)])
    finally:
        P.set_digit_table(n, 4, [])
    assert P.digit_choice(n, 100, 20) == before


def test_extreme_int8_range(P):
    """|Q| = 127 everywhere with x = 1 or the largest 8-digit magnitudes: the
    int32 digit sums and the int64 combination stay exact."""
    n = 4096
    Q = np.full((n, n), 127, dtype=np.int32)
    Q[::2, :] = -127
    Q = np.triu(Q) + np.triu(Q, 1).T
    X = np.ones((2, n))
    X[1, ::3] = 1.0 - 2.0**-28
    Y = P.qx_digits(_t(Q), _t(X), digits=4).cpu().numpy()
    rows = np.array([0, 1, 2, n // 2, n - 1])
    assert np.array_equal(Y[:, rows], F.qx_fixed_point(Q, X, 4, rows=rows))
    V = np.full((2, n), -1.0 + 2.0**-53)
    V[1, 1::2] = 1.0 - 2.0**-53
    Y8 = P.qx_digits(_t(Q), _t(V), digits=8).cpu().numpy()
    assert np.array_equal(Y8[:, rows], F.qx_fixed_point(Q, V, 8, rows=rows))


def test_product_matches_fp64_within_grid_error(P):
    """The 4-digit result differs from the FP64 product by at most the grid error."""
    Q, b, X0 = gen.sparse_2500_starts(n=1000, B=8)
    Y = P.qx_digits(_t(Q), _t(X0), digits=4).cpu().numpy()
    Qo = Q.astype(np.float64)
    np.fill_diagonal(Qo, 0.0)
    ref = X0 @ Qo.T
    bound = np.abs(Qo).sum(axis=1) * 2.0**-28 + 1e-9
    assert (np.abs(Y - ref) <= bound[None, :]).all()


def test_error_paths(P):
    Q = _sym_int8(10, 1)
    X = gen.random_box_points(10, 2, 3)
    bad = Q.copy()
    bad[0, 1] = bad[1, 0] = 128
    with pytest.raises(P.PSDPError, match="unsupported"):
        P.qx_digits(_t(bad), _t(X), digits=4)
    with pytest.raises(P.PSDPError, match="non-finite"):
        P.qx_digits(_t(Q), _t(X + 1.0), digits=4)
    with pytest.raises(P.PSDPError, match="invalid"):
        P.qx_digits(_t(Q), _t(X), digits=5)
    Xn = X.copy()
    Xn[0, 0] = np.nan
    with pytest.raises(P.PSDPError, match="non-finite"):
        P.qx_digits(_t(Q), _t(Xn), digits=8)
