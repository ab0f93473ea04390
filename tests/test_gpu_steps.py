"""Step-level parity at full size: the first penalty update and K subproblem
iterations of Algorithm 2 on the GPU against the oracle, element by element,
for every per-column kernel instantiation (one, two, four and six elements
per thread with the iterate kept in registers, and four per thread over
several chunks), plus the batched path's floating-point products against
their FP64 definition.

The penalty step alpha of the update (eqs. (alpha), (alpha1)) is computed
here by the oracle (dense eigensolver at the start point, p = 0) and handed
to the GPU through the replay hook, so both sides run the subproblem at the
same penalty p = alpha z (eq. (pp1)) from the same start; the GPU's own
lambda_min (LOBPCG) is compared with the oracle's value. With the integer
products the oracle applies the same 2^-27 operand grid, and both sides
take the BB inner products and rho as exact values rounded once, so the
iterates must be identical; with FP64 products (another summation order)
they must agree to 1e-9.
"""
import numpy as np
import pytest

from oracle import fixed_point as FP
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


_CASES = {}


def _case(n, B):
    """Instance, starts and the oracle's first penalty update of each start."""
    key = (n, B)
    if key not in _CASES:
        from threadpoolctl import threadpool_limits
        Q, b = gen.sparse_int(n, 40 + n % 97)
        X0 = gen.random_box_points(n, B, 7 + n)
        prm = O.Params()
        gam = O.reformation_gamma(Q, b)
        Q_r, b_r = Q + np.diag(gam), b - gam
        norms = O._RowNorms(Q_r)
        ups = []
        for c in range(B):
            with threadpool_limits(16):
                lam, I, z = O.lambda_min_scaled(Q_r, np.zeros(n), X0[c])
            rho0 = norms.rho(b_r, np.zeros(n))
            alpha = prm.eta * max(lam, prm.lambda_floor_rel * rho0)
            p = np.zeros(n)
            p[I] += alpha * z
            ups.append((lam, alpha, p, norms.rho(b_r, p)))
        _CASES[key] = (Q, b, X0, Q_r, b_r, ups)
    return _CASES[key]


# n -> (starts, per-thread elements of the column kernel at that size)
_SIZES = [(300, 4, "1 per thread"), (1000, 4, "2 per thread"), (1500, 3, "4 per thread, registers/LDS"),
          (2500, 4, "6 per thread, registers/LDS"), (4000, 2, "4 per thread, several chunks")]


@pytest.mark.parametrize("n,B,layout", _SIZES, ids=[f"n{n}" for n, _, _ in _SIZES])
@pytest.mark.parametrize("qdt", ["i8", "f64"])
def test_first_update_and_k_subproblem_steps_elementwise(P, n, B, layout, qdt):
    Q, b, X0, Q_r, b_r, ups = _case(n, B)
    A = np.array([[u[1]] for u in ups])
    mode = "i8" if qdt == "i8" else "fp64"
    gp = FP.GridProduct(Q_r) if qdt == "i8" else None
    for K in (1, 5, 20):
        r = P.solve(_t(Q), _t(b), X0=_t(X0), qx_dtype=qdt, alpha=A, max_outer=1, max_inner=K, trace_cap=2)
        X = r.X.cpu().numpy()
        worst = 0.0
        for c in range(B):
            lam, alpha, p, rho = ups[c]
            ref, it, rel, _ = O.solve_subproblem_pabb(Q_r, b_r, p, X0[c], O.Params(max_inner=K, product=mode),
                                                      rho=rho, grid_product=gp)
            d = float(np.abs(X[c] - ref).max())
            worst = max(worst, d)
            assert r.trace[c, 0, 4] == it, (K, c)                      # subproblem length
            assert r.trace[c, 0, 3] == alpha                           # the replayed step
            assert abs(r.trace[c, 0, 2] - lam) <= 5e-5 * abs(lam)      # LOBPCG vs dense lambda_min
            if qdt == "i8":
                assert np.array_equal(X[c], ref), (K, c, d)
            else:
                assert d <= 1e-9, (K, c, d)
        print(f"n={n} ({layout}) {qdt} K={K}: max |x_gpu - x_oracle| = {worst:.2e} over {B} starts", flush=True)


@pytest.mark.parametrize("B", [8, 16, 32, 64, 256])
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_float_products_elementwise_n2500(P, B, dtype):
    """psdp_qx_dense runs the product kernel the solver picks for B live
    columns (streaming MFMA kernel with 1, 2 or 4 column tiles up to 64
    columns, LDS-tiled MFMA GEMM above) and sums its K slices as the column
    kernel does. Against the FP64 definition Q_off X: FP64 within the
    accumulation bound 2 n u sum_j |Q_ij x_j| (u = 2^-53); FP32 within
    (n + 2) 2^-24 sum_j |Q_ij| |x_j| (the rounding of x to float and the
    FP32 accumulation)."""
    n = 2500
    Q, _, X = gen.sparse_2500_starts(n=n, B=B, seed_x=11)
    Qo = Q.astype(np.float64)
    np.fill_diagonal(Qo, 0.0)
    Y = P.qx_dense(_t(Q), _t(X), dtype=dtype).cpu().numpy()
    ref = X @ Qo.T
    scale = np.abs(X) @ np.abs(Qo).T
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    bound = (2 * n * u if dtype == "f64" else (n + 2) * u) * scale
    ratio = float((np.abs(Y - ref) / np.maximum(bound, 1e-300)).max())
    print(f"n={n} B={B} {dtype}: max error / bound = {ratio:.2e}, max error {np.abs(Y - ref).max():.2e}", flush=True)
    assert (np.abs(Y - ref) <= bound).all()
