"""GPU parity of the single-step kernels against the FP64 oracle.

Penalty value and gradient (eq. (p1), eq. (kkt1)), the adjoint, the
perturbation generator (bit-exact) and the exact rounding/objective step
(bit-exact), at sizes that span several tiles plus a ragged tail and at the
n = 4096, B = 64 differentiation workload.
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


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t.to(dtype) if dtype is not None else t


def _scales(Q, b, p, X):
    """Absolute-value scales of h and grad h (normwise error denominators)."""
    aQ = np.abs(Q)
    sh = np.array([np.abs(x) @ aQ @ np.abs(x) + np.abs(b) @ np.abs(x) + np.abs(p) @ np.abs(x - x * x) for x in X])
    sG = np.stack([2 * aQ @ np.abs(x) + np.abs(b) + np.abs(p) * (1 + 2 * np.abs(x)) for x in X])
    return sh, sG


@pytest.mark.parametrize("n,B", [(40, 3), (200, 5), (1000, 7), (256, 64), (1000, 130)])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_eval_penalty_grad_matches_oracle(P, n, B, prec):
    import torch
    rng = np.random.default_rng(n + B)
    Q = rng.standard_normal((n, n)); Q = (Q + Q.T) / 2
    b = rng.standard_normal(n); p = rng.uniform(0, 2, n); X = rng.random((B, n))
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[prec]
    vdt = torch.float64 if prec == "f64" else torch.float32
    print(f"eval n={n} B={B} {prec}", flush=True)
    h, G = P.eval_penalty_grad(_t(Q, tdt), _t(b, vdt), _t(p, vdt), _t(X, tdt))
    torch.cuda.synchronize()
    hr, Gr = O.penalty_batch(Q, b.astype(np.float64), p, X)
    sh, sG = _scales(Q, b, p, X)
    eh = np.max(np.abs(h.double().cpu().numpy() - hr) / sh)
    eG = np.max(np.abs(G.double().cpu().numpy() - Gr)) / np.max(sG)
    tol = {"f64": 1e-13, "f32": 1e-5, "bf16": 5e-3}[prec]
    assert eh < tol and eG < tol, (eh, eG)


@pytest.mark.parametrize("n,B", [(100, 4), (512, 16), (1000, 33)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_adjoint_matches_oracle(P, n, B, prec):
    import torch
    rng = np.random.default_rng(7 * n + B)
    Q = rng.standard_normal((n, n)); Q = (Q + Q.T) / 2
    b = rng.standard_normal(n); p = rng.uniform(0, 2, n)
    X = rng.uniform(1e-3, 1 - 1e-3, (B, n)); w = rng.standard_normal(B)
    tdt = torch.float64 if prec == "f64" else torch.float32
    print(f"adjoint n={n} B={B} {prec}", flush=True)
    Xt = _t(X, tdt)
    h, G = P.eval_penalty_grad(_t(Q, tdt), _t(b, tdt), _t(p, tdt), Xt)
    dX, dQ, db, dp = P.penalty_adjoint(Xt, G, _t(w, tdt))
    torch.cuda.synchronize()
    rX, rQ, rb, rp = O.penalty_adjoint(Q, b, p, X, w)
    tol = 1e-12 if prec == "f64" else 2e-5
    aw = np.abs(w)
    sQ = (np.abs(X).T * aw) @ np.abs(X)
    assert np.max(np.abs(dQ.double().cpu().numpy() - rQ) / np.maximum(sQ, 1e-300)) < tol
    assert np.max(np.abs(db.double().cpu().numpy() - rb)) / np.max(aw @ np.abs(X)) < tol
    assert np.max(np.abs(dp.double().cpu().numpy() - rp)) / np.max(aw @ np.abs(X - X * X)) < tol
    _, sG = _scales(Q, b, p, X)
    assert np.max(np.abs(dX.double().cpu().numpy() - rX)) / np.max(aw[:, None] * sG) < tol


def test_penalty_fn_autograd_fd_differentiation_workload(P):
    """n = 4096, B = 64 FP32: PenaltyFn gradients vs the FP64 oracle and FD."""
    import torch
    Q, b, X, p, w = gen.dense_normal_batch(5)
    n, B = len(b), len(X)
    print(f"autograd n={n} B={B}", flush=True)
    Xt = _t(X).requires_grad_(True); Qt = _t(Q).requires_grad_(True)
    bt = _t(b).requires_grad_(True); pt = _t(p).requires_grad_(True)
    h = P.penalty_fn().apply(Xt, Qt, bt, pt)
    (h * _t(w)).sum().backward()
    torch.cuda.synchronize()
    Q64, b64, X64, p64, w64 = (a.astype(np.float64) for a in (Q, b, X, p, w))
    # oracle on sampled entries (the full oracle adjoint is O(B n^2))
    rng = np.random.default_rng(0)
    cols = rng.choice(B, 4, replace=False)
    for c in cols:
        g = O.penalty_grad(Q64, b64, p64, X64[c])
        got = Xt.grad[c].double().cpu().numpy()
        assert np.max(np.abs(got - w64[c] * g)) / np.max(np.abs(w64[c]) * (2 * np.abs(Q64) @ X64[c] + 3)) < 1e-5
    ii = rng.choice(n, 16); jj = rng.choice(n, 16)
    dQ = Qt.grad.double().cpu().numpy()
    ref = np.array([np.sum(w64 * X64[:, i] * X64[:, j]) for i, j in zip(ii, jj)])
    sc = np.array([np.sum(np.abs(w64) * X64[:, i] * X64[:, j]) for i, j in zip(ii, jj)])
    assert np.max(np.abs(dQ[ii, jj] - ref) / sc) < 1e-5
    assert np.max(np.abs(bt.grad.double().cpu().numpy() - w64 @ X64)) / np.max(np.abs(w64) @ X64) < 1e-5
    assert np.max(np.abs(pt.grad.double().cpu().numpy() - w64 @ (X64 - X64 ** 2))) / np.max(
        np.abs(w64) @ (X64 - X64 ** 2)) < 1e-5
    # central differences (h = 1e-3) of L = w^T h along random directions, FP64 evaluation
    Qd, bd, pd, Xd = (_t(a) for a in (Q64, b64, p64, X64))
    wd = _t(w64)

    def L(Q_, b_, p_, X_):
        hh, _ = P.eval_penalty_grad(Q_, b_, p_, X_, want_grad=False)
        return float((hh * wd).sum())

    for k in range(4):
        r = np.random.default_rng(100 + k)
        E = r.standard_normal((n, n)); E = (E + E.T) / 2
        Et = _t(E)
        fd = (L(Qd + 1e-3 * Et, bd, pd, Xd) - L(Qd - 1e-3 * Et, bd, pd, Xd)) / 2e-3
        an = float((Qt.grad.double() * Et).sum())
        assert abs(fd - an) <= 1e-5 * (abs(fd) + np.sum(np.abs(E) * np.abs(dQ)))
        D = r.standard_normal((B, n)); Dt = _t(D)
        fd = (L(Qd, bd, pd, Xd + 1e-3 * Dt) - L(Qd, bd, pd, Xd - 1e-3 * Dt)) / 2e-3
        an = float((Xt.grad.double() * Dt).sum())
        assert abs(fd - an) <= 1e-4 * (abs(fd) + float((Xt.grad.double().abs() * Dt.abs()).sum()))


@pytest.mark.parametrize("n,mode,sigma,seed", [(7, "full", 1.0, 0), (33, "full", 0.37, 5), (50, "diag", 2.5, 9),
                                               (64, "full", 1e-3, 2**63 + 7)])
def test_perturbation_bit_exact(P, n, mode, sigma, seed):
    import torch
    print(f"perturbation n={n} {mode}", flush=True)
    mu = P.perturbation(n, sigma, seed, mode)
    torch.cuda.synchronize()
    ref = O.perturbation(n, sigma, seed, mode)
    assert np.array_equal(mu.cpu().numpy(), ref)


@pytest.mark.parametrize("n,B", [(17, 3), (300, 9), (2500, 40)])
def test_round_objective_bit_exact(P, n, B):
    import torch
    Q, b = gen.dense_int(n, n) if n < 100 else gen.sparse_int(n, n)
    b = np.random.default_rng(1).integers(-100, 101, n).astype(np.int32)
    X = np.random.default_rng(2).random((B, n))
    X[0, : n // 2] = 0.5  # exact ties round to 0
    print(f"round_objective n={n} B={B}", flush=True)
    xh, obj = P.round_objective(_t(Q), _t(b), _t(X))
    torch.cuda.synchronize()
    xh = xh.cpu().numpy(); obj = obj.cpu().numpy()
    Q64 = Q.astype(np.int64)
    for c in range(B):
        ref_x = O.round_binary(X[c])
        assert np.array_equal(xh[c], ref_x)
        v = ref_x.astype(np.int64)
        exact = int(v @ Q64 @ v + b.astype(np.int64) @ v)   # exact in int64 at these sizes
        assert obj[c] == exact
    assert obj[0] == O.objective_exact(Q, b, O.round_binary(X[0]))
