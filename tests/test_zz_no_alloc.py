"""psdp_eval_penalty_grad_noalloc (the evaluation with a fixed device
workspace, for callers that cannot allocate) against psdp_eval_penalty_grad,
through the C ABI, on two calls in a row, the second with a smaller input."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    from paper_2408_04875_amd import binding
    assert torch.cuda.is_available()
    return binding.load()


def _call(lib, name, Q, b, p, X, dt, vt):
    import torch
    from paper_2408_04875_amd import binding
    n = b.shape[0]
    B = X.shape[0]
    h = torch.full((B,), float("nan"), dtype=b.dtype, device="cuda")
    G = torch.full((B, n), float("nan"), dtype=b.dtype, device="cuda")
    st = getattr(lib, name)(dt, vt, Q.data_ptr(), Q.stride(0), b.data_ptr(), p.data_ptr(), X.data_ptr(), n, B,
                            h.data_ptr(), G.data_ptr(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, lib.psdp_last_error().decode()
    torch.cuda.synchronize()
    return h.cpu().numpy(), G.cpu().numpy()


@pytest.mark.parametrize("qdt,vdt", [("f64", "f64"), ("f32", "f32"), ("bf16", "f64")])
def test_noalloc_eval_equals_allocating_eval_twice(lib, qdt, vdt):
    import torch
    from paper_2408_04875_amd import binding
    tq = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[qdt]
    tv = {"f64": torch.float64, "f32": torch.float32}[vdt]
    code = {"f64": binding.F64, "f32": binding.F32, "bf16": binding.BF16}
    # the first call fills the workspace with a larger problem (MFMA path for
    # aligned F32/F64 shapes), the second is smaller and ragged (FMA path)
    for n, B, seed in ((1024, 96, 1), (333, 7, 2)):
        rng = np.random.default_rng(seed)
        A = rng.standard_normal((n, n))
        Q = torch.from_numpy((A + A.T) / 2).to(tq).cuda()
        b = torch.from_numpy(rng.standard_normal(n)).to(tv).cuda()
        p = torch.from_numpy(rng.uniform(0, 2, n)).to(tv).cuda()
        X = torch.from_numpy(rng.random((B, n))).to(tq).cuda()
        h0, G0 = _call(lib, "psdp_eval_penalty_grad", Q, b, p, X, code[qdt], code[vdt])
        h1, G1 = _call(lib, "psdp_eval_penalty_grad_noalloc", Q, b, p, X, code[qdt], code[vdt])
        assert np.array_equal(h0, h1) and np.array_equal(G0, G1), (n, B)


def test_noalloc_eval_rejects_oversize(lib):
    import torch
    from paper_2408_04875_amd import binding
    n, B = 4096, 1100   # 8 n B > 32 MiB
    z = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = lib.psdp_eval_penalty_grad_noalloc(binding.F64, binding.F64, z.data_ptr(), n, z.data_ptr(), z.data_ptr(),
                                            z.data_ptr(), n, B, z.data_ptr(), None, None)
    assert st == -7  # PSDP_E_UNSUPPORTED
    assert "32 MiB" in lib.psdp_last_error().decode()
