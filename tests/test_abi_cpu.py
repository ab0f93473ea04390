"""The C-ABI library loads and exports what include/psdp.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psdp.h")


def _declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:psdp_status|void|const char \*|int32_t)\s*(psdp_\w+)\(", txt, re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 12
    for nm in names:
        assert hasattr(lib, nm), nm


def test_binding_signatures_cover_header():
    from paper_2408_04875_amd import binding
    assert sorted(binding.SIGNATURES) == _declared()


def test_params_defaults_and_struct_size(lib):
    from paper_2408_04875_amd import binding
    p = binding.default_params()
    assert p.struct_size == ctypes.sizeof(binding.Params)
    assert (p.max_inner, p.max_outer, p.tol_kkt) == (10000, 1000, 1e-5)   # Section 5
    assert p.eta == 0.999 and p.stall_outer == 2
    assert p.poll_sweeps == 64 and p.sparse == -1 and p.graph == 1
    assert p.eig_tol == 1e-7 and p.eig_maxit == 500
    assert p.lambda_reuse == 1
    assert p.gemv_sym == -1 and p.slots == 0
    q = binding.default_params(inner="ppa", qx_dtype="f32", perturb="diag", sigma=0.5)
    assert (q.inner, q.qx_dtype, q.perturb, q.sigma) == (1, 1, 2, 0.5)
    with pytest.raises(TypeError):
        binding.default_params(bogus=1)


def test_status_strings(lib):
    for code in range(0, -9, -1):
        s = lib.psdp_status_string(code).decode()
        assert s and s != "unknown status"
    assert lib.psdp_status_string(-99).decode() == "unknown status"
    assert lib.psdp_version() == 10000


def test_invalid_arguments_fail_before_device_work(lib):
    from paper_2408_04875_amd import binding
    p = binding.default_params()
    st = lib.psdp_solve_i32(None, None, 4, None, None, 1, ctypes.byref(p), None, None, None, None, None, None)
    assert st == -1
    assert "null" in lib.psdp_last_error().decode()
    bad = binding.default_params(eta=1.5)
    dummy = ctypes.c_void_p(16)
    st = lib.psdp_solve_i32(dummy, dummy, 4, None, None, 1, ctypes.byref(bad), dummy, dummy, None, None,
                            None, None)
    assert st == -1 and "eta" in lib.psdp_last_error().decode()
    wrong = binding.default_params()
    wrong.struct_size = 8
    st = lib.psdp_solve_i32(dummy, dummy, 4, None, None, 1, ctypes.byref(wrong), dummy, dummy, None, None,
                            None, None)
    assert st == -1 and "struct_size" in lib.psdp_last_error().decode()
    for kw, code, word in ((dict(sparse=2), -1, "sparse"), (dict(sparse=1, qx_dtype="f64"), -7, "I8"),
                           (dict(lanes=5), -1, "lanes"), (dict(lanes=-1), -1, "lanes")):
        sp = binding.default_params(**kw)
        st = lib.psdp_solve_i32(dummy, dummy, 4, None, None, 1, ctypes.byref(sp), dummy, dummy, None, None,
                                None, None)
        assert st == code and word in lib.psdp_last_error().decode()
    st = lib.psdp_eval_penalty_grad(7, 0, dummy, 4, dummy, dummy, dummy, 4, 1, dummy, None, None)
    assert st == -1
    st = lib.psdp_penalty_adjoint(2, 0, dummy, dummy, dummy, 4, 1, None, None, None, None, None)
    assert st == -7
    st = lib.psdp_perturbation(0, 1.0, 0, 1, dummy, None)
    assert st == -1


def test_product_path_has_no_oracle_or_fallback():
    pkg = os.path.join(ROOT, "paper_2408_04875_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "workloads" not in txt, f


@pytest.mark.parametrize("B", [1, 7, 256])
def test_list_indexed_buffers_hold_the_zero_column(lib, B):
    """Every buffer that the product kernels read through a live-column list
    (the lists, the digit planes, the sparse operand words) holds the extra
    all-zero column that an empty list slot names (index zero_col = ncol).
    The solve allocates from this plan and refuses to run when the check
    fails; here the plan is taken for B starts with every operand type, with
    and without the sparse copy, and with queued starts."""
    from paper_2408_04875_amd import binding
    seen = 0
    for qdt in ("i8", "f32", "f64", "bf16"):
        for sparse in (False, True):
            for slots in sorted({0, 1, 3, max(1, B // 2), B, 2 * B}):
                if qdt == "bf16" and B > 1:
                    continue
                for n in (1, 63, 64, 2500):
                    pl = binding.plan_columns(n, B, sparse_copy=sparse, qx_dtype=qdt, slots=slots)
                    batched = B > 1 or qdt == "i8"
                    ncol = slots if (batched and 0 < slots < B) else B
                    assert pl["ncol"] == ncol
                    assert pl["zero_col"] == ncol
                    need = pl["zero_col"] + 1
                    assert pl["list_len"] >= need
                    if qdt == "i8":
                        assert pl["digit_cols"] >= need
                        assert pl["ld"] % 64 == 0 and pl["ld"] >= n
                        assert pl["word_cols"] >= need if sparse else pl["word_cols"] == 0
                    else:
                        assert pl["digit_cols"] == 0 and pl["word_cols"] == 0
                        assert pl["ld"] % 32 == 0 and pl["ld"] >= n
                    assert pl["ok"] == 1
                    seen += 1
    assert seen > 0
    with pytest.raises(binding.PSDPError, match="invalid"):
        binding.plan_columns(0, B)
    with pytest.raises(binding.PSDPError, match="slots"):
        binding.plan_columns(10, B, slots=-1)
