"""CPU tier for the Python binding's operand checks: B and C tensors that do
not match a plan (dtype, rows, columns) are refused with ValueError before
any pointer reaches the C ABI, for spmm_run, spmm_run_timed, spmm_submit and
spmm_autotune.  (The ABI sees only pointers and leading dimensions, so such a
tensor would otherwise make the kernels read or write out of bounds.)"""
import numpy as np
import pytest
import torch

from paper_2606_22482_amd import api, synth

M, K, N = 40, 24, 16


@pytest.fixture(scope="module")
def plans():
    A = synth.random_csr(M, K, 0.2, seed=3)
    f32 = api.Plan(A, N, "f32", api.default_opts(mode="plain"), upload=False)
    bf16 = api.Plan(A, N, "bf16", api.default_opts(mode="plain"), upload=False)
    return A, f32, bf16


def _bad_cases(kind):
    dt = {"f32": torch.float32, "bf16": torch.bfloat16}[kind]
    other = torch.float16
    ok_b, ok_c = torch.zeros(K, N, dtype=dt), torch.zeros(M, N)
    return [
        (torch.zeros(K, N, dtype=other), ok_c, "B must be"),
        (torch.zeros(K - 1, N, dtype=dt), ok_c, "B must be at least"),
        (torch.zeros(K, N - 1, dtype=dt), ok_c, "B must be at least"),
        (ok_b, torch.zeros(M, N, dtype=torch.float64), "C must be torch.float32"),
        (ok_b, torch.zeros(M - 1, N), "C must be at least"),
        (ok_b, torch.zeros(M, N - 1), "C must be at least"),
        (torch.zeros(K * N, dtype=dt), ok_c, "B must be at least"),
    ]


@pytest.mark.parametrize("kind", ["f32", "bf16"])
def test_run_refuses_mismatched_operands(plans, kind):
    _, pf, pb = plans
    plan = pf if kind == "f32" else pb
    for B, Cout, msg in _bad_cases(kind):
        with pytest.raises(ValueError, match=msg):
            plan.run(B, Cout)
        with pytest.raises(ValueError, match=msg):
            plan.run_timed(B, Cout, timer=None)
        with pytest.raises(ValueError, match=msg):
            api.spmm_submit([api.WorkItem(plan, B, Cout)])


def test_matching_host_tensors_still_refused_as_not_on_device(plans):
    _, pf, _ = plans
    B, Cout = torch.zeros(K, N), torch.zeros(M, N)
    with pytest.raises(ValueError, match="device tensor"):
        pf.run(B, Cout)
    # a wider B / C (row stride above N) passes the shape checks
    with pytest.raises(ValueError, match="device tensor"):
        pf.run(torch.zeros(K, N + 8)[:, :N], torch.zeros(M + 3, N + 4)[:, :N])


def test_autotune_refuses_mismatched_operands(plans):
    A = plans[0]
    with pytest.raises(ValueError, match="B must be"):
        api.spmm_autotune(A, torch.zeros(K, N, dtype=torch.float16), torch.zeros(M, N), "f32")
    with pytest.raises(ValueError, match="C must be at least"):
        api.spmm_autotune(A, torch.zeros(K, N), torch.zeros(M - 1, N), "f32")


def test_operand_check_is_exact_at_the_boundary():
    # at exactly k x n and m x n the checks pass and only the device check remains
    B = torch.zeros(K, N, dtype=torch.float16)
    with pytest.raises(ValueError, match="device tensor"):
        api._operands(M, K, N, "f16", B, torch.zeros(M, N))
    assert np.dtype(np.float32).itemsize == 4


def test_autotune_context_is_validated(plans):
    """spmm_autotune refuses a tuning context other than run or submit before
    it touches the device."""
    import ctypes as C
    from paper_2606_22482_amd import _lib as L
    A = plans[0]
    lib = L.load()
    csr, keep = api._csr_struct(A)
    o, rep = L.Opts(), L.TuneReport()
    st = lib.spmm_autotune(C.byref(csr), N, L.F32, L.F32, None, N, None, N, None, 10.0, 7,
                           C.byref(o), C.byref(rep))
    assert st == L.SPMM_ERR_INVALID
    assert b"context" in lib.spmm_last_error()
    del keep


def test_gather_probe_argument_checks():
    """spmm_gather_bandwidth refuses bad sizes and pointers with INVALID
    before any device call (the pointers here are never dereferenced)."""
    import ctypes as C
    from paper_2606_22482_amd import _lib as L
    lib = L.load()
    out = C.c_double()
    fake = C.c_void_p(0x100000)  # 16-byte aligned, never touched
    bad = [
        (None, 16, fake, 8, 128, 128, 1),      # no row ids
        (fake, 16, None, 8, 128, 128, 1),      # no B
        (fake, 0, fake, 8, 128, 128, 1),       # empty sequence
        (fake, 16, fake, 0, 128, 128, 1),      # no rows in B
        (fake, 16, fake, 8, 128, 130, 1),      # rows wider than 128 f32
        (fake, 16, fake, 8, 128, 6, 1),        # not a multiple of 4
        (fake, 16, fake, 8, 64, 128, 1),       # ldb below n_cols
        (fake, 16, fake, 8, 130, 128, 1),      # ldb not a multiple of 4
        (fake, 16, fake, 8, 128, 128, 0),      # no repetitions
        (fake, 16, C.c_void_p(0x100004), 8, 128, 128, 1),  # B not 16-byte aligned
        (fake, 16, fake, 1 << 31, 128, 128, 1),  # k beyond int32
    ]
    for rows, n, B, k, ldb, ncols, reps in bad:
        st = lib.spmm_gather_bandwidth(rows, n, B, k, ldb, ncols, reps, None, C.byref(out))
        assert st == L.SPMM_ERR_INVALID, (n, k, ldb, ncols, reps)
    assert lib.spmm_gather_bandwidth(fake, 16, fake, 8, 128, 128, 1, None, None) == L.SPMM_ERR_INVALID
