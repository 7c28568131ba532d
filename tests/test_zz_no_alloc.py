"""GPU tier for spmm_run_noalloc (the run for callers that cannot allocate,
working from the library's fixed device scratch array): through the C ABI
its C equals spmm_run's bit for bit, and the FP64 oracle exactly on
integer-valued inputs, on two calls in a row, the second with a smaller
problem; a run whose workspace exceeds the array is refused with BUDGET
before anything is launched."""
import numpy as np
import pytest

from gpu_util import device_B, device_C, exact
from paper_2606_22482_amd import _lib as L
from paper_2606_22482_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def int_graph(n, seed, wmax):
    A = synth.chung_lu_graph(n, 2.1, 16.0, wmax, seed)
    A.vals = np.random.default_rng(seed).integers(-2, 3, A.nnz).astype(np.float32)
    return A


def check(A, B, bk, opts):
    import torch
    n = B.shape[1]
    p = api.Plan(A, n, bk, api.default_opts(**opts))
    Bd = device_B(B, bk)
    C_run = device_C(A.m, n)
    p.run(Bd, C_run)
    C_na = device_C(A.m, n)
    p.run_noalloc(Bd, C_na)
    torch.cuda.synchronize()
    assert torch.equal(C_na, C_run)
    exact(C_na, A, B, bk)
    return p


@pytest.mark.parametrize("exec_form", [L.EXEC_TWO_GRIDS, L.EXEC_SERIAL])
def test_noalloc_equals_run_two_calls_second_smaller(exec_form):
    # call 1: a mixed plan with split rows inside windows and partial tiles
    A = int_graph(50000, 21, 4000.0)
    B = synth.int_dense(22, (50000, 128), -8, 8, kind="f32")
    print("call 1", exec_form, A.m, A.nnz, flush=True)
    p1 = check(A, B, "f32", dict(mode="mixed", row_order="length_sorted", t_row=8, seg_len=32,
                                 exec=exec_form))
    st = p1.stats()
    assert st["segments"] > 0 and st["tiles"] > 0
    # call 2: a smaller plain plan with hub rows split into segments
    A = int_graph(8000, 23, 1500.0)
    B = synth.int_dense(24, (8000, 64), -8, 8, kind="f32")
    print("call 2", exec_form, A.m, A.nnz, flush=True)
    p2 = check(A, B, "f32", dict(mode="plain", seg_len=16, exec=exec_form))
    assert p2.stats()["segments"] > 0


def test_noalloc_16bit_windows():
    A, _ = synth.block_community(n=8192, band=8, n_cols=8, seed=5, val_kind="bf16")
    A.vals[:] = synth.to_bf16_bits(np.round(np.random.default_rng(5).uniform(-2, 2, A.nnz)))
    B = synth.int_dense(6, (8192, 256), -8, 8, kind="bf16")
    check(A, B, "bf16", dict(mode="mixed", row_order="original_ranges"))


def test_noalloc_refuses_runs_beyond_the_scratch():
    import torch
    # 500k segments of 8 entries x 32 columns: a 64 MB workspace
    A = synth.random_csr(4000, 4000, 0.25, 9, int_values=(-2, 2))
    B = synth.int_dense(10, (4000, 32), -8, 8, kind="f32")
    p = api.Plan(A, 32, "f32", api.default_opts(mode="plain", seg_len=8))
    assert p.stats()["workspace_bytes"] > 32 << 20
    C = device_C(A.m, 32)
    with pytest.raises(L.SpmmError) as ei:
        p.run_noalloc(device_B(B, "f32"), C)
    assert ei.value.status == L.SPMM_ERR_BUDGET
    torch.cuda.synchronize()
    assert torch.isnan(C).all()  # nothing was launched
    # the ordinary run takes it
    p.run(device_B(B, "f32"), C)
    torch.cuda.synchronize()
    exact(C, A, B, "f32")
