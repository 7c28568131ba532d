"""GPU parity over seeded random problems and plan options: every case is
integer-valued (all partial sums exact in FP32, all values exact in the 16-bit
types), so the HIP result must equal the FP64 oracle bit for bit whatever the
path, variant, window height, row order, segment length or leading dimension.
The cases cover ragged shapes (N from 1 to 300, empty and duplicate-heavy
rows, tiny and empty matrices) that the fixed cases do not."""
import numpy as np
import pytest

from gpu_util import device_B, device_C, exact
from paper_2606_22482_amd import api, synth

pytestmark = pytest.mark.gpu

KINDS = [("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"), ("f16", "f16")]
MODES = ["plain", "mixed", "mixed", "mfma_only", "auto"]
ORDERS = ["original_ranges", "compacted", "length_sorted", "clustered"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def draw(seed):
    r = np.random.default_rng(1000 + seed)
    vk, bk = KINDS[r.integers(len(KINDS))]
    m = int(r.choice([0, 1, 17, int(r.integers(2, 2500))]))
    k = int(r.choice([1, 31, int(r.integers(2, 2500))]))
    n = int(r.choice([1, 7, 8, 32, 33, 64, 100, 128, 129, 256, int(r.integers(1, 301))]))
    mode = MODES[r.integers(len(MODES))]
    order = ORDERS[r.integers(len(ORDERS))]
    opts = dict(mode=mode, row_order=order, window_h=int(r.choice([16, 32, 64])),
                t_row=int(r.integers(0, 9)), alpha=float(r.choice([0.0, 0.0, 0.02, 0.1, 0.5])),
                alpha_c=float(r.choice([0.0, 1 / 16, 1 / 8])),
                seg_len=int(r.choice([3, 7, 64, 256])), pipeline=int(r.integers(0, 4)),
                win_sched=int(r.integers(0, 2)), exec=int(r.choice([1, 2, 2, 3])))
    if r.random() < 0.25:
        opts["n_panel"] = int(r.choice([8, 32, 48, 64, 96]))
    if order != "original_ranges" and r.random() < 0.3:
        opts["local_reorder"] = int(r.choice([16, 64, 200]))
    density = float(r.choice([0.002, 0.01, 0.04, 0.1]))
    pads = (int(r.choice([0, 3])), int(r.choice([0, 5])))
    return vk, bk, m, k, n, density, opts, pads


@pytest.mark.parametrize("seed", range(120))
def test_random_case_exact(seed):
    import torch
    vk, bk, m, k, n, density, opts, (pad_b, pad_c) = draw(seed)
    print("case", seed, vk, bk, m, k, n, density, opts, pad_b, pad_c, flush=True)
    A = synth.random_csr(m, k, density, 50 + seed, val_kind=vk, int_values=(-2, 2),
                         dup_frac=0.03, empty_rows=0.05)
    B = synth.int_dense(70 + seed, (k, n), -8, 8, kind=bk)
    p = api.Plan(A, n, bk, api.default_opts(**opts))
    Bd = device_B(B, bk, pad_cols=pad_b)
    C = device_C(A.m, n, pad_cols=pad_c)
    p.run(Bd, C)
    torch.cuda.synchronize()
    exact(C, A, B, bk)


@pytest.mark.parametrize("seed", range(20))
def test_random_batch_exact(seed):
    """A submission of 2-7 random problems (each with its own options and
    types): every batched result equals its solo run bit for bit and the
    oracle exactly."""
    import torch
    r = np.random.default_rng(5000 + seed)
    count = int(r.integers(2, 8))
    items, solos, cases = [], [], []
    for j in range(count):
        case = 200 + 10 * seed + j
        vk, bk, m, k, n, density, opts, _ = draw(case)
        A = synth.random_csr(m, k, density, 50 + case, val_kind=vk, int_values=(-2, 2),
                             dup_frac=0.03, empty_rows=0.05)
        B = synth.int_dense(70 + case, (k, n), -8, 8, kind=bk)
        p = api.Plan(A, n, bk, api.default_opts(**opts))
        Bd = device_B(B, bk)
        Cs = device_C(A.m, n)
        p.run(Bd, Cs)
        Cb = device_C(A.m, n)
        items.append(api.WorkItem(p, Bd, Cb))
        solos.append(Cs)
        cases.append((A, B, bk, p))
    print("batch", seed, count, flush=True)
    torch.cuda.synchronize()
    t = api.spmm_submit(items)
    api.spmm_wait(t)
    torch.cuda.synchronize()
    for it, Cs, (A, B, bk, _) in zip(items, solos, cases):
        assert torch.equal(it.C, Cs)
        exact(it.C, A, B, bk)
