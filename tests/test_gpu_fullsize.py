"""GPU parity at the full workload sizes, in the launch configurations that
bench.py times, on sampled rows the FP64 oracle computes one by one: the
longest (segmented) rows, the first and last rows and a seeded random
sample.  Plus maximum-size shapes: N over several column panels and
column indices near a large K."""
import numpy as np
import pytest

from gpu_util import TOL_16, TOL_F32, device_B, device_C, parity
from paper_2606_22482_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_22482_amd import _lib
    _lib.load()


def sample_rows(A, n_random=3000, n_long=64, seed=0):
    lens = np.diff(A.rowptr)
    longest = np.argsort(-lens, kind="stable")[:n_long]
    rnd = np.random.default_rng(seed).choice(A.m, min(n_random, A.m), replace=False)
    return np.unique(np.concatenate([longest, rnd, [0, A.m - 1]]))


def run_sampled(A, B, kind, opts, tol):
    import torch
    p = api.Plan(A, B.shape[1], kind, opts)
    Bd = device_B(B, kind)
    C = device_C(A.m, B.shape[1])
    for _ in range(2):  # the timed configuration runs repeatedly on the same buffers
        p.run(Bd, C)
    torch.cuda.synchronize()
    assert not torch.isnan(C).any()
    rows = sample_rows(A)
    err = parity(C, A, B, kind, tol, rows=rows)
    return p, err


@pytest.mark.parametrize("n,mode", [(128, "plain"), (128, "mixed"), (64, "plain")])
def test_gnn_graph_2p20(n, mode):
    A, B = synth.gnn_graph(n_cols=n)
    kw = dict(mode=mode)
    if mode == "mixed":
        kw.update(row_order="length_sorted", t_row=16)
    p, err = run_sampled(A, B, "f32", api.default_opts(**kw), TOL_F32 if mode == "plain" else TOL_16)
    st = p.stats()
    assert st["segments"] > 0
    print("gnn", n, mode, err, flush=True)


@pytest.mark.parametrize("mode", ["mixed", "plain"])
def test_block_community_262144(mode):
    A, B = synth.block_community()
    kw = dict(mode=mode)
    if mode == "mixed":
        kw.update(row_order="original_ranges")
    p, err = run_sampled(A, B, "bf16", api.default_opts(**kw), TOL_16 if mode == "mixed" else TOL_F32)
    if mode == "mixed":
        assert p.stats()["nnz_tiles"] > 0.9 * A.nnz
    print("block", mode, err, flush=True)


@pytest.mark.parametrize("mode", ["mixed", "plain"])
def test_attention_mask_32768(mode):
    """The attention-mask workload as bench.py times it: 32,768 rows, 124 M
    entries, N = 256 bf16; mixed with 64-row windows whose items take 128
    tiles (no partial item), or plain."""
    import numpy as np
    A = synth.attention_mask(32768, seed=3, val_kind="bf16")
    B = synth.dense_values(np.random.default_rng(11), (A.k, 256), "bf16")
    kw = dict(mode=mode)
    if mode == "mixed":
        kw.update(row_order="original_ranges", window_h=64)
    p, err = run_sampled(A, B, "bf16", api.default_opts(**kw), TOL_16 if mode == "mixed" else TOL_F32)
    if mode == "mixed":
        assert p.stats()["nnz_tiles"] > 0.99 * A.nnz and p.export()["wpart_win"].size == 0
    print("mask", mode, err, flush=True)


def test_batch_512_uneven():
    """All 512 matrices in one submission (as bench.py times it); sampled rows
    of every 16th matrix against the oracle, and one matrix against its solo
    run bit for bit."""
    import torch
    specs = synth.batch_specs(count=512, seed=4)
    items, mats = [], []
    for i, sp in enumerate(specs):
        A, B = synth.batch_matrix(i, sp, seed=4)
        p = api.Plan(A, B.shape[1], "f16", api.default_opts(mode="auto"))
        items.append(api.WorkItem(p, device_B(B, "f16"), device_C(A.m, B.shape[1])))
        mats.append((A, B))
    for _ in range(2):
        api.spmm_wait(api.spmm_submit(items))
    torch.cuda.synchronize()
    for i in range(0, 512, 16):
        A, B = mats[i]
        parity(items[i].C, A, B, "f16", TOL_F32, rows=sample_rows(A, n_random=300, n_long=8))
    solo = device_C(mats[7][0].m, mats[7][1].shape[1])
    items[7].plan.run(items[7].B, solo)
    torch.cuda.synchronize()
    assert torch.equal(solo, items[7].C)


@pytest.mark.parametrize("n,kind", [(1000, "f32"), (520, "bf16"), (1024, "f16")])
def test_many_column_panels(n, kind):
    """N beyond one vector panel (512 f32 / 1024 16-bit columns) and many
    64-column MFMA panels, with mixed windows and split rows."""
    vk = "f16" if kind == "f16" else "f32"
    A0, _ = synth.block_community(n=4096, band=4, n_cols=8, seed=12, val_kind=vk)
    B = synth.dense_values(np.random.default_rng(n), (A0.k, n), kind)
    for mode in ("plain", "mixed"):
        run_sampled(A0, B, kind, api.default_opts(mode=mode, seg_len=24),
                    TOL_F32 if mode == "plain" else TOL_16)


def test_large_k_column_indices():
    """K = 2^26 columns (B holds 2^26 rows, N = 4): column indices near the
    top of the range, long rows split into segments."""
    K = 1 << 26
    rng = np.random.default_rng(3)
    m, per = 2048, 40
    rows = np.repeat(np.arange(m), per)
    cols = np.concatenate([rng.integers(K - 1000, K, m * per // 2), rng.integers(0, K, m * per // 2)])
    rng.shuffle(cols)
    vals = rng.uniform(-1, 1, rows.size).astype(np.float32)
    A = synth.csr_from_coo(m, K, rows, cols, vals, "f32")
    B = rng.standard_normal((K, 4)).astype(np.float32)
    run_sampled(A, B, "f32", api.default_opts(mode="plain", seg_len=16), TOL_F32)
