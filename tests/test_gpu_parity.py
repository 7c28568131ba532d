"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Floating point: normalised error <= 1e-5 on the FP32 path, <= 2e-2 where MFMA
operands are 16-bit.  Integer-valued inputs (every partial sum exact in FP32
and every value exact in bf16/f16) must match the oracle bit for bit on every
path.  Edge cases: empty matrix, empty rows, NaN-prefilled C, N in {1, 7, 33}
with padded leading dimensions, long rows split into segments.
"""
import numpy as np
import pytest

from gpu_util import TOL_16, TOL_F32, device_B, device_C, exact, parity
from paper_2606_22482_amd import _lib as L
from paper_2606_22482_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_22482_amd import _lib
    _lib.load()


def run(A, B, b_kind, opts, n=None, pad_b=0, pad_c=0, fill=float("nan")):
    import torch
    n = B.shape[1] if n is None else n
    p = api.Plan(A, n, b_kind, opts)
    Bd = device_B(B, b_kind, pad_cols=pad_b)
    Cd = device_C(A.m, n, fill=fill, pad_cols=pad_c)
    p.run(Bd, Cd)
    torch.cuda.synchronize()
    return p, Cd


MODES = ["plain", "mixed", "mfma_only"]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("kinds", [("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"),
                                   ("f16", "f16")])
@pytest.mark.parametrize("n", [1, 7, 32, 33, 64, 128, 256])
def test_integer_exact_all_paths(mode, kinds, n):
    vk, bk = kinds
    A = synth.random_csr(700, 500, 0.03, 11 + n, val_kind=vk, int_values=(-2, 2),
                         dup_frac=0.03, empty_rows=0.05)
    B = synth.int_dense(n, (500, n), -8, 8, kind=bk)
    kw = dict(mode=mode, seg_len=13)
    if mode == "mixed":
        kw.update(window_h=16, t_row=2, alpha_c=1 / 16, alpha=0.0, row_order="length_sorted")
    print("case", mode, kinds, n, flush=True)
    p, C = run(A, B, bk, api.default_opts(**kw), pad_b=3 if n % 2 else 0, pad_c=5 if n == 7 else 0)
    if mode != "plain":
        assert p.stats()["tiles"] > 0
    exact(C, A, B, bk)


@pytest.mark.parametrize("mode", ["plain", "mixed"])
@pytest.mark.parametrize("kinds,n", [(("f32", "f32"), 40), (("bf16", "bf16"), 128)])
def test_b_spanning_4gib_exact(mode, kinds, n):
    """B rows 2 GiB apart (a span beyond 4 GiB): the gathers cannot use a
    32-bit buffer resource and take predicated plain loads, and the window
    kernel stages B (direct to LDS for bf16 with whole 128-column panels)
    with 64-bit addresses.  Integer-exact against the oracle."""
    import torch
    vk, bk = kinds
    k = 3
    A = synth.random_csr(300, k, 0.7, 21, val_kind=vk, int_values=(-2, 2), empty_rows=0.05)
    B = synth.int_dense(5, (k, n), -8, 8, kind=bk)
    esize = 4 if bk == "f32" else 2
    ldb = (1 << 31) // esize + 64
    Bt = device_B(B, bk)
    big = torch.zeros((k - 1) * ldb + n, dtype=Bt.dtype, device="cuda")
    Bv = big.as_strided((k, n), (ldb, 1))
    Bv.copy_(Bt)
    kw = dict(mode=mode, seg_len=13)
    if mode == "mixed":
        kw.update(window_h=16, t_row=2, alpha_c=1 / 16, alpha=0.0)
    print("case", mode, kinds, n, ldb, flush=True)
    p = api.Plan(A, n, bk, api.default_opts(**kw))
    C = device_C(A.m, n)
    p.run(Bv, C)
    torch.cuda.synchronize()
    if mode == "mixed":
        assert p.stats()["tiles"] > 0
    exact(C, A, B, bk)
    del big, Bv
    torch.cuda.empty_cache()


@pytest.mark.parametrize("H", [16, 32, 64])
@pytest.mark.parametrize("order", ["original_ranges", "compacted", "length_sorted"])
def test_window_heights_and_orders_exact(H, order):
    A, _ = synth.block_community(n=4096, band=4, n_cols=8, seed=H, val_kind="bf16")
    A.vals[:] = synth.to_bf16_bits(np.round(np.random.default_rng(H).uniform(-2, 2, A.nnz)))
    B = synth.int_dense(H, (4096, 96), -8, 8, kind="bf16")
    print("case", H, order, flush=True)
    p, C = run(A, B, "bf16", api.default_opts(mode="mixed", window_h=H, t_row=1,
                                              alpha_c=1 / H, alpha=0.0, row_order=order,
                                              seg_len=17))
    assert p.stats()["tiles"] > 0
    exact(C, A, B, "bf16")


@pytest.mark.parametrize("H", [16, 64])
def test_windows_with_many_tiles_exact(H):
    # wide dense-ish rows: hundreds of tiles per window, split into partial items
    A = synth.random_csr(200, 9000, 0.25, 17 + H, val_kind="bf16", int_values=(-2, 2))
    B = synth.int_dense(3, (9000, 160), -8, 8, kind="bf16")
    p, C = run(A, B, "bf16", api.default_opts(mode="mfma_only", window_h=H, seg_len=40))
    d = p.export()
    assert d["wpart_win"].size > 10
    exact(C, A, B, "bf16")
    # the same through a batched submission
    import torch
    Bd = device_B(B, "bf16")
    C2 = device_C(A.m, 160)
    api.spmm_wait(api.spmm_submit([api.WorkItem(p, Bd, C2)]))
    torch.cuda.synchronize()
    assert torch.equal(C, C2)


def test_identity_returns_B_bitwise():
    import torch
    n = 2048
    for mode, bk in [("plain", "f32"), ("mfma_only", "bf16"), ("mixed", "bf16")]:
        vk = "f32" if mode == "plain" else "bf16"
        vals = np.ones(n, np.float32) if vk == "f32" else synth.to_bf16_bits(np.ones(n))
        A = synth.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                      vals, vk)
        B = synth.dense_values(np.random.default_rng(1), (n, 64), bk)
        p, C = run(A, B, bk, api.default_opts(mode=mode, t_row=-1, alpha_c=0.0, alpha=0.0))
        Bd = device_B(B, bk).float()
        assert torch.equal(C, Bd), mode


def test_empty_matrix_and_empty_rows():
    import torch
    A = synth.CSR(300, 50, np.zeros(301, np.int64), np.zeros(0, np.int32),
                  np.zeros(0, np.float32), "f32")
    B = np.ones((50, 40), np.float32)
    for mode in MODES:
        _, C = run(A, B, "f32", api.default_opts(mode=mode))
        assert torch.all(C == 0)
    A = synth.random_csr(1000, 300, 0.05, 3, empty_rows=0.5)
    B = np.random.default_rng(2).standard_normal((300, 64)).astype(np.float32)
    for mode in MODES:
        _, C = run(A, B, "f32", api.default_opts(mode=mode))
        parity(C, A, B, "f32", TOL_F32 if mode == "plain" else TOL_16)


def test_uniform_4096_n32_all_modes():
    A, B = synth.uniform_rows()
    for mode, tol in [("plain", TOL_F32), ("auto", TOL_F32), ("mixed", TOL_16),
                      ("mfma_only", TOL_16)]:
        print("case", mode, flush=True)
        _, C = run(A, B, "f32", api.default_opts(mode=mode))
        parity(C, A, B, "f32", tol)


def test_long_rows_segments():
    # hub rows of up to 20,000 entries split into segments of 64
    A = synth.chung_lu_graph(50000, 2.1, 16.0, 20000.0, 7, val_kind="f32")
    B = np.random.default_rng(3).standard_normal((50000, 128)).astype(np.float32)
    for mode, tol in [("plain", TOL_F32), ("mixed", TOL_16)]:
        kw = dict(mode=mode, seg_len=64)
        if mode == "mixed":
            kw.update(row_order="length_sorted", t_row=8)
        p, C = run(A, B, "f32", api.default_opts(**kw))
        assert p.stats()["segments"] > 0
        parity(C, A, B, "f32", tol)


def test_mixed_without_tiles_bitwise_equals_plain():
    import torch
    A = synth.chung_lu_graph(20000, 2.1, 16.0, 5000.0, 9)
    B = np.random.default_rng(4).standard_normal((20000, 64)).astype(np.float32)
    _, C1 = run(A, B, "f32", api.default_opts(mode="plain", seg_len=100))
    _, C2 = run(A, B, "f32", api.default_opts(mode="mixed", alpha=1.5, seg_len=100))
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("n,kind", [(128, "f32"), (64, "f32"), (33, "f32"), (256, "bf16")])
def test_pipelined_vector_kernel_bitwise_equals_row_by_row(n, kind):
    import torch
    A = synth.chung_lu_graph(30000, 2.1, 16.0, 3000.0, 12)
    B = synth.dense_values(np.random.default_rng(5), (30000, n), kind)
    outs = []
    for pipe in (0, 1):
        for hot in (0, -1):
            _, C = run(A, B, kind, api.default_opts(mode="plain", seg_len=50, pipeline=pipe,
                                                    hot_cols=hot))
            outs.append(C)
    for C in outs[1:]:
        assert torch.equal(outs[0], C)
    parity(outs[0], A, B, kind, TOL_F32)
    # packed short rows: a different fixed order, same tolerance, same result in mixed(no tiles)
    _, P1 = run(A, B, kind, api.default_opts(mode="plain", seg_len=50, pipeline=2))
    _, P2 = run(A, B, kind, api.default_opts(mode="mixed", alpha=1.5, seg_len=50, pipeline=2))
    assert torch.equal(P1, P2)
    parity(P1, A, B, kind, TOL_F32)


@pytest.mark.parametrize("n,kinds", [(32, ("f16", "f16")), (128, ("f32", "f32")),
                                     (7, ("bf16", "bf16"))])
def test_packed_rows_integer_exact(n, kinds):
    vk, bk = kinds
    A = synth.random_csr(3000, 1500, 0.006, 31 + n, val_kind=vk, int_values=(-2, 2),
                         empty_rows=0.1)
    # a few long rows (segments) between the short ones
    B = synth.int_dense(n + 1, (1500, n), -8, 8, kind=bk)
    for seg in (5, 300):
        _, C = run(A, B, bk, api.default_opts(mode="plain", pipeline=2, seg_len=seg))
        exact(C, A, B, bk)


def _lane_shape(n, kind):
    """(lane groups G, unroll U) of the vector kernel for N = n: 16-byte chunks
    of 4 f32 or 8 16-bit values (one value per lane when N is not a multiple),
    chunk lanes per row the power of two >= the chunk count (at most 64)."""
    e = 4 if kind == "f32" else 8
    if n % e:
        e = 1
    chunks = n // e
    lpr = 1
    while lpr < min(chunks, 64):
        lpr *= 2
    u = 4 if e == 1 else (8 if chunks <= 64 else 4)
    return 64 // lpr, u


@pytest.mark.parametrize("n,kinds", [(32, ("f16", "f16")), (64, ("f16", "f16")),
                                     (128, ("f16", "f16")), (128, ("f32", "f32")),
                                     (256, ("bf16", "bf16")), (33, ("f32", "f32")),
                                     (8, ("f32", "bf16"))])
def test_class_packed_variant(n, kinds):
    """Rows packed by size class: within the FP32 bound of the oracle, and bit
    for bit equal to the packed-short-row variant on every row whose class is
    1 (at most 2U entries) or all groups (more than U*G entries), which both
    variants sum in the same order."""
    import torch
    vk, bk = kinds
    A = synth.chung_lu_graph(20000, 2.2, 20.0, 1500.0, 40 + n, val_kind=vk, values="uniform")
    B = synth.dense_values(np.random.default_rng(n), (20000, n), bk)
    print("case", n, kinds, flush=True)
    p3, C3 = run(A, B, bk, api.default_opts(mode="plain", pipeline=3, seg_len=300))
    parity(C3, A, B, bk, TOL_F32)
    _, C2 = run(A, B, bk, api.default_opts(mode="plain", pipeline=2, seg_len=300))
    G, U = _lane_shape(n, bk)
    L = np.diff(A.rowptr)
    same = torch.from_numpy((L <= 2 * U) | (L > U * G)).cuda()
    if G > 2:
        assert int((~same).sum()) > 100
    assert torch.equal(C2[same], C3[same])
    assert p3.stats()["segments"] > 0


@pytest.mark.parametrize("n,kinds", [(32, ("f16", "f16")), (7, ("bf16", "bf16"))])
def test_class_packed_integer_exact(n, kinds):
    vk, bk = kinds
    A = synth.random_csr(3000, 1500, 0.02, 57 + n, val_kind=vk, int_values=(-2, 2),
                         empty_rows=0.1)
    B = synth.int_dense(n + 3, (1500, n), -8, 8, kind=bk)
    for seg in (5, 40, 300):
        _, C = run(A, B, bk, api.default_opts(mode="plain", pipeline=3, seg_len=seg,
                                              item_cost=200))
        exact(C, A, B, bk)


def test_submit_class_packed_matches_solo_bitwise():
    import torch
    specs = synth.batch_specs(count=6, seed=9, rows_lo=2000, rows_hi=40000)
    items, solos = [], []
    for i, sp in enumerate(specs):
        A, B = synth.batch_matrix(i, sp, seed=9)
        p = api.Plan(A, B.shape[1], "f16", api.default_opts(mode="plain", pipeline=3, seg_len=64))
        Bd = device_B(B, "f16")
        Cs = device_C(A.m, B.shape[1])
        p.run(Bd, Cs)
        items.append(api.WorkItem(p, Bd, device_C(A.m, B.shape[1])))
        solos.append((Cs, A, B))
    for _ in range(2):
        api.spmm_wait(api.spmm_submit(items))
    torch.cuda.synchronize()
    for it, (Cs, A, B) in zip(items, solos):
        assert torch.equal(it.C, Cs)
    parity(items[0].C, solos[0][1], solos[0][2], "f16", TOL_F32)


def test_deterministic_and_nan_prefill():
    import torch
    A, B = synth.block_community(n=16384, band=8, n_cols=256, seed=8)
    p = api.Plan(A, 256, "bf16", api.default_opts(mode="mixed", row_order="original_ranges"))
    Bd = device_B(B, "bf16")
    C1 = device_C(A.m, 256, fill=float("nan"))
    C2 = device_C(A.m, 256, fill=12345.0)
    p.run(Bd, C1)
    p.run(Bd, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    assert p.stats()["tiles"] > 0
    parity(C1, A, B, "bf16", TOL_16)


def test_block_community_scaled():
    A, B = synth.block_community(n=65536, band=32, n_cols=256, seed=3)
    for mode, tol in [("mixed", TOL_16), ("plain", TOL_F32)]:
        p, C = run(A, B, "bf16", api.default_opts(mode=mode, row_order="original_ranges"))
        print(mode, p.stats()["nnz_tiles"] / A.nnz, flush=True)
        parity(C, A, B, "bf16", tol)


def test_submit_matches_solo_bitwise():
    """Batched persistent launch (graph replay) vs solo runs, bit for bit, over
    several submissions with new B between replays and eager work around
    them; mixed dtypes and N make several kernel variants in one batch."""
    import torch
    specs = synth.batch_specs(count=8, seed=4, rows_lo=1000, rows_hi=30000)
    plans, mats = [], []
    for i, sp in enumerate(specs):
        A, B = synth.batch_matrix(i, sp, seed=4)
        mode = ["auto", "plain", "mixed", "mfma_only"][i % 4]
        kw = dict(mode=mode, seg_len=64)
        if mode == "mixed":
            kw.update(row_order="length_sorted", t_row=4)
        plans.append(api.Plan(A, B.shape[1], "f16", api.default_opts(**kw)))
        mats.append((A, B))
    # one f32 matrix with an odd N (scalar variant) in the same submission
    Af = synth.random_csr(3000, 2000, 0.01, 9)
    Bf = np.random.default_rng(1).standard_normal((2000, 33)).astype(np.float32)
    plans.append(api.Plan(Af, 33, "f32", api.default_opts(mode="plain", seg_len=16)))
    mats.append((Af, Bf))
    kinds = ["f16"] * len(specs) + ["f32"]
    for rnd in range(3):
        items, solos = [], []
        for p, (A, B), kind in zip(plans, mats, kinds):
            Bd = device_B(B, kind)
            if rnd:
                Bd = Bd * (rnd + 1)  # new values each round (exact in f16/f32: powers of two)
            Cs = device_C(A.m, B.shape[1])
            p.run(Bd, Cs)
            torch.cuda.synchronize()
            Cb = device_C(A.m, B.shape[1])
            items.append(api.WorkItem(p, Bd, Cb))
            solos.append(Cs)
        t = api.spmm_submit(items)
        _ = torch.ones(1000, device="cuda").sum().item()  # eager work while it runs
        api.spmm_wait(t)
        assert api.spmm_poll(t)
        torch.cuda.synchronize()
        for it, Cs in zip(items, solos):
            assert torch.equal(it.C, Cs), "round %d" % rnd
    for p, (A, B), kind in zip(plans, mats, kinds):
        Bd = device_B(B, kind)
        Cs = device_C(A.m, B.shape[1])
        p.run(Bd, Cs)
        torch.cuda.synchronize()
        parity(Cs, A, B, kind, TOL_16 if kind == "f16" else TOL_F32)


@pytest.mark.parametrize("a0", [0.9, 0.004])
def test_adapt_epochs(a0):
    """Epoch-level re-partition from a threshold that keeps no tile (0.9) and
    from one that keeps very sparse tiles (0.004): every epoch's C matches the
    oracle, the state's bookkeeping holds, and it stops within 7 rounds."""
    import torch
    A, B = synth.block_community(n=32768, band=16, n_cols=128, seed=6)
    Bd = device_B(B, "bf16")
    p = api.Plan(A, 128, "bf16", api.default_opts(mode="mixed", alpha=a0))
    p.run(Bd, device_C(A.m, 128))  # first launch of these kernels: not an epoch
    torch.cuda.synchronize()
    st = api.adapt_state()
    rows = np.sort(np.random.default_rng(0).choice(A.m, 3000, replace=False))
    alphas = []
    for epoch in range(9):
        C = device_C(A.m, 128)
        alphas.append(p.stats()["opts"]["alpha"])
        p.adapt_epoch(A, Bd, C, st)
        print("epoch", epoch, alphas[-1], st.alpha_star, st.skew, st.t_vec_ms, st.t_mfma_ms,
              flush=True)
        parity(C, A, B, "bf16", TOL_16, rows=rows)
        if not st.replanned:
            break
        assert p.stats()["opts"]["alpha"] == pytest.approx(st.alpha, rel=1e-6)
    assert st.rounds <= 7 and (st.converged or st.rounds == 7)
    assert st.p_vec > 0 and st.p_mfma > 0 and 0 < st.alpha_star <= 1
    C = device_C(A.m, 128)
    p.run(Bd, C)
    torch.cuda.synchronize()
    parity(C, A, B, "bf16", TOL_16)


@pytest.mark.parametrize("order", ["compacted", "length_sorted", "clustered"])
def test_local_reorder_exact(order):
    A = synth.random_csr(2000, 800, 0.02, 21, int_values=(-2, 2), dup_frac=0.02,
                         empty_rows=0.05)
    B = synth.int_dense(5, (800, 64), -8, 8, kind="bf16")
    p, C = run(A, B, "bf16", api.default_opts(mode="mixed", window_h=16, t_row=2,
                                              alpha_c=1 / 16, alpha=0.0, row_order=order,
                                              local_reorder=64, seg_len=11))
    assert p.stats()["tiles"] > 0
    exact(C, A, B, "bf16")


def test_local_reorder_shuffled_communities():
    """Row-shuffled community matrix: the rebuilt windows put most entries
    back into dense tiles, and the result stays within the 16-bit bound."""
    A0, B = synth.block_community(n=16384, band=8, n_cols=64, seed=4)
    A = synth.permute_rows(A0, 3)
    kw = dict(mode="mixed", row_order="compacted", t_row=1, alpha=1 / 16)
    p0 = api.Plan(A, 64, "bf16", api.default_opts(**kw), upload=False)
    p1, C = run(A, B, "bf16", api.default_opts(local_reorder=256, **kw))
    s0, s1 = p0.stats(), p1.stats()
    assert s1["nnz_tiles"] > 3 * s0["nnz_tiles"]
    assert s1["mean_tile_density"] > s0["mean_tile_density"]
    parity(C, A, B, "bf16", TOL_16)


@pytest.mark.parametrize("shape", ["equal16", "one_big", "two_big_many_small"])
def test_submit_xcd_assignment_bitwise(shape):
    """16 matrices of equal work (whole matrices per XCD); one large matrix
    with three small ones (every matrix cut into 8 chunks, one per XCD); two
    large matrices with 20 small ones (the two cut, the small ones whole):
    all equal their solo runs bit for bit."""
    import torch
    if shape == "equal16":
        mats = [synth.random_csr(3000, 3000, 0.004, 60 + i) for i in range(16)]
    elif shape == "one_big":
        mats = [synth.chung_lu_graph(60000, 2.1, 16.0, 3000.0, 61)] + \
               [synth.random_csr(500, 500, 0.01, 62 + i) for i in range(3)]
    else:
        mats = [synth.chung_lu_graph(60000, 2.1, 16.0, 3000.0, 61 + i) for i in range(2)] + \
               [synth.random_csr(1500, 1500, 0.004, 70 + i) for i in range(20)]
    items, solos = [], []
    for i, A in enumerate(mats):
        B = np.random.default_rng(i).standard_normal((A.k, 64)).astype(np.float32)
        p = api.Plan(A, 64, "f32", api.default_opts(mode="plain", seg_len=40))
        Bd = device_B(B, "f32")
        Cs = device_C(A.m, 64)
        p.run(Bd, Cs)
        items.append(api.WorkItem(p, Bd, device_C(A.m, 64)))
        solos.append((Cs, A, B))
    for _ in range(2):
        api.spmm_wait(api.spmm_submit(items))
    torch.cuda.synchronize()
    for it, (Cs, A, B) in zip(items, solos):
        assert torch.equal(it.C, Cs)
    parity(items[0].C, solos[0][1], solos[0][2], "f32", TOL_F32)


def test_plan_image_runs_bitwise():
    """A plan loaded from its image (uploaded anew) gives the same C bit for
    bit as the plan it was written from."""
    import torch
    A, B = synth.block_community(n=8192, band=8, n_cols=64, seed=2)
    p = api.Plan(A, 64, "bf16", api.default_opts(mode="mixed", seg_len=20))
    q = api.Plan.deserialize(p.serialize())
    Bd = device_B(B, "bf16")
    C1, C2 = device_C(A.m, 64), device_C(A.m, 64)
    p.run(Bd, C1)
    q.run(Bd, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    parity(C2, A, B, "bf16", TOL_16)


@pytest.mark.parametrize("policy", [2, 16, 18])
def test_cold_gather_policies_bitwise(policy):
    """Gathers of cold B rows with non-temporal / sc1 cache policies (and the
    hottest rows with the default one) change only where lines are cached:
    C equals the default-policy run bit for bit, segments included."""
    import torch
    A = synth.chung_lu_graph(30000, 2.1, 16.0, 3000.0, 71)
    B = np.random.default_rng(8).standard_normal((30000, 64)).astype(np.float32)
    p0, C0 = run(A, B, "f32", api.default_opts(mode="plain", seg_len=60, pipeline=0))
    p1, C1 = run(A, B, "f32", api.default_opts(mode="plain", seg_len=60, cold_policy=policy))
    s1 = p1.stats()
    assert s1["opts"]["pipeline"] == 0 and s1["hot_cols"] > 0 and s1["segments"] > 0
    assert torch.equal(C0, C1)
    parity(C1, A, B, "f32", TOL_F32)


def test_destroy_busy_plan_rejected():
    import torch
    A = synth.random_csr(2000, 2000, 0.01, 3)
    B = np.random.default_rng(2).standard_normal((2000, 64)).astype(np.float32)
    p = api.Plan(A, 64, "f32", api.default_opts(mode="plain"))
    Bd = device_B(B, "f32")
    C = device_C(A.m, 64)
    t = api.spmm_submit([api.WorkItem(p, Bd, C), api.WorkItem(p, Bd, device_C(A.m, 64))])
    # the ticket is outstanding until spmm_poll or spmm_wait retires it, so
    # destroy refuses with BUSY however far the device has got, and leaves
    # the plan usable
    with pytest.raises(L.SpmmError) as ei:
        p.destroy()
    assert ei.value.status == L.SPMM_ERR_BUSY
    assert p.handle and p.stats()["m"] == A.m
    api.spmm_wait(t)
    p.destroy()  # the ticket is retired, so destroy succeeds
    assert p.handle is None
    torch.cuda.synchronize()
    parity(C, A, B, "f32", TOL_F32)


def test_autotune_picks_and_caches():
    import torch
    api.tune_cache_clear()
    A, B = synth.block_community(n=32768, band=16, n_cols=128, seed=6)
    Bd = device_B(B, "bf16")
    C = device_C(A.m, 128)
    opts, rep = api.spmm_autotune(A, Bd, C, "bf16", budget_ms=8000)
    assert rep["candidates"] >= 4 and rep["best_ms"] <= rep["default_ms"] * 1.02
    assert 0 < rep["alpha_cost"] <= 1 and rep["p_vec"] > 0 and rep["p_mfma"] > 0
    key = api.spmm_profile_key(A, 128, "bf16")
    assert api.opts_dict(api.tune_cache_get(key)) == api.opts_dict(opts)
    p = api.Plan(A, 128, "bf16", api.default_opts(mode="auto"))
    assert p.stats()["opts"]["mode"] == opts.mode
    C2 = device_C(A.m, 128)
    p.run(Bd, C2)
    torch.cuda.synchronize()
    # the plan states its precision class; the tolerance follows it
    st = p.stats()
    assert st["tol_class"] == (1 if st["tiles"] > 0 else 0)
    parity(C2, A, B, "bf16", TOL_16 if st["tol_class"] == L.SPMM_TOL_ROUNDED16 else TOL_F32)
    api.tune_cache_clear()


def test_timer_and_copy_bandwidth():
    import torch
    A, B = synth.uniform_rows()
    p = api.Plan(A, 32, "f32", api.default_opts(mode="plain"))
    Bd = device_B(B, "f32")
    C = device_C(A.m, 32)
    t = api.Timer(16)
    for _ in range(3):
        p.run_timed(Bd, C, t)
    rec = t.read()
    # a plain plan is one co-scheduled grid by default (segments and vector items)
    assert len(rec) == 3 and all(name == "vector_path" and ms > 0 for name, ms in rec)
    t.reset()
    ps = api.Plan(A, 32, "f32", api.default_opts(mode="plain", exec=1))
    ps.run_timed(Bd, C, t)
    assert [name for name, _ in t.read()] == ["vector"]
    bw = api.spmm_copy_bandwidth(1 << 28)
    assert bw > 1e11
    torch.cuda.synchronize()


def test_gather_probe():
    """spmm_gather_bandwidth over random row ids (ids outside [0, k) are
    clamped), at full and partial row widths; the rate is positive and the
    caller's tensors are untouched."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(5)
    k = 4096
    B = torch.randn(k, 128, device="cuda", generator=g)
    rows = torch.randint(-50, k + 50, (1 << 18,), dtype=torch.int32, device="cuda", generator=g)
    B0, r0 = B.clone(), rows.clone()
    for ncols in (128, 64, 4):
        bw = api.spmm_gather_bandwidth(rows, B, ncols, reps=3)
        assert bw > 1e10, (ncols, bw)
    torch.cuda.synchronize()
    assert torch.equal(B, B0) and torch.equal(rows, r0)
