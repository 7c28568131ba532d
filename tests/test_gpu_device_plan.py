"""Plans built on the device (spmm_plan_device) from a CSR in device memory --
plain plans, and mixed plans with original-ranges windows (the column stage,
K-tiles, density test, bitmaps and packed values computed on the device) --
equal the host builder's plans array for array, run to the same C bit for
bit, and a malformed device CSR is refused by the device-side checks."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import TOL_F32, device_B, device_C, parity
from paper_2606_22482_amd import _lib as L
from paper_2606_22482_amd import api, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()


def device_csr(A):
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(A.rowptr, dtype=np.int64)).cuda()
    ci = torch.from_numpy(np.ascontiguousarray(A.colidx, dtype=np.int32)).cuda()
    v = np.ascontiguousarray(A.vals)
    if A.val_kind == "f32":
        vt = torch.from_numpy(v.astype(np.float32)).cuda()
    else:
        vt = torch.from_numpy(v.view(np.int16)).view(
            torch.bfloat16 if A.val_kind == "bf16" else torch.float16).cuda()
    return rp, ci, vt


CASES = [
    ("graph", "f32", "f32", 64, dict(seg_len=40)),
    ("graph", "f16", "f16", 32, dict(seg_len=50)),                      # size-class variant
    ("graph", "bf16", "bf16", 128, dict(seg_len=7, item_cost=100)),
    ("graph", "f32", "f32", 33, dict(seg_len=300, pipeline=0)),
    ("random", "f32", "bf16", 16, dict(seg_len=5, item_cost=4096, pipeline=3)),
    ("empty", "f32", "f32", 8, dict()),
]


def _matrix(kind, vk):
    if kind == "graph":
        return synth.chung_lu_graph(20000, 2.1, 14.0, 2500.0, 31, val_kind=vk, values="uniform")
    if kind == "random":
        return synth.random_csr(5000, 3000, 0.004, 9, val_kind=vk, dup_frac=0.05, empty_rows=0.2)
    return synth.random_csr(0, 50, 0.1, 1, val_kind=vk)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_device_plan_equals_host_plan(case):
    kind, vk, bk, n, kw = CASES[case]
    A = _matrix(kind, vk)
    _compare(A, n, bk, api.default_opts(mode="plain", **kw), case)


@pytest.mark.parametrize("seed", range(30))
def test_device_plan_random(seed):
    """Seeded random shapes, types and plain-plan options: device plan =
    host plan array for array, and the same C bit for bit."""
    r = np.random.default_rng(700 + seed)
    vk, bk = [("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"), ("f16", "f16")][r.integers(4)]
    m = int(r.choice([1, 3, int(r.integers(2, 6000))]))
    k = int(r.choice([1, int(r.integers(2, 4000))]))
    A = synth.random_csr(m, k, float(r.choice([0.001, 0.01, 0.05])), 800 + seed, val_kind=vk,
                         dup_frac=0.03, empty_rows=float(r.choice([0.0, 0.3])))
    n = int(r.choice([1, 8, 33, 64, 128, int(r.integers(1, 200))]))
    kw = dict(seg_len=int(r.choice([2, 9, 64, 256])), pipeline=int(r.integers(0, 4)),
              item_cost=int(r.choice([0, 16, 300, 4096])))
    print("case", seed, vk, bk, m, k, n, kw, flush=True)
    _compare(A, n, bk, api.default_opts(mode="plain", **kw), seed)


def _compare(A, n, bk, opts, case):
    import torch
    host = api.Plan(A, n, bk, opts)
    rp, ci, vt = device_csr(A)
    dev = api.Plan.on_device(rp, ci, vt, A.m, A.k, n, bk, opts)
    sh, sd = host.stats(), dev.stats()
    for key in ("vector_items", "segments", "k_ref", "workspace_bytes", "nnz_remainder",
                "vector_rows", "algorithmic_bytes"):
        assert sh[key] == sd[key], key
    assert sh["opts"] == sd["opts"]
    dh, dd = host.export(), dev.export()
    for key in ("rem_ptr", "rem_src", "vector_rows", "nseg", "vitem_ptr", "vitem_seg",
                "vexec_rows", "seg_row", "seg_begin", "seg_end", "rem_col_dev"):
        assert np.array_equal(dh[key], dd[key]), key
    if A.m == 0:
        return
    B = synth.dense_values(np.random.default_rng(case), (A.k, n), bk)
    Bd = device_B(B, bk)
    C1, C2 = device_C(A.m, n), device_C(A.m, n)
    host.run(Bd, C1)
    dev.run(Bd, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    parity(C2, A, B, bk, TOL_F32)
    # the device plan's image loads as an ordinary plan
    q = api.Plan.deserialize(dev.serialize())
    C3 = device_C(A.m, n)
    q.run(Bd, C3)
    torch.cuda.synchronize()
    assert torch.equal(C1, C3)


def _status(rp, ci, vt, m, k, opts=None):
    lib = L.load()
    csr = L.Csr(m, k, int(ci.numel()), rp.data_ptr(), ci.data_ptr(), vt.data_ptr(), L.F32, 0)
    h = C.c_void_p()
    st = lib.spmm_plan_device(C.byref(csr), 8, L.F32, L.F32,
                              C.byref(opts) if opts is not None else None, None, C.byref(h))
    if st == L.SPMM_OK:
        lib.spmm_plan_destroy(h)
    return st, lib.spmm_last_error().decode()


def test_device_checks_refuse_a_bad_csr():
    A = synth.random_csr(300, 200, 0.05, 4)
    rp, ci, vt = device_csr(A)
    assert _status(rp, ci, vt, A.m, A.k)[0] == L.SPMM_OK
    bad_rp = rp.clone()
    bad_rp[10], bad_rp[11] = rp[11] + 1, rp[10]          # not monotone
    assert _status(bad_rp, ci, vt, A.m, A.k) == (L.SPMM_ERR_INVALID, "rowptr not monotone from 0 to nnz")
    bad_ci = ci.clone()
    bad_ci[7] = A.k                                    # column out of range
    assert _status(rp, bad_ci, vt, A.m, A.k) == (L.SPMM_ERR_INVALID, "column index out of range")
    # clustered windows and local reordering are built on the host only
    st, _ = _status(rp, ci, vt, A.m, A.k, api.default_opts(mode="mixed", row_order="clustered"))
    assert st == L.SPMM_ERR_UNSUPPORTED
    st, _ = _status(rp, ci, vt, A.m, A.k, api.default_opts(mode="mixed", row_order="compacted",
                                                           local_reorder=32))
    assert st == L.SPMM_ERR_UNSUPPORTED
    for order in ("original_ranges", "compacted", "length_sorted"):
        opts = api.default_opts(mode="mixed", row_order=order)
        assert _status(rp, ci, vt, A.m, A.k, opts)[0] == L.SPMM_OK, order


MIXED_KEYS = ("windows", "tile_window", "tile_cols", "tile_bitmap", "tile_val_ptr", "tile_vals",
              "tile_src", "rem_ptr", "rem_src", "vector_rows", "nseg", "vitem_ptr", "vitem_seg",
              "vexec_rows", "seg_row", "seg_begin", "seg_end", "win_seg", "win_order", "rem_col_dev",
              "win_part", "wpart_win", "wpart_t0", "wpart_t1", "seg_win", "win_dep", "win_nsseg")
MIXED_STATS = ("windows", "tiles", "nnz_tiles", "nnz_remainder", "vector_rows", "segments",
               "vector_items", "k_ref", "workspace_bytes", "algorithmic_bytes", "tol_class")


def _compare_mixed(A, n, bk, opts, case, exact_ints):
    import torch
    from gpu_util import TOL_16, exact
    host = api.Plan(A, n, bk, opts)
    rp, ci, vt = device_csr(A)
    dev = api.Plan.on_device(rp, ci, vt, A.m, A.k, n, bk, opts)
    sh, sd = host.stats(), dev.stats()
    for key in MIXED_STATS:
        assert sh[key] == sd[key], key
    assert sh["opts"] == sd["opts"]
    dh, dd = host.export(), dev.export()
    assert dh["n_dep"] == dd["n_dep"]
    for key in MIXED_KEYS:
        assert np.array_equal(dh[key], dd[key]), key
    if A.m == 0:
        return sh
    if exact_ints:
        B = synth.int_dense(case, (A.k, n), -8, 8, kind=bk)
    else:
        B = synth.dense_values(np.random.default_rng(case), (A.k, n), bk)
    Bd = device_B(B, bk)
    C1, C2 = device_C(A.m, n), device_C(A.m, n)
    host.run(Bd, C1)
    dev.run(Bd, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    if exact_ints:
        exact(C2, A, B, bk)
    else:
        parity(C2, A, B, bk, TOL_16)
    q = api.Plan.deserialize(dev.serialize())
    C3 = device_C(A.m, n)
    q.run(Bd, C3)
    torch.cuda.synchronize()
    assert torch.equal(C1, C3)
    return sh


def _int_vals(A, seed):
    v = np.random.default_rng(seed).integers(-2, 3, A.nnz).astype(np.float32)
    A.vals = v if A.val_kind == "f32" else (synth.to_bf16_bits(v) if A.val_kind == "bf16"
                                            else synth.to_f16_bits(v))
    return A


MIXED_CASES = [
    # block community, bf16 values and B: dense windows, every tile kept
    ("block", "bf16", "bf16", 256, dict(mode="mixed")),
    # f32 values and B: tiles round both to bf16
    ("block", "f32", "f32", 96, dict(mode="mixed", window_h=32)),
    # duplicates and empty rows, low thresholds: repeated pairs, sparse tiles demoted
    ("random", "f32", "bf16", 64, dict(mode="mixed", t_row=2, alpha_c=1 / 16, alpha=0.05, seg_len=9)),
    # every row in a window, every column in a tile
    ("graph", "f16", "f16", 40, dict(mode="mfma_only", window_h=64, seg_len=33)),
    # windows of hundreds of tiles (partial items) and split remainders
    ("wide", "bf16", "bf16", 160, dict(mode="mixed", window_h=16, t_row=-1, alpha_c=0.0, alpha=0.2,
                                       seg_len=40)),
    # length-sorted windows over a power-law graph (the GNN mixed plan's order)
    ("graph", "f32", "f32", 128, dict(mode="mixed", row_order="length_sorted", t_row=8, alpha=0.05,
                                      seg_len=24)),
    # compacted windows, empty rows passing the row stage (t_row = -1), duplicates
    ("random", "bf16", "bf16", 48, dict(mode="mixed", row_order="compacted", t_row=-1, alpha_c=1 / 16,
                                        alpha=0.02, window_h=32)),
    # length-sorted, every row in a window (many equal lengths: ties keep row order)
    ("block", "f16", "f16", 64, dict(mode="mfma_only", row_order="length_sorted", window_h=64)),
    # no tile dense enough: every window dissolves into vector rows
    ("graph", "f32", "f32", 32, dict(mode="mixed", alpha=2.0)),
]


def _mixed_matrix(kind, vk, seed):
    if kind == "block":
        A, _ = synth.block_community(n=8192, band=8, n_cols=8, seed=seed, val_kind=vk)
        return A
    if kind == "random":
        return synth.random_csr(3001, 2000, 0.01, seed, val_kind=vk, dup_frac=0.1, empty_rows=0.2)
    if kind == "wide":
        return synth.random_csr(300, 9000, 0.2, seed, val_kind=vk)
    return synth.chung_lu_graph(6000, 2.1, 14.0, 1500.0, seed, val_kind=vk, values="uniform")


@pytest.mark.parametrize("case", range(len(MIXED_CASES)))
def test_device_mixed_plan_equals_host_plan(case):
    kind, vk, bk, n, kw = MIXED_CASES[case]
    A = _int_vals(_mixed_matrix(kind, vk, 40 + case), case)
    print("case", case, kind, vk, bk, n, kw, flush=True)
    sh = _compare_mixed(A, n, bk, api.default_opts(**kw), case, exact_ints=True)
    if case < len(MIXED_CASES) - 1:
        assert sh["tiles"] > 0
    else:
        assert sh["tiles"] == 0 and sh["windows"] == 0


@pytest.mark.parametrize("seed", range(24))
def test_device_mixed_plan_random(seed):
    """Seeded random shapes, types and mixed-plan options (window height, row
    and column thresholds, tile density, segment length, variants, launch
    forms): device plan = host plan array for array, same C bit for bit,
    integer-exact against the oracle."""
    r = np.random.default_rng(900 + seed)
    vk, bk = [("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"), ("f16", "f16")][r.integers(4)]
    m = int(r.choice([1, 17, int(r.integers(2, 5000))]))
    k = int(r.choice([1, 31, int(r.integers(2, 3000))]))
    A = synth.random_csr(m, k, float(r.choice([0.005, 0.02, 0.08, 0.2])), 950 + seed, val_kind=vk,
                         int_values=(-2, 2), dup_frac=float(r.choice([0.0, 0.05])),
                         empty_rows=float(r.choice([0.0, 0.3])))
    H = int(r.choice([16, 32, 64]))
    n = int(r.choice([1, 8, 33, 64, 128, 256, int(r.integers(1, 300))]))
    kw = dict(mode=str(r.choice(["mixed", "mixed", "mfma_only"])), window_h=H,
              t_row=int(r.choice([-1, 0, 2, 8])), alpha_c=float(r.choice([0.0, 1.0 / H, 2.0 / H])),
              alpha=float(r.choice([0.0, 0.02, 0.1, 0.5])), seg_len=int(r.choice([3, 17, 64, 256])),
              pipeline=int(r.integers(0, 4)), win_sched=int(r.integers(0, 2)),
              exec=int(r.choice([1, 2, 3])))
    print("case", seed, vk, bk, m, k, n, kw, flush=True)
    _compare_mixed(A, n, bk, api.default_opts(**kw), seed, exact_ints=True)


@pytest.mark.parametrize("seed", range(16))
def test_device_mixed_plan_random_orders(seed):
    """As above with compacted and length-sorted windows: device plan = host
    plan array for array, same C bit for bit, integer-exact."""
    r = np.random.default_rng(1900 + seed)
    vk, bk = [("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"), ("f16", "f16")][r.integers(4)]
    m = int(r.choice([17, int(r.integers(200, 5000)), int(r.integers(200, 5000))]))
    if r.integers(2):
        k = int(r.choice([31, int(r.integers(50, 3000))]))
        A = synth.random_csr(m, k, float(r.choice([0.02, 0.08, 0.2])), 1950 + seed, val_kind=vk,
                             int_values=(-2, 2), dup_frac=float(r.choice([0.0, 0.05])),
                             empty_rows=float(r.choice([0.0, 0.3])))
    else:
        A = _int_vals(synth.chung_lu_graph(max(m, 200), 2.1, 12.0, 800.0, 1950 + seed, val_kind=vk,
                                           values="uniform"), seed)
    H = int(r.choice([16, 32, 64]))
    n = int(r.choice([1, 8, 33, 64, 128, 256, int(r.integers(1, 300))]))
    kw = dict(mode=str(r.choice(["mixed", "mixed", "mfma_only"])), window_h=H,
              row_order=str(r.choice(["compacted", "length_sorted"])),
              t_row=int(r.choice([-1, 0, 2, 8])), alpha_c=float(r.choice([0.0, 1.0 / H])),
              alpha=float(r.choice([0.0, 0.02, 0.1])), seg_len=int(r.choice([3, 17, 64, 256])),
              pipeline=int(r.integers(0, 4)), win_sched=int(r.integers(0, 2)),
              exec=int(r.choice([1, 2, 3])))
    print("case", seed, vk, bk, A.m, A.k, n, kw, flush=True)
    _compare_mixed(A, n, bk, api.default_opts(**kw), seed, exact_ints=True)
