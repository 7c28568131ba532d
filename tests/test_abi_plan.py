"""CPU tier for the library: it loads and exports every declared symbol, the
ABI structs match, validation returns the documented codes, and the C++ plan
builder equals the independent numpy reference bit for bit (NeutronSparse
Sec. 5.2.2 / Sec. 6.1 partition), with a valid schedule on top."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle import plan_ref as pr
from paper_2606_22482_amd import _lib as L
from paper_2606_22482_amd import api, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return L.load()


def declared_functions():
    names = []
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if not hdr.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", hdr)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"^[A-Za-z_][\w \*]*?\b(spmm_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, "binding lacks " + n
    assert lib.spmm_abi_version() == 1


def _csr(A):
    rp = np.ascontiguousarray(A.rowptr, np.int64)
    ci = np.ascontiguousarray(A.colidx, np.int32)
    v = np.ascontiguousarray(A.vals)
    return L.Csr(A.m, A.k, int(rp[-1]), rp.ctypes.data, ci.ctypes.data, v.ctypes.data,
                 L.KIND_CODE[A.val_kind], 0), (rp, ci, v)


def _status(lib, A, n=8, bt=L.F32, ct=L.F32, opts=None):
    csr, keep = _csr(A)
    h = C.c_void_p()
    st = lib.spmm_plan_build(C.byref(csr), n, bt, ct, C.byref(opts) if opts else None, C.byref(h))
    if st == 0:
        lib.spmm_plan_destroy(h)
    return st


def test_validation_codes(lib):
    A = synth.random_csr(20, 10, 0.2, 1)
    assert _status(lib, A) == L.SPMM_OK
    bad = synth.CSR(A.m, A.k, A.rowptr.copy(), A.colidx.copy(), A.vals, "f32")
    bad.colidx[3] = 10
    assert _status(lib, bad) == L.SPMM_ERR_INVALID
    bad = synth.CSR(A.m, A.k, A.rowptr.copy(), A.colidx, A.vals, "f32")
    bad.rowptr[5], bad.rowptr[6] = bad.rowptr[6] + 1, bad.rowptr[5]
    assert _status(lib, bad) == L.SPMM_ERR_INVALID
    bad = synth.CSR(A.m, A.k, A.rowptr.copy(), A.colidx, A.vals, "f32")
    bad.rowptr[0] = 1
    assert _status(lib, bad) == L.SPMM_ERR_INVALID
    assert _status(lib, A, n=0) == L.SPMM_ERR_INVALID
    assert _status(lib, A, bt=L.F16) == L.SPMM_ERR_UNSUPPORTED     # f32 vals with f16 B
    assert _status(lib, A, ct=L.BF16) == L.SPMM_ERR_UNSUPPORTED
    assert _status(lib, A, opts=api.default_opts(window_h=24)) == L.SPMM_ERR_UNSUPPORTED
    assert _status(lib, A, opts=api.default_opts(kt=16)) == L.SPMM_ERR_UNSUPPORTED
    assert _status(lib, A, opts=api.default_opts(win_sched=2)) == L.SPMM_ERR_UNSUPPORTED
    assert _status(lib, A, opts=api.default_opts(cold_policy=2, pipeline=2)) == L.SPMM_ERR_UNSUPPORTED
    assert _status(lib, A, opts=api.default_opts(cold_policy=2)) == L.SPMM_OK
    assert _status(lib, A, opts=api.default_opts(mode="mixed", row_order="original_ranges",
                                                  local_reorder=32)) == L.SPMM_ERR_UNSUPPORTED
    assert _status(lib, A, opts=api.default_opts(mode="mixed", row_order="compacted",
                                                  local_reorder=32)) == L.SPMM_OK
    assert _status(lib, A, opts=api.default_opts(alpha=float("nan"), mode="mixed")) in (
        L.SPMM_OK, L.SPMM_ERR_UNSUPPORTED)
    h = C.c_void_p()
    assert lib.spmm_plan_build(None, 8, 0, 0, None, C.byref(h)) == L.SPMM_ERR_INVALID
    assert b"null" in lib.spmm_last_error()


def test_run_needs_upload_and_checks_ld(lib):
    A = synth.random_csr(20, 10, 0.2, 1)
    p = api.Plan(A, 8, "f32", api.default_opts(mode="plain"), upload=False)
    st = lib.spmm_run(p.handle, C.c_void_p(16), 8, C.c_void_p(16), 8, None)
    assert st == L.SPMM_ERR_UNSUPPORTED
    s = p.stats()
    assert s["uploaded"] == 0 and s["nnz"] == A.nnz and s["n"] == 8
    assert s["flops"] == 2 * A.nnz * 8


def _cmp_plan(A, dump, ref):
    assert np.array_equal(dump["windows"], ref.windows)
    assert np.array_equal(dump["tile_window"], ref.tile_window)
    assert np.array_equal(dump["tile_cols"], ref.tile_cols)
    assert np.array_equal(dump["tile_bitmap"], ref.tile_bitmap)
    assert np.array_equal(dump["tile_val_ptr"], ref.tile_val_ptr)
    assert np.array_equal(dump["tile_vals"], ref.tile_vals)
    assert np.array_equal(dump["tile_src"], ref.tile_src)
    assert np.array_equal(dump["rem_ptr"], ref.rem_ptr)
    assert np.array_equal(dump["rem_src"], ref.rem_src)
    assert np.array_equal(dump["vector_rows"], ref.vector_rows)
    assert np.array_equal(dump["nseg"], ref.nseg)


def _win_tiles(d, n):
    """Tiles an owner window item computes, by the scheduling rule: the least
    power of two in [16, 128] that is at least the plan's tiles times its
    128-column panels over 1024."""
    want = -(-d["tile_window"].size * ((n + 127) // 128) // 1024)
    k = 16
    while k < 128 and k < want:
        k *= 2
    return k


def _check_schedule(A, d, seg_len, pipeline=2, n=8):
    m = A.m
    vr = d["vector_rows"]
    ve = d["vexec_rows"]
    vp = d["vitem_ptr"]
    assert vp[0] == 0 and vp[-1] == vr.size and np.all(np.diff(vp) > 0)
    # segments: walk items then windows in order, ids must be consecutive
    rem_len = np.diff(d["rem_ptr"])
    sid = 0
    for i in range(vp.size - 1):
        assert d["vitem_seg"][i] == sid
        part = ve[vp[i]:vp[i + 1]]
        # an item's launch order is a permutation of its vector rows: the same
        # rows for every variant; variant 3 takes them longest first (split
        # rows last), ties in row order
        assert np.array_equal(np.sort(part), vr[vp[i]:vp[i + 1]])
        if pipeline == 3:
            key = np.where(d["nseg"][part] > 0, -1, rem_len[part])
            assert np.all(np.diff(key) <= 0)
            assert np.all(np.diff(part)[np.diff(key) == 0] > 0)
        else:
            assert np.array_equal(part, vr[vp[i]:vp[i + 1]])
        for r in part:
            for j in range(d["nseg"][r]):
                assert d["seg_row"][sid] == r
                assert d["seg_begin"][sid] == d["rem_ptr"][r] + j * seg_len
                assert d["seg_end"][sid] == min(d["rem_ptr"][r] + (j + 1) * seg_len,
                                                d["rem_ptr"][r + 1])
                sid += 1
    for w in range(d["windows"].shape[0]):
        assert d["win_seg"][w] == sid
        for r in d["windows"][w]:
            if r >= 0:
                sid += d["nseg"][r]
    assert sid == d["seg_row"].size
    assert np.array_equal(np.sort(d["win_order"]), np.arange(d["windows"].shape[0]))
    # window partial items: tiles beyond a window's first K, in chunks of K, in order
    K = _win_tiles(d, n)
    wt = np.bincount(d["tile_window"], minlength=d["windows"].shape[0])
    tstart = np.concatenate([[0], np.cumsum(wt)])
    k = 0
    for w in range(d["windows"].shape[0]):
        assert d["win_part"][w] == k
        for t in range(tstart[w] + K, tstart[w + 1], K):
            assert d["wpart_win"][k] == w and d["wpart_t0"][k] == t
            assert d["wpart_t1"][k] == min(t + K, tstart[w + 1])
            k += 1
    assert d["win_part"][-1] == k == d["wpart_win"].size
    # every row is owned exactly once
    owners = np.concatenate([vr, d["windows"][d["windows"] >= 0]])
    assert np.array_equal(np.sort(owners), np.arange(m))
    assert np.all(d["nseg"] == np.where(rem_len > seg_len, -(-rem_len // seg_len), 0))


CASES = [
    # (matrix kind, val kind, b kind, options)
    ("random", "f32", "f32", dict(mode="mixed", window_h=16, t_row=3, alpha_c=1 / 16, alpha=0.05,
                                  row_order="length_sorted", seg_len=7)),
    ("random", "f32", "bf16", dict(mode="mixed", window_h=32, t_row=0, alpha_c=1 / 32, alpha=0.0,
                                   row_order="original_ranges", seg_len=5)),
    ("random", "bf16", "bf16", dict(mode="mixed", window_h=64, t_row=-1, alpha_c=0.0, alpha=0.01,
                                    row_order="compacted", seg_len=11)),
    ("random", "f16", "f16", dict(mode="mfma_only", window_h=16, seg_len=4)),
    ("random", "f32", "f32", dict(mode="plain", seg_len=6)),
    ("random", "f32", "f32", dict(mode="mixed", t_row=-1, alpha_c=0.0, alpha=1.5, seg_len=6)),
    ("block", "f32", "bf16", dict(mode="mixed", window_h=16, t_row=1, alpha_c=1 / 16,
                                  alpha=1 / 16, row_order="original_ranges", seg_len=16)),
    ("random", "f32", "f32", dict(mode="mixed", window_h=16, t_row=3, alpha_c=1 / 16, alpha=0.02,
                                  row_order="compacted", seg_len=7, local_reorder=40)),
    ("random", "f16", "f16", dict(mode="mixed", window_h=32, t_row=2, alpha_c=1 / 32, alpha=0.0,
                                  row_order="length_sorted", seg_len=9, local_reorder=96)),
    ("block", "f32", "bf16", dict(mode="mixed", window_h=16, t_row=1, alpha_c=1 / 16,
                                  alpha=1 / 16, row_order="compacted", seg_len=16,
                                  local_reorder=256)),
    ("random", "f32", "f32", dict(mode="mixed", window_h=16, t_row=2, alpha_c=1 / 16, alpha=0.02,
                                  row_order="clustered", seg_len=7)),
    ("shuffled", "f32", "bf16", dict(mode="mixed", window_h=16, t_row=1, alpha_c=1 / 16,
                                     alpha=1 / 16, row_order="clustered", seg_len=16,
                                     local_reorder=64)),
    ("shuffled", "bf16", "bf16", dict(mode="mixed", window_h=32, t_row=1, alpha_c=1 / 32,
                                      alpha=0.03, row_order="clustered", seg_len=16)),
]


def _matrix(kind, vk):
    if kind == "random":
        return synth.random_csr(400, 300, 0.04, 7, val_kind=vk, dup_frac=0.05, empty_rows=0.05)
    A, _ = synth.block_community(n=2048, band=4, n_cols=8, seed=5, val_kind=vk)
    return synth.permute_rows(A, 2) if kind == "shuffled" else A


@pytest.mark.parametrize("case", range(len(CASES)))
def test_plan_bit_exact_vs_reference(lib, case):
    kind, vk, bk, kw = CASES[case]
    A = _matrix(kind, vk)
    o = api.default_opts(**kw)
    p = api.Plan(A, 8, bk, o, upload=False)
    st = p.stats()
    ro = st["opts"]
    mode = ro["mode"]
    ref = pr.build_plan(A.rowptr, A.colidx, A.vals, k=A.k, mode=mode, window_h=ro["window_h"],
                        t_row=ro["t_row"], alpha_c=ro["alpha_c"], alpha=ro["alpha"],
                        kt=ro["kt"], row_order=ro["row_order"], seg=ro["seg_len"],
                        tile_kind="f16" if bk == "f16" else "bf16", val_kind=vk,
                        local_reorder_rows=ro["local_reorder"])
    d = p.export()
    _cmp_plan(A, d, ref)
    _check_schedule(A, d, ro["seg_len"], ro["pipeline"])
    assert np.all(pr.coverage(ref) == 1)
    if mode == L.MODE_MIXED and kw.get("alpha", 0) <= 1.0:
        assert st["tiles"] > 0
    assert st["nnz_tiles"] + st["nnz_remainder"] == A.nnz


def test_many_tiles_make_window_partials(lib):
    A = synth.random_csr(64, 8192, 0.3, 6)
    p = api.Plan(A, 32, "f32", api.default_opts(mode="mfma_only", window_h=16), upload=False)
    d = p.export()
    assert d["wpart_win"].size > 0
    _check_schedule(A, d, p.stats()["opts"]["seg_len"], p.stats()["opts"]["pipeline"], n=32)


@pytest.mark.parametrize("n, K", [(128, 32), (256, 64)])
def test_window_items_grow_with_the_tile_count(lib, n, K):
    """A plan of 32,768 tiles: window items of K tiles (the least power of
    two in [16, 128] that brings tiles x panels down to about 1024 items);
    the partial items cover the rest exactly, and a plan image keeps them."""
    A = synth.random_csr(2048, 8192, 0.5, 12)
    p = api.Plan(A, n, "bf16", api.default_opts(mode="mfma_only", window_h=16), upload=False)
    d = p.export()
    assert d["tile_window"].size == 32768
    assert _win_tiles(d, n) == K
    assert d["wpart_win"].size == 128 * (256 // K - 1)
    _check_schedule(A, d, p.stats()["opts"]["seg_len"], p.stats()["opts"]["pipeline"], n=n)
    q = api.Plan.deserialize(p.serialize(), upload=False)
    dq = q.export()
    for key in ("win_part", "wpart_win", "wpart_t0", "wpart_t1", "win_order"):
        assert np.array_equal(d[key], dq[key]), key


def _window_costs(d, kt, h, n):
    """Per-window work estimate of the schedule: the owner's tiles (at most K)
    times kt, H per partial item, and 4 + entries (or segments) per row."""
    nw = d["windows"].shape[0]
    wt = np.bincount(d["tile_window"], minlength=nw)
    rem_len = np.diff(d["rem_ptr"])
    cost = np.minimum(wt, _win_tiles(d, n)) * kt + np.diff(d["win_part"]) * h
    for w in range(nw):
        for r in d["windows"][w]:
            if r >= 0:
                cost[w] += 4 + (d["nseg"][r] if d["nseg"][r] else rem_len[r])
    return cost


@pytest.mark.parametrize("sched", [0, 1])
def test_window_launch_order(lib, sched):
    A, _ = synth.block_community(n=8192, band=8, n_cols=8, seed=4)
    p = api.Plan(A, 64, "bf16", api.default_opts(mode="mixed", win_sched=sched, seg_len=8),
                 upload=False)
    d = p.export()
    ro = p.stats()["opts"]
    nw = d["windows"].shape[0]
    assert nw > 100 and ro["win_sched"] == sched
    if sched == 0:
        assert np.array_equal(d["win_order"], np.arange(nw))
    else:
        cost = _window_costs(d, ro["kt"], ro["window_h"], 64)
        c = cost[d["win_order"]]
        assert np.all(np.diff(c) <= 0) and np.unique(c).size > 1
        # stable: equal costs keep window id order
        same = np.diff(c) == 0
        assert np.all(np.diff(d["win_order"])[same] > 0)
    _check_schedule(A, d, ro["seg_len"], ro["pipeline"], n=64)


@pytest.mark.parametrize("pipeline", [2, 3])
def test_vector_launch_order(lib, pipeline):
    A = synth.chung_lu_graph(6000, 2.2, 12.0, 700.0, 8, val_kind="f16")
    p = api.Plan(A, 32, "f16", api.default_opts(mode="plain", pipeline=pipeline, seg_len=40,
                                                item_cost=300), upload=False)
    d = p.export()
    assert d["vitem_ptr"].size > 10 and d["seg_row"].size > 0
    _check_schedule(A, d, 40, pipeline)
    if pipeline == 3:
        assert not np.array_equal(d["vexec_rows"], d["vector_rows"])


def test_auto_vector_variant(lib):
    A = synth.random_csr(200, 200, 0.05, 2, val_kind="f16")
    pick = lambda n, bk: api.Plan(A, n, bk, api.default_opts(mode="plain"),
                                  upload=False).stats()["opts"]["pipeline"]
    assert pick(32, "f16") == 3 and pick(128, "f16") == 3 and pick(256, "f16") == 2
    Af = synth.random_csr(200, 200, 0.05, 2)
    assert api.Plan(Af, 64, "f32", None, upload=False).stats()["opts"]["pipeline"] == 2
    assert api.Plan(Af, 64, "bf16", None, upload=False).stats()["opts"]["pipeline"] == 3


def test_default_window_order_is_by_id(lib):
    A, _ = synth.block_community(n=2048, band=4, n_cols=8, seed=5)
    p = api.Plan(A, 8, "bf16", api.default_opts(mode="mixed"), upload=False)
    assert p.stats()["opts"]["win_sched"] == 0


def test_mixed_without_tiles_equals_plain(lib):
    A = synth.random_csr(300, 300, 0.03, 9)
    p1 = api.Plan(A, 16, "f32", api.default_opts(mode="plain", seg_len=9), upload=False)
    p2 = api.Plan(A, 16, "f32", api.default_opts(mode="mixed", alpha=2.0, seg_len=9),
                  upload=False)
    d1, d2 = p1.export(), p2.export()
    for key in ("rem_ptr", "rem_src", "vector_rows", "nseg", "vitem_ptr", "vitem_seg",
                "seg_begin", "seg_end"):
        assert np.array_equal(d1[key], d2[key]), key
    assert d2["windows"].shape[0] == 0


def test_auto_mode_falls_back_to_plain_without_tiles(lib):
    A = synth.random_csr(500, 5000, 0.001, 3)
    p = api.Plan(A, 16, "f32", None, upload=False)
    assert p.stats()["opts"]["mode"] == L.MODE_PLAIN_F32
    B, _ = synth.block_community(n=1024, band=4, n_cols=8, seed=2)
    # 16-bit B: the tiles hold most entries, so AUTO keeps the mixed plan (its
    # tiles round the f32 values to bf16, which the plan reports)
    q = api.Plan(B, 16, "bf16", None, upload=False)
    assert q.stats()["opts"]["mode"] == L.MODE_MIXED and q.stats()["tiles"] > 0
    assert q.stats()["tol_class"] == L.SPMM_TOL_ROUNDED16
    # f32 B is the FP32 path: AUTO never rounds its operands
    r = api.Plan(B, 16, "f32", None, upload=False)
    assert r.stats()["opts"]["mode"] == L.MODE_PLAIN_F32 and r.stats()["tiles"] == 0
    assert r.stats()["tol_class"] == L.SPMM_TOL_FP32
    # an explicit mixed plan of f32 B rounds, and says so
    x = api.Plan(B, 16, "f32", api.default_opts(mode="mixed"), upload=False)
    assert x.stats()["tiles"] > 0 and x.stats()["tol_class"] == L.SPMM_TOL_ROUNDED16
    # 16-bit values and B: the tiles' products are exact, so the class stays FP32
    Bb = synth.CSR(B.m, B.k, B.rowptr, B.colidx, synth.to_bf16_bits(B.vals), "bf16")
    y = api.Plan(Bb, 16, "bf16", api.default_opts(mode="mixed"), upload=False)
    assert y.stats()["tiles"] > 0 and y.stats()["tol_class"] == L.SPMM_TOL_FP32


def test_plan_stats_consistency(lib):
    A, _ = synth.block_community(n=4096, band=8, n_cols=8, seed=3)
    p = api.Plan(A, 64, "bf16", api.default_opts(mode="mixed", row_order="original_ranges"),
                 upload=False)
    s = p.stats()
    assert s["k_ref"] == np.unique(A.colidx).size
    expect = 4 * (A.m + 1) + A.nnz * 8 + s["k_ref"] * 64 * 2 + A.m * 64 * 4
    assert s["algorithmic_bytes"] == expect
    assert 0 < s["mean_tile_density"] <= 1
    assert abs(s["zero_fraction_tiles"] - (1 - s["mean_tile_density"])) < 1e-12


def test_hot_columns_are_most_gathered(lib):
    A = synth.chung_lu_graph(5000, 2.1, 16.0, 800.0, 4)
    for hot in (0, 37, 10 ** 9):
        p = api.Plan(A, 64, "f32", api.default_opts(mode="plain", hot_cols=hot), upload=False)
        d = p.export()
        dev = d["rem_col_dev"]
        cols = A.colidx[d["rem_src"]]
        assert np.array_equal(dev & 0x7FFFFFFF, cols)
        flagged = np.unique(cols[dev < 0])
        counts = np.bincount(cols, minlength=A.k)
        used = np.nonzero(counts)[0]
        order = sorted(used.tolist(), key=lambda c: (-counts[c], c))
        want = np.sort(np.array(order[:min(hot, used.size)], dtype=np.int64))
        assert np.array_equal(flagged, want)
        assert p.stats()["hot_cols"] == want.size
    # auto: 80% of a 4 MiB L2 in rows of N * 4 bytes when cold rows get their own policy
    p = api.Plan(A, 64, "f32", api.default_opts(mode="plain", cold_policy=2), upload=False)
    assert p.stats()["opts"]["hot_cols"] == int(0.8 * 4 * 1024 * 1024 / (64 * 4))
    q = api.Plan(A, 64, "f32", api.default_opts(mode="plain"), upload=False)
    assert q.stats()["opts"]["cold_policy"] == 0 and q.stats()["opts"]["hot_cols"] == 0


def _path_work(d, h, kt):
    """Entries of the vector path (all segments, unsplit vector rows), tile
    slots, and unsplit window rows' remainder entries, from the export."""
    rem_len = np.diff(d["rem_ptr"])
    wv = float(np.sum(d["seg_end"] - d["seg_begin"]))
    vr = d["vector_rows"]
    wv += float(rem_len[vr][d["nseg"][vr] == 0].sum())
    wr_rows = d["windows"][d["windows"] >= 0]
    wr = float(rem_len[wr_rows][d["nseg"][wr_rows] == 0].sum())
    return wv, float(d["tile_window"].size * h * kt), wr


def test_plan_path_work(lib):
    A, _ = synth.block_community(n=4096, band=8, n_cols=8, seed=3)
    for alpha in (0.05, 0.3, 2.0):
        p = api.Plan(A, 64, "bf16", api.default_opts(mode="mixed", alpha=alpha, seg_len=24),
                     upload=False)
        st, d = p.stats(), p.export()
        wv, wt, wr = _path_work(d, st["opts"]["window_h"], st["opts"]["kt"])
        assert (st["work_vec"], st["work_tile"], st["work_winrem"]) == (wv, wt, wr)
        assert wv + wr + st["nnz_tiles"] == A.nnz


def test_adapt_next_matches_reference(lib):
    from oracle import cost_model as cm
    rng = np.random.default_rng(11)
    for _ in range(200):
        g = rng.uniform(0, 2)
        a0 = float(np.exp(rng.uniform(np.log(0.002), 0)))
        at = float(np.exp(rng.uniform(np.log(0.01), np.log(0.8))))
        st = api.adapt_state(a0)
        lo = hi = pa = ps = 0.0
        rounds = capped = 0
        for _ in range(9):
            alpha = st.alpha
            a_meas = min(1.0, at * (at / alpha) ** g * float(np.exp(rng.uniform(-0.05, 0.05))))
            # epoch times that measure P_vec = a_meas, P_mat = 1 (per second)
            t_vec, t_mat, wr = 2.0, 3.0, 0.5e-3 * a_meas
            w_vec = a_meas * t_vec * 1e-3
            w_tile = (t_mat * 1e-3 - wr / a_meas) * 1.0
            api.adapt_next(st, t_vec, t_mat, w_vec, w_tile, wr, 0.0, 0.0, 0.05)
            p_vec, p_mat = cm.path_throughputs(t_vec * 1e-3, t_mat * 1e-3, w_vec, w_tile, wr,
                                               0.0, 0.0)
            nxt, lo, hi, rounds, a_s, s, replan, capped = cm.adapt_next(
                alpha, lo, hi, rounds, pa, ps, capped, p_vec, p_mat, 0.05)
            assert st.alpha_star == pytest.approx(a_s, rel=1e-12)
            assert st.skew == pytest.approx(s, rel=1e-12)
            assert bool(st.replanned) == replan
            if not replan:
                assert st.converged == int(s <= 1.05)
                break
            assert st.alpha == pytest.approx(nxt, rel=1e-12)
            assert (st.lo, st.hi, st.rounds, st.capped) == (lo, hi, rounds, capped)
            pa, ps = alpha, a_s
        assert st.converged


def test_adapt_loop_on_plans(lib):
    """The host loop on real plans with a model device whose per-path rates
    are fixed: one re-partition reaches the crossover, and the plan's split
    follows the threshold."""
    A, _ = synth.block_community(n=4096, band=8, n_cols=8, seed=3)
    n, pv, pm = 64, 3.0e11, 2.0e12
    for a0 in (0.9, 0.01):
        st = api.adapt_state(a0)
        tiles = []
        for epoch in range(9):
            p = api.Plan(A, n, "bf16", api.default_opts(mode="mixed", alpha=st.alpha),
                         upload=False)
            s = p.stats()
            tiles.append(s["tiles"])
            t_vec = s["work_vec"] * n / pv * 1e3
            t_mat = (s["work_tile"] * n / pm + s["work_winrem"] * n / pv) * 1e3
            api.adapt_next(st, t_vec, t_mat, s["work_vec"] * n, s["work_tile"] * n,
                           s["work_winrem"] * n, pv, pm, 0.05)
            if not st.replanned:
                break
        assert st.converged and epoch <= 7
        assert abs(np.log(st.alpha / (pv / pm))) <= np.log(1.05) + 1e-12
        if a0 == 0.9:  # no tile is that dense; at the crossover most are kept
            assert tiles[0] == 0 and tiles[-1] > 0


def test_adapt_next_keeps_the_last_measured_rate(lib):
    st = api.adapt_state(0.3)
    # both paths measured: P_vec = 1e9, P_mfma = 4e9 per second -> alpha* = 0.25
    api.adapt_next(st, 1.0, 1.0, 1e6, 4e6, 0.0, 5e8, 1e12, 0.05)
    assert st.alpha_star == pytest.approx(0.25) and st.p_mfma == pytest.approx(4e9)
    # no tiles in this epoch: the last measured P_mfma, not the dry run's
    api.adapt_next(st, 1.0, 0.0, 1e6, 0.0, 0.0, 5e8, 1e12, 0.05)
    assert st.alpha_star == pytest.approx(0.25) and st.converged
    # a fresh state without measurements takes the dry run
    st2 = api.adapt_state(0.3)
    api.adapt_next(st2, 1.0, 0.0, 1e6, 0.0, 0.0, 5e8, 1e12, 0.05)
    assert st2.p_mfma == 1e12 and st2.alpha_star == pytest.approx(1e9 / 1e12)


@pytest.mark.parametrize("order,local", [("original_ranges", 0), ("compacted", 0), ("clustered", 0),
                                         ("compacted", 64), ("clustered", 256)])
def test_plan_same_for_any_thread_count(order, local, monkeypatch):
    """The column stage, the remainder and the local reordering run ranges of
    windows, rows or clusters on threads and append their output in order:
    the plan is the same array for array whatever the thread count
    (SPMM_PLAN_THREADS)."""
    A, _ = synth.block_community(n=8192, band=8, n_cols=8, seed=3)
    A = synth.permute_rows(A, 4) if local else A
    kw = dict(mode="mixed", row_order=order, seg_len=16, alpha=0.05, local_reorder=local)
    dumps = []
    for nth in ("1", "5", "16"):
        monkeypatch.setenv("SPMM_PLAN_THREADS", nth)
        p = api.Plan(A, 8, "bf16", api.default_opts(**kw), upload=False)
        dumps.append(p.export())
    assert dumps[0]["tile_window"].size > 0
    for d in dumps[1:]:
        for key in dumps[0]:
            if isinstance(dumps[0][key], np.ndarray):
                assert np.array_equal(dumps[0][key], d[key]), key


def _exec_tables_ref(d):
    """The co-scheduling tables written out from their definition: window w
    owns the segments of its rows (consecutive ids from win_seg[w], in slot
    order); a window gets a slot, in window order, when it has partial items
    or rows split into segments."""
    W, H = d["windows"].shape
    S = d["seg_row"].size
    seg_win = np.full(S, -1, np.int32)
    win_dep = np.full(W, -1, np.int32)
    win_nsseg = np.zeros(W, np.int32)
    slot = 0
    for w in range(W):
        rows = [r for r in d["windows"][w] if r >= 0]
        ns = int(sum(d["nseg"][r] for r in rows))
        # the segments' rows, in slot order, are exactly the window's split rows
        got = d["seg_row"][d["win_seg"][w]: d["win_seg"][w] + ns]
        want = np.concatenate([np.full(d["nseg"][r], r, np.int32) for r in rows]) if rows else []
        assert np.array_equal(got, np.asarray(want, np.int32))
        seg_win[d["win_seg"][w]: d["win_seg"][w] + ns] = w
        win_nsseg[w] = ns
        if ns > 0 or d["win_part"][w + 1] > d["win_part"][w]:
            win_dep[w] = slot
            slot += 1
    return seg_win if W else np.zeros(0, np.int32), win_dep, win_nsseg, slot


@pytest.mark.parametrize("case", range(6))
def test_exec_tables_match_definition(lib, case):
    r = np.random.default_rng(900 + case)
    if case < 3:
        A = synth.chung_lu_graph(4000, 2.1, 16.0, 1500.0, 30 + case)
        opts = dict(mode="mixed", row_order="length_sorted", t_row=int(r.integers(4, 16)),
                    seg_len=int(r.choice([16, 40, 128])), window_h=int(r.choice([16, 32])))
    else:
        A = synth.random_csr(300, 9000, 0.2, 40 + case, val_kind="bf16", int_values=(-2, 2))
        opts = dict(mode="mixed", window_h=16, t_row=-1, alpha_c=0.0, alpha=0.22,
                    seg_len=int(r.choice([40, 200])))
    p = api.Plan(A, 64, "bf16", api.default_opts(**opts), upload=False)
    d = p.export()
    seg_win, win_dep, win_nsseg, n_dep = _exec_tables_ref(d)
    assert d["n_dep"] == n_dep and n_dep > 0
    assert np.array_equal(d["seg_win"], seg_win)
    assert np.array_equal(d["win_dep"], win_dep)
    assert np.array_equal(d["win_nsseg"], win_nsseg)
    # plain plans: no windows, no slots
    q = api.Plan(A, 64, "bf16", api.default_opts(mode="plain"), upload=False).export()
    assert q["n_dep"] == 0 and q["seg_win"].size == 0


def test_exec_option_range(lib):
    A = synth.random_csr(50, 50, 0.1, 3)
    for bad in (4, 9):
        assert _status(lib, A, opts=api.default_opts(exec=bad)) == L.SPMM_ERR_UNSUPPORTED
    # a cold policy needs the serial kernels
    assert _status(lib, A, opts=api.default_opts(mode="plain", cold_policy=2, pipeline=0,
                                                 exec=2)) == L.SPMM_ERR_UNSUPPORTED
    for ok in (1, 2, 3):
        assert _status(lib, A, opts=api.default_opts(exec=ok)) == L.SPMM_OK
    p = api.Plan(A, 8, "f32", None, upload=False)
    assert p.stats()["opts"]["exec"] == L.EXEC_TWO_GRIDS
