"""Pins for the numpy partition reference (NeutronSparse Sec. 5.2.2, Sec. 6.1):
hand-worked examples, the printed tie rules of Eq. 5, coverage, the
reduction cases and an FP64 re-execution of the decomposition."""
import os

import numpy as np
import pytest
import torch

from oracle import plan_ref as pr
from paper_2606_22482_amd import synth


def csr_from_dense_pattern(P, vals=None):
    m, k = P.shape
    rows, cols = np.nonzero(P)
    v = (np.arange(1, rows.size + 1, dtype=np.float32) if vals is None else vals)
    return synth.csr_from_coo(m, k, rows, cols, v, "f32")


def execute_plan_f64(plan, A, B, kind="bf16"):
    """Re-execute the decomposition in FP64: tiles from bitmap + packed values,
    remainder from its CSR entries."""
    C = np.zeros((A.m, B.shape[1]))
    Bd = B.astype(np.float64)
    tv = (plan.tile_vals.astype(np.uint32) << 16).view(np.float32).astype(np.float64) \
        if kind == "bf16" else plan.tile_vals.view(np.float16).astype(np.float64)
    for t in range(plan.tile_window.size):
        slots = plan.windows[plan.tile_window[t]]
        q = plan.tile_val_ptr[t]
        for s, r in enumerate(slots):
            word = int(plan.tile_bitmap[t, s])
            for j in range(plan.kt):
                if word >> j & 1:
                    assert r >= 0
                    C[r] += tv[q] * Bd[plan.tile_cols[t, j]]
                    q += 1
        assert q == plan.tile_val_ptr[t + 1]
    rows = np.repeat(np.arange(A.m), np.diff(A.rowptr))
    for p in plan.rem_src:
        C[rows[p]] += float(A.vals[p]) * Bd[A.colidx[p]]
    return C


def test_hand_example_one_dense_block():
    # rows 0..15 hold the dense block of columns 0..31 plus one private column 40+r
    P = np.zeros((32, 64), dtype=bool)
    P[:16, :32] = True
    for r in range(16):
        P[r, 40 + r] = True
    P[20, 3] = True   # a row outside the block, length 1
    A = csr_from_dense_pattern(P)
    plan = pr.build_plan(A.rowptr, A.colidx, A.vals, k=64, mode=pr.MODE_MIXED, window_h=16,
                         t_row=1, alpha_c=1 / 16, alpha=0.5, row_order=pr.ORDER_COMPACTED)
    # row stage: rows 0..15 (Len 33 > 1) pass; row 20 (Len 1 <= 1) stays vector
    assert plan.windows.shape == (1, 16)
    assert list(plan.windows[0]) == list(range(16))
    # column stage: columns 0..31 counted 16 > floor(16/16) = 1; private columns counted 1
    assert plan.tile_cols.shape == (1, 32)
    assert list(plan.tile_cols[0]) == list(range(32))
    assert np.all(plan.tile_bitmap == 0xFFFFFFFF)
    # remainder: one private entry per block row, the whole of row 20
    rem_rows = np.repeat(np.arange(32), np.diff(A.rowptr))[plan.rem_src]
    assert sorted(rem_rows.tolist()) == list(range(16)) + [20]
    assert set(A.colidx[plan.rem_src].tolist()) == set(range(40, 56)) | {3}
    assert list(plan.vector_rows) == list(range(16, 32))
    # packed values in row-major bit order: row r's 32 block values in column order
    want = np.concatenate([A.vals[A.rowptr[r]:A.rowptr[r] + 32] for r in range(16)])
    assert np.array_equal(plan.tile_vals, pr.f32_to_bf16_bits(want))


def test_eq5_ties():
    # Len == t_row -> vector (Len <= Thres); count == floor(alpha_c*H) -> vector;
    # density == alpha -> matrix engine.
    P = np.zeros((16, 32), dtype=bool)
    P[:8, :4] = True          # rows 0..7: Len 4
    P[8:12, :2] = True        # rows 8..11: Len 2 (tie with t_row = 2 -> vector)
    A = csr_from_dense_pattern(P)
    plan = pr.build_plan(A.rowptr, A.colidx, A.vals, k=32, mode=pr.MODE_MIXED, window_h=16,
                         t_row=2, alpha_c=8 / 16 - 1 / 16, alpha=32 / (16 * 32),
                         row_order=pr.ORDER_COMPACTED)
    # window = rows 0..7; columns 0..3 have count 8 > floor(7/16*16) = 7
    assert list(plan.windows[0][:8]) == list(range(8)) and np.all(plan.windows[0][8:] == -1)
    assert list(plan.tile_cols[0][:4]) == [0, 1, 2, 3]
    # tile nnz 32 == alpha * 16 * 32 -> kept
    assert plan.tile_val_ptr[-1] == 32
    # raise the column threshold to exactly the count: columns leave, window dissolves
    plan2 = pr.build_plan(A.rowptr, A.colidx, A.vals, k=32, mode=pr.MODE_MIXED, window_h=16,
                          t_row=2, alpha_c=8 / 16, alpha=0.0, row_order=pr.ORDER_COMPACTED)
    assert plan2.windows.shape[0] == 0 and plan2.rem_src.size == A.nnz
    # density just above the tile's: demoted
    plan3 = pr.build_plan(A.rowptr, A.colidx, A.vals, k=32, mode=pr.MODE_MIXED, window_h=16,
                          t_row=2, alpha_c=0.0, alpha=np.nextafter(np.float32(32 / 512),
                                                                    np.float32(1)),
                          row_order=pr.ORDER_COMPACTED)
    assert plan3.tile_window.size == 0


@pytest.mark.parametrize("order", [pr.ORDER_ORIGINAL_RANGES, pr.ORDER_COMPACTED,
                                   pr.ORDER_LENGTH_SORTED])
@pytest.mark.parametrize("H", [16, 32])
def test_coverage_and_reexecution(order, H):
    A = synth.random_csr(300, 200, 0.06, 3, int_values=(-2, 2), dup_frac=0.05, empty_rows=0.05)
    B = synth.int_dense(1, (200, 6), -8, 8)
    plan = pr.build_plan(A.rowptr, A.colidx, A.vals, k=200, mode=pr.MODE_MIXED, window_h=H,
                         t_row=8, alpha_c=1 / H, alpha=0.02, row_order=order, seg=7)
    assert np.all(pr.coverage(plan) == 1)
    assert plan.tile_window.size > 0
    ref = A  # integer values: every path is exact
    dense = np.zeros((A.m, A.k))
    np.add.at(dense, (np.repeat(np.arange(A.m), np.diff(A.rowptr)), A.colidx), A.vals)
    assert np.array_equal(execute_plan_f64(plan, ref, B), dense @ B.astype(np.float64))
    # every row is in exactly one kept window slot or in the vector rows
    in_win = plan.windows[plan.windows >= 0]
    assert np.unique(in_win).size == in_win.size
    assert np.array_equal(np.sort(np.concatenate([in_win, plan.vector_rows])),
                          np.arange(A.m))
    # segments: ceil(remainder length / seg) for rows longer than seg
    rem_len = np.diff(plan.rem_ptr)
    assert np.array_equal(plan.nseg, np.where(rem_len > 7, -(-rem_len // 7), 0))


def test_length_sorted_and_original_ranges_order():
    A = synth.random_csr(100, 100, 0.05, 4)
    lens = np.diff(A.rowptr)
    plan = pr.build_plan(A.rowptr, A.colidx, A.vals, k=100, mode=pr.MODE_MIXED, window_h=16,
                         t_row=-1, alpha_c=0.0, alpha=0.0, row_order=pr.ORDER_LENGTH_SORTED)
    order = sorted(range(100), key=lambda r: (-lens[r], r))
    got = [r for r in plan.windows.reshape(-1) if r >= 0]
    assert got == order
    plan = pr.build_plan(A.rowptr, A.colidx, A.vals, k=100, mode=pr.MODE_MIXED, window_h=16,
                         t_row=2, alpha_c=0.0, alpha=0.0, row_order=pr.ORDER_ORIGINAL_RANGES)
    for w, slots in enumerate(plan.windows):
        for s, r in enumerate(slots):
            assert r == -1 or r % 16 == s


def test_reductions_plain_and_mfma_only():
    A = synth.random_csr(200, 150, 0.05, 5, dup_frac=0.05)
    # alpha > 1: no tile can be kept, so the partition is the plain one
    p = pr.build_plan(A.rowptr, A.colidx, A.vals, k=150, mode=pr.MODE_MIXED, window_h=16,
                      t_row=-1, alpha_c=0.0, alpha=1.5)
    assert p.tile_window.size == 0 and np.array_equal(p.rem_src, np.arange(A.nnz))
    assert np.array_equal(p.vector_rows, np.arange(A.m))
    q = pr.build_plan(A.rowptr, A.colidx, A.vals, k=150, mode=pr.MODE_PLAIN)
    assert np.array_equal(q.rem_src, p.rem_src) and np.array_equal(q.rem_ptr, p.rem_ptr)
    # matrix engine only: every entry except repeated (row, col) pairs is in a tile
    z = pr.build_plan(A.rowptr, A.colidx, A.vals, k=150, mode=pr.MODE_MFMA_ONLY, window_h=16)
    rows = np.repeat(np.arange(A.m), np.diff(A.rowptr))
    key = rows * 150 + A.colidx
    _, first = np.unique(key, return_index=True)
    assert z.tile_src.size == first.size
    assert np.array_equal(np.sort(z.rem_src), np.setdiff1d(np.arange(A.nnz), first))


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([
        rng.standard_normal(100000).astype(np.float32),
        (rng.integers(0, 2**32, 100000, dtype=np.uint64).astype(np.uint32)).view(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 3.4e38],
                 dtype=np.float32),
    ])
    x = x[~np.isnan(x)]
    ours = pr.f32_to_bf16_bits(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)
    # NaN stays NaN
    nan_bits = pr.f32_to_bf16_bits(np.array([np.nan], dtype=np.float32))[0]
    assert (nan_bits & 0x7F80) == 0x7F80 and (nan_bits & 0x7F) != 0


# ---- Sec. 6.1 local reordering ------------------------------------------------------------

def _csr_rows(rows):
    rp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int64)
    ci = np.array([c for r in rows for c in r], dtype=np.int64)
    return rp, ci


def test_jaccard_values():
    from fractions import Fraction
    assert pr.jaccard({1, 2}, {2, 3}) == Fraction(1, 3)
    assert pr.jaccard({1, 2}, {1, 2}) == 1
    assert pr.jaccard(set(), set()) == 0 and pr.jaccard({4}, set()) == 0


def test_local_reorder_hand_example():
    # H = 2, one cluster of 4 rows: windows [r0 r1] [r2 r3] give anchors r0
    # (longest of window 0) and then r3 (the only unassigned row of window 1).
    # J(r0, r1) = 0, J(r0, r2) = 2/3, J(r0, r3) = 0 -> {r0, r2};
    # J(r3, r1) = 1/3 -> {r3, r1}.
    rp, ci = _csr_rows([[1, 2, 3], [7, 8], [1, 2], [7, 9]])
    assert pr.local_reorder([0, 1, 2, 3], 2, 4, rp, ci) == [[0, 2], [3, 1]]
    # clusters of 2 rows: no row may leave its cluster; in [r2 r3] both have
    # length 2, so the earlier one is the anchor
    assert pr.local_reorder([0, 1, 2, 3], 2, 2, rp, ci) == [[0, 1], [2, 3]]


def test_local_reorder_recovers_planted_groups():
    """32 rows in 4 planted groups of 8 (shared columns plus one private
    column each), shuffled: every rebuilt window is exactly one group."""
    rng = np.random.default_rng(7)
    rows, group = [], []
    for g in range(4):
        base = list(range(100 * g, 100 * g + 10))
        for j in range(8):
            rows.append(base + [1000 + 8 * g + j])
            group.append(g)
    perm = rng.permutation(32)
    rows = [rows[i] for i in perm]
    group = [group[i] for i in perm]
    rp, ci = _csr_rows(rows)
    wins = pr.local_reorder(list(range(32)), 8, 32, rp, ci)
    assert len(wins) == 4
    for w in wins:
        assert len({group[r] for r in w}) == 1 and len(w) == 8


def test_local_reorder_is_a_partition():
    A = synth.random_csr(300, 200, 0.05, 3)
    D = [r for r in range(A.m) if A.rowptr[r + 1] - A.rowptr[r] > 4]
    for H, C in [(16, 64), (16, 48), (32, 96), (16, 1000)]:
        wins = pr.local_reorder(D, H, C, A.rowptr, A.colidx)
        flat = [r for w in wins for r in w if r >= 0]
        assert sorted(flat) == sorted(D) and all(len(w) == H for w in wins)
        # rows never leave their cluster
        where = {r: i // C for i, r in enumerate(D)}
        for w in wins:
            assert len({where[r] for r in w if r >= 0}) == 1


def test_local_reorder_raises_tile_density():
    """Shuffled community rows: the rebuilt windows keep more entries in
    tiles at a higher density than the shuffled order (Sec. 8.4 measure)."""
    A, _ = synth.block_community(n=2048, band=4, n_cols=8, seed=5)
    rng = np.random.default_rng(1)
    perm = rng.permutation(A.m)
    rows = [A.colidx[A.rowptr[r]:A.rowptr[r + 1]].tolist() for r in perm]
    rp, ci = _csr_rows(rows)
    vals = np.ones(ci.size, dtype=np.float32)
    kw = dict(k=A.k, mode=pr.MODE_MIXED, window_h=16, t_row=1, alpha_c=1 / 16, alpha=1 / 16,
              row_order=pr.ORDER_COMPACTED)
    before = pr.build_plan(rp, ci, vals, **kw)
    after = pr.build_plan(rp, ci, vals, local_reorder_rows=256, **kw)
    assert after.stats["nnz_tiles"] > 2 * before.stats["nnz_tiles"]
    assert after.stats["mean_tile_density"] > before.stats["mean_tile_density"]


# ---- Sec. 6.1 global stage (Rabbit Order on the bipartite row-column graph) ------------------

def _modularity(edges, n, comm):
    """Q from its definition: (1/2M) sum_ij [A_ij - d_i d_j / 2M] [c_i == c_j],
    A the symmetric adjacency (multi-edges counted)."""
    A = np.zeros((n, n))
    for a, b in edges:
        A[a, b] += 1
        A[b, a] += 1
    d = A.sum(axis=1)
    two_m = A.sum()
    same = np.equal.outer(comm, comm)
    return float(((A - np.outer(d, d) / two_m) * same).sum() / two_m)


def test_rabbit_gain_is_the_modularity_gain():
    """The integer gain w_uv * 2M - d_u * d_v is (Q_after - Q_before) * (2M)^2 / 2
    for merging two communities, Q computed by brute force."""
    rng = np.random.default_rng(4)
    m, k = 7, 6
    edges = [(int(r), m + int(c)) for r, c in zip(rng.integers(0, m, 30), rng.integers(0, k, 30))]
    n = m + k
    comm = np.arange(n)
    comm[[0, 3]] = 0          # a few communities already merged
    comm[[m + 1, m + 4]] = m + 1
    d = np.zeros(n)
    for a, b in edges:
        d[a] += 1
        d[b] += 1
    two_m = 2 * len(edges)
    for cu, cv in [(0, m + 1), (2, m + 1), (0, 5)]:
        before = _modularity(edges, n, comm)
        merged = np.where(comm == cu, cv, comm)
        after = _modularity(edges, n, merged)
        w = sum(1 for a, b in edges if (comm[a], comm[b]) in ((cu, cv), (cv, cu)))
        du, dv = d[comm == cu].sum(), d[comm == cv].sum()
        assert (after - before) * two_m ** 2 / 2 == pytest.approx(w * two_m - du * dv, abs=1e-9)


def test_rabbit_order_hand_worked_example():
    """The clustering order on a 4 x 4 matrix of two interleaved communities,
    worked by hand from the algorithm's definition (tests/golden): pins the
    visit order, the exact gain comparison and its tie rule, and the
    depth-first walk of the merge tree."""
    import json
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rabbit_order_hand_example.json")))
    rank = pr.rabbit_order(np.array(g["rowptr"]), np.array(g["colidx"]), g["m"], g["k"])
    assert rank.tolist() == g["rank"]


def test_rabbit_order_keeps_components_together():
    """Two disconnected groups of rows (each a dense biclique on its own
    columns), interleaved: each group occupies a contiguous rank range."""
    rows = []
    for r in range(20):
        g = r % 2
        rows.append(list(range(10 * g, 10 * g + 6)))
    rp, ci = _csr_rows(rows)
    rank = pr.rabbit_order(rp, ci, 20, 20)
    assert sorted(rank.tolist()) == list(range(20))
    for g in range(2):
        rk = sorted(rank[g::2].tolist())
        assert rk[-1] - rk[0] == 9


def test_rabbit_order_recovers_shuffled_communities():
    A0, _ = synth.block_community(n=4096, band=8, n_cols=8, seed=5)
    A = synth.permute_rows(A0, 3)
    rank = pr.rabbit_order(A.rowptr, A.colidx, A.m, A.k)
    assert sorted(rank.tolist()) == list(range(A.m))
    kw = dict(k=A.k, mode=pr.MODE_MIXED, window_h=16, t_row=1, alpha_c=1 / 16, alpha=1 / 16)
    v = np.ones(A.nnz, dtype=np.float32)
    shuffled = pr.build_plan(A.rowptr, A.colidx, v, row_order=pr.ORDER_COMPACTED, **kw)
    clustered = pr.build_plan(A.rowptr, A.colidx, v, row_order=pr.ORDER_CLUSTERED, **kw)
    both = pr.build_plan(A.rowptr, A.colidx, v, row_order=pr.ORDER_CLUSTERED,
                         local_reorder_rows=256, **kw)
    assert clustered.stats["nnz_tiles"] > 4 * shuffled.stats["nnz_tiles"]
    assert both.stats["nnz_tiles"] > clustered.stats["nnz_tiles"]
    assert both.stats["mean_tile_density"] > shuffled.stats["mean_tile_density"]
