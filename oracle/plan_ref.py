"""Reference for the integer partition of A (TEST INFRASTRUCTURE ONLY).

Written from NeutronSparse Sec. 5.2.2 (two-stage row-column extraction,
Eq. 4-5), Sec. 5.1 / Sec. 5.2.1 (tiles whose density is below alpha go to the
vector engine), Sec. 6.1 (row windows whose height is the tile height; empty
columns of a window are compacted away when its tiles are built) and the
storage choice at the end of Sec. 5.2.2 (the matrix-engine core as a bitmap,
the vector-engine fringes as index/value lists).

Readings where the paper is silent (each is listed in the design notes):

* Two thresholds.  The row stage compares Len(row) with an absolute row
  length ``t_row`` (Eq. 5 with Thres = alpha * K, K = the row dimension, so
  t_row = alpha_row * K).  The column stage is applied per row window, with
  the window height H as the "vector dimension" of Eq. 5, so a column of a
  window goes to the matrix engine iff its count in that window exceeds
  floor(alpha_c * H).  A tile is kept iff its density nnz / (H * Kt) is at
  least alpha (Sec. 5.2.1: below alpha -> vector engine).
* Ties follow Eq. 5 as printed: Len <= Thres -> vector; density >= alpha ->
  matrix engine.
* Bitmap: one Kt-bit word per window row, bit j <-> the j-th column of the
  tile, least significant bit first; the packed values follow the set bits
  in row-major order.  A (row, column) pair stored twice in the CSR puts its
  first occurrence in the tile and the rest in the remainder.
* A window that keeps no tile is dissolved: its rows are plain vector rows.
* Remainder rows longer than ``seg`` entries are cut into consecutive
  segments of ``seg`` entries (the last one shorter).

Row orders for forming windows: ``original_ranges`` (fixed ranges [wH, wH+H),
rows failing the row stage leave holes), ``compacted`` (rows passing the row
stage, in their original order) and ``length_sorted`` (by Len descending,
ties by row id), the last being the degree-grouping the local reordering of
Sec. 6.1 starts from.

Local reordering (Sec. 6.1, ``local_reorder`` = rows per cluster, rounded up
to a multiple of H): the row list is cut into clusters of consecutive rows;
inside a cluster the current windows are visited in order, one
representative row of each -- read as its longest unassigned row, ties to the
earlier one -- becomes an anchor, and the anchor takes the H-1 unassigned
rows of the cluster most similar to it by Jaccard similarity of their
distinct column sets (ties to the earlier row; an empty union counts as 0).
Rows left unassigned after all windows were visited form windows in list
order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

ORDER_ORIGINAL_RANGES = 1
ORDER_COMPACTED = 2
ORDER_LENGTH_SORTED = 3
ORDER_CLUSTERED = 4

MODE_PLAIN = 1
MODE_MIXED = 2
MODE_MFMA_ONLY = 3


def Len(rowptr: np.ndarray) -> np.ndarray:
    """Eq. 4: the number of stored entries of each row."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    return rowptr[1:] - rowptr[:-1]


def row_stage(rowptr: np.ndarray, t_row: int) -> np.ndarray:
    """Eq. 5, row stage: True for rows that go on to the matrix-engine
    candidate set (Len > Thres); rows with Len <= Thres stay on the vector
    path."""
    return Len(rowptr) > t_row


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round binary32 to bfloat16 with round-to-nearest, ties to even, written
    from the definition: keep the top 16 bits, add half an ulp of the kept
    part plus the kept part's lowest bit as the tie-breaker; NaNs stay quiet
    NaNs."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) & np.uint64(0xFFFF)
    nan = np.isnan(np.ascontiguousarray(x, dtype=np.float32))
    r = np.where(nan, ((u >> np.uint64(16)) | np.uint64(0x40)) & np.uint64(0xFFFF), r)
    return r.astype(np.uint16)


@dataclass
class PlanRef:
    m: int
    k: int
    nnz: int
    window_h: int
    kt: int
    seg: int
    windows: np.ndarray            # int32 [W_kept, H]: original row per slot, -1 = empty slot
    tile_window: np.ndarray        # int32 [T]: index of the kept window owning the tile
    tile_cols: np.ndarray          # int32 [T, Kt]: compacted columns, -1 = padding
    tile_bitmap: np.ndarray        # uint32 [T, H]: one word per window slot
    tile_val_ptr: np.ndarray       # int64 [T+1]: offsets into tile_vals / tile_src
    tile_vals: np.ndarray          # uint16 bit patterns (bf16 or f16)
    tile_src: np.ndarray           # int64: CSR entry index of each packed value
    rem_ptr: np.ndarray            # int64 [M+1]
    rem_src: np.ndarray            # int64: CSR entry index of each remainder entry
    vector_rows: np.ndarray        # int32: rows not covered by a kept window (ascending)
    nseg: np.ndarray               # int32 [M]: segments of each row's remainder (0 if <= seg)
    stats: dict = field(default_factory=dict)


def rabbit_order(rowptr, colidx, m, k):
    """Global clustering order of the rows (Sec. 6.1, global stage), from the
    published Rabbit Order algorithm (community detection by incremental
    aggregation, then a depth-first walk of the merge dendrogram), applied
    to the bipartite graph of A: vertices 0..m-1 are rows, m..m+k-1 columns,
    one unit-weight edge per stored entry.

    Vertices are visited once, in increasing degree (ties: lower id).  A
    visited vertex u is the root of its community (whatever merged into it
    so far); it joins the neighbouring community v with the largest
    modularity gain, 2 * (w_uv / 2M - d_u * d_v / (2M)^2) > 0, compared
    exactly as w_uv * 2M - d_u * d_v (ties: lower root id), where w_uv counts
    the edges between the two communities, d the summed degrees and M the
    edge count; otherwise it stays a root.  The order lists the roots in the
    order they were visited, each followed depth first by what merged into
    it, children in the order they merged.  Returns the rank of each row in
    that order (rows only)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    n = m + k
    nnz = int(rowptr[-1])
    adj = [[] for _ in range(n)]
    for r in range(m):
        for p in range(rowptr[r], rowptr[r + 1]):
            c = m + int(colidx[p])
            adj[r].append(c)
            adj[c].append(r)
    two_m = 2 * nnz
    deg = [len(a) for a in adj]
    parent = list(range(n))
    members = [[v] for v in range(n)]
    children = [[] for _ in range(n)]

    def find(v):
        while parent[v] != v:
            v = parent[v]
        return v

    visited_roots = []
    for u in sorted(range(n), key=lambda v: (deg[v], v)):
        w = {}
        for x in members[u]:
            for y in adj[x]:
                ry = find(y)
                if ry != u:
                    w[ry] = w.get(ry, 0) + 1
        best, best_gain = -1, 0
        for v in sorted(w):
            gain = w[v] * two_m - deg[u] * deg[v]
            if gain > best_gain:
                best, best_gain = v, gain
        if best < 0:
            visited_roots.append(u)
            continue
        parent[u] = best
        children[best].append(u)
        members[best].extend(members[u])
        deg[best] += deg[u]
    order = []
    for root in [v for v in visited_roots if parent[v] == v]:
        stack = [root]
        while stack:
            v = stack.pop()
            order.append(v)
            stack.extend(reversed(children[v]))
    rank = np.empty(m, dtype=np.int64)
    pos = 0
    for v in order:
        if v < m:
            rank[v] = pos
            pos += 1
    return rank


def jaccard(a: set, b: set) -> Fraction:
    """|a & b| / |a | b| as an exact fraction (0 when both are empty)."""
    union = len(a | b)
    return Fraction(len(a & b), union) if union else Fraction(0)


def local_reorder(D, H, cluster_rows, rowptr, colidx):
    """Windows (lists of H slots, -1 padded) of the rows in D after the local
    reordering of Sec. 6.1 (see the module docstring)."""
    out = []
    for c0 in range(0, len(D), cluster_rows):
        cluster = list(D[c0:c0 + cluster_rows])
        colsets = [set(int(c) for c in colidx[rowptr[r]:rowptr[r + 1]]) for r in cluster]
        length = [int(rowptr[r + 1] - rowptr[r]) for r in cluster]
        unassigned = set(range(len(cluster)))
        for w0 in range(0, len(cluster), H):
            members = [i for i in range(w0, min(w0 + H, len(cluster))) if i in unassigned]
            if not members:
                continue
            anchor = min(members, key=lambda i: (-length[i], i))
            unassigned.discard(anchor)
            ranked = sorted(unassigned, key=lambda i: (-jaccard(colsets[anchor], colsets[i]), i))
            picked = ranked[:H - 1]
            for i in picked:
                unassigned.discard(i)
            window = [cluster[anchor]] + [cluster[i] for i in picked]
            out.append(window + [-1] * (H - len(window)))
        rest = [cluster[i] for i in sorted(unassigned)]
        for w in range(0, len(rest), H):
            chunk = rest[w:w + H]
            out.append(chunk + [-1] * (H - len(chunk)))
    return out


def build_plan(rowptr, colidx, vals, *, k: int, mode: int, window_h: int = 16, t_row: int = 0,
               alpha_c: float = 1.0 / 16, alpha: float = 0.0, kt: int = 32,
               row_order: int = ORDER_LENGTH_SORTED, seg: int = 256,
               tile_kind: str = "bf16", val_kind: str = "f32",
               local_reorder_rows: int = 0) -> PlanRef:
    """Build the partition of A for the given options (see module docstring).

    ``vals`` holds the stored values: float32, or uint16 bit patterns for
    ``val_kind`` "bf16" / "f16".  Tile values are the stored values rounded
    to ``tile_kind`` ("bf16": RNE from f32, unchanged from bf16; "f16":
    unchanged from f16).
    """
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    m = rowptr.size - 1
    nnz = int(rowptr[-1])
    H = int(window_h)
    if mode == MODE_MFMA_ONLY:
        t_row, alpha_c, alpha = -1, 0.0, 0.0
    lens = Len(rowptr)

    # ---- row stage + windows -------------------------------------------------
    windows = []
    if mode != MODE_PLAIN:
        inD = row_stage(rowptr, t_row)
        if row_order == ORDER_ORIGINAL_RANGES:
            for w in range((m + H - 1) // H):
                slots = [r if (r < m and inD[r]) else -1 for r in range(w * H, w * H + H)]
                windows.append(slots)
        else:
            D = [r for r in range(m) if inD[r]]
            if row_order == ORDER_LENGTH_SORTED:
                D.sort(key=lambda r: (-int(lens[r]), r))
            elif row_order == ORDER_CLUSTERED:
                rank = rabbit_order(rowptr, colidx, m, k)
                D.sort(key=lambda r: int(rank[r]))
            elif row_order != ORDER_COMPACTED:
                raise ValueError("unknown row order")
            if local_reorder_rows > 0:
                crows = (local_reorder_rows + H - 1) // H * H
                windows = local_reorder(D, H, crows, rowptr, colidx)
            else:
                for w in range(0, len(D), H):
                    chunk = D[w:w + H]
                    windows.append(chunk + [-1] * (H - len(chunk)))

    # ---- column stage, K-tiles, density test, packing -----------------------
    col_thr = math.floor(float(np.float32(alpha_c)) * H)
    keep_thr = float(np.float32(alpha)) * float(H * kt)
    in_tile = np.zeros(nnz, dtype=bool)
    kept_windows, t_window, t_cols, t_bitmap, t_ptr, t_src = [], [], [], [], [0], []
    for slots in windows:
        cnt = {}
        for r in slots:
            if r < 0:
                continue
            for p in range(rowptr[r], rowptr[r + 1]):
                c = int(colidx[p])
                cnt[c] = cnt.get(c, 0) + 1
        mcols = sorted(c for c, n in cnt.items() if n > col_thr)
        w_tiles = []
        for j0 in range(0, len(mcols), kt):
            tc = mcols[j0:j0 + kt]
            if float(sum(cnt[c] for c in tc)) >= keep_thr:
                w_tiles.append(tc)
        if not w_tiles:
            continue  # dissolved window: its rows stay on the vector path
        widx = len(kept_windows)
        kept_windows.append(slots)
        for tc in w_tiles:
            pos = {c: j for j, c in enumerate(tc)}
            bitmap = np.zeros(H, dtype=np.uint32)
            src = []
            for s, r in enumerate(slots):
                if r < 0:
                    continue
                seen = {}
                for p in range(rowptr[r], rowptr[r + 1]):
                    c = int(colidx[p])
                    if c in pos and c not in seen:
                        seen[c] = p
                for j, c in enumerate(tc):
                    if c in seen:
                        bitmap[s] |= np.uint32(1 << j)
                        src.append(seen[c])
                        in_tile[seen[c]] = True
            t_window.append(widx)
            t_cols.append(tc + [-1] * (kt - len(tc)))
            t_bitmap.append(bitmap)
            t_src.extend(src)
            t_ptr.append(len(t_src))

    # ---- tile values ---------------------------------------------------------
    t_src_arr = np.asarray(t_src, dtype=np.int64)
    vals = np.asarray(vals)
    if t_src_arr.size:
        picked = vals[t_src_arr]
        if tile_kind == "bf16":
            if val_kind == "f32":
                tvals = f32_to_bf16_bits(picked.astype(np.float32))
            elif val_kind == "bf16":
                tvals = picked.view(np.uint16) if picked.dtype != np.uint16 else picked
            else:
                raise ValueError("bf16 tiles need f32 or bf16 values")
        elif tile_kind == "f16":
            if val_kind != "f16":
                raise ValueError("f16 tiles need f16 values")
            tvals = picked.view(np.uint16) if picked.dtype != np.uint16 else picked
        else:
            raise ValueError("tile kind")
        tvals = np.ascontiguousarray(tvals, dtype=np.uint16)
    else:
        tvals = np.zeros(0, dtype=np.uint16)

    # ---- remainder, vector rows, segments -------------------------------------
    keep_mask = ~in_tile
    rem_src = np.nonzero(keep_mask)[0].astype(np.int64)
    row_of = np.repeat(np.arange(m, dtype=np.int64), lens)
    rem_len = np.bincount(row_of[rem_src], minlength=m) if nnz else np.zeros(m, dtype=np.int64)
    rem_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(rem_len, out=rem_ptr[1:])
    covered = np.zeros(m, dtype=bool)
    for slots in kept_windows:
        for r in slots:
            if r >= 0:
                covered[r] = True
    vector_rows = np.nonzero(~covered)[0].astype(np.int32)
    nseg = np.where(rem_len > seg, (rem_len + seg - 1) // seg, 0).astype(np.int32)

    T = len(t_window)
    plan = PlanRef(
        m=m, k=int(k), nnz=nnz, window_h=H, kt=kt, seg=seg,
        windows=np.asarray(kept_windows, dtype=np.int32).reshape(-1, H),
        tile_window=np.asarray(t_window, dtype=np.int32),
        tile_cols=np.asarray(t_cols, dtype=np.int32).reshape(T, kt),
        tile_bitmap=np.asarray(t_bitmap, dtype=np.uint32).reshape(T, H),
        tile_val_ptr=np.asarray(t_ptr, dtype=np.int64),
        tile_vals=tvals,
        tile_src=t_src_arr,
        rem_ptr=rem_ptr,
        rem_src=rem_src,
        vector_rows=vector_rows,
        nseg=nseg,
    )
    plan.stats = {
        "nnz_tiles": int(t_src_arr.size),
        "nnz_remainder": int(rem_src.size),
        "windows": int(plan.windows.shape[0]),
        "tiles": T,
        "mean_tile_density": (t_src_arr.size / (T * H * kt)) if T else 0.0,
    }
    return plan


def coverage(plan: PlanRef) -> np.ndarray:
    """How many times each CSR entry is placed (tile slot or remainder).  The
    partition is complete and disjoint iff every count is exactly 1."""
    cnt = np.zeros(plan.nnz, dtype=np.int64)
    np.add.at(cnt, plan.tile_src, 1)
    np.add.at(cnt, plan.rem_src, 1)
    return cnt
