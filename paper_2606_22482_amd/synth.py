"""Seeded synthetic inputs shaped like the paper's workloads.

The paper evaluates on GNN graphs and SuiteSparse matrices (Sec. 8.1,
Table 2) that are not available here; these generators are stand-ins with the
shapes, value distributions and structure of the workloads this library is
measured on.  They contain none of the SpMM method's arithmetic: they only
draw random structure and values, and are shared by the tests, the
benchmark and the oracle's callers.

All generators use ``numpy.random.default_rng`` with sub-streams spawned from
``SeedSequence(seed)``, so a (config, seed) pair always yields the same bits.
16-bit values are produced as uint16 bit patterns by the libraries' own
round-to-nearest-even conversions (numpy for f16, torch for bf16).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class CSR:
    m: int
    k: int
    rowptr: np.ndarray   # int64 [m+1]
    colidx: np.ndarray   # int32 [nnz]
    vals: np.ndarray     # float32, or uint16 bit patterns for bf16 / f16
    val_kind: str        # "f32" | "bf16" | "f16"

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def _rngs(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bfloat16 bit patterns via torch's conversion (RNE)."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(torch.bfloat16)
    return t.view(torch.int16).numpy().view(np.uint16).copy()


def to_f16_bits(x: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.float32).astype(np.float16).view(np.uint16)


def dense_values(rng, shape, kind: str) -> np.ndarray:
    """N(0,1) values stored in ``kind``."""
    x = rng.standard_normal(shape, dtype=np.float32)
    if kind == "f32":
        return x
    if kind == "bf16":
        return to_bf16_bits(x)
    if kind == "f16":
        return to_f16_bits(x)
    raise ValueError(kind)


def uniform_values(rng, n, kind: str, lo=-1.0, hi=1.0) -> np.ndarray:
    x = rng.uniform(lo, hi, size=n).astype(np.float32)
    if kind == "f32":
        return x
    if kind == "bf16":
        return to_bf16_bits(x)
    if kind == "f16":
        return to_f16_bits(x)
    raise ValueError(kind)


def csr_from_coo(m: int, k: int, rows: np.ndarray, cols: np.ndarray, vals: np.ndarray,
                 val_kind: str) -> CSR:
    """Stable sort by (row, col) into CSR; duplicates are kept as entries."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    order = np.lexsort((cols, rows))
    counts = np.bincount(rows, minlength=m)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return CSR(m, k, rowptr, cols[order].astype(np.int32), np.asarray(vals)[order], val_kind)


# --------------------------------------------------------------------------------------------
# Plain uniform matrix: 16 distinct random columns per row.
# --------------------------------------------------------------------------------------------
def uniform_rows(m=4096, k=4096, per_row=16, n=32, seed=1, val_kind="f32", b_kind="f32"):
    """A m x k with exactly ``per_row`` distinct uniformly random columns per
    row (sorted), values U(-1,1); B k x n N(0,1)."""
    r_struct, r_val, r_b = _rngs(seed, 3)
    cols = np.empty((m, per_row), dtype=np.int64)
    for i in range(m):
        cols[i] = np.sort(r_struct.choice(k, size=per_row, replace=False))
    rowptr = np.arange(0, m * per_row + 1, per_row, dtype=np.int64)
    vals = uniform_values(r_val, m * per_row, val_kind)
    A = CSR(m, k, rowptr, cols.reshape(-1).astype(np.int32), vals, val_kind)
    B = dense_values(r_b, (k, n), b_kind)
    return A, B


# --------------------------------------------------------------------------------------------
# Chung-Lu power-law graphs.
# --------------------------------------------------------------------------------------------
def chung_lu_weights(n: int, gamma: float, mean: float, wmax: float) -> np.ndarray:
    """Expected degrees w_i = c (i + i0)^(-1/(gamma-1)), with i0 found by
    bisection so that w_0 / mean(w) = wmax / mean, and c so that mean(w) =
    mean.  (Degree exponent gamma <-> rank exponent 1/(gamma-1).)"""
    beta = 1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)
    target = wmax / mean

    def ratio(i0):
        f = (i + i0) ** (-beta)
        return f[0] / f.mean()

    lo, hi = 1e-6, float(n)
    if ratio(lo) < target:   # even the steepest profile cannot reach wmax
        i0 = lo
    else:
        for _ in range(200):
            mid = math.sqrt(lo * hi)
            if ratio(mid) > target:
                lo = mid
            else:
                hi = mid
        i0 = math.sqrt(lo * hi)
    f = (i + i0) ** (-beta)
    return f * (mean / f.mean())


def chung_lu_graph(n: int, gamma: float, mean: float, wmax: float, seed: int, *,
                   val_kind="f32", values="sym_norm"):
    """Symmetric Chung-Lu graph on n vertices.

    E = round(sum(w)/2) endpoint pairs are drawn with both endpoints
    proportional to w; self-loops are dropped, duplicate edges merged, the
    edge set symmetrised, and vertex ids randomly permuted.  Values are
    1/sqrt(d_i d_j) with the realised degrees (``values="sym_norm"``, the GCN
    normalisation without self loops) or U(-1,1) (``values="uniform"``).
    """
    r_pair, r_perm, r_val = _rngs(seed, 3)
    w = chung_lu_weights(n, gamma, mean, wmax)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    e = int(round(w.sum() / 2.0))
    u = np.searchsorted(cdf, r_pair.random(e), side="right")
    v = np.searchsorted(cdf, r_pair.random(e), side="right")
    np.minimum(u, n - 1, out=u)
    np.minimum(v, n - 1, out=v)
    keep = u != v
    u, v = u[keep], v[keep]
    perm = r_perm.permutation(n)
    u, v = perm[u], perm[v]
    key = np.unique(np.concatenate([u * n + v, v * n + u]))
    rows = key // n
    cols = key % n
    deg = np.bincount(rows, minlength=n).astype(np.float64)
    if values == "sym_norm":
        vals = (1.0 / np.sqrt(deg[rows] * deg[cols])).astype(np.float32)
        if val_kind == "bf16":
            vals = to_bf16_bits(vals)
        elif val_kind == "f16":
            vals = to_f16_bits(vals)
    else:
        vals = uniform_values(r_val, rows.size, val_kind)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return CSR(n, n, rowptr, cols.astype(np.int32), vals, val_kind)


def gnn_graph(n=1 << 20, n_cols=128, seed=2, b_kind="f32"):
    """GNN aggregation workload: Chung-Lu (exponent 2.1, mean degree 16,
    max expected degree 20,000), symmetric-normalised f32 values; B n x n_cols
    N(0,1)."""
    A = chung_lu_graph(n, 2.1, 16.0, 20000.0, seed, val_kind="f32")
    (r_b,) = _rngs(seed + 1000, 1)
    B = dense_values(r_b, (n, n_cols), b_kind)
    return A, B


# --------------------------------------------------------------------------------------------
# Block-community matrix.
# --------------------------------------------------------------------------------------------
def block_community(n=262144, block=16, blocks_per_row=8, band=32, fill=0.3, off_block=2,
                    n_cols=256, seed=3, val_kind="f32", b_kind="bf16"):
    """16x16 blocks along a banded community structure: each block-row picks
    ``blocks_per_row`` distinct block-columns uniformly from the band
    {r-band, ..., r+band-1} (mod the block count); every slot of a chosen
    block is present independently with probability ``fill``; each row also
    gets ``off_block`` uniformly random columns outside its blocks (redrawn on
    collision).  Values U(-1,1); B n x n_cols N(0,1)."""
    r_blk, r_fill, r_off, r_val, r_b = _rngs(seed, 5)
    nb = n // block
    width = 2 * band
    bc = np.empty((nb, blocks_per_row), dtype=np.int64)
    for br in range(nb):
        pick = r_blk.choice(width, size=blocks_per_row, replace=False)
        bc[br] = (br - band + pick) % nb
    rows_l, cols_l = [], []
    # block entries
    present = r_fill.random((nb, blocks_per_row, block, block)) < fill
    br_i, b_i, ri, ci = np.nonzero(present)
    rows_blk = br_i * block + ri
    cols_blk = bc[br_i, b_i] * block + ci
    rows_l.append(rows_blk)
    cols_l.append(cols_blk)
    # off-block entries, redrawn until they avoid the row's blocks and each other
    own = np.zeros((n, blocks_per_row), dtype=np.int64)
    own[:] = np.repeat(bc, block, axis=0)
    off = r_off.integers(0, n, size=(n, off_block))
    for _ in range(1000):
        bad = np.zeros(off.shape, dtype=bool)
        for j in range(off_block):
            bad[:, j] = np.any((off[:, j:j + 1] // block) == own, axis=1)
            for jj in range(j):
                bad[:, j] |= off[:, j] == off[:, jj]
        if not bad.any():
            break
        off[bad] = r_off.integers(0, n, size=int(bad.sum()))
    rows_l.append(np.repeat(np.arange(n, dtype=np.int64), off_block))
    cols_l.append(off.reshape(-1))
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = uniform_values(r_val, rows.size, val_kind)
    A = csr_from_coo(n, n, rows, cols, vals, val_kind)
    B = dense_values(r_b, (n, n_cols), b_kind)
    return A, B


# --------------------------------------------------------------------------------------------
# Batched uneven matrices.
# --------------------------------------------------------------------------------------------
def permute_rows(A: "CSR", seed: int) -> "CSR":
    """A with its rows in a seeded random order (each row keeps its columns
    and values): community structure that the row order no longer shows."""
    (r,) = _rngs(seed, 1)
    perm = r.permutation(A.m)
    lens = np.diff(A.rowptr)[perm]
    rowptr = np.zeros(A.m + 1, dtype=np.int64)
    np.cumsum(lens, out=rowptr[1:])
    idx = np.concatenate([np.arange(A.rowptr[q], A.rowptr[q + 1]) for q in perm]) \
        if A.nnz else np.zeros(0, dtype=np.int64)
    return CSR(A.m, A.k, rowptr, A.colidx[idx], A.vals[idx], A.val_kind)


def batch_specs(count=512, seed=4, rows_lo=1000, rows_hi=200000):
    """Per-matrix (rows, mean degree, wmax, N) for the batched workload."""
    (r,) = _rngs(seed, 1)
    specs = []
    for _ in range(count):
        rows = int(round(math.exp(r.uniform(math.log(rows_lo), math.log(rows_hi)))))
        mean = float(r.uniform(8.0, 32.0))
        n_cols = int(r.choice([32, 64, 128]))
        specs.append((rows, mean, min(20000.0, rows / 8.0), n_cols))
    return specs


def batch_matrix(i: int, spec, seed=4, kind="f16"):
    """Matrix i of the batched workload: Chung-Lu exponent 2.3, U(-1,1) values
    and N(0,1) B, both stored in ``kind``."""
    rows, mean, wmax, n_cols = spec
    sub = 1_000_003 * (seed + 1) + i
    A = chung_lu_graph(rows, 2.3, mean, max(wmax, mean * 1.01), sub, val_kind=kind,
                       values="uniform")
    (r_b,) = _rngs(sub + 7, 1)
    B = dense_values(r_b, (rows, n_cols), kind)
    return A, B


# --------------------------------------------------------------------------------------------
# Small helpers for tests.
# --------------------------------------------------------------------------------------------
def random_csr(m, k, density, seed, val_kind="f32", int_values=None, dup_frac=0.0,
               empty_rows=0.0):
    """Uniformly random CSR (for tests).  ``int_values=(lo, hi)`` draws small
    integers; ``dup_frac`` appends duplicated (row, col) entries; a fraction
    ``empty_rows`` of rows is emptied."""
    r_s, r_v, r_d = _rngs(seed, 3)
    nnz = int(round(m * k * density))
    rows = r_s.integers(0, m, size=nnz)
    cols = r_s.integers(0, k, size=nnz)
    key = np.unique(rows * k + cols) if m * k > 0 else np.zeros(0, np.int64)
    rows, cols = key // max(k, 1), key % max(k, 1)
    if empty_rows > 0 and m > 0:
        dead = r_s.random(m) < empty_rows
        keep = ~dead[rows]
        rows, cols = rows[keep], cols[keep]
    if dup_frac > 0 and rows.size:
        nd = int(rows.size * dup_frac)
        pick = r_d.integers(0, rows.size, size=nd)
        rows = np.concatenate([rows, rows[pick]])
        cols = np.concatenate([cols, cols[pick]])
    if int_values is not None:
        v = r_v.integers(int_values[0], int_values[1] + 1, size=rows.size).astype(np.float32)
        if val_kind == "bf16":
            v = to_bf16_bits(v)
        elif val_kind == "f16":
            v = to_f16_bits(v)
    else:
        v = uniform_values(r_v, rows.size, val_kind)
    return csr_from_coo(m, k, rows, cols, v, val_kind)


def int_dense(rng_seed, shape, lo, hi, kind="f32"):
    (r,) = _rngs(rng_seed, 1)
    x = r.integers(lo, hi + 1, size=shape).astype(np.float32)
    if kind == "bf16":
        return to_bf16_bits(x)
    if kind == "f16":
        return to_f16_bits(x)
    return x


# --------------------------------------------------------------------------------------------
# Serving stream.
# --------------------------------------------------------------------------------------------
def attention_mask(rows: int, block=64, block_density=0.1, band=512, seed=0, val_kind="f32"):
    """Block-sparse attention mask: each 64-row block-row holds
    ceil(block_density * nb) distinct uniformly drawn dense 64x64 blocks, plus
    the sliding window |i - j| < band/2 (i - band/2 <= j < i + band/2);
    values U(0,1)."""
    r_blk, r_val = _rngs(seed, 2)
    nb = (rows + block - 1) // block
    per = max(1, int(math.ceil(block_density * nb)))
    rows_l, cols_l = [], []
    bi = np.repeat(np.arange(nb), per)
    bj = np.concatenate([np.sort(r_blk.choice(nb, size=per, replace=False)) for _ in range(nb)])
    ii, jj = np.meshgrid(np.arange(block), np.arange(block), indexing="ij")
    r = (bi[:, None, None] * block + ii[None]).reshape(-1)
    c = (bj[:, None, None] * block + jj[None]).reshape(-1)
    keep = (r < rows) & (c < rows)
    rows_l.append(r[keep])
    cols_l.append(c[keep])
    half = band // 2
    i = np.repeat(np.arange(rows), band)
    j = i - half + np.tile(np.arange(band), rows)
    keep = (j >= 0) & (j < rows)
    rows_l.append(i[keep])
    cols_l.append(j[keep])
    key = np.unique(np.concatenate(rows_l).astype(np.int64) * rows + np.concatenate(cols_l))
    rr, cc = key // rows, key % rows
    vals = uniform_values(r_val, rr.size, val_kind, 0.0, 1.0)
    rowptr = np.zeros(rows + 1, dtype=np.int64)
    np.cumsum(np.bincount(rr, minlength=rows), out=rowptr[1:])
    return CSR(rows, rows, rowptr, cc.astype(np.int32), vals, val_kind)


class DeviceCSR:
    """A CSR held in torch tensors (``rowptr`` int64, ``colidx`` int32,
    ``vals``) on one device, with the host CSR's size attributes."""

    def __init__(self, m, k, rowptr, colidx, vals, val_kind):
        self.m, self.k = int(m), int(k)
        self.rowptr, self.colidx, self.vals, self.val_kind = rowptr, colidx, vals, val_kind

    @property
    def nnz(self) -> int:
        return int(self.colidx.numel())

    def host_rows(self, rows):
        """A host CSR of the given rows only (in that order), for checks."""
        import torch
        rp = self.rowptr.cpu().numpy()
        rows = np.asarray(rows, dtype=np.int64)
        lens = rp[rows + 1] - rp[rows]
        rowptr = np.zeros(rows.size + 1, dtype=np.int64)
        np.cumsum(lens, out=rowptr[1:])
        idx = torch.from_numpy(np.concatenate([np.arange(rp[r], rp[r + 1]) for r in rows])
                               if rows.size else np.zeros(0, np.int64)).to(self.colidx.device)
        cols = self.colidx[idx].cpu().numpy()
        v = self.vals[idx].cpu()
        if self.val_kind == "f32":
            vals = v.numpy().astype(np.float32)
        else:
            vals = v.view(torch.int16).numpy().view(np.uint16)
        return CSR(int(rows.size), self.k, rowptr, cols.astype(np.int32), vals, self.val_kind)


def attention_mask_device(rows: int, block=64, block_density=0.1, band=512, seed=0, val_kind="f32",
                          device="cuda", chunk_entries=1 << 27):
    """attention_mask's structure built with torch on ``device`` (the same
    block draws from the same seed, so the same rows and columns), for masks
    too large to build on the host: every row's columns are the union of its
    block-row's dense blocks and the sliding window, laid out as sorted
    intervals and expanded chunk by chunk.  Values U(0,1) from torch's
    generator on the device (not attention_mask's values).  Returns a
    DeviceCSR."""
    import torch
    r_blk, _ = _rngs(seed, 2)
    nb = (rows + block - 1) // block
    per = max(1, int(math.ceil(block_density * nb)))
    bj = np.stack([np.sort(r_blk.choice(nb, size=per, replace=False)) for _ in range(nb)])
    dev = torch.device(device)
    bjt = torch.from_numpy(bj.astype(np.int64)).to(dev)                       # nb x per
    present = torch.zeros((nb, nb), dtype=torch.bool, device=dev)
    present.scatter_(1, bjt, True)
    half = band // 2
    ncand = band // block + 2                                                   # block columns a window touches
    # row lengths and, per row, its sorted intervals [start, end)
    def intervals(r0, r1):
        rr = torch.arange(r0, r1, device=dev)
        bi = rr // block
        ps = bjt[bi] * block                                                    # R x per
        pe = torch.clamp(ps + block, max=rows)
        lo = torch.clamp(rr - half, min=0)
        hi = torch.clamp(rr + half, max=rows)
        cb = (lo // block)[:, None] + torch.arange(ncand, device=dev)[None, :]  # R x ncand
        cs = torch.maximum(lo[:, None], cb * block)
        ce = torch.minimum(hi[:, None], cb * block + block)
        inb = cb < nb
        pres = torch.zeros_like(inb)
        pres[inb] = present[bi[:, None].expand_as(cb)[inb], cb[inb]]
        ok = inb & (cs < ce) & ~pres
        cs = torch.where(ok, cs, torch.full_like(cs, rows))                      # invalid: empty, sorted last
        ce = torch.where(ok, ce, torch.full_like(ce, rows))
        st = torch.cat([ps, cs], dim=1)
        en = torch.cat([pe, ce], dim=1)
        order = torch.argsort(st, dim=1, stable=True)
        st = torch.gather(st, 1, order)
        en = torch.gather(en, 1, order)
        return st, en
    lens = torch.zeros(rows, dtype=torch.int64, device=dev)
    step = max(1, chunk_entries // (per * block + band))
    for r0 in range(0, rows, step):
        st, en = intervals(r0, min(rows, r0 + step))
        lens[r0:r0 + st.shape[0]] = (en - st).sum(dim=1)
    rowptr = torch.zeros(rows + 1, dtype=torch.int64, device=dev)
    rowptr[1:] = torch.cumsum(lens, 0)
    nnz = int(rowptr[-1])
    colidx = torch.empty(nnz, dtype=torch.int32, device=dev)
    for r0 in range(0, rows, step):
        st, en = intervals(r0, min(rows, r0 + step))
        ln = (en - st).reshape(-1)
        s0 = st.reshape(-1)
        keep = ln > 0
        ln, s0 = ln[keep], s0[keep]
        total = int(ln.sum())
        if total == 0:
            continue
        off = torch.cumsum(ln, 0) - ln
        col = torch.repeat_interleave(s0 - off, ln) + torch.arange(total, device=dev)
        b = int(rowptr[r0])
        colidx[b:b + total] = col.to(torch.int32)
    g = torch.Generator(device=dev)
    g.manual_seed(seed * 7 + 3)
    vals = torch.rand(nnz, generator=g, device=dev, dtype=torch.float32)
    if val_kind == "bf16":
        vals = vals.to(torch.bfloat16)
    elif val_kind == "f16":
        vals = vals.to(torch.float16)
    return DeviceCSR(rows, rows, rowptr, colidx, vals, val_kind)


def serving_pool(n_graphs=64, n_masks=16, seed=5, max_rows=500000, max_mask_rows=16384,
                 device_masks=False):
    """Resident matrices the serving stream draws from: power-law graphs
    (Chung-Lu exponent 2.1, mean degree 16, rows log-uniform in [1e3,
    max_rows]) and block-sparse attention masks (rows log-uniform in [1e3,
    max_mask_rows]; with ``device_masks`` built on the GPU as DeviceCSR),
    values in f32.  Returns a list of dicts."""
    (r,) = _rngs(seed, 1)
    pool = []
    for g in range(n_graphs):
        rows = int(round(math.exp(r.uniform(math.log(1000), math.log(max_rows)))))
        A = chung_lu_graph(rows, 2.1, 16.0, min(20000.0, rows / 8.0), seed * 7919 + g)
        pool.append({"kind": "graph", "A": A})
    for k in range(n_masks):
        rows = int(round(math.exp(r.uniform(math.log(1000), math.log(max_mask_rows)))))
        if device_masks:
            A = attention_mask_device(rows, seed=seed * 104729 + k)
        else:
            A = attention_mask(rows, seed=seed * 104729 + k)
        pool.append({"kind": "mask", "A": A})
    return pool


def serving_requests(count, pool_size, n_graphs, seed=5, rate=None):
    """Request list: matrix drawn 50/50 between graphs and masks (uniform
    within each kind), N uniform in {32, 64, 128, 256}, B type 50/50 f32 /
    bf16, a per-request seed for B, and Poisson arrival times at ``rate``
    requests/s (None: all at time 0)."""
    (r,) = _rngs(seed + 17, 1)
    reqs = []
    t = 0.0
    for i in range(count):
        if r.random() < 0.5 or n_graphs == pool_size:
            mid = int(r.integers(0, n_graphs))
        else:
            mid = int(r.integers(n_graphs, pool_size))
        n = int(r.choice([32, 64, 128, 256]))
        kind = "f32" if r.random() < 0.5 else "bf16"
        if rate:
            t += float(r.exponential(1.0 / rate))
        reqs.append({"rid": i, "matrix": mid, "n": n, "b_kind": kind,
                     "seed": int(r.integers(0, 2**31 - 1)), "arrival": t})
    return reqs
