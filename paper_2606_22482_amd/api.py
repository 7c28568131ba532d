"""Thin Python binding over the C ABI (``include/spmm.h``).

Same names as the ABI.  Host arrays are numpy; device buffers are torch
tensors, used only as memory and streams.  Every step of the computation runs
in ``libspmm.so``; nothing here computes.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L

__all__ = ["Plan", "Timer", "spmm_plan", "spmm_run", "spmm_submit", "spmm_poll", "spmm_wait",
           "spmm_dryrun", "spmm_copy_bandwidth", "spmm_gather_bandwidth", "default_opts",
           "SpmmError"]

SpmmError = L.SpmmError


def default_opts(**kw) -> L.Opts:
    """spmm_opts_default() with fields overridden by keyword (names as in the
    C struct; ``mode``/``row_order`` also accept the names without prefix)."""
    lib = L.load()
    o = L.Opts()
    lib.spmm_opts_default(C.byref(o))
    modes = {"auto": L.MODE_AUTO, "plain": L.MODE_PLAIN_F32, "plain_f32": L.MODE_PLAIN_F32,
             "mixed": L.MODE_MIXED, "mfma_only": L.MODE_MFMA_ONLY}
    orders = {"auto": L.ORDER_AUTO, "original_ranges": L.ORDER_ORIGINAL_RANGES,
              "compacted": L.ORDER_COMPACTED, "length_sorted": L.ORDER_LENGTH_SORTED,
              "clustered": L.ORDER_CLUSTERED}
    for k, v in kw.items():
        if k == "mode" and isinstance(v, str):
            v = modes[v]
        if k == "row_order" and isinstance(v, str):
            v = orders[v]
        setattr(o, k, v)
    return o


def device_tensor(x: np.ndarray, kind: str):
    """Copy a host array (float32, or uint16 bit patterns for "bf16"/"f16")
    to a device tensor of the matching torch dtype."""
    import torch
    if kind == "f32":
        t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32))
    else:
        t = torch.from_numpy(np.ascontiguousarray(x).view(np.int16))
        t = t.view(torch.bfloat16 if kind == "bf16" else torch.float16)
    return t.cuda()


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _kind_of_tensor(t):
    import torch
    return {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16"}[t.dtype]


def _dev2d(t, what):
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("%s must be a 2-D tensor with unit column stride" % what)
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % what)
    return t.data_ptr(), t.stride(0)


_TORCH_DTYPE = {"f32": "float32", "bf16": "bfloat16", "f16": "float16"}


def _operands(m: int, k: int, n: int, b_kind: str, B, Cout):
    """Device pointers and leading dimensions of B and C after checking them
    against the problem, before anything reaches the device: B of the plan's
    B type with at least k rows and n columns, C float32 with at least m rows
    and n columns, both 2-D device tensors with unit column stride.  (The C
    ABI only sees pointers and leading dimensions, so a wrong dtype or a short
    B would make the kernels read or write out of bounds.)"""
    import torch
    want = getattr(torch, _TORCH_DTYPE[b_kind])
    if B.dtype != want:
        raise ValueError("B must be %s for this plan (B type %s), got %s" % (want, b_kind, B.dtype))
    if Cout.dtype != torch.float32:
        raise ValueError("C must be torch.float32, got %s" % Cout.dtype)
    if B.dim() != 2 or B.shape[0] < k or B.shape[1] < n:
        raise ValueError("B must be at least %d x %d, got %s" % (k, n, tuple(B.shape)))
    if Cout.dim() != 2 or Cout.shape[0] < m or Cout.shape[1] < n:
        raise ValueError("C must be at least %d x %d, got %s" % (m, n, tuple(Cout.shape)))
    bp, ldb = _dev2d(B, "B")
    cp, ldc = _dev2d(Cout, "C")
    return bp, ldb, cp, ldc


def _csr_struct(A):
    rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(A.colidx, dtype=np.int32)
    vals = np.ascontiguousarray(A.vals)
    csr = L.Csr(int(A.m), int(A.k), int(rowptr[-1]) if rowptr.size else 0, rowptr.ctypes.data,
                colidx.ctypes.data, vals.ctypes.data, L.KIND_CODE[A.val_kind], 0)
    return csr, (rowptr, colidx, vals)


def opts_dict(o: L.Opts) -> dict:
    return {f: getattr(o, f) for f, _ in L.Opts._fields_}


class Plan:
    """A plan built by ``spmm_plan`` (or ``spmm_plan_build`` when
    ``upload=False``).  ``A`` needs ``m, k, rowptr, colidx, vals, val_kind``."""

    def __init__(self, A, n: int, b_kind: str, opts: L.Opts | None = None, upload=True):
        lib = L.load()
        self._lib = lib
        rowptr = np.ascontiguousarray(A.rowptr, dtype=np.int64)
        colidx = np.ascontiguousarray(A.colidx, dtype=np.int32)
        vals = np.ascontiguousarray(A.vals)
        self._keep = (rowptr, colidx, vals)
        csr = L.Csr(int(A.m), int(A.k), int(rowptr[-1]) if rowptr.size else 0,
                    rowptr.ctypes.data, colidx.ctypes.data, vals.ctypes.data,
                    L.KIND_CODE[A.val_kind], 0)
        self.n = int(n)
        self.m = int(A.m)
        self.k = int(A.k)
        self.b_kind = b_kind
        h = C.c_void_p()
        fn = lib.spmm_plan if upload else lib.spmm_plan_build
        L.check(fn(C.byref(csr), self.n, L.KIND_CODE[b_kind], L.F32,
                   C.byref(opts) if opts is not None else None, C.byref(h)))
        self._h = h
        self._keep = None

    @property
    def handle(self):
        return self._h

    def serialize(self) -> bytes:
        """spmm_plan_serialize: the plan image as bytes."""
        size = C.c_int64()
        L.check(self._lib.spmm_plan_serialize(self._h, None, 0, C.byref(size)))
        buf = C.create_string_buffer(size.value)
        L.check(self._lib.spmm_plan_serialize(self._h, buf, size.value, C.byref(size)))
        return buf.raw[: size.value]

    @classmethod
    def on_device(cls, rowptr, colidx, vals, m: int, k: int, n: int, b_kind: str,
                  opts: "L.Opts | None" = None, stream=None) -> "Plan":
        """spmm_plan_device: a plain plan built on the device from device
        tensors rowptr (int64, m+1), colidx (int32, nnz) and vals (nnz)."""
        import torch
        lib = L.load()
        for t, what in ((rowptr, "rowptr"), (colidx, "colidx"), (vals, "vals")):
            if not t.is_cuda or not t.is_contiguous():
                raise ValueError("%s must be a contiguous device tensor" % what)
        if rowptr.dtype != torch.int64 or colidx.dtype != torch.int32:
            raise ValueError("rowptr must be int64 and colidx int32")
        kind = _kind_of_tensor(vals)
        csr = L.Csr(int(m), int(k), int(colidx.numel()), rowptr.data_ptr(), colidx.data_ptr(),
                    vals.data_ptr(), L.KIND_CODE[kind], 0)
        h = C.c_void_p()
        L.check(lib.spmm_plan_device(C.byref(csr), int(n), L.KIND_CODE[b_kind], L.F32,
                                     C.byref(opts) if opts is not None else None,
                                     _stream_handle(stream), C.byref(h)))
        p = cls.__new__(cls)
        p._lib, p._h, p._keep = lib, h, None
        p.n, p.m, p.k, p.b_kind = int(n), int(m), int(k), b_kind
        return p

    @classmethod
    def deserialize(cls, image: bytes, upload=True) -> "Plan":
        """spmm_plan_deserialize: a plan from an image written by serialize."""
        lib = L.load()
        h = C.c_void_p()
        L.check(lib.spmm_plan_deserialize(image, len(image), 1 if upload else 0, C.byref(h)))
        p = cls.__new__(cls)
        p._lib, p._h, p._keep = lib, h, None
        st = p.stats()
        p.n, p.m, p.k = int(st["n"]), int(st["m"]), int(st["k"])
        p.b_kind = {0: "f32", 1: "bf16", 2: "f16"}[int(st["b_type"])]
        return p

    def upload(self):
        L.check(self._lib.spmm_plan_upload(self._h))

    def stats(self) -> dict:
        s = L.PlanStats()
        L.check(self._lib.spmm_plan_stats(self._h, C.byref(s)))
        out = {f: getattr(s, f) for f, _ in L.PlanStats._fields_ if f not in ("opts", "reserved")}
        out["opts"] = {f: getattr(s.opts, f) for f, _ in L.Opts._fields_ if f != "reserved"}
        return out

    def export(self) -> dict:
        """Copies of the plan's host arrays (see spmm_plan_dump_t)."""
        d = L.PlanDump()
        L.check(self._lib.spmm_plan_export(self._h, C.byref(d)))

        def arr(ptr, n, dt):
            if n == 0 or not ptr:
                return np.zeros(0, dtype=dt)
            buf = (C.c_char * (n * np.dtype(dt).itemsize)).from_address(ptr)
            return np.frombuffer(buf, dtype=dt).copy()

        H, kt, W, T = d.window_h, d.kt, d.n_windows, d.n_tiles
        tvp = arr(d.tile_val_ptr, T + 1, np.int64)
        rp = arr(d.rem_ptr, d.m + 1, np.int64)
        nv = d.n_vitems
        return {
            "window_h": H, "kt": kt,
            "windows": arr(d.windows, W * H, np.int32).reshape(W, H),
            "tile_window": arr(d.tile_window, T, np.int32),
            "tile_cols": arr(d.tile_cols, T * kt, np.int32).reshape(T, kt),
            "tile_bitmap": arr(d.tile_bitmap, T * H, np.uint32).reshape(T, H),
            "tile_val_ptr": tvp,
            "tile_vals": arr(d.tile_vals, int(tvp[-1]), np.uint16),
            "tile_src": arr(d.tile_src, int(tvp[-1]), np.int64),
            "rem_ptr": rp,
            "rem_src": arr(d.rem_src, int(rp[-1]), np.int64),
            "vector_rows": arr(d.vector_rows, d.n_vector_rows, np.int32),
            "nseg": arr(d.nseg, d.m, np.int32),
            "vitem_ptr": arr(d.vitem_ptr, nv + 1, np.int32),
            "vitem_seg": arr(d.vitem_seg, nv, np.int32),
            "seg_row": arr(d.seg_row, d.n_segments, np.int32),
            "seg_begin": arr(d.seg_begin, d.n_segments, np.int32),
            "seg_end": arr(d.seg_end, d.n_segments, np.int32),
            "win_seg": arr(d.win_seg, W, np.int32),
            "win_order": arr(d.win_order, W, np.int32),
            "rem_col_dev": arr(d.rem_col_dev, int(rp[-1]), np.int32),
            "win_part": arr(d.win_part, W + 1, np.int32),
            "wpart_win": arr(d.wpart_win, d.n_wparts, np.int32),
            "wpart_t0": arr(d.wpart_t0, d.n_wparts, np.int32),
            "wpart_t1": arr(d.wpart_t1, d.n_wparts, np.int32),
            "vexec_rows": arr(d.vexec_rows, d.n_vector_rows, np.int32),
            "n_dep": int(d.n_dep),
            "seg_win": arr(d.seg_win, d.n_segments if d.seg_win else 0, np.int32),
            "win_dep": arr(d.win_dep, W, np.int32),
            "win_nsseg": arr(d.win_nsseg, W, np.int32),
        }

    def operands(self, B, Cout):
        """(B pointer, ldb, C pointer, ldc) after checking B and C against
        this plan (see _operands)."""
        return _operands(self.m, self.k, self.n, self.b_kind, B, Cout)

    def run(self, B, Cout, stream=None):
        """spmm_run: Cout = A @ B on the stream (torch's current one by default)."""
        bp, ldb, cp, ldc = self.operands(B, Cout)
        L.check(self._lib.spmm_run(self._h, bp, ldb, cp, ldc, _stream_handle(stream)))

    def run_bytes(self, ldb: int | None = None, ldc: int | None = None, batched=False,
                  budget: int = -1):
        """spmm_run_bytes: (status, bytes) of one execution (B, C, scratch;
        not the plan).  status is SPMM_OK or SPMM_ERR_BUDGET (bytes > budget)."""
        out = C.c_int64()
        st = self._lib.spmm_run_bytes(self._h, int(ldb or self.n), int(ldc or self.n),
                                      1 if batched else 0, int(budget), C.byref(out))
        if st not in (L.SPMM_OK, L.SPMM_ERR_BUDGET):
            L.check(st)
        return st, out.value

    def run_noalloc(self, B, Cout, stream=None):
        """spmm_run_noalloc: as run, with the library's fixed scratch array
        instead of a per-stream workspace (no allocation)."""
        bp, ldb, cp, ldc = self.operands(B, Cout)
        L.check(self._lib.spmm_run_noalloc(self._h, bp, ldb, cp, ldc, _stream_handle(stream)))

    def run_timed(self, B, Cout, timer: "Timer", stream=None):
        bp, ldb, cp, ldc = self.operands(B, Cout)
        L.check(self._lib.spmm_run_timed(self._h, bp, ldb, cp, ldc, _stream_handle(stream),
                                         timer.handle))

    def adapt_epoch(self, A, B, Cout, state: "L.AdaptState", eps: float = 0.05, stream=None):
        """spmm_adapt_epoch: one timed run (Cout = A @ B, the stream is
        synchronised), then the adaptive re-partition step; when it rebuilds
        the plan, this object takes the new plan's handle.  A must be the
        matrix this plan was built from.  Returns ``state``."""
        csr, keep = _csr_struct(A)
        bp, ldb, cp, ldc = self.operands(B, Cout)
        L.check(self._lib.spmm_adapt_epoch(C.byref(csr), C.byref(self._h), bp, ldb, cp, ldc,
                                           _stream_handle(stream), float(eps), C.byref(state)))
        del keep
        return state

    def destroy(self):
        if self._h:
            L.check(self._lib.spmm_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            if getattr(self, "_h", None):
                self._lib.spmm_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


def spmm_plan(A, n, b_kind, opts=None, upload=True) -> Plan:
    return Plan(A, n, b_kind, opts, upload)


def spmm_run(plan: Plan, B, Cout, stream=None):
    plan.run(B, Cout, stream)


class Timer:
    """spmm_timer_*: per-kernel HIP event pairs recorded by run_timed."""

    def __init__(self, capacity=4096):
        self._lib = L.load()
        h = C.c_void_p()
        L.check(self._lib.spmm_timer_create(int(capacity), C.byref(h)))
        self.handle = h
        self.capacity = int(capacity)

    def reset(self):
        L.check(self._lib.spmm_timer_reset(self.handle))

    def read(self):
        ids = (C.c_int32 * self.capacity)()
        ms = (C.c_float * self.capacity)()
        n = C.c_int32()
        L.check(self._lib.spmm_timer_read(self.handle, ids, ms, self.capacity, C.byref(n)))
        return [(L.KERNEL_NAMES[ids[i]], ms[i]) for i in range(n.value)]

    def __del__(self):
        try:
            self._lib.spmm_timer_destroy(self.handle)
        except Exception:
            pass


@dataclass
class WorkItem:
    plan: Plan
    B: object
    C: object


def spmm_submit(items, stream=None) -> int:
    lib = L.load()
    arr = (L.Work * max(1, len(items)))()
    for i, it in enumerate(items):
        bp, ldb, cp, ldc = it.plan.operands(it.B, it.C)
        arr[i] = L.Work(it.plan.handle.value, bp, ldb, cp, ldc)
    t = C.c_uint64()
    L.check(lib.spmm_submit(arr, len(items), _stream_handle(stream), C.byref(t)))
    return t.value


def spmm_poll(ticket: int) -> bool:
    lib = L.load()
    d = C.c_int32()
    L.check(lib.spmm_poll(C.c_uint64(ticket), C.byref(d)))
    return bool(d.value)


def spmm_wait(ticket: int):
    L.check(L.load().spmm_wait(C.c_uint64(ticket)))


def spmm_dryrun(n: int, b_kind: str, stream=None):
    lib = L.load()
    pv, pm = C.c_double(), C.c_double()
    L.check(lib.spmm_dryrun(int(n), L.KIND_CODE[b_kind], _stream_handle(stream), C.byref(pv),
                            C.byref(pm)))
    return pv.value, pm.value


def spmm_autotune(A, B, Cout, b_kind: str, budget_ms: float = 20000.0, stream=None,
                  batched: bool = False):
    """spmm_autotune: returns (opts, report dict); also caches the options
    under A's profile key for spmm_plan(mode=AUTO).  ``batched`` times the
    candidates as spmm_submit batches of copies of A (their throughput among
    other work, for plans that will run in batches)."""
    lib = L.load()
    csr, keep = _csr_struct(A)
    bp, ldb, cp, ldc = _operands(int(A.m), int(A.k), int(B.shape[1]), b_kind, B, Cout)
    o = L.Opts()
    rep = L.TuneReport()
    L.check(lib.spmm_autotune(C.byref(csr), int(B.shape[1]), L.KIND_CODE[b_kind], L.F32, bp, ldb,
                              cp, ldc, _stream_handle(stream), float(budget_ms),
                              L.TUNE_SUBMIT if batched else L.TUNE_RUN, C.byref(o), C.byref(rep)))
    del keep
    return o, {f: getattr(rep, f) for f, _ in L.TuneReport._fields_ if f != "reserved"}


def spmm_profile_key(A, n: int, b_kind: str) -> str:
    lib = L.load()
    csr, keep = _csr_struct(A)
    buf = C.create_string_buffer(1024)
    L.check(lib.spmm_profile_key(C.byref(csr), int(n), L.KIND_CODE[b_kind], buf, 1024))
    del keep
    return buf.value.decode()


def tune_cache_put(key: str, opts: L.Opts):
    L.check(L.load().spmm_tune_cache_put(key.encode(), C.byref(opts)))


def tune_cache_get(key: str):
    o = L.Opts()
    found = C.c_int32()
    L.check(L.load().spmm_tune_cache_get(key.encode(), C.byref(o), C.byref(found)))
    return o if found.value else None


def tune_cache_save(path: str):
    L.check(L.load().spmm_tune_cache_save(path.encode()))


def tune_cache_load(path: str):
    L.check(L.load().spmm_tune_cache_load(path.encode()))


def tune_cache_clear():
    L.load().spmm_tune_cache_clear()


def spmm_copy_bandwidth(nbytes: int, stream=None) -> float:
    lib = L.load()
    out = C.c_double()
    L.check(lib.spmm_copy_bandwidth(int(nbytes), _stream_handle(stream), C.byref(out)))
    return out.value


def spmm_gather_bandwidth(rows, B, n_cols: int = None, reps: int = 10, stream=None) -> float:
    """Bytes per second at which the device gathers the B rows named by the
    int32 device tensor ``rows`` (the first ``n_cols`` f32 of each row of the
    f32 device matrix ``B``) with nothing else done."""
    import torch
    if rows.dtype != torch.int32 or not rows.is_cuda or not rows.is_contiguous():
        raise ValueError("rows must be a contiguous int32 device tensor")
    if B.dtype != torch.float32 or not B.is_cuda or B.dim() != 2 or B.stride(1) != 1:
        raise ValueError("B must be a row-major f32 device matrix")
    n_cols = B.shape[1] if n_cols is None else n_cols
    lib = L.load()
    out = C.c_double()
    L.check(lib.spmm_gather_bandwidth(C.c_void_p(rows.data_ptr()), rows.numel(),
                                      C.c_void_p(B.data_ptr()), B.shape[0], B.stride(0),
                                      int(n_cols), int(reps), _stream_handle(stream), C.byref(out)))
    return out.value


def adapt_state(alpha: float = 0.0) -> L.AdaptState:
    """A zeroed adaptive re-partition state (alpha <= 0: start from the plan's
    own threshold)."""
    st = L.AdaptState()
    st.alpha = alpha
    return st


def adapt_next(state: L.AdaptState, t_vec_ms, t_mfma_ms, w_vec, w_tile, w_winrem,
               p_vec_dry=0.0, p_mfma_dry=0.0, eps=0.05) -> L.AdaptState:
    """spmm_adapt_next: the host update of one epoch (see include/spmm.h)."""
    lib = L.load()
    L.check(lib.spmm_adapt_next(C.byref(state), t_vec_ms, t_mfma_ms, w_vec, w_tile, w_winrem,
                                p_vec_dry, p_mfma_dry, eps))
    return state
