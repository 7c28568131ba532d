"""Helpers shared by the GPU tests: device tensors from generator outputs and
the parity check against the FP64 oracle."""
import numpy as np

import oracle

TOL_F32 = 1e-5     # FP32 path, error normalised by sum |A||B|
TOL_16 = 2e-2      # 16-bit MFMA operands
# FP32 path, plain relative error |C - C*| / |C*| on the entries whose |C*| is
# at least REL_FLOOR * sum |A||B| (below it cancellation makes the relative
# error unbounded for any FP32 summation and the normalised error applies)
REL_FLOOR = 0.1


def max_relative_error(C, Cs, S, floor=REL_FLOOR):
    """max |C - C*| / |C*| over entries with |C*| >= floor * S, and how many
    entries that covers."""
    sel = np.abs(Cs) >= floor * S
    sel &= S > 0
    if not sel.any():
        return 0.0, 0
    return float(np.max(np.abs(C[sel] - Cs[sel]) / np.abs(Cs[sel]))), int(sel.sum())


def device_B(B, kind, pad_cols=0):
    """B (generator output: float32 or uint16 bit patterns) as a device tensor,
    optionally with extra columns so that the row stride exceeds N."""
    import torch
    if kind == "f32":
        t = torch.from_numpy(np.ascontiguousarray(B, dtype=np.float32))
    else:
        t = torch.from_numpy(np.ascontiguousarray(B).view(np.int16))
        t = t.view(torch.bfloat16 if kind == "bf16" else torch.float16)
    if pad_cols:
        full = torch.zeros((t.shape[0], t.shape[1] + pad_cols), dtype=t.dtype)
        full[:, : t.shape[1]] = t
        return full.cuda()[:, : t.shape[1]]
    return t.cuda()


def device_C(m, n, fill=float("nan"), pad_cols=0):
    import torch
    full = torch.full((m, n + pad_cols), fill, dtype=torch.float32, device="cuda")
    return full[:, :n] if pad_cols else full


def oracle_of(A, B, b_kind, rows=None, nthreads=8):
    return oracle.spmm(A.rowptr, A.colidx, A.vals, B, val_kind=A.val_kind, b_kind=b_kind,
                       rows=rows, nthreads=nthreads)


def parity(Cdev, A, B, b_kind, tol, rows=None):
    """Max normalised error of the device result against the oracle; asserts
    it is within ``tol`` and returns it."""
    C = Cdev.cpu().numpy().astype(np.float64)
    if rows is not None:
        C = C[rows]
    Cs, S = oracle_of(A, B, b_kind, rows=rows)
    err = oracle.max_normalised_error(C, Cs, S)
    assert err <= tol, "normalised error %g > %g" % (err, tol)
    if tol <= TOL_F32:
        rel, count = max_relative_error(C, Cs, S)
        assert rel <= TOL_F32, "relative error %g > %g over %d entries" % (rel, TOL_F32, count)
    return err


def exact(Cdev, A, B, b_kind):
    C = Cdev.cpu().numpy().astype(np.float64)
    Cs, _ = oracle_of(A, B, b_kind)
    assert np.array_equal(C, Cs), "max abs diff %g" % np.max(np.abs(C - Cs))
