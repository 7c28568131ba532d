"""Pins for the FP64 oracle against things other than itself: dense brute
force with numpy, scipy.sparse, closed-form special cases and exact
invariants (NeutronSparse Sec. 5.1 defines the product being computed)."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2606_22482_amd import synth


def widen_test(x, kind):
    """The test's own exact widening (independent of the oracle's decoder)."""
    x = np.asarray(x)
    if kind == "f32":
        return x.astype(np.float64)
    if kind == "bf16":
        return (x.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    if kind == "f16":
        return x.view(np.float16).astype(np.float64)
    raise ValueError(kind)


def dense_of(A, kind, absolute=False):
    """Densify A (duplicates add); with ``absolute`` the entries' |v| add."""
    D = np.zeros((A.m, A.k), dtype=np.float64)
    rows = np.repeat(np.arange(A.m), np.diff(A.rowptr))
    v = widen_test(A.vals, kind)
    np.add.at(D, (rows, A.colidx.astype(np.int64)), np.abs(v) if absolute else v)
    return D


KINDS = [("f32", "f32"), ("f32", "bf16"), ("bf16", "bf16"), ("f16", "f16")]


@pytest.mark.parametrize("vk,bk", KINDS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bruteforce_dense(oracle_lib, vk, bk, seed):
    m, k, n = 37, 53, 19
    A = synth.random_csr(m, k, 0.15, seed, val_kind=vk, dup_frac=0.1, empty_rows=0.1)
    B = synth.dense_values(np.random.default_rng(seed + 100), (k, n), bk)
    C, S = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B, val_kind=vk, b_kind=bk)
    Da = dense_of(A, vk)
    Db = widen_test(B, bk)
    ref = Da @ Db
    Sref = dense_of(A, vk, absolute=True) @ np.abs(Db)
    # dense products of duplicates merged first: agree to rounding of the sums
    assert np.all(np.abs(C - ref) <= 1e-12 * np.maximum(Sref, 1e-300))
    np.testing.assert_allclose(S, Sref, rtol=1e-12, atol=0)


def test_scipy_medium(oracle_lib):
    A = synth.random_csr(2000, 1500, 0.01, 7)
    B = np.random.default_rng(3).standard_normal((1500, 33)).astype(np.float32)
    C, S = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B)
    M = sp.csr_matrix((A.vals.astype(np.float64), A.colidx, A.rowptr), shape=(A.m, A.k))
    ref = M @ B.astype(np.float64)
    assert oracle_lib.max_normalised_error(C, ref, S) <= 1e-12


def test_identity_returns_B_bitwise(oracle_lib):
    n = 300
    A = synth.CSR(n, n, np.arange(n + 1, dtype=np.int64), np.arange(n, dtype=np.int32),
                  np.ones(n, dtype=np.float32), "f32")
    B = np.random.default_rng(5).standard_normal((n, 7)).astype(np.float32)
    C, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B)
    assert np.array_equal(C, B.astype(np.float64))


def test_empty_matrix_and_rows(oracle_lib):
    A = synth.CSR(5, 4, np.zeros(6, dtype=np.int64), np.zeros(0, np.int32),
                  np.zeros(0, np.float32), "f32")
    B = np.ones((4, 3), np.float32)
    C, S = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B)
    assert C.shape == (5, 3) and np.all(C == 0) and np.all(S == 0)


def test_row_permutation_bitwise(oracle_lib):
    A = synth.random_csr(200, 150, 0.05, 11)
    B = np.random.default_rng(1).standard_normal((150, 16)).astype(np.float32)
    C, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B)
    perm = np.random.default_rng(2).permutation(A.m)
    lens = np.diff(A.rowptr)[perm]
    rp = np.zeros(A.m + 1, np.int64)
    np.cumsum(lens, out=rp[1:])
    idx = np.concatenate([np.arange(A.rowptr[r], A.rowptr[r + 1]) for r in perm])
    C2, _ = oracle_lib.spmm(rp, A.colidx[idx], A.vals[idx], B)
    assert np.array_equal(C2, C[perm])


def test_column_permutation_bitwise(oracle_lib):
    # A Q^T with Q B: same sum order per row, so bitwise equal
    A = synth.random_csr(120, 90, 0.08, 12)
    B = np.random.default_rng(4).standard_normal((90, 10)).astype(np.float32)
    q = np.random.default_rng(5).permutation(A.k)
    C, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B)
    Bq = np.empty_like(B)
    Bq[q] = B
    C2, _ = oracle_lib.spmm(A.rowptr, q[A.colidx].astype(np.int32), A.vals, Bq)
    assert np.array_equal(C, C2)


def test_linearity_in_B_exact(oracle_lib):
    A = synth.random_csr(64, 80, 0.1, 13, int_values=(-2, 2))
    B1 = synth.int_dense(1, (80, 9), -8, 8)
    B2 = synth.int_dense(2, (80, 9), -8, 8)
    a, b = 0.5, -2.0
    C1, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B1)
    C2, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B2)
    C3, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, (a * B1 + b * B2).astype(np.float32))
    assert np.array_equal(C3, a * C1 + b * C2)


def test_row_scaling_exact(oracle_lib):
    A = synth.random_csr(50, 40, 0.2, 14, int_values=(-2, 2))
    B = synth.int_dense(3, (40, 5), -8, 8)
    s = np.array([2.0 ** (i % 5 - 2) for i in range(A.m)], dtype=np.float32)
    rows = np.repeat(np.arange(A.m), np.diff(A.rowptr))
    C, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B)
    Cs, _ = oracle_lib.spmm(A.rowptr, A.colidx, (A.vals * s[rows]).astype(np.float32), B)
    assert np.array_equal(Cs, C * s[:, None].astype(np.float64))


def test_integer_values_exact(oracle_lib):
    A = synth.random_csr(100, 100, 0.2, 15, int_values=(-2, 2), dup_frac=0.05)
    B = synth.int_dense(4, (100, 12), -8, 8)
    C, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B)
    ref = dense_of(A, "f32") @ B.astype(np.float64)
    assert np.array_equal(C, ref)


def test_threads_and_row_subset_bitwise(oracle_lib):
    A = synth.random_csr(500, 300, 0.05, 16)
    B = np.random.default_rng(6).standard_normal((300, 24)).astype(np.float32)
    C1, S1 = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B, nthreads=1)
    C4, S4 = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B, nthreads=4)
    assert np.array_equal(C1, C4) and np.array_equal(S1, S4)
    rows = np.array([499, 0, 17, 17, 250])
    Cr, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, B, rows=rows)
    assert np.array_equal(Cr, C1[rows])


def test_strided_B(oracle_lib):
    A = synth.random_csr(40, 30, 0.2, 17)
    Bfull = np.random.default_rng(7).standard_normal((30, 20)).astype(np.float32)
    Bv = Bfull[:, :11]  # row stride 20 > N = 11
    C, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, Bv)
    C2, _ = oracle_lib.spmm(A.rowptr, A.colidx, A.vals, np.ascontiguousarray(Bv))
    assert np.array_equal(C, C2)


def test_decoders_exhaustive(oracle_lib):
    bits = np.arange(65536, dtype=np.uint16)
    f16 = oracle_lib.widen(bits, "f16")
    ref16 = bits.view(np.float16).astype(np.float64)
    nan = np.isnan(ref16)
    assert np.array_equal(np.isnan(f16), nan)
    assert np.array_equal(f16[~nan], ref16[~nan])
    assert np.array_equal(np.signbit(f16[~nan]), np.signbit(ref16[~nan]))
    bf = oracle_lib.widen(bits, "bf16")
    refb = widen_test(bits, "bf16")
    nanb = np.isnan(refb)
    assert np.array_equal(np.isnan(bf), nanb)
    assert np.array_equal(bf[~nanb], refb[~nanb])


def test_error_metric(oracle_lib):
    Cs = np.array([[1.0, 0.0], [2.0, -3.0]])
    S = np.array([[2.0, 0.0], [4.0, 3.0]])
    assert oracle_lib.max_normalised_error(Cs, Cs, S) == 0.0
    C = Cs.copy()
    C[1, 0] += 0.04
    assert abs(oracle_lib.max_normalised_error(C, Cs, S) - 0.01) < 1e-15
    C = Cs.copy()
    C[0, 1] = 1e-30  # S == 0 entries must be exactly zero
    assert oracle_lib.max_normalised_error(C, Cs, S) == float("inf")
    C = Cs.copy()
    C[1, 1] = np.nan
    assert oracle_lib.max_normalised_error(C, Cs, S) == float("inf")


@pytest.mark.parametrize("mutation", ["drop_term", "flip_sign", "transpose_B", "shift_col"])
def test_pins_catch_planted_mistakes(oracle_lib, mutation):
    """A plausible mistake planted in the oracle's input (standing in for a
    bug in its loop) must fail the dense brute-force pin."""
    A = synth.random_csr(30, 30, 0.2, 21)
    B = np.random.default_rng(9).standard_normal((30, 30)).astype(np.float32)
    ref = dense_of(A, "f32") @ B.astype(np.float64)
    rp, ci, v, Bm = A.rowptr.copy(), A.colidx.copy(), A.vals.copy(), B
    if mutation == "drop_term":
        v[5] = 0
    elif mutation == "flip_sign":
        v[3] = -v[3]
    elif mutation == "transpose_B":
        Bm = np.ascontiguousarray(B.T)
    elif mutation == "shift_col":
        ci[7] = (ci[7] + 1) % 30
    C, S = oracle_lib.spmm(rp, ci, v, Bm)
    assert oracle_lib.max_normalised_error(C, ref, dense_of(A, "f32", absolute=True) @ np.abs(B)) > 1e-6
