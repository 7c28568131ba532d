"""CPU tier for the input generators of the serving stream: the attention
mask built with torch (for masks too large for the host) has exactly the
rows and columns of the host generator from the same seed -- dense 64x64
blocks of each block-row plus the sliding window, sorted, no duplicates."""
import numpy as np
import pytest

from paper_2606_22482_amd import synth


@pytest.mark.parametrize("rows,seed,chunk", [(64, 3, 1 << 16), (700, 4, 1 << 12), (1000, 1, 1 << 20),
                                             (4097, 2, 1 << 15), (3001, 9, 1 << 14)])
def test_device_mask_structure_equals_host(rows, seed, chunk):
    A = synth.attention_mask(rows, seed=seed)
    D = synth.attention_mask_device(rows, seed=seed, device="cpu", chunk_entries=chunk)
    assert D.m == D.k == rows and D.nnz == A.nnz
    assert np.array_equal(A.rowptr, D.rowptr.numpy())
    assert np.array_equal(A.colidx, D.colidx.numpy())
    v = D.vals.numpy()
    assert v.dtype == np.float32 and (v >= 0).all() and (v < 1).all()
    # the structure's definition, row by row on a sample
    nb = (rows + 63) // 64
    per = max(1, int(np.ceil(0.1 * nb)))
    r_blk, _ = synth._rngs(seed, 2)
    blocks = [np.sort(r_blk.choice(nb, size=per, replace=False)) for _ in range(nb)]
    for r in np.random.default_rng(seed).choice(rows, min(rows, 40), replace=False):
        want = set()
        for b in blocks[r // 64]:
            want.update(range(64 * b, min(rows, 64 * b + 64)))
        want.update(range(max(0, r - 256), min(rows, r + 256)))
        got = D.colidx.numpy()[D.rowptr[r]: D.rowptr[r + 1]]
        assert list(got) == sorted(want)


def test_host_rows_view():
    D = synth.attention_mask_device(900, seed=5, device="cpu")
    rows = np.array([0, 17, 899, 400])
    H = D.host_rows(rows)
    assert H.m == 4 and H.k == 900
    for i, r in enumerate(rows):
        b, e = int(D.rowptr[r]), int(D.rowptr[r + 1])
        assert np.array_equal(H.colidx[H.rowptr[i]: H.rowptr[i + 1]], D.colidx.numpy()[b:e])
        assert np.array_equal(H.vals[H.rowptr[i]: H.rowptr[i + 1]], D.vals.numpy()[b:e])
