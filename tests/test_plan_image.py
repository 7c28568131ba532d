"""Plan images (spmm_plan_serialize / spmm_plan_deserialize): round trips are
exact, and a damaged or crafted image is refused before any kernel could
index with it.  CPU only (plans are built and loaded without upload)."""
import ctypes as C
import struct

import numpy as np
import pytest

from paper_2606_22482_amd import _lib as L
from paper_2606_22482_amd import api, synth

# array order and element sizes of the image (after the fixed header)
ARRAYS = [("windows", 4), ("tile_window", 4), ("tile_cols", 4), ("tile_bitmap", 4),
          ("tile_val_ptr", 8), ("tile_vals", 2), ("tile_src", 8), ("rem_ptr", 8), ("rem_src", 8),
          ("vector_rows", 4), ("nseg", 4), ("vexec", 4), ("vitem_ptr", 4), ("vitem_seg", 4),
          ("seg_row", 4), ("seg_begin", 4), ("seg_end", 4), ("win_tile_ptr", 4), ("win_seg", 4),
          ("win_order", 4), ("win_part", 4), ("wpart_win", 4), ("wpart_t0", 4), ("wpart_t1", 4),
          ("rem_ptr32", 4), ("rem_col", 4), ("rem_val", 1)]


def fnv1a(b: bytes) -> int:
    h = 1469598103934665603
    for x in b:
        h = ((h ^ x) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def array_offsets(img: bytes) -> dict:
    """Byte offset and count of every array in an image."""
    lib = L.load()
    at = 8 + 4 + 4 + 3 * 8 + 5 * 4 + lib.spmm_sizeof(1) + 4 + 2 * 8 + 8
    out = {}
    for name, size in ARRAYS:
        (count,) = struct.unpack_from("<Q", img, at)
        out[name] = (at + 8, count, size)
        at += 8 + count * size
    assert at == len(img) - 8
    return out


def reseal(img: bytearray) -> bytes:
    img[-8:] = struct.pack("<Q", fnv1a(bytes(img[:-8])))
    return bytes(img)


def load(img: bytes):
    lib = L.load()
    h = C.c_void_p()
    st = lib.spmm_plan_deserialize(img, len(img), 0, C.byref(h))
    if st == L.SPMM_OK:
        lib.spmm_plan_destroy(h)
    return st, lib.spmm_last_error().decode()


PLANS = [
    ("random", dict(mode="mixed", window_h=16, t_row=3, alpha_c=1 / 16, alpha=0.02,
                    row_order="length_sorted", seg_len=7)),
    ("random", dict(mode="plain", seg_len=5, pipeline=3)),
    ("random", dict(mode="mfma_only", window_h=32, seg_len=9)),
    ("block", dict(mode="mixed", row_order="original_ranges", seg_len=16, win_sched=1)),
    ("block", dict(mode="mixed", row_order="clustered", local_reorder=64, seg_len=16)),
    ("wide", dict(mode="mfma_only", window_h=16)),
]


def _matrix(kind):
    if kind == "random":
        return synth.random_csr(400, 300, 0.04, 7, dup_frac=0.05, empty_rows=0.05), "f32"
    if kind == "wide":
        return synth.random_csr(64, 8192, 0.3, 6), "f32"
    A, _ = synth.block_community(n=1024, band=4, n_cols=8, seed=5)
    return A, "bf16"


@pytest.mark.parametrize("case", range(len(PLANS)))
def test_round_trip_is_exact(case):
    kind, kw = PLANS[case]
    A, bk = _matrix(kind)
    p = api.Plan(A, 8, bk, api.default_opts(**kw), upload=False)
    img = p.serialize()
    q = api.Plan.deserialize(img, upload=False)
    d1, d2 = p.export(), q.export()
    for key in d1:
        if isinstance(d1[key], np.ndarray):
            assert np.array_equal(d1[key], d2[key]), key
    s1, s2 = p.stats(), q.stats()
    for key in s1:
        assert s1[key] == s2[key], key
    assert q.serialize() == img
    if kind == "wide":
        assert d1["wpart_win"].size > 0


def test_damaged_images_are_refused():
    A, bk = _matrix("random")
    img = api.Plan(A, 8, bk, api.default_opts(mode="mixed", alpha=0.02), upload=False).serialize()
    assert load(img)[0] == L.SPMM_OK
    flipped = bytearray(img)
    flipped[len(img) // 2] ^= 0x10
    assert load(bytes(flipped)) == (L.SPMM_ERR_INVALID, "plan image: checksum")
    assert load(img[:-20])[0] == L.SPMM_ERR_INVALID
    assert load(b"NOTAPLAN" + img[8:])[0] == L.SPMM_ERR_INVALID
    other = bytearray(img)
    other[8] = 99  # format version
    assert load(reseal(other))[0] == L.SPMM_ERR_UNSUPPORTED


def _crafted(img, name, index, value):
    off, count, size = array_offsets(img)[name]
    assert index < count
    b = bytearray(img)
    fmt = {1: "<B", 2: "<H", 4: "<i", 8: "<q"}[size]
    struct.pack_into(fmt, b, off + index * size, value)
    return reseal(b)


@pytest.mark.parametrize("name,index,value,msg", [
    ("rem_col", 3, 10 ** 6, "remainder column"),
    ("rem_ptr", 5, 10 ** 7, "remainder row pointers"),
    ("windows", 2, 400, "window row"),
    ("tile_cols", 1, 10 ** 6, "tile column"),
    ("tile_val_ptr", 1, 0, "tile value"),
    ("vitem_ptr", 1, 10 ** 6, "vector items"),
    ("seg_begin", 0, 0, "segments"),
    ("win_order", 0, 10 ** 6, "window order"),
    ("vitem_seg", 1, 10 ** 6, "item segment ids"),
])
def test_crafted_images_are_refused(name, index, value, msg):
    """An image whose checksum is valid but one index is out of range or
    inconsistent is refused by the invariant checks."""
    A, bk = _matrix("random")
    p = api.Plan(A, 8, bk, api.default_opts(mode="mixed", alpha=0.02, seg_len=7), upload=False)
    img = p.serialize()
    st, err = load(_crafted(img, name, index, value))
    assert st == L.SPMM_ERR_INVALID and msg in err, err


def test_windows_without_tiles_and_tiles_without_values_are_refused():
    """The window kernel reads a round's tile data at clamped indices and takes
    its rows' metadata in the first tile round, so an image with an empty
    window or a tile without values is refused."""
    A, bk = _matrix("block")
    p = api.Plan(A, 8, bk, api.default_opts(mode="mixed", row_order="original_ranges"),
                 upload=False)
    img = p.serialize()
    offs = array_offsets(img)
    assert offs["win_tile_ptr"][1] > 2
    # window 0 without tiles: its tiles moved to window 1 (win_tile_ptr[1] = 0)
    st, err = load(_crafted(img, "win_tile_ptr", 1, 0))
    assert st == L.SPMM_ERR_INVALID and "window without tiles" in err, err
    # tile 0 without values: bitmap words and value count both zero
    H = p.export()["window_h"]
    b = bytearray(img)
    off, _, _ = offs["tile_bitmap"]
    for s in range(H):
        struct.pack_into("<I", b, off + 4 * s, 0)
    off, _, _ = offs["tile_val_ptr"]
    struct.pack_into("<q", b, off + 8, 0)
    st, err = load(reseal(b))
    assert st == L.SPMM_ERR_INVALID and "tile without values" in err, err


def test_size_query_and_small_buffer():
    lib = L.load()
    A, bk = _matrix("random")
    p = api.Plan(A, 8, bk, api.default_opts(mode="plain"), upload=False)
    size = C.c_int64()
    assert lib.spmm_plan_serialize(p.handle, None, 0, C.byref(size)) == L.SPMM_OK
    buf = C.create_string_buffer(size.value)
    assert lib.spmm_plan_serialize(p.handle, buf, size.value - 1, C.byref(size)) == L.SPMM_ERR_INVALID
    assert lib.spmm_plan_deserialize(None, 0, 0, C.byref(C.c_void_p())) == L.SPMM_ERR_INVALID
