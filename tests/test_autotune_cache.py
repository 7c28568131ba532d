"""CPU tier for the autotuner's host side: the sparsity-profile key and the
tuned-options cache that spmm_plan(mode=AUTO) consults."""
import os

import numpy as np

from paper_2606_22482_amd import _lib as L
from paper_2606_22482_amd import api, synth


def test_profile_key_deterministic_and_structural():
    A = synth.chung_lu_graph(20000, 2.1, 16.0, 2000.0, 3)
    k1 = api.spmm_profile_key(A, 64, "f32")
    assert k1 == api.spmm_profile_key(A, 64, "f32")
    assert k1 != api.spmm_profile_key(A, 128, "f32")
    Bc, _ = synth.block_community(n=16384, band=8, n_cols=8, seed=2)
    kb = api.spmm_profile_key(Bc, 64, "f32")
    assert kb != k1
    # block structure shares columns inside 16-row windows, the random graph does not
    share = lambda k: int(k.split(" w")[-1])
    assert share(kb) >= 7 and share(k1) <= 2
    # histogram tenths: the uniform matrix has all entries in the 16..31 bucket
    U, _ = synth.uniform_rows()
    hist = api.spmm_profile_key(U, 32, "f32").split(" h")[1].split(" ")[0].split(",")
    assert hist[4] == "10" and sum(int(x) for x in hist) == 10


def test_cache_put_get_save_load(tmp_path):
    api.tune_cache_clear()
    o = api.default_opts(mode="mixed", window_h=32, t_row=5, alpha_c=0.125, alpha=0.25,
                         row_order="length_sorted", seg_len=77)
    api.tune_cache_put("key one", o)
    got = api.tune_cache_get("key one")
    assert api.opts_dict(got) == api.opts_dict(o)
    assert api.tune_cache_get("missing") is None
    path = str(tmp_path / "tune.txt")
    api.tune_cache_save(path)
    api.tune_cache_clear()
    assert api.tune_cache_get("key one") is None
    api.tune_cache_load(path)
    assert api.opts_dict(api.tune_cache_get("key one")) == api.opts_dict(o)
    api.tune_cache_clear()


def test_auto_plan_uses_cached_profile():
    api.tune_cache_clear()
    A = synth.random_csr(600, 6000, 0.001, 5)
    key = api.spmm_profile_key(A, 16, "f32")
    p = api.Plan(A, 16, "f32", api.default_opts(mode="auto"), upload=False)
    assert p.stats()["opts"]["mode"] == L.MODE_PLAIN_F32       # heuristic: too few tiles
    tuned = api.default_opts(mode="mixed", window_h=32, t_row=-1, alpha_c=0.0, alpha=0.0,
                             seg_len=33)
    api.tune_cache_put(key, tuned)
    # f32 B: the profile's other options apply, but AUTO stays on the FP32 path
    q = api.Plan(A, 16, "f32", api.default_opts(mode="auto"), upload=False)
    so = q.stats()["opts"]
    assert so["mode"] == L.MODE_PLAIN_F32 and so["seg_len"] == 33 and q.stats()["tiles"] == 0
    # 16-bit B (its own profile key): the tuned mixed plan is used as stored
    key16 = api.spmm_profile_key(A, 16, "bf16")
    assert key16 != key
    api.tune_cache_put(key16, tuned)
    q = api.Plan(A, 16, "bf16", api.default_opts(mode="auto"), upload=False)
    so = q.stats()["opts"]
    assert so["mode"] == L.MODE_MIXED and so["window_h"] == 32 and so["seg_len"] == 33
    assert q.stats()["tiles"] > 0
    # explicit modes are not overridden
    r = api.Plan(A, 16, "f32", api.default_opts(mode="plain"), upload=False)
    assert r.stats()["opts"]["mode"] == L.MODE_PLAIN_F32
    api.tune_cache_clear()
