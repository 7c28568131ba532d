"""GPU tests of the continuous-batching server: every result is bitwise the
same alone and in the mix; results match the FP64 oracle; requests that can
never fit the HBM budget are rejected while the rest are served."""
import numpy as np
import pytest

from gpu_util import TOL_16, TOL_F32, oracle_of
import oracle
from paper_2606_22482_amd import api, serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pool():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return synth.serving_pool(n_graphs=4, n_masks=2, seed=7, max_rows=20000, max_mask_rows=4096)


def test_mix_equals_solo_and_oracle(pool):
    import torch
    reqs = synth.serving_requests(60, len(pool), 4, seed=7, rate=2000.0)
    srv = serve.Server(pool, n_streams=3, max_batch=8, keep_results=True)
    stats = srv.run(reqs, realtime=True)
    s = stats.summary()
    assert s["completed"] == 60 and s["rejected"] == 0
    assert s["batches"] >= 2 and s["p99_ms"] >= s["p50_ms"] > 0
    for d, r in zip(reqs, srv.requests):
        B, C = srv.solo(d)
        assert torch.equal(B, r.B)
        assert torch.equal(C, r.C), "request %d differs alone vs in the mix" % r.rid
    for r in srv.requests:
        A = pool[r.matrix]["A"]
        Bh = r.B.float().cpu().numpy()
        Cs, S = oracle_of(A, Bh, "f32")
        err = oracle.max_normalised_error(r.C.cpu().numpy(), Cs, S)
        plan = srv.plans.plans[(r.matrix, r.n, r.b_kind)][0]
        tol = TOL_16 if plan.stats()["tol_class"] == 1 else TOL_F32
        assert err <= tol, (r.rid, err, tol)


def test_budget_rejects_and_keeps_serving(pool):
    reqs = synth.serving_requests(30, len(pool), 4, seed=8, rate=None)
    sizes = [pool[d["matrix"]]["A"].m for d in reqs]
    # a budget that the largest requests can never fit: the median B + C footprint
    foot = sorted(pool[d["matrix"]]["A"].m * d["n"] * (8 if d["b_kind"] == "f32" else 6)
                  for d in reqs)
    budget = foot[len(foot) // 2]
    srv = serve.Server(pool, budget_bytes=budget, n_streams=2, max_batch=4)
    s = srv.run(reqs, realtime=False).summary()
    assert s["rejected"] > 0 and s["completed"] > 0
    assert s["completed"] + s["rejected"] == 30
    for d, r in zip(reqs, srv.requests):
        # what the request occupies: B and C at least, plus its plan
        A = pool[r.matrix]["A"]
        io = A.k * r.n * (4 if r.b_kind == "f32" else 2) + A.m * r.n * 4
        assert r.footprint >= io and r.need > r.footprint
        if r.status == "rejected":
            assert r.need > budget, (r.rid, r.need, budget)
        else:
            assert r.status == "done" and r.need <= budget, (r.rid, r.need, budget)
    assert max(sizes) > 0


def test_library_footprint_and_budget_status(pool):
    """spmm_run_bytes: B + C + workspace (batched: the serial workspace; a
    run: the stream's workspace and counters), BUDGET above the budget."""
    from paper_2606_22482_amd import _lib as L
    A = pool[0]["A"]
    p = api.Plan(A, 64, "f32", api.default_opts(mode="plain", seg_len=32))
    st = p.stats()
    io = A.k * 64 * 4 + A.m * 64 * 4
    s0, b_batch = p.run_bytes(batched=True)
    s1, b_run = p.run_bytes(batched=False)
    assert s0 == s1 == L.SPMM_OK
    assert b_batch == io + st["workspace_bytes"]
    assert b_run >= b_batch  # plus the arrival counters of a co-scheduled run
    s2, b = p.run_bytes(batched=True, budget=b_batch - 1)
    assert s2 == L.SPMM_ERR_BUDGET and b == b_batch
    assert p.run_bytes(batched=True, budget=b_batch)[0] == L.SPMM_OK
    # wider leading dimensions count
    assert p.run_bytes(ldb=80, ldc=96, batched=True)[1] == b_batch + A.k * 16 * 4 + A.m * 32 * 4


def test_device_mask_pool_mix_equals_solo_and_oracle():
    """A pool with an attention mask built on the device (and planned there):
    every request equals its solo run bit for bit; sampled rows of every
    request match the oracle."""
    import torch
    pool = synth.serving_pool(n_graphs=2, n_masks=0, seed=9, max_rows=8000)
    pool.append({"kind": "mask", "A": synth.attention_mask_device(12000, seed=31)})
    reqs = synth.serving_requests(40, len(pool), 2, seed=9, rate=3000.0)
    srv = serve.Server(pool, n_streams=3, max_batch=8, keep_results=True)
    s = srv.run(reqs, realtime=True).summary()
    assert s["completed"] == 40 and s["rejected"] == 0
    masks = [r for r in srv.requests if pool[r.matrix]["kind"] == "mask"]
    assert masks
    mplan = srv.plans.plans[(masks[0].matrix, masks[0].n, masks[0].b_kind)][0]
    assert mplan.stats()["tiles"] > 0 and mplan.stats()["opts"]["window_h"] == 64
    rng = np.random.default_rng(4)
    for d, r in zip(reqs, srv.requests):
        B, C = srv.solo(d)
        assert torch.equal(C, r.C), "request %d differs alone vs in the mix" % r.rid
        A = pool[r.matrix]["A"]
        plan = srv.plans.plans[(r.matrix, r.n, r.b_kind)][0]
        tol = TOL_16 if plan.stats()["tol_class"] == 1 else TOL_F32
        Bh = r.B.float().cpu().numpy()
        if hasattr(A, "host_rows"):
            rows = np.unique(np.concatenate([rng.choice(A.m, 200, replace=False), [0, A.m - 1]]))
            Ar = A.host_rows(rows)
            Cs, S = oracle_of(Ar, Bh, "f32")
            err = oracle.max_normalised_error(r.C.cpu().numpy()[rows], Cs, S)
        else:
            Cs, S = oracle_of(A, Bh, "f32")
            err = oracle.max_normalised_error(r.C.cpu().numpy(), Cs, S)
        assert err <= tol, (r.rid, err, tol)


def test_large_requests_run_alone_and_small_ones_keep_a_stream(pool):
    """With every request classed large (threshold 0), each request runs
    alone (as a run, on one stream at a time by default); results equal the
    solo runs.  With no request large the classes do not change the results."""
    import torch
    reqs = synth.serving_requests(24, len(pool), 4, seed=12, rate=None)
    for large_ms, one_each in ((0.0, True), (1e9, False)):
        srv = serve.Server(pool, n_streams=3, max_batch=8, keep_results=True, large_ms=large_ms)
        s = srv.run(reqs, realtime=False).summary()
        assert s["completed"] == 24 and s["rejected"] == 0
        assert s["large"] == (24 if one_each else 0)
        if one_each:
            assert s["batches"] == 24 and s["mean_batch"] == 1.0
        for d, r in zip(reqs, srv.requests):
            B, C = srv.solo(d)
            assert torch.equal(C, r.C), (large_ms, r.rid)
