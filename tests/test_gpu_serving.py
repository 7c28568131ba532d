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
    for r in srv.requests[:6]:
        A = pool[r.matrix]["A"]
        Bh = r.B.float().cpu().numpy()
        Cs, S = oracle_of(A, Bh, "f32")
        err = oracle.max_normalised_error(r.C.cpu().numpy(), Cs, S)
        plan = srv.plans.plans[(r.matrix, r.n, r.b_kind)][0]
        tol = TOL_F32 if plan.stats()["opts"]["mode"] == 1 else TOL_16
        assert err <= tol


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
        if r.status == "rejected":
            A = pool[r.matrix]["A"]
            assert A.k * r.n * (4 if r.b_kind == "f32" else 2) + A.m * r.n * 4 > 0
        else:
            assert r.status == "done"
    assert max(sizes) > 0
