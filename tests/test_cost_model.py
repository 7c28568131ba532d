"""Pins for the cost model (Eq. 1-3, 6, 8) and the statistics of Tables 1-2."""
import csv
import json
import os

import numpy as np
import pytest

from oracle import cost_model as cm
from oracle import stats
from paper_2606_22482_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("m,k,pv,pm,r", [(4, 5, 3.0, 7.0, 2.0), (6, 6, 1.0, 9.0, 1.0),
                                           (3, 7, 2.5, 4.0, 2.0), (5, 5, 10.0, 1.0, 0.5)])
def test_eq2_bruteforce_matches_eq3(m, k, pv, pm, r):
    nstar = cm.nnz_star_bruteforce(m, k, pv, pm, r)
    alpha = cm.alpha_closed_form(pv, pm, r)
    target = alpha * m * k
    if target >= m * k:
        assert nstar == m * k
    else:
        lo = int(np.floor(target))
        best = lo if (target - lo) <= (lo + 1 - target) else lo + 1
        assert nstar == best


def test_eq8_with_ascend_constants():
    g = json.load(open(os.path.join(GOLDEN, "eq8_ascend.json")))
    caps = g["capacities_bytes"]
    assert cm.tile_limits(caps["L0A"], caps["L0B"], caps["L0C"]) == tuple(g["limits_MK_NK_MN"])
    for shape, kb in g["input_traffic_kb"].items():
        m, n, k = (int(x) for x in shape.split(","))
        assert cm.tile_input_bytes(m, n, k) == kb * 1024
        assert cm.tile_feasible(m, n, k, caps["L0A"], caps["L0B"], caps["L0C"])
    # one step past the chosen tile breaks the output-buffer limit
    assert not cm.tile_feasible(128, 512, 32, caps["L0A"], caps["L0B"], caps["L0C"])
    assert not cm.tile_feasible(128, 256, 72, caps["L0A"], caps["L0B"], caps["L0C"])


def test_eq6_skew_and_trigger():
    assert cm.skew(2.0, 1.0) == cm.skew(1.0, 2.0) == 2.0
    assert cm.skew(3.0, 3.0) == 1.0
    assert not cm.should_migrate(1.05, 1.0)
    assert cm.should_migrate(1.0501, 1.0)
    assert cm.thres(0.002, 1000) == pytest.approx(2.0)


def _table2():
    with open(os.path.join(GOLDEN, "table2_stats.csv")) as f:
        rows = [r for r in csv.reader(f) if r and not r[0].startswith("#")]
    return rows[1:]


@pytest.mark.parametrize("row", _table2(), ids=lambda r: r[0])
def test_table2_avgl_and_density(row):
    abbr, n, nnz, avgl, dens, _ = row
    n, nnz = int(n), int(nnz)
    # AvgL printed to one decimal (one row differs by one unit in that digit)
    assert abs(stats.avg_len(nnz, n) - float(avgl)) <= 0.1 + 1e-9
    # Dens printed in units of 1e-3 to two decimals
    assert round(stats.density(nnz, n, n) * 1e3, 2) == pytest.approx(float(dens), abs=1e-9)


def test_row_skew_bruteforce():
    A = synth.random_csr(97, 50, 0.1, 8)
    lens = np.diff(A.rowptr)
    top = int(np.ceil(0.1 * lens.size))
    expect = sum(sorted(lens.tolist(), reverse=True)[:top]) / lens.sum()
    assert stats.row_skew(A.rowptr) == pytest.approx(expect)


def _zero_fraction_loops(P, t):
    m, k = P.shape
    z = a = 0
    for i in range(0, m, t):
        for j in range(0, k, t):
            blk = np.zeros((t, t), dtype=bool)
            sub = P[i:i + t, j:j + t]
            blk[:sub.shape[0], :sub.shape[1]] = sub
            if blk.any():
                a += t * t
                z += t * t - blk.sum()
    return z / a if a else 0.0


@pytest.mark.parametrize("t", [4, 16])
def test_table1_measure(t):
    rng = np.random.default_rng(1)
    P = rng.random((70, 45)) < 0.05
    A = synth.csr_from_coo(70, 45, *np.nonzero(P), np.ones(P.sum(), np.float32), "f32")
    assert stats.active_tile_zero_fraction(A.rowptr, A.colidx, 70, 45, t) == pytest.approx(
        _zero_fraction_loops(P, t))
    # closed forms: a diagonal gives 1 - 1/t; a full matrix gives 0
    n = 64
    D = synth.csr_from_coo(n, n, np.arange(n), np.arange(n), np.ones(n, np.float32), "f32")
    assert stats.active_tile_zero_fraction(D.rowptr, D.colidx, n, n, t) == pytest.approx(1 - 1 / t)
    F = np.ones((32, 32), dtype=bool)
    Af = synth.csr_from_coo(32, 32, *np.nonzero(F), np.ones(1024, np.float32), "f32")
    assert stats.active_tile_zero_fraction(Af.rowptr, Af.colidx, 32, 32, t) == 0.0
    assert stats.empty_tile_fraction(D.rowptr, D.colidx, n, n, 16) == pytest.approx(1 - 4 / 16)
