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


# ---- Sec. 5.3 adaptive re-partition (Eq. 6-7, one pool of CUs) -------------------------

def _plant(alpha, a_true, gamma):
    """Model device: the crossover measured at threshold alpha drifts from the
    true one as the split moves (log-linear, slope -gamma)."""
    return min(1.0, a_true * (a_true / alpha) ** gamma)


def _run_ref(a0, a_true, gamma, eps=0.05, max_epochs=9):
    alpha, lo, hi, rounds, pa, ps, capped = a0, 0.0, 0.0, 0, 0.0, 0.0, 0
    trace = []
    for _ in range(max_epochs):
        a_star = _plant(alpha, a_true, gamma)
        nxt, lo, hi, rounds2, a_s, s, replan, capped = cm.adapt_next(alpha, lo, hi, rounds, pa,
                                                                     ps, capped, a_star, 1.0,
                                                                     eps)
        trace.append((alpha, a_s, s, replan, lo, hi))
        if not replan:
            break
        pa, ps = alpha, a_s
        alpha, rounds = nxt, rounds2
    return trace


def test_adapt_fixed_point_trigger_and_direction():
    # alpha = alpha*: Eq. 6 skew 1, nothing moves
    nxt, lo, hi, rounds, a_s, s, replan, _ = cm.adapt_next(0.2, 0, 0, 0, 0, 0, 0, 2.0, 10.0)
    assert a_s == pytest.approx(0.2) and s == pytest.approx(1.0) and not replan
    # the trigger is Eq. 6's: Skew > 1 + eps
    for ratio in (1.04, 1.0499, 1.0501, 1.2, 1 / 1.2, 1 / 1.0501):
        a_star = 0.1 * ratio
        out = cm.adapt_next(0.1, 0, 0, 0, 0, 0, 0, a_star, 1.0)
        assert out[6] == cm.should_migrate(0.1, a_star)
    # direction: alpha* above -> threshold rises, lower bracket end set
    nxt, lo, hi, *_ = cm.adapt_next(0.05, 0, 0, 0, 0, 0, 0, 0.3, 1.0)
    assert nxt == pytest.approx(0.3) and lo == 0.05 and hi == 0
    nxt, lo, hi, *_ = cm.adapt_next(0.5, 0, 0, 0, 0, 0, 0, 0.1, 1.0)
    assert nxt == pytest.approx(0.1) and hi == 0.5 and lo == 0
    # never past the geometric midpoint towards a known bracket end
    nxt, lo, hi, *_ = cm.adapt_next(0.05, 0.0, 0.2, 1, 0, 0, 0, 0.9, 1.0)
    assert nxt == pytest.approx((0.05 * 0.2) ** 0.5)
    # at most 7 re-partitions
    assert not cm.adapt_next(0.05, 0, 0, 7, 0, 0, 0, 0.9, 1.0)[6]


def test_adapt_balance_at_the_crossover():
    """Eq. 7 with r = 1: at alpha = P_vec / P_mat a tile of threshold density
    costs the same on both paths (Eq. 1)."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        pv, pm = rng.uniform(1, 100, size=2)
        if pv >= pm:
            continue
        a = cm.adapt_next(0.5, 0, 0, 0, 0, 0, 0, pv, pm)[4]
        m, k = 16, 32
        assert cm.cost_vec(a * m * k, pv) == pytest.approx(cm.cost_mat(m, k, pm), rel=1e-12)


@pytest.mark.parametrize("gamma", [0.0, 0.3, 0.6, 0.9, 1.2, 1.5, 1.9, 3.0])
def test_adapt_converges_on_a_model_device(gamma):
    for a0 in (0.002, 0.01, 0.05, 0.3, 1.0):
        for a_true in (0.02, 0.1, 0.5):
            tr = _run_ref(a0, a_true, gamma)
            last = tr[-1]
            assert not last[3] and last[2] <= 1.05, (gamma, a0, a_true, tr)
            assert len(tr) - 1 <= 7
            for alpha, _, _, replan, lo, hi in tr[:-1]:
                # the bracket always contains the next threshold
                assert (lo == 0 or lo <= alpha) and (hi == 0 or alpha <= hi)


def test_path_throughputs():
    # window kernels: tiles plus window-row remainders charged at the vector rate
    pv, pm = cm.path_throughputs(2.0, 3.0, 100.0, 400.0, 50.0, 1.0, 1.0)
    assert pv == 50.0 and pm == pytest.approx(400.0 / (3.0 - 1.0))
    # a path without work takes the dry run
    assert cm.path_throughputs(0.0, 3.0, 0.0, 400.0, 0.0, 7.0, 9.0)[0] == 7.0
    assert cm.path_throughputs(2.0, 0.0, 100.0, 0.0, 0.0, 7.0, 9.0)[1] == 9.0
    # the tiles keep at least a tenth of the window time
    assert cm.path_throughputs(1.0, 1.0, 100.0, 10.0, 1000.0, 1, 1)[1] == pytest.approx(100.0)


def test_adapt_secant_never_extrapolates_wildly():
    # two epochs whose crossovers barely differ put the secant root far away
    # (about 4e-6 here); the step falls back to alpha* itself
    nxt, lo, hi, rounds, a_s, s, replan, _ = cm.adapt_next(0.2596, 0.0, 0.9, 1, 0.9, 0.2596, 0,
                                                           0.085, 1.0)
    assert replan and nxt == pytest.approx(0.085) and hi == 0.2596
    # a secant root on alpha*'s side within twice its distance is taken: on a
    # log-linear device (crossover 0.1 * (0.1 / alpha) ** 0.5) it is exact
    plant = lambda a: 0.1 * (0.1 / a) ** 0.5
    nxt, lo, hi, *_ = cm.adapt_next(0.2, 0.0, 0.4, 1, 0.4, plant(0.4), 0, plant(0.2), 1.0)
    assert nxt == pytest.approx(0.1, rel=1e-12) and hi == 0.2


def test_adapt_drops_a_contradicted_bracket_end():
    # an early outlier set lo = 0.12; later epochs keep measuring 0.10 below it
    nxt, lo, hi, _, _, _, replan, capped = cm.adapt_next(0.15, 0.12, 0.2, 2, 0, 0, 0, 0.10, 1.0)
    assert replan and nxt == pytest.approx((0.15 * 0.12) ** 0.5) and capped == -1
    nxt, lo, hi, _, _, _, replan, capped = cm.adapt_next(nxt, lo, hi, 3, 0, 0, capped, 0.10, 1.0)
    assert replan and nxt == pytest.approx(0.10) and lo == 0.0 and capped == 0


@pytest.mark.parametrize("outlier", [1.6, 0.6])
def test_adapt_converges_after_an_outlier(outlier):
    rng = np.random.default_rng(5)
    for _ in range(100):
        g = rng.uniform(0, 2)
        a0 = float(np.exp(rng.uniform(np.log(0.002), 0)))
        at = float(np.exp(rng.uniform(np.log(0.01), np.log(0.8))))
        alpha, lo, hi, rounds, pa, ps, capped = a0, 0.0, 0.0, 0, 0.0, 0.0, 0
        for epoch in range(9):
            a_star = _plant(alpha, at, g) * (outlier if epoch == 1 else 1.0)
            nxt, lo, hi, rounds, a_s, s, replan, capped = cm.adapt_next(
                alpha, lo, hi, rounds, pa, ps, capped, min(a_star, 1.0), 1.0)
            if not replan:
                break
            pa, ps, alpha = alpha, a_s, nxt
        assert s <= 1.05 and rounds <= 7
