"""Cost-model and tile-shape formulas of NeutronSparse (TEST INFRASTRUCTURE ONLY).

* Eq. 1: Cost_vec(NNZ) = NNZ / P_vec and Cost_mat = M*K / P_mat (vector cost
  proportional to stored entries, matrix cost to the full tile volume).
* Eq. 2: NNZ* = argmin over NNZ of (Cost_vec(NNZ)/Cost_mat - r)^2.
* Eq. 3: alpha = NNZ*/(M*K) = r * P_vec / P_mat.
* Eq. 5: Thres = alpha * K (a density turned into a length).
* Eq. 6: Skew = max(dt_a, dt_b) / min(dt_a, dt_b) >= 1; rebalancing triggers
  only when Skew > 1 + eps (Sec. 5.3, eps = 0.05).
* Sec. 5.3 (Eq. 6-7) read for one engine pool: an epoch measures the two
  paths' times, turns them into throughputs (Eq. 1 inverted), takes the
  crossover alpha* = P_vec / P_mat (Eq. 3 and Eq. 7 with r = 1), and applies
  Eq. 6 to the two paths' times for a tile of the current threshold density
  (which reduces to max(alpha, alpha*) / min(alpha, alpha*)).  Above 1 + eps
  the threshold moves towards alpha* inside a bracket of earlier thresholds
  (a secant step on log(alpha*/alpha) over two epochs when it falls inside,
  else at most the geometric midpoint to the bracket end, and a bracket end
  contradicted by two capped steps is dropped), at most 7 rounds.
* Eq. 8: double-buffered residency limits for an (M, N, K) tile:
  2*M*K <= C_A/2, 2*N*K <= C_B/2, 4*M*N <= C_C/2; fp16 input traffic of a
  tile is 2*(M*K + N*K) bytes (Sec. 6.2.2).
"""
from __future__ import annotations

import math


def cost_vec(nnz, p_vec):
    """Eq. 1, vector engine."""
    return nnz / p_vec


def cost_mat(m, k, p_mat):
    """Eq. 1, matrix engine."""
    return (m * k) / p_mat


def nnz_star_bruteforce(m, k, p_vec, p_mat, r):
    """Eq. 2 by exhaustive search over the integers 0..M*K (ties -> smaller)."""
    best, best_val = 0, None
    cm = cost_mat(m, k, p_mat)
    for nnz in range(m * k + 1):
        val = (cost_vec(nnz, p_vec) / cm - r) ** 2
        if best_val is None or val < best_val:
            best, best_val = nnz, val
    return best


def alpha_closed_form(p_vec, p_mat, r):
    """Eq. 3."""
    return r * p_vec / p_mat


def thres(alpha, k):
    """Eq. 5."""
    return alpha * k


def skew(dt_a, dt_b):
    """Eq. 6."""
    return max(dt_a, dt_b) / min(dt_a, dt_b)


def should_migrate(dt_a, dt_b, eps=0.05):
    """Sec. 5.3: rebalance only when Skew exceeds 1 + eps."""
    return skew(dt_a, dt_b) > 1.0 + eps


def tile_limits(cap_a, cap_b, cap_c, in_bytes=2, acc_bytes=4):
    """Eq. 8 solved for the products: returns (max MK, max NK, max MN) with
    every buffer double-buffered (each tile may use half of it)."""
    return (cap_a // 2 // in_bytes, cap_b // 2 // in_bytes, cap_c // 2 // acc_bytes)


def tile_feasible(m, n, k, cap_a, cap_b, cap_c, in_bytes=2, acc_bytes=4, multiple=16):
    """Eq. 8 feasibility of an (M, N, K) tile, plus the multiple-of-16 rule."""
    mk, nk, mn = tile_limits(cap_a, cap_b, cap_c, in_bytes, acc_bytes)
    return (m * k <= mk and n * k <= nk and m * n <= mn
            and m % multiple == 0 and n % multiple == 0 and k % multiple == 0)


def tile_input_bytes(m, n, k, in_bytes=2):
    """Input traffic of one tile: the A tile plus the B tile (Sec. 6.2.2)."""
    return in_bytes * (m * k + n * k)


def path_throughputs(t_vec, t_mat, w_vec, w_tile, w_winrem, p_vec_dry, p_mat_dry):
    """Eq. 1 inverted on one epoch.  t_vec: time of the vector path (segment
    and vector kernels), which gathered w_vec entries; t_mat: time of the
    window kernels, which computed w_tile tile slots and also gathered
    w_winrem remainder entries of window rows (charged at P_vec).  A path
    with no work takes the fallback throughput (the last one measured, else
    the dry run's)."""
    if w_vec > 0 and t_vec > 0:
        p_vec = w_vec / t_vec
    else:
        p_vec = p_vec_dry
    if w_tile > 0 and t_mat > 0:
        t_tiles = t_mat - w_winrem / p_vec
        if t_tiles < 0.1 * t_mat:
            t_tiles = 0.1 * t_mat
        p_mat = w_tile / t_tiles
    else:
        p_mat = p_mat_dry
    return p_vec, p_mat


def adapt_next(alpha, lo, hi, rounds, prev_alpha, prev_star, capped, p_vec, p_mat, eps=0.05,
               r=1.0, max_rounds=7):
    """One epoch of the adaptive re-partition.  (lo, hi) bracket the
    threshold (0 = open); (prev_alpha, prev_star) is the previous epoch's
    threshold and measured crossover (0 = none); capped is +1 / -1 when the
    previous step was cut at the bracket midpoint going up / down, else 0.
    Returns (next alpha, lo, hi, rounds, alpha*, skew, replan, capped).

    The next threshold is the secant estimate of where the measured
    crossover meets the threshold (in logarithms, from this epoch and the
    previous one) when it lies strictly inside the updated bracket, on
    alpha*'s side of alpha and at most twice as far (in logarithms) as
    alpha*; else alpha* itself, but never more than the geometric midpoint
    towards a known bracket end -- unless the previous step was cut the same
    way, in which case that bracket end is dropped (two newer measurements
    outvote the one that set it) and the step goes to alpha*."""
    a_star = min(1.0, alpha_closed_form(p_vec, p_mat, r))
    s = skew(alpha, a_star)
    if s <= 1.0 + eps or rounds >= max_rounds:
        return alpha, lo, hi, rounds, a_star, s, False, capped
    raise_it = a_star > alpha
    # bracket: the threshold must rise above alpha, or fall below it
    if raise_it:
        lo = alpha
    else:
        hi = alpha
    if prev_alpha > 0 and prev_star > 0 and prev_alpha != alpha:
        f = math.log(a_star / alpha)
        f_prev = math.log(prev_star / prev_alpha)
        if f != f_prev:
            x = math.log(alpha) - f * (math.log(alpha) - math.log(prev_alpha)) / (f - f_prev)
            cand = math.exp(x)
            d = x - math.log(alpha)
            inside = (lo <= 0 or cand > lo) and (hi <= 0 or cand < hi)
            if inside and d * f > 0 and abs(d) <= 2.0 * abs(f):
                return cand, lo, hi, rounds + 1, a_star, s, True, 0
    if raise_it:
        # the tiles at the threshold cost more on the matrix path: move the
        # sparser tiles to the vector path
        if hi > 0 and a_star >= math.sqrt(alpha * hi):
            if capped == 1:
                return a_star, lo, 0.0, rounds + 1, a_star, s, True, 0
            return math.sqrt(alpha * hi), lo, hi, rounds + 1, a_star, s, True, 1
    else:
        # rows just below the threshold cost more on the vector path: pack
        # them into tiles
        if lo > 0 and a_star <= math.sqrt(alpha * lo):
            if capped == -1:
                return a_star, 0.0, hi, rounds + 1, a_star, s, True, 0
            return math.sqrt(alpha * lo), lo, hi, rounds + 1, a_star, s, True, -1
    return a_star, lo, hi, rounds + 1, a_star, s, True, 0
