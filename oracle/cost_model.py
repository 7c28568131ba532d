"""Cost-model and tile-shape formulas of NeutronSparse (TEST INFRASTRUCTURE ONLY).

* Eq. 1: Cost_vec(NNZ) = NNZ / P_vec and Cost_mat = M*K / P_mat (vector cost
  proportional to stored entries, matrix cost to the full tile volume).
* Eq. 2: NNZ* = argmin over NNZ of (Cost_vec(NNZ)/Cost_mat - r)^2.
* Eq. 3: alpha = NNZ*/(M*K) = r * P_vec / P_mat.
* Eq. 5: Thres = alpha * K (a density turned into a length).
* Eq. 6: Skew = max(dt_a, dt_b) / min(dt_a, dt_b) >= 1; rebalancing triggers
  only when Skew > 1 + eps (Sec. 5.3, eps = 0.05).
* Eq. 8: double-buffered residency limits for an (M, N, K) tile:
  2*M*K <= C_A/2, 2*N*K <= C_B/2, 4*M*N <= C_C/2; fp16 input traffic of a
  tile is 2*(M*K + N*K) bytes (Sec. 6.2.2).
"""
from __future__ import annotations


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
