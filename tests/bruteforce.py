"""Brute-force references used to pin the oracle, independent of its code.

Dynamic-programming path costs are checked against explicit enumeration of
every disparity assignment along a short scanline (section 3.1.3: a path cost
is the smallest sum of matching costs plus smoothness penalties over all
disparity sequences reaching the pixel).  Only pure Python, tiny inputs.
"""
from __future__ import annotations

import itertools


def penalty(d_prev: int, d: int, p1: int, p2: int) -> int:
    """Smoothness penalty between consecutive pixels of a path: 0 for the same
    disparity, P1 for a change of one, P2 for any larger change."""
    k = abs(d - d_prev)
    return 0 if k == 0 else (p1 if k == 1 else p2)


def path_energy_min(costs, p1, p2):
    """BF_n(d): min over every assignment (d_1 .. d_n) with d_n = d of
    sum_i C_i(d_i) + sum_i penalty(d_{i-1}, d_i).  costs: list of n lists of D."""
    n, D = len(costs), len(costs[0])
    best = [None] * D
    for seq in itertools.product(range(D), repeat=n):
        e = sum(costs[i][seq[i]] for i in range(n))
        e += sum(penalty(seq[i - 1], seq[i], p1, p2) for i in range(1, n))
        if best[seq[-1]] is None or e < best[seq[-1]]:
            best[seq[-1]] = e
    return best


def normalised_path_costs(costs, p1, p2):
    """L_r along a scanline by enumeration.  The recurrence subtracts the
    predecessor's minimum after every pixel, which telescopes to
    L(p_n, d) = BF_n(d) - min_k BF_{n-1}(k)   (and L(p_1, d) = C_1(d))."""
    out = [list(costs[0])]
    for n in range(2, len(costs) + 1):
        bf_n = path_energy_min(costs[:n], p1, p2)
        prev_min = min(path_energy_min(costs[: n - 1], p1, p2))
        out.append([v - prev_min for v in bf_n])
    return out


def right_disparity_loop(S):
    """D_R(x, y) = first argmin over d < min(D, W - x) of S[y][x + d][d]."""
    H, W, D = len(S), len(S[0]), len(S[0][0])
    out = [[0] * W for _ in range(H)]
    for y in range(H):
        for x in range(W):
            best, bv = 0, S[y][x][0]
            for d in range(1, min(D, W - x)):
                if S[y][x + d][d] < bv:
                    best, bv = d, S[y][x + d][d]
            out[y][x] = best
    return out


def popcount(v: int) -> int:
    return bin(v).count("1")
