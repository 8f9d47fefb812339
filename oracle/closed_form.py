"""Closed forms for N independent cyclic L-state processes — TEST INFRASTRUCTURE.

Each process steps l -> (l + 1) mod L with no guard, interleaved.  A state is
a vector of N local states; BFS distance from the all-zero vector is the sum of
the locals (each local can only be advanced one step at a time, and reaching l
needs exactly l steps of that process, 0 <= l < L).  Hence:

* total reachable states  = L^N
* edges (every state enables N steps) = N * L^N
* deadlocks = 0 for L >= 2 (for L == 1 every step is a self-loop: still 0)
* number of levels = N (L - 1) + 1
* level_counts[d] = #{x in [0, L)^N : sum(x) = d}
                  = [x^d] ((1 - x^L) / (1 - x))^N
                  = sum_j (-1)^j C(N, j) C(d - j L + N - 1, N - 1)
  (inclusion-exclusion over the j coordinates forced to be >= L).
"""
from __future__ import annotations

from math import comb


def cyclic_level_counts(N: int, L: int) -> list[int]:
    out = []
    for d in range(N * (L - 1) + 1):
        c = 0
        for j in range(N + 1):
            m = d - j * L + N - 1
            if m < N - 1:
                break
            c += (-1) ** j * comb(N, j) * comb(m, N - 1)
        out.append(c)
    return out


def cyclic_summary(N: int, L: int) -> dict:
    lv = cyclic_level_counts(N, L)
    return dict(total=L ** N, n_levels=len(lv), level_counts=lv,
                edges=N * L ** N, deadlocks=0, capped=False)


def cyclic_capped(N: int, L: int, cap: int) -> dict:
    """Level-prefix cap applied to the closed form."""
    lv = cyclic_level_counts(N, L)
    if not cap or sum(lv) <= cap:
        return cyclic_summary(N, L)
    acc, last = 0, -1
    for d, c in enumerate(lv):
        if acc + c > cap:
            break
        acc += c
        last = d
    kept = lv[: last + 1]
    # every state has exactly N successors; levels 0..last-1 are expanded
    return dict(total=acc, n_levels=len(kept), level_counts=kept,
                edges=N * sum(kept[:-1]), deadlocks=0, capped=True)
