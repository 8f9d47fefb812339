"""Brute-force reachability by product enumeration — TEST INFRASTRUCTURE ONLY.

An algorithm independent of the BFS oracle, used to pin it: no hash set, no
queue.  Every state of the product space (locals in [0, L)^P, shared values in
[0, D)^S) gets an index in mixed radix.  For every (process, transition) pair
the successor index of every product state is computed at once with numpy, and
BFS distances from s0 come from repeated relaxation
``dist[v] = min(dist[v], dist[u] + 1)`` over all enabled edges until nothing
changes (Bellman-Ford on unit weights).  Reachable = finite distance.

The next-state semantics are the same definition as the oracle's (asynchronous
interleaving, guard read on the source state), written out again here in array
form.  The cap rule is the level-prefix reading: keep the longest prefix of
levels whose cumulative count is <= cap; if that cuts anything off, edges and
deadlocks cover only the levels before the last kept one.
"""
from __future__ import annotations

import numpy as np

NONE = 0xFFFFFFFF
MAX_PRODUCT = 1 << 22


def product_size(model) -> int:
    return int(model.L) ** model.P * int(max(model.D, 1)) ** model.S


def brute(model, cap: int | None = None, with_states: bool = False) -> dict:
    cap = model.cap if cap is None else cap
    P, L, S, K = model.P, model.L, model.S, model.K
    D = max(model.D, 1)
    W = P + S
    radix = np.array([L] * P + [D] * S, dtype=np.int64)
    N = int(np.prod(radix))
    if N > MAX_PRODUCT:
        raise ValueError(f"product space {N} too large for brute force")
    init = np.asarray(model.init, dtype=np.int64)
    if np.any(init >= radix):
        raise ValueError("initial state outside the product domain")

    # decode every product index into its state vector (mixed radix, word 0
    # least significant)
    place = np.cumprod(np.concatenate([[1], radix[:-1]]))
    idx = np.arange(N, dtype=np.int64)
    states = (idx[:, None] // place[None, :]) % radix[None, :]      # [N, W]

    trans = np.asarray(model.trans, dtype=np.int64)                 # [P, L, K, 5]
    succ_idx = []      # per (p, k): successor index of each product state
    enabled = []       # per (p, k): bool mask
    for p in range(P):
        for k in range(K):
            t = trans[p, states[:, p], k]                           # [N, 5]
            gvar, gval, evar, evl = t[:, 1], t[:, 2], t[:, 3], t[:, 4]
            ok = gvar == NONE
            has_g = ~ok
            if np.any(has_g):
                col = (P + gvar[has_g]).astype(np.int64)
                ok[has_g] = states[has_g, col] == gval[has_g]
            nxt = states.copy()
            nxt[:, p] = t[:, 0]
            has_e = evar != NONE
            if np.any(has_e):
                col = (P + evar[has_e]).astype(np.int64)
                nxt[has_e, col] = evl[has_e]
            # successors must stay inside the enumerated domain
            inside = np.all(nxt < radix[None, :], axis=1)
            if np.any(ok & ~inside):
                raise ValueError("successor outside the product domain")
            succ_idx.append((nxt * place[None, :]).sum(axis=1))
            enabled.append(ok)

    INF = np.iinfo(np.int64).max // 2
    dist = np.full(N, INF, dtype=np.int64)
    dist[int((init * place).sum())] = 0
    while True:
        before = dist.copy()
        for si, ok in zip(succ_idx, enabled):
            src = ok & (dist < INF)
            np.minimum.at(dist, si[src], dist[src] + 1)
        if np.array_equal(before, dist):
            break

    reach = dist < INF
    outdeg = np.zeros(N, dtype=np.int64)
    for ok in enabled:
        outdeg += ok
    levels = np.bincount(dist[reach]).astype(np.int64)
    cum = np.cumsum(levels)
    capped = bool(cap) and int(cum[-1]) > cap
    if capped:
        last = int(np.nonzero(cum <= cap)[0].max())
        levels = levels[: last + 1]
        expanded = reach & (dist < last)
    else:
        expanded = reach
    out = dict(total=int(levels.sum()), n_levels=len(levels),
               level_counts=[int(x) for x in levels],
               edges=int(outdeg[expanded].sum()),
               deadlocks=int((outdeg[expanded] == 0).sum()),
               capped=capped)
    if with_states:
        keep = reach & (dist < len(levels))
        out["states"] = states[keep].astype(np.uint32)      # product-index order
        out["dist"] = dist[keep]
    return out
