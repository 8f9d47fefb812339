"""How often a successor repeats another successor of the same expansion pass
(CPU, no GPU): the premise of merging equal successors of a pass before
find-or-put.

Interleavings of independent moves reach one state from several frontier
states (a -> b -> d and a -> c -> d), and a level's states are appended in
the order they were found, so neighbouring frontier states share
successors.  This replays the 12x16 benchmark model's BFS in that order,
cuts each level into tiles of 256 states and each tile's successors into
passes of 256 (the expansion's shapes), and counts the successors that equal
an earlier successor of their pass or tile.  Successors come from the
oracle's successor function; the order is sequential, which is the order a
workgroup appends a tile's new states in."""
import numpy as np

import gen
import oracle

TILE = PASS = 256


def repeat_rates(model, cap):
    s0 = np.asarray(model.init, dtype=np.uint32)
    seen = {s0.tobytes()}
    front = [s0]
    edges = in_pass = in_tile = 0
    while front and len(seen) < cap:
        nxt = []
        for t0 in range(0, len(front), TILE):
            succ = [s.tobytes() for st in front[t0:t0 + TILE] for s in oracle.successors(model, st)]
            tile_set = set()
            for p0 in range(0, len(succ), PASS):
                pass_set = set()
                for b in succ[p0:p0 + PASS]:
                    edges += 1
                    in_pass += b in pass_set
                    in_tile += b in tile_set
                    pass_set.add(b)
                    tile_set.add(b)
                    if b not in seen:
                        seen.add(b)
                        nxt.append(np.frombuffer(b, dtype=np.uint32))
        front = nxt
    return edges, in_pass / edges, in_tile / edges


def test_pass_repeats_of_the_benchmark_model():
    edges, pass_rate, tile_rate = repeat_rates(gen.big_model(cap=1 << 18), 1 << 18)
    print(f"\n{edges} edges: {pass_rate:.3f} repeat within their pass, {tile_rate:.3f} within their tile")
    # a pass is part of its tile, so its repeats are a subset of the tile's
    assert pass_rate <= tile_rate
    # about a quarter of the successors repeat within their pass (23-25 %)
    assert 0.18 < pass_rate < 0.32


def test_no_repeats_without_shared_successors():
    # one process stepping round a cycle of 3000 local states: every state
    # has one successor (the last one's is the initial state), and no two
    # states share one
    edges, pass_rate, tile_rate = repeat_rates(gen.chain_model(3000), 1 << 20)
    assert edges == 3000 and pass_rate == 0.0 and tile_rate == 0.0
