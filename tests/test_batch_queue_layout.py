"""The work tables of the batch queue launch, built by the library's own host code
(fe_batch_queue_layout; no device work), checked for the properties the kernel relies on:

* every (matrix, tile, layer) item appears exactly once, all of a matrix's items in one queue;
* each queue is layer-major, and an item's `need` is its layer times the matrix's upper tiles;
* every item's dependencies (the matrix's items of earlier layers) come before it in its queue,
  so the smallest unfinished ticket can always proceed;
* matrices are dealt, in batch order, to the queue with the least work so far (tiles x size).

A discrete-event run of the protocol (workers take tickets in order, an item starts once its
matrix's completion count reaches `need`) then completes every item, in every tried order of
completion times.
"""
import os

import numpy as np
import pytest

from paper_2605_08523_amd import api


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(api.LIB_PATH):
        pytest.fail("libfe.so is not built (python -m paper_2605_08523_amd.build)")
    api.lib()


def batch(rng, count, tile, sort):
    nps = [int(rng.integers(1, 768 // tile + 1)) * tile for _ in range(count)]
    Ls = [int(rng.integers(1, 9)) for _ in range(count)]
    if sort:   # the plan's order: more layers first, then larger matrices
        order = sorted(range(count), key=lambda i: (-Ls[i], -nps[i]))
        nps, Ls = [nps[i] for i in order], [Ls[i] for i in order]
    return nps, Ls


def simulate(items, qoff, counts, workers, rng):
    """Workers of each queue take tickets in order; a worker starts its item once the matrix has
    completed `need` items, and finishes it after a random time. Returns True when all items
    finish (False: no worker could ever proceed)."""
    done = np.zeros(len(counts), dtype=np.int64)
    for x in range(len(qoff) - 1):
        q = items[qoff[x]:qoff[x + 1]]
        nxt = 0
        busy = []   # [finish time, matrix] of running items; waiting tickets held in `held`
        held = []
        t = 0.0
        while nxt < len(q) or busy or held:
            while len(busy) + len(held) < workers and nxt < len(q):
                held.append(q[nxt])
                nxt += 1
            started = True
            while started:
                started = False
                for it in list(held):
                    if done[it[0]] >= it[3]:
                        held.remove(it)
                        busy.append([t + rng.uniform(0.5, 2.0), it[0]])
                        started = True
            if not busy:
                return False
            busy.sort()
            t, m = busy.pop(0)
            done[m] += 1
    return bool(np.all(done == counts))


@pytest.mark.parametrize("tile", [128, 64])
@pytest.mark.parametrize("nq", [1, 3, 8])
@pytest.mark.parametrize("sort", [True, False])
def test_queue_tables(tile, nq, sort):
    rng = np.random.default_rng(1000 * tile + 10 * nq + sort)
    for trial in range(12):
        count = int(rng.integers(1, 30))
        nps, Ls = batch(rng, count, tile, sort)
        items, qoff = api.batch_queue_layout(nps, Ls, tile, nq)
        T = [n // tile for n in nps]
        nt = [t * (t + 1) // 2 for t in T]
        assert qoff[0] == 0 and qoff[-1] == len(items) and np.all(np.diff(qoff) >= 0)
        assert len(items) == sum(nt[m] * Ls[m] for m in range(count))
        seen = set()
        queue_of = {}
        for x in range(nq):
            q = items[qoff[x]:qoff[x + 1]]
            assert np.all(np.diff(q[:, 2]) >= 0), "layer-major"
            before = np.zeros(count, dtype=np.int64)   # items of each matrix earlier in the queue
            for m, t, layer, need in q:
                assert 0 <= m < count and 0 <= t < nt[m] and 0 <= layer < Ls[m]
                assert (m, t, layer) not in seen
                seen.add((m, t, layer))
                assert queue_of.setdefault(m, x) == x, "one queue per matrix"
                assert need == layer * nt[m]
                assert before[m] >= need, "dependencies precede the item"
                before[m] += 1
        assert len(seen) == len(items)
        # the dealing rule: in batch order, to the queue with the least tiles x size so far
        load = [0.0] * nq
        for m in range(count):
            x = min(range(nq), key=lambda y: (load[y], y))
            assert queue_of[m] == x
            load[x] += nt[m] * nps[m]
        counts = np.array([nt[m] * Ls[m] for m in range(count)])
        for workers in (1, 2, 5):
            assert simulate(items, qoff, counts, workers, rng)


def test_bad_arguments_are_refused():
    with pytest.raises(api.FeError):
        api.batch_queue_layout([100], [3], 128, 8)       # not a multiple of the tile
    with pytest.raises(api.FeError):
        api.batch_queue_layout([128], [0], 128, 8)       # no layers
    with pytest.raises(api.FeError):
        api.batch_queue_layout([128], [3], 96, 8)        # tile
    with pytest.raises(api.FeError):
        api.batch_queue_layout([128], [3], 128, 17)      # queues
