"""The server's admission bookkeeping on the CPU: its first-fit arena
allocator, replayed through pf_arena_replay, against a plain model (a
sorted free list, 256-byte granules, lowest address first, neighbouring
free runs merged), on random sequences and on the cases that matter for
admission (exhaustion, reuse after release, full coalescing)."""
import numpy as np
import pytest

import paper_1302_5586_amd as pf


@pytest.fixture(scope="module")
def lib():
    import os
    if not os.path.exists(pf.LIB_PATH):
        from paper_1302_5586_amd import build as b
        b.build()
    return pf.load()


def _model(budget, ops):
    free = [(0, budget)]       # sorted (offset, length)
    live, res, used = {}, [], 0
    up = lambda b: (b + 255) // 256 * 256  # noqa: E731
    for i, op in enumerate(ops):
        if op > 0:
            b = up(op)
            for k, (o, ln) in enumerate(free):
                if ln >= b:
                    free[k:k + 1] = [(o + b, ln - b)] if ln > b else []
                    live[i] = (o, b)
                    used += b
                    res.append(o)
                    break
            else:
                res.append(-1)
        else:
            o, b = live.pop(-op - 1)
            used -= b
            free.append((o, b))
            free.sort()
            merged = []
            for fo, fl in free:
                if merged and merged[-1][0] + merged[-1][1] == fo:
                    merged[-1] = (merged[-1][0], merged[-1][1] + fl)
                else:
                    merged.append((fo, fl))
            free = merged
            res.append(0)
    return res, used


def test_random_sequences_match_the_model(lib):
    rng = np.random.default_rng(12)
    for trial in range(40):
        budget = int(rng.integers(1, 64)) * 4096
        ops, live = [], []
        for i in range(300):
            if live and rng.random() < 0.45:
                j = live.pop(int(rng.integers(0, len(live))))
                ops.append(-j - 1)
            else:
                ops.append(int(rng.integers(1, 20000)))
                # only allocations that fit become live (and may be freed later)
                res, _ = _model(budget, ops)
                if res[-1] >= 0:
                    live.append(i)
        want, want_used = _model(budget, ops)
        got, used = pf.arena_replay(budget, ops)
        assert list(got) == want and used == want_used, trial
        # live allocations never overlap and stay inside the budget
        spans = sorted((got[i], (ops[i] + 255) // 256 * 256) for i in live)
        assert all(o >= 0 and o + ln <= budget for o, ln in spans)
        assert all(spans[k][0] + spans[k][1] <= spans[k + 1][0] for k in range(len(spans) - 1))


def test_exhaustion_reuse_and_coalescing(lib):
    budget = 4 * 256
    res, used = pf.arena_replay(budget, [256, 256, 256, 256, 1])
    assert list(res) == [0, 256, 512, 768, -1] and used == budget
    # free the two middle blocks: their runs merge and fit a 512-byte request
    res, used = pf.arena_replay(budget, [256, 256, 256, 256, -2, -3, 512, 300])
    assert list(res) == [0, 256, 512, 768, 0, 0, 256, -1] and used == budget
    # free everything: one run again, the whole budget fits
    res, used = pf.arena_replay(budget, [100, 200, 300, -1, -3, -2, 1024])
    assert res[-1] == 0 and used == 1024
    with pytest.raises(pf.PFInvalid):
        pf.arena_replay(budget, [256, -1, -1])      # double free
    with pytest.raises(pf.PFInvalid):
        pf.arena_replay(budget, [2048, -1])         # free of an allocation that failed
