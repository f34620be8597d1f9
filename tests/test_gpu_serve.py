"""The continuous-batching server on the GPU: results against the oracle,
each request's result the same alone and inside a mixed stream, admission
under a tiny HBM budget, upload mode, and the open-loop trace driver."""
import time

import numpy as np
import pytest

import oracle
import paper_1302_5586_amd as pf
import synth
from gpu_util import assert_close, device, tolerance_sep

pytestmark = pytest.mark.gpu


def _requests(seed, n, hi=400):
    rng = np.random.default_rng(seed)
    reqs = []
    for _ in range(n):
        h, w = int(rng.integers(1, hi)), int(rng.integers(1, hi))
        r = int(rng.integers(1, 5))
        g = synth.gaussian_1d(r, float(rng.uniform(0.5, 2.0)))
        reqs.append((rng.random((h, w), dtype=np.float32), r, np.concatenate([g, g])))
    return reqs


def test_alone_equals_mixed_and_oracle():
    dev = device()
    import torch
    reqs = _requests(21, 80)
    xs = [torch.from_numpy(img).to(dev) for img, _, _ in reqs]
    torch.cuda.synchronize()
    alone = []
    with pf.Server(1 << 30, n_streams=1, max_batch=1) as s:
        for x, (img, r, f) in zip(xs, reqs):
            t = s.submit(x, r, pf.KIND_SEP, f)
            s.wait(t, timeout_s=30)
            alone.append(s.result(t, *img.shape))
    with pf.Server(1 << 30, n_streams=3, max_batch=16) as s:
        tickets = [s.submit(x, r, pf.KIND_SEP, f) for x, (img, r, f) in zip(xs, reqs)]
        mixed = []
        for t, (img, _, _) in zip(tickets, reqs):
            s.wait(t, timeout_s=30)
            mixed.append(s.result(t, *img.shape))
        st = s.stats()
    assert st["completed"] == len(reqs) and st["batches"] < len(reqs)
    for i, (img, r, f) in enumerate(reqs):
        assert np.array_equal(alone[i], mixed[i]), "request %d differs alone vs mixed" % i
        k = 2 * r + 1
        ref = oracle.filter_sep_f32(img, f[:k], f[k:])
        assert_close(mixed[i], ref, tolerance_sep(img, f[:k], f[k:]), "served request %d" % i)


def test_budget_admission_and_upload():
    device()
    reqs = _requests(22, 30, hi=200)
    biggest = max(img.nbytes for img, _, _ in reqs)
    # room for about two uploaded requests at a time: admission must queue
    budget = 4 * (biggest + 256) + 4096
    with pf.Server(budget, n_streams=2, max_batch=8) as s:
        tickets = [s.submit(img, r, pf.KIND_SEP, f) for img, r, f in reqs]   # host arrays: upload mode
        outs = []
        for t, (img, _, _) in zip(tickets, reqs):
            s.wait(t, timeout_s=60)
            outs.append(s.result(t, *img.shape))
        st = s.stats()
        assert st["bytes_high_water"] <= budget
        assert st["completed"] == len(reqs)
        with pytest.raises(pf.PFBudget):
            s.submit(np.zeros((2048, 2048), np.float32), 1, pf.KIND_SEP, np.ones(6, np.float32))
    for (img, r, f), o in zip(reqs, outs):
        k = 2 * r + 1
        assert_close(o, oracle.filter_sep_f32(img, f[:k], f[k:]), tolerance_sep(img, f[:k], f[k:]), "upload")


def test_ticket_errors_and_timeout():
    dev = device()
    import torch
    with pf.Server(1 << 26, n_streams=1, max_batch=4) as s:
        with pytest.raises(pf.PFInvalid):
            s.wait(12345, timeout_s=0.01)
        x = torch.rand(64, 64, device=dev)
        t = s.submit(x, 1, pf.KIND_2D, np.full(9, 1.0 / 9, np.float32))
        s.wait(t, timeout_s=30)
        assert s.poll(t)
        s.release(t)
        with pytest.raises(pf.PFInvalid):
            s.release(t)


def test_run_trace_small():
    dev = device()
    import torch
    pool = synth.batch_f32(n=32, seed=41, hi=256)
    offs, o = np.zeros(pool.n, np.int64), 0
    for i in range(pool.n):
        offs[i] = o
        o += int(pool.h[i] * pool.w[i])
    arena = np.concatenate([im.ravel() for im in pool.images])
    pool_dev = torch.from_numpy(arena).to(dev)
    tr = synth.arrival_trace(rate=2000.0, duration=0.25, seed=5, pool_size=pool.n)
    fls, foffs, fo = [], np.zeros(tr.n, np.int64), 0
    for i in range(tr.n):
        g = synth.gaussian_1d(int(tr.r[i]), float(tr.sigma[i]))
        fls += [g, g]
        foffs[i] = fo
        fo += 2 * g.size
    pi = tr.pool_index
    t0 = time.time()
    with pf.Server(1 << 30, n_streams=2, max_batch=32) as s:
        st = s.run_trace((tr.t * 1e9).astype(np.int64), pool.h[pi], pool.w[pi], tr.r, offs[pi], foffs, pool_dev,
                         np.concatenate(fls))
    assert time.time() - t0 >= 0.2
    assert st["completed"] == tr.n and st["p50_us"] > 0 and st["p99_us"] >= st["p50_us"]
