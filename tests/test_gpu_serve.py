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


def test_reductions_served_with_filters():
    """Sums and histograms batched with filter requests: every sum bit for
    bit equal to pf_sum_f32 (and within its bound of the oracle), every
    histogram equal to the oracle's, alone and mixed alike."""
    dev = device()
    import torch
    rng = np.random.default_rng(31)
    sums = [(rng.standard_normal(n) * 10).astype(np.float32) for n in (1, 65535, 65536, 200001, (1 << 20) + 3)]
    hists = [rng.integers(0, 256, n).astype(np.uint8) for n in (1, 5, 262144, 262145, 3 * 262144 + 17)]
    filt = _requests(32, 12, hi=300)
    xs = [torch.from_numpy(a).to(dev) for a in sums]
    hb = [torch.from_numpy(np.concatenate([np.zeros(1, np.uint8), a])).to(dev) for a in hists]
    hs = [t[1:] for t in hb]                    # device views one byte into their buffers
    fx = [torch.from_numpy(img).to(dev) for img, _, _ in filt]

    def run(server):
        tk = []
        for x in xs:
            tk.append(("sum", server.submit_sum(x)))
        for i, (x, (img, r, f)) in enumerate(zip(fx, filt)):
            tk.append(("flt", server.submit(x, r, pf.KIND_SEP, f)))
            if i < len(hs):
                tk.append(("hist", server.submit_hist(hs[i])))
        tk.append(("sum", server.submit_sum(sums[3])))      # host input, uploaded
        tk.append(("hist", server.submit_hist(hists[4])))   # host input, uploaded
        out = []
        fi = 0
        for kind, t in tk:
            server.wait(t, timeout_s=60)
            if kind == "sum":
                out.append(server.result_sum(t))
            elif kind == "hist":
                out.append(server.result_hist(t))
            else:
                out.append(server.result(t, *filt[fi][0].shape))
                fi += 1
        return out

    with pf.Server(1 << 30, n_streams=1, max_batch=1) as s:
        alone = run(s)
    with pf.Server(1 << 30, n_streams=3, max_batch=16) as s:
        mixed = run(s)
        assert s.stats()["batches"] < len(mixed)
    for a, b in zip(alone, mixed):
        assert np.array_equal(a, b)
    k = 0
    for x, a in zip(xs, sums):
        want = pf.sum_f32(x).cpu().numpy()
        assert np.array_equal(mixed[k], want), k
        tol = 2.0 * max(a.size - 1, 1) * 2.0 ** -53 * float(np.abs(a.astype(np.float64)).sum())
        assert abs(mixed[k][0] - oracle.sum_f32(a)) <= tol
        k += 1
    for i, (img, r, f) in enumerate(filt):
        kk = 2 * r + 1
        assert_close(mixed[k], oracle.filter_sep_f32(img, f[:kk], f[kk:]), tolerance_sep(img, f[:kk], f[kk:]),
                     "filter %d" % i)
        k += 1
        if i < len(hists):
            assert np.array_equal(mixed[k], oracle.hist256_u8(hists[i])), i
            k += 1
    assert np.array_equal(mixed[k], pf.sum_f32(xs[3]).cpu().numpy())
    assert np.array_equal(mixed[k + 1], oracle.hist256_u8(hists[4]))


def test_submit_orders_after_the_producer_stream():
    """A device input still being written on the caller's stream (and
    dropped by the caller right after submit) is read only after it is
    complete."""
    dev = device()
    import torch
    h, w = 1024, 1536
    g = synth.gaussian_1d(2, 1.3)
    f = np.concatenate([g, g])
    side = torch.cuda.Stream()
    with pf.Server(1 << 30, n_streams=2, max_batch=8) as s:
        tickets = []
        for seed in range(4):
            busy = torch.randn(3000, 3000, device=dev)
            for _ in range(3):
                busy = busy @ busy.t().contiguous() * 1e-3       # keep the stream busy for a while
            gen = torch.Generator(device=dev)
            gen.manual_seed(seed)
            tickets.append(s.submit(torch.rand((h, w), generator=gen, device=dev), 2, pf.KIND_SEP, f))
            with torch.cuda.stream(side):
                gen2 = torch.Generator(device=dev)
                gen2.manual_seed(100 + seed)
                y = torch.rand((h, w), generator=gen2, device=dev) * 2.0
                tickets.append(s.submit(y, 2, pf.KIND_SEP, f, stream=side))
                tickets.append(s.submit_sum(y.reshape(-1), stream=side))
            del y
        outs = []
        for i, t in enumerate(tickets):
            s.wait(t, timeout_s=60)
            outs.append(s.result_sum(t) if i % 3 == 2 else s.result(t, h, w))
    for seed in range(4):
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        a = torch.rand((h, w), generator=gen, device=dev).cpu().numpy()
        gen2 = torch.Generator(device=dev)
        gen2.manual_seed(100 + seed)
        b = (torch.rand((h, w), generator=gen2, device=dev) * 2.0).cpu().numpy()
        for img, got in ((a, outs[3 * seed]), (b, outs[3 * seed + 1])):
            assert_close(got, oracle.filter_sep_f32(img, g, g), tolerance_sep(img, g, g), "ordered input")
        assert np.array_equal(outs[3 * seed + 2], pf.sum_f32(torch.from_numpy(b.reshape(-1)).to(dev)).cpu().numpy())


def test_queue_full_budget_and_shutdown():
    """Admission under a budget for two uploaded requests: finished results
    that are not fetched hold the arena, later requests queue, a full queue
    refuses with PF_EAGAIN, a request larger than the budget with
    PF_EBUDGET, releasing a result admits the next, and closing the server
    with a request that can never be admitted returns at once (that request
    fails with PF_EAGAIN)."""
    device()
    rng = np.random.default_rng(33)
    img = rng.random((64, 64), dtype=np.float32)
    f = np.concatenate([synth.gaussian_1d(1, 1.0)] * 2)
    per = 2 * img.nbytes                         # uploaded: input and output in the arena
    s = pf.Server(2 * per, n_streams=1, max_batch=4, max_queue=2)
    t1 = s.submit(img, 1, pf.KIND_SEP, f)
    t2 = s.submit(img, 1, pf.KIND_SEP, f)
    s.wait(t1, timeout_s=30)
    s.wait(t2, timeout_s=30)
    t3 = s.submit(img, 1, pf.KIND_SEP, f)        # no room: stays queued
    t4 = s.submit(img, 1, pf.KIND_SEP, f)
    time.sleep(0.1)
    assert not s.poll(t3) and not s.poll(t4)
    with pytest.raises(pf.PFAgain):
        s.submit(img, 1, pf.KIND_SEP, f)         # two already waiting
    with pytest.raises(pf.PFBudget):
        s.submit(np.zeros((128, 128), np.float32), 1, pf.KIND_SEP, f)
    s.release(t1)                                # frees room for t3
    s.wait(t3, timeout_s=30)
    ref = oracle.filter_sep_f32(img, f[:3], f[3:])
    assert_close(s.result(t3, 64, 64), ref, tolerance_sep(img, f[:3], f[3:]), "admitted after release")
    st = s.stats()
    assert st["rejected"] == 2 and st["queue_high_water"] == 2 and st["bytes_high_water"] <= 2 * per
    t0 = time.time()
    s.close()                                    # t4 can never be admitted while t2's result is held
    assert time.time() - t0 < 5.0
