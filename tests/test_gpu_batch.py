"""Batch plans on the GPU: every image of a persistent launch against the
oracle, and bit-identical to the single-image call with the same variant
(variant choice depends only on kind, radius and size), with and without
graph replay, across replays and re-pointed arenas."""
import numpy as np
import pytest

import oracle
import paper_1302_5586_amd as pf
import synth
from gpu_util import assert_close, device, tolerance_2d, tolerance_sep

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _mixed_batch(seed, n, hi=300, rmax=4):
    """n images with mixed kinds, radii 0..rmax and ragged sizes."""
    rng = np.random.default_rng(seed)
    imgs, filts, kinds = [], [], []
    for i in range(n):
        h = int(rng.integers(1, hi))
        w = int(rng.integers(1, hi))
        r = int(rng.integers(0, rmax + 1))
        k = int(rng.integers(0, 2))
        imgs.append(rng.random((h, w), dtype=np.float32))
        if k == pf.KIND_2D:
            filts.append(rng.standard_normal((2 * r + 1) ** 2).astype(np.float32))
        else:
            filts.append(rng.standard_normal(2 * (2 * r + 1)).astype(np.float32))
        kinds.append(k)
    return imgs, filts, kinds


def _oracle_and_tol(img, filt, kind, r):
    k = 2 * r + 1
    if kind == pf.KIND_2D:
        f2 = filt.reshape(k, k)
        return oracle.filter2d_f32(img, f2), tolerance_2d(img, f2, r)
    fx, fy = filt[:k], filt[k:]
    return oracle.filter_sep_f32(img, fx, fy), tolerance_sep(img, fx, fy)


def _single(xi, fi, kind, r, var, dev):
    """The single-image call with a given variant and default shape."""
    if kind == pf.KIND_2D:
        return pf.filter2d(xi, fi.view(2 * r + 1, 2 * r + 1))
    if var == pf.VAR_SEPARABLE:
        k = 2 * r + 1
        return pf.filter_sep(xi, fi[:k], fi[k:])
    return pf.filter_shaped(xi, fi, r, kind, var, 16, 4)


@pytest.mark.parametrize("graph", [False, True])
def test_mixed_batch_against_oracle_and_single(graph):
    dev = device()
    import torch
    imgs, filts, kinds = _mixed_batch(11, 60)
    pk = pf.pack_batch(imgs, filts, kinds)
    x, fl = _t(pk.pixels, dev), _t(pk.filters, dev)
    out = torch.full_like(x, float("nan"))
    plan = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel(), graph=graph)
    info = plan.info()
    assert info["launches"] == 1
    var = plan.variants()
    plan.run(x, fl, out)
    got = out.cpu().numpy()
    for i in range(len(imgs)):
        h, w, r, k = int(pk.h[i]), int(pk.w[i]), int(pk.r[i]), int(pk.kind[i])
        gi = got[pk.pix_off[i]:pk.pix_off[i] + h * w].reshape(h, w)
        ref, tol = _oracle_and_tol(imgs[i], filts[i], k, r)
        assert_close(gi, ref, tol, "batch image %d (%dx%d r=%d kind=%d)" % (i, h, w, r, k))
        xi = x[pk.pix_off[i]:pk.pix_off[i] + h * w].view(h, w)
        fi = fl[pk.filt_off[i]:pk.filt_off[i] + filts[i].size]
        alone = _single(xi, fi, k, r, int(var[i]), dev).cpu().numpy()
        assert np.array_equal(alone, gi), "image %d differs between batch and single launch" % i
    # padding between images is never written
    mask = np.ones(got.size, bool)
    for i in range(len(imgs)):
        mask[pk.pix_off[i]:pk.pix_off[i] + int(pk.h[i]) * int(pk.w[i])] = False
    assert np.isnan(got[mask]).all()


@pytest.mark.parametrize("side_stream", [False, True])
def test_graph_replay_and_repoint(side_stream):
    dev = device()
    import torch
    if side_stream:
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            _replay_and_repoint(dev)
        st.synchronize()
    else:
        _replay_and_repoint(dev)


def _replay_and_repoint(dev):
    import torch
    imgs, filts, kinds = _mixed_batch(12, 25, hi=200, rmax=4)
    pk = pf.pack_batch(imgs, filts, kinds)
    x, fl = _t(pk.pixels, dev), _t(pk.filters, dev)
    plan = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel(), graph=True)
    ref_plan = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel(), graph=False)
    want = torch.zeros_like(x)      # padding between images stays 0 in every arena
    ref_plan.run(x, fl, want)
    want = want.cpu().numpy()
    outs = [torch.zeros_like(x) for _ in range(3)]
    for rep in range(3):
        for j, o in enumerate(outs):
            o.zero_()
            plan.run(x, fl, o)      # new arena pointer on each call: node re-pointed
            torch.cuda.synchronize()
            g = o.cpu().numpy()
            bad = np.flatnonzero(g != want)
            assert bad.size == 0, "replay %d arena %d: %d differ, first %d of %d" % (rep, j, bad.size, bad[0], g.size)
    # a different input arena through the same graph
    x2 = x * 2
    o2 = torch.zeros_like(x)
    plan.run(x2, fl, o2)
    outs[0].zero_()
    ref_plan.run(x2, fl, outs[0])
    assert np.array_equal(o2.cpu().numpy(), outs[0].cpu().numpy())


def test_exact_batch_matches_oracle_bitwise():
    dev = device()
    import torch
    imgs, filts, kinds = _mixed_batch(13, 20, hi=150, rmax=4)
    pk = pf.pack_batch(imgs, filts, kinds)
    x, fl = _t(pk.pixels, dev), _t(pk.filters, dev)
    out = torch.empty_like(x)
    plan = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel(), exact=True)
    plan.run(x, fl, out)
    got = out.cpu().numpy()
    for i in range(len(imgs)):
        h, w, r, k = int(pk.h[i]), int(pk.w[i]), int(pk.r[i]), int(pk.kind[i])
        ref, _ = _oracle_and_tol(imgs[i], filts[i], k, r)
        assert np.array_equal(got[pk.pix_off[i]:pk.pix_off[i] + h * w].reshape(h, w), ref), i


def test_config_batch_512():
    """The 512-image batch (seed 3), in the launch configuration the
    benchmark times (the committed MI355X tune table, graph replay): every
    element of every image against the separable oracle within 1e-5 * D,
    and every image bit-identical to its single-image launch."""
    dev = device()
    import os
    import torch
    table = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1302_5586_amd",
                         "tune_mi355x.json")
    pf.tune_load(table)
    try:
        _config_batch_512(dev, torch)
    finally:
        pf.tune_reset()


def _config_batch_512(dev, torch):
    b = synth.config_batch()
    filts = [np.concatenate([b.fx[i], b.fx[i]]) for i in range(b.n)]
    pk = pf.pack_batch(b.images, filts, [pf.KIND_SEP] * b.n)
    x, fl = _t(pk.pixels, dev), _t(pk.filters, dev)
    out = torch.full_like(x, float("nan"))
    plan = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel(), graph=True)
    plan.run(x, fl, out)
    plan.run(x, fl, out)
    var = plan.variants()
    got = out.cpu().numpy()
    worst_abs, worst_rel = 0.0, 0.0
    for i in range(b.n):
        h, w, r = int(pk.h[i]), int(pk.w[i]), int(pk.r[i])
        gi = got[pk.pix_off[i]:pk.pix_off[i] + h * w].reshape(h, w)
        ref, tol = _oracle_and_tol(b.images[i], filts[i], pf.KIND_SEP, r)
        err, rel = assert_close(gi, ref, tol, "batch512 image %d (%dx%d r=%d)" % (i, h, w, r))
        worst_abs, worst_rel = max(worst_abs, err), max(worst_rel, rel)
        xi = x[pk.pix_off[i]:pk.pix_off[i] + h * w].view(h, w)
        fi = fl[pk.filt_off[i]:pk.filt_off[i] + 2 * (2 * r + 1)]
        alone = _single(xi, fi, pf.KIND_SEP, r, int(var[i]), dev).cpu().numpy()
        assert np.array_equal(alone, gi), "image %d differs between batch and single launch" % i
    print("batch512: %d images, %d px, every element checked; max abs %.3g, max rel %.3g"
          % (b.n, b.pixels, worst_abs, worst_rel))


def test_batch_autotune_keeps_results(tmp_path):
    """Tuning the table on a batch changes only launch shapes: the tuned plan
    still matches the oracle, and the saved table reloads."""
    dev = device()
    import torch
    imgs, filts, kinds = _mixed_batch(21, 40, hi=700, rmax=4)
    pk = pf.pack_batch(imgs, filts, kinds)
    x, fl = _t(pk.pixels, dev), _t(pk.filters, dev)
    out = torch.zeros_like(x)
    path = str(tmp_path / "tuned.json")
    try:
        pf.autotune_batch(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x, fl, out, reps=2, path=path)
        pf.tune_reset()
        pf.tune_load(path)
        out.zero_()
        plan = pf.BatchPlan(pk.h, pk.w, pk.r, pk.kind, pk.pix_off, pk.filt_off, x.numel(), fl.numel())
        plan.run(x, fl, out)
        got = out.cpu().numpy()
        for i in range(len(imgs)):
            h, w, r, k = int(pk.h[i]), int(pk.w[i]), int(pk.r[i]), int(pk.kind[i])
            gi = got[pk.pix_off[i]:pk.pix_off[i] + h * w].reshape(h, w)
            ref, tol = _oracle_and_tol(imgs[i], filts[i], k, r)
            assert_close(gi, ref, tol, "tuned batch image %d (%dx%d r=%d kind=%d)" % (i, h, w, r, k))
    finally:
        pf.tune_reset()
