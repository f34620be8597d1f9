"""OP2-style edge-to-cell increment on the GPU against the oracle's loop.

The plan path adds every cell's increments in the loop's own order, so it
must equal the oracle bit for bit. The atomic path adds them in whatever
order the atomics land: each cell with k increments is within
2 k 2^-53 (|cell| + sum |edge|) of the loop's result."""
import numpy as np
import pytest

import oracle
import paper_1302_5586_amd as pf
import synth
from gpu_util import device

pytestmark = pytest.mark.gpu


def _t(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def _random_mesh(seed, ncells, nedges):
    rng = np.random.default_rng(seed)
    e2c = rng.integers(0, ncells, (nedges, 2)).astype(np.int32)
    if nedges > 4:
        e2c[1, 1] = e2c[1, 0]          # a self-loop: its cell is incremented twice
        e2c[3] = e2c[2]                # a repeated edge
    return e2c, rng.standard_normal(nedges), rng.standard_normal(ncells)


@pytest.mark.parametrize("ncells,nedges", [(1, 0), (1, 5), (7, 3), (100, 1000), (5000, 12345), (70000, 300000)])
def test_plan_bitwise(ncells, nedges):
    dev = device()
    e2c, edge, cell = _random_mesh(ncells + nedges, ncells, nedges)
    plan = pf.IncPlan(ncells, e2c)
    got = plan.run(_t(edge, dev), _t(cell, dev)).cpu().numpy()
    ref = oracle.edge_inc_f64(ncells, e2c, edge, cell)
    assert np.array_equal(got, ref)
    plan.close()


def test_plan_mesh_bitwise_and_repeatable():
    dev = device()
    m = synth.config_mesh()
    plan = pf.IncPlan(m.ncells, m.edge_to_cells)
    ed, c0 = _t(m.edge, dev), _t(m.cell, dev)
    c = c0.clone()
    plan.run(ed, c)
    ref = oracle.edge_inc_f64(m.ncells, m.edge_to_cells, m.edge, m.cell)
    assert np.array_equal(c.cpu().numpy(), ref)
    c2 = c0.clone()
    plan.run(ed, c2)
    assert np.array_equal(c2.cpu().numpy(), ref)
    plan.close()


def test_atomic_within_rounding():
    dev = device()
    m = synth.quad_mesh(300, 200, 9)
    got = pf.edge_inc_atomic(_t(m.edge_to_cells.reshape(-1), dev), _t(m.edge, dev), _t(m.cell, dev)).cpu().numpy()
    ref = oracle.edge_inc_f64(m.ncells, m.edge_to_cells, m.edge, m.cell)
    k = np.bincount(m.edge_to_cells.reshape(-1), minlength=m.ncells)
    mag = np.abs(m.cell).copy()
    np.add.at(mag, m.edge_to_cells[:, 0], np.abs(m.edge))
    np.add.at(mag, m.edge_to_cells[:, 1], np.abs(m.edge))
    assert np.all(np.abs(got - ref) <= 2 * np.maximum(k, 1) * 2.0 ** -53 * mag)


def test_atomic_skips_out_of_range_entries():
    dev = device()
    e2c = np.array([[0, 1], [1, 7], [-3, 2]], np.int32)   # 7 and -3 are outside 0..2
    edge = np.array([1.0, 2.0, 4.0])
    cell = np.zeros(3)
    got = pf.edge_inc_atomic(_t(e2c.reshape(-1), dev), _t(edge, dev), _t(cell, dev)).cpu().numpy()
    assert np.array_equal(got, [1.0, 3.0, 4.0])


def test_plan_rejects():
    dev = device()
    with pytest.raises(pf.PFInvalid):
        pf.IncPlan(3, np.array([[0, 3]], np.int32))
    plan = pf.IncPlan(3, np.array([[0, 1]], np.int32))
    import torch
    with pytest.raises(ValueError):
        plan.run(torch.zeros(2, dtype=torch.float64, device=dev), torch.zeros(3, dtype=torch.float64, device=dev))
    x = torch.zeros(8, dtype=torch.float64, device=dev)
    with pytest.raises(pf.PFAlias):
        pf._check(pf.load().pf_inc_plan_run(plan._h, 3, 1, x.data_ptr(), x.data_ptr(), None))
    plan.close()
