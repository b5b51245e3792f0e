"""Batched persistent forward + adjoint of the 32-volume workload.

Every volume's field and gradient must equal the per-volume launches bit for
bit (same routines, schedule-independent arithmetic), under every schedule, in a
direct launch and in repeated HIP-graph replays; every volume is also checked
against the FP64 oracle on every element."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2004_05962_amd as bsi
import workloads
from gpu_util import dev, host, max_abs, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def batch():
    dims, spac = workloads.cfg5_geometry()
    vols = [workloads.cfg5_volume(tuple(d), tuple(s), i) for i, (d, s) in enumerate(zip(dims, spac))]
    grids = [dev(g) for g, _ in vols]
    dfields = [dev(f) for _, f in vols]
    return dims, spac, vols, grids, dfields


def _outputs(dims, spac):
    fields = [torch.empty(bsi.field_shape(d), device="cuda") for d in dims]
    grads = [torch.empty(bsi.grid_shape(d, s), device="cuda") for d, s in zip(dims, spac)]
    return fields, grads


def _force(plan, index):
    os.environ["BSI_FORCE_CONFIG"] = str(index)
    try:
        plan.tune()
    finally:
        del os.environ["BSI_FORCE_CONFIG"]
    assert plan.config()[0] == index


def _covering_schedules(plan):
    """Schedule indices that together take every value of every knob (greedy
    over the whole space, which is enumerated through the plan's own text)."""
    n = plan.config()[1]
    items = []
    for idx in range(n):
        _force(plan, idx)
        items.append(set(plan.describe().split()))
    universe = set().union(*items)
    chosen, covered = [0], set(items[0])
    while covered != universe:
        best = max(range(n), key=lambda i: len(items[i] - covered))
        chosen.append(best)
        covered |= items[best]
    return chosen, universe


def test_batched_equals_per_volume_bits(batch):
    dims, spac, vols, grids, dfields = batch
    say("batch: per-volume reference")
    ref_f, ref_g = _outputs(dims, spac)
    for i in range(len(dims)):
        bsi.forward(grids[i], dims[i], spac[i], out=ref_f[i])
        bsi.adjoint(dfields[i], dims[i], spac[i], out=ref_g[i])
    plan = bsi.BatchPlan(dims, spac)
    f, g = _outputs(dims, spac)
    plan.bind(grids, f, dfields, g)
    schedules, universe = _covering_schedules(plan)
    say("batch: schedules", schedules, "cover", len(universe), "knob values")
    assert len(universe) == 3 + 3 + 4 + 4 + 2 + 3 + 2 + 2 + 2
    for sched in schedules:
        _force(plan, sched)
        for t in f + g:
            t.fill_(float("nan"))
        say("batch: schedule", sched, plan.describe())
        plan.run()
        torch.cuda.synchronize()
        for i in range(len(dims)):
            assert torch.equal(f[i], ref_f[i]), (sched, i)
            assert torch.equal(g[i], ref_g[i]), (sched, i)
    say("batch: separate launches")
    for t in f + g:
        t.fill_(float("nan"))
    plan.run_separate()
    torch.cuda.synchronize()
    for i in range(len(dims)):
        assert torch.equal(f[i], ref_f[i]) and torch.equal(g[i], ref_g[i])
    plan.close()


def test_graph_replays(batch):
    dims, spac, vols, grids, dfields = batch
    plan = bsi.BatchPlan(dims, spac)
    f, g = _outputs(dims, spac)
    plan.bind(grids, f, dfields, g)
    say("batch: eager run")
    plan.run()
    torch.cuda.synchronize()
    ref_f = [t.clone() for t in f]
    ref_g = [t.clone() for t in g]
    say("batch: capture")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan.capture(stream)
    for rep in range(3):
        for t in f + g:
            t.zero_()
        torch.cuda.synchronize()
        say("batch: replay", rep)
        plan.launch()
        torch.cuda.synchronize()
        for i in range(len(dims)):
            assert torch.equal(f[i], ref_f[i]) and torch.equal(g[i], ref_g[i]), (rep, i)
    plan.close()


def test_every_volume_against_oracle(batch):
    """All 32 volumes of the batched graph's workload against the FP64 oracle on
    every voxel and every control point (the forward by the triple sum, the
    adjoint by the per-point gather)."""
    dims, spac, vols, grids, dfields = batch
    plan = bsi.BatchPlan(dims, spac)
    f, g = _outputs(dims, spac)
    plan.bind(grids, f, dfields, g)
    say("batch: oracle parity, 32 volumes")
    plan.run()
    torch.cuda.synchronize()
    for i in range(len(dims)):
        d, s = tuple(int(v) for v in dims[i]), tuple(int(v) for v in spac[i])
        grid, dfield = vols[i]
        ref_f = oracle.forward(grid, d, s)
        assert max_abs(host(f[i]), ref_f) <= 1e-5 * float(np.abs(grid).max()), i
        del ref_f
        ref_g = oracle.adjoint_gather(dfield, d, s)
        assert max_abs(host(g[i]), ref_g) <= 1e-5 * float(np.abs(ref_g).max()), i
    plan.close()


def test_tune_persists_choice(batch, tmp_path):
    dims, spac, vols, grids, dfields = batch
    path = str(tmp_path / "tune.json")
    os.environ["BSI_TUNE_CACHE"] = path
    try:
        plan = bsi.BatchPlan(dims[:6], spac[:6])
        f, g = _outputs(dims[:6], spac[:6])
        plan.bind(grids[:6], f, dfields[:6], g)
        say("batch: tune")
        chosen, n = plan.tune()
        assert 0 <= chosen < n
        data = json.load(open(path))
        assert list(data.values()) == [chosen]
        again = bsi.BatchPlan(dims[:6], spac[:6])
        assert again.config()[0] == chosen
        assert again.describe() == plan.describe()
        plan.close()
        again.close()
    finally:
        del os.environ["BSI_TUNE_CACHE"]


def test_forward_only_and_single_volume():
    say("batch: forward-only single volume")
    d, s = (70, 33, 21), (5, 4, 3)
    grid = dev(workloads.random_grid(d, s, 2.0, seed=77))
    plan = bsi.BatchPlan([d], [s])
    out = torch.empty(bsi.field_shape(d), device="cuda")
    plan.bind(grids=[grid], fields=[out])
    plan.run()
    torch.cuda.synchronize()
    assert torch.equal(out, bsi.forward(grid, d, s))
    plan.close()


def test_bind_rejects_short_or_misshaped_lists():
    """A list shorter than the plan, or a tensor of another volume's shape, raises
    ValueError in the binding, before the library stores any pointer."""
    say("batch: bind argument checks")
    dims, spac = [(40, 30, 20), (33, 21, 17)], [(5, 5, 5), (4, 4, 4)]
    plan = bsi.BatchPlan(dims, spac)
    grids = [torch.zeros(bsi.grid_shape(d, s), device="cuda") for d, s in zip(dims, spac)]
    fields = [torch.empty(bsi.field_shape(d), device="cuda") for d in dims]
    with pytest.raises(ValueError):
        plan.bind(grids[:1], fields[:1])
    with pytest.raises(ValueError):
        plan.bind(grids, fields[::-1])
    with pytest.raises(ValueError):
        plan.bind(grids, fields, dfields=[fields[0]], grid_grads=[grids[0]])
    plan.bind(grids, fields)
    plan.run()
    torch.cuda.synchronize()
    for g, f, d, s in zip(grids, fields, dims, spac):
        assert torch.equal(f, bsi.forward(g, d, s))
    plan.close()


def test_invalid_forced_schedule_rejected(batch):
    dims, spac, vols, grids, dfields = batch
    say("batch: invalid BSI_FORCE_CONFIG")
    plan = bsi.BatchPlan(dims[:2], spac[:2])
    f, g = _outputs(dims[:2], spac[:2])
    plan.bind(grids[:2], f, dfields[:2], g)
    n = plan.config()[1]
    for bad in (str(n), "-1", "7x"):
        os.environ["BSI_FORCE_CONFIG"] = bad
        try:
            with pytest.raises(bsi.BSIError):
                plan.tune()
            with pytest.raises(bsi.BSIError):
                bsi.BatchPlan(dims[:2], spac[:2])
        finally:
            del os.environ["BSI_FORCE_CONFIG"]
    plan.close()
