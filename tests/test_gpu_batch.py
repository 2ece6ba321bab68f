"""GPU parity of the batched mode: many clustered sets of uneven size built and
queried together must give, set by set, exactly the single-tree results and
the oracle's (kNN k = 8 of every point, friends-of-friends b = 0.2)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _batch(sizes, seed_base, d=3):
    if d == 3:
        x, off = workloads.batched_clustered(np.asarray(sizes, np.int64), seed_base)
    else:
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        x = np.concatenate([workloads.uniform(int(s), d, seed_base + i) for i, s in enumerate(sizes)])
    lens = np.array([np.float32(0.2 * (1.0 / s) ** (1.0 / 3.0)) for s in sizes], np.float32)
    return x, off, lens


@pytest.mark.parametrize("d,traversal", ((3, 0), (3, 1), (2, 0), (8, 0), (8, 1)))
def test_batch_matches_per_set_and_oracle(d, traversal):
    dev()
    sizes = [1, 2, 33, 700, 5000, 20011, 64, 3, 12000, 257]
    x, off, lens = _batch(sizes, 900, d)
    say(f"batch d={d} traversal={traversal} sets={len(sizes)} total={off[-1]}")
    plan = kdt.BatchPlan(off, d, 8, traversal=traversal)
    xt, lt = to_dev(x), to_dev(lens)
    outs = {}
    for mode in (1, 2, 0, 1):
        outs.setdefault(mode, []).append([to_host(a) for a in plan.launch(xt, lt, use_graph=mode)])
    ref = outs[0][0]
    for mode, runs in outs.items():
        for r in runs:
            for a, b in zip(r, ref):
                np.testing.assert_array_equal(a, b)
    idx, d2, lab = ref
    for s, n in enumerate(sizes):
        xs = x[off[s]:off[s + 1]]
        t = oracle.Tree(xs, 32)
        oi, od = t.knn(xs, 8)
        np.testing.assert_array_equal(idx[off[s]:off[s + 1]], oi)
        np.testing.assert_array_equal(d2[off[s]:off[s + 1]], od)
        np.testing.assert_array_equal(lab[off[s]:off[s + 1]], t.fof(float(lens[s])))
    plan.close()


def test_graph_replays_stay_exact_with_eager_work_between():
    dev()
    sizes = workloads.batch_sizes(40, 2.0, 4.5, seed=8)
    x, off, lens = _batch(sizes, 5000)
    plan = kdt.BatchPlan(off, 3, 8)
    xt, lt = to_dev(x), to_dev(lens)
    ref = [to_host(a) for a in plan.launch(xt, lt, use_graph=0)]
    out = plan.launch(xt, lt, use_graph=1)
    for rep in range(4):
        say(f"graph replay {rep}")
        junk = torch.randn(1 << 20, device=xt.device).sum()  # eager work in between
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        out = plan.launch(xt, lt, use_graph=1, out=out)
        for a, b in zip(out, ref):
            np.testing.assert_array_equal(to_host(a), b)
    # new output buffers force a fresh capture
    out2 = plan.launch(xt, lt, use_graph=1)
    for a, b in zip(out2, ref):
        np.testing.assert_array_equal(to_host(a), b)
    plan.close()


def test_batch_rejects_bad_arguments():
    dev()
    with pytest.raises(kdt.KdtError) as e:
        kdt.BatchPlan(np.array([0, 10, 5], np.int64), 3, 8)
    assert e.value.status == kdt.KDT_EINVAL
    with pytest.raises(kdt.KdtError) as e:
        kdt.BatchPlan(np.array([0, 10], np.int64), 5, 8)
    assert e.value.status == kdt.KDT_EUNSUPPORTED
    with pytest.raises(kdt.KdtError) as e:
        kdt.BatchPlan(np.array([0, 10], np.int64), 3, 65)
    assert e.value.status == kdt.KDT_EUNSUPPORTED
