"""Out-of-memory paths of every entry point that allocates device scratch.

kdt_debug_fail_alloc(after) makes the after-th next device allocation of the
library fail as if the device were full.  For each entry point the test arms
the hook with after = 1, 2, ... in turn: every call that meets the failure
must return KDT_ENOMEM with an error text, and the first call that no longer
reaches the failing allocation must return the results of a call made with
no failure.  So every allocation of the call is failed once, and the library
is shown to stay usable (trees, streams and cached scratch intact) after each
failure."""
import numpy as np
import pytest
import torch

from paper_2609_18316_amd import kdt, workloads
from tests.gpu_util import dev, say, to_dev, to_host

pytestmark = pytest.mark.gpu

MAX_ALLOCS = 64


def _same(a, b):
    if isinstance(a, (tuple, list)):
        assert len(a) == len(b)
        for u, v in zip(a, b):
            _same(u, v)
    elif isinstance(a, torch.Tensor):
        np.testing.assert_array_equal(to_host(a), to_host(b))
    else:
        assert a == b


def _each_allocation_fails_once(name, call, check=None):
    """Arms the hook at 1, 2, ... allocations until `call` succeeds; returns
    the number of allocations the call made."""
    want = call()
    torch.cuda.synchronize()
    for after in range(1, MAX_ALLOCS + 1):
        say(f"ENOMEM {name}: allocation {after} fails")
        kdt.fail_alloc(after)
        try:
            got = call()
        except kdt.KdtError as e:
            assert e.status == kdt.KDT_ENOMEM, (name, after, e)
            assert str(e), name
            continue
        finally:
            kdt.fail_alloc(0)
        torch.cuda.synchronize()
        (check or _same)(got, want)
        return after - 1
    raise AssertionError(f"{name}: still failing after {MAX_ALLOCS} allocations")


def test_every_allocation_of_every_entry_point_can_fail():
    dev()
    n, nq = 20011, 3000
    x = to_dev(workloads.clustered(n, 91))
    q = to_dev(workloads.uniform(nq, 3, 92))
    m = to_dev(workloads.masses(n, 93))
    fails = {}

    def build(rule):
        def call():
            t = kdt.build(x, leaf_size=16, split_rule=rule)
            e = t.export()
            t.close()
            return tuple(torch.from_numpy(np.ascontiguousarray(e[k])) for k in ("perm", "pts"))
        return call

    def check_export(a, b):
        for u, v in zip(a, b):
            np.testing.assert_array_equal(u.numpy(), v.numpy())

    fails["build median"] = _each_allocation_fails_once("build median", build(kdt.SPLIT_MEDIAN),
                                                        check_export)
    fails["build midpoint"] = _each_allocation_fails_once(
        "build midpoint", build(kdt.SPLIT_MIDPOINT), check_export)

    for rule in (kdt.SPLIT_MEDIAN, kdt.SPLIT_MIDPOINT):
        t = kdt.build(x, leaf_size=16, split_rule=rule)
        tag = "median" if rule == kdt.SPLIT_MEDIAN else "midpoint"
        fails[f"knn {tag}"] = _each_allocation_fails_once(f"knn {tag}", lambda: t.knn(q, 16))
        fails[f"hsml {tag}"] = _each_allocation_fails_once(
            f"hsml {tag}", lambda: t.knn(None, 32, kth_only=2))
        fails[f"range lists {tag}"] = _each_allocation_fails_once(
            f"range lists {tag}", lambda: t.range(q, 0.03, lists=True))
        fails[f"fof {tag}"] = _each_allocation_fails_once(
            f"fof {tag}", lambda: t.fof(0.004, count_groups=True))
        if rule == kdt.SPLIT_MEDIAN:
            fails["knn k=200"] = _each_allocation_fails_once("knn k=200", lambda: t.knn(q, 200))
            lo, hi = (q - 0.02).contiguous(), (q + 0.02).contiguous()
            fails["box lists"] = _each_allocation_fails_once(
                "box lists", lambda: t.box(lo, hi, lists=True))
            qp = torch.remainder(q, 1.0).contiguous()
            fails["torus knn"] = _each_allocation_fails_once(
                "torus knn", lambda: t.knn(qp, 16, period=1.0))
            fails["torus range lists"] = _each_allocation_fails_once(
                "torus range lists", lambda: t.range(qp, 0.03, lists=True, period=1.0))
            fails["torus fof"] = _each_allocation_fails_once(
                "torus fof", lambda: t.fof(0.004, count_groups=True, period=1.0))
            h = t.knn(None, 32, kth_only=2)
            g = torch.randn((64,) * 3, device=dev(), generator=torch.Generator(dev()).manual_seed(3))
            # P2M keeps its scratch per stream between calls: releasing it
            # first makes every call allocate
            for name, fn in (
                    ("p2m", lambda: kdt.p2m(x, m, h, (0, 0, 0), 1 / 64, (64,) * 3)),
                    ("p2m periodic", lambda: kdt.p2m(x, m, h, (0, 0, 0), 1 / 64, (64,) * 3,
                                                     periodic=True)),
                    ("p2m tsc", lambda: kdt.p2m_cloud(x, m, (0, 0, 0), 1 / 64, (64,) * 3, "tsc")),
                    ("p2m backward", lambda: kdt.p2m_backward(x, m, h, (0, 0, 0), 1 / 64,
                                                              (64,) * 3, g))):
                def call(fn=fn):
                    kdt.stream_release()
                    return fn()

                def close(a, b):
                    for u, v in zip(a if isinstance(a, tuple) else (a,),
                                    b if isinstance(b, tuple) else (b,)):
                        np.testing.assert_allclose(to_host(u), to_host(v), rtol=1e-6, atol=1e-6)
                fails[name] = _each_allocation_fails_once(name, call, close)
        t.close()
    say(f"allocations failed per entry point: {fails}")
    for name, k in fails.items():
        if name.startswith("hsml"):
            # the self-query kNN walks the tree order in place: no scratch
            assert k == 0, name
        else:
            assert k >= 1, f"{name} made no device allocation the hook could fail"
