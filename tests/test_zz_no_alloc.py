"""The allocation-free bake entry point (sdfddgi_bake_sdf_noalloc) against the
allocating one (sdfddgi_bake_sdf), through the C ABI: identical bits for the
distance grid and the nearest-primitive albedo, on two calls in a row (the second
smaller, so stale staging from the first would show), with zero primitives, and
at the staging limit; and the limit's error."""
import sys

import numpy as np
import pytest

import scenegen

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def S():
    import torch
    from paper_2007_14394_amd import sdfddgi
    assert torch.cuda.is_available(), "GPU tests need a visible gfx950 device"
    sdfddgi.load_library()
    return sdfddgi


def prims(seed, count):
    rng = np.random.default_rng(seed)
    return scenegen.open_scene_primitives(rng, count, (-8.0, 0.0, -8.0), (8.0, 4.0, 8.0),
                                          size_range=(0.2, 3.0))


def both(S, p, n, origin, spacing, empty=1e30):
    import torch
    a = S.sdfddgi_bake_sdf(p.kind, p.center, p.half, p.albedo, n, origin, spacing, empty)
    # the no-alloc call fills buffers the caller allocated beforehand
    out = (torch.full((n[2], n[1], n[0]), -7.0, device="cuda:0"),
           torch.full((n[2], n[1], n[0], 3), -7.0, device="cuda:0"))
    b = S.sdfddgi_bake_sdf(p.kind, p.center, p.half, p.albedo, n, origin, spacing, empty,
                           out=out, noalloc=True)
    torch.cuda.synchronize()
    for x, y, name in ((a[0], b[0], "sdf"), (a[1], b[1], "albedo")):
        assert torch.equal(x.view(torch.int32), y.view(torch.int32)), name
    return a


def test_noalloc_bake_matches_the_allocating_bake_on_two_calls(S):
    big = prims(1, 300)
    announce("no-alloc bake: 300 primitives on 96x80x72, then 40 on 33x20x41")
    sdf, alb = both(S, big, (96, 80, 72), (-9.0, -1.0, -9.0), 0.21)
    assert float(sdf.min()) < 0.0 < float(sdf.max()) and float(alb.max()) > 0.0
    small = prims(2, 40)
    both(S, small, (33, 20, 41), (-8.5, -0.5, -8.5), 0.43)


def test_noalloc_bake_edge_cases(S):
    from paper_2007_14394_amd.sdfddgi import SDFDDGI_BAKE_NOALLOC_MAX_PRIMS as MAXP
    announce("no-alloc bake: zero primitives, the staging limit, one past it")
    empty = scenegen.Primitives(np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros((0, 3)),
                                np.zeros((0, 3)))
    sdf, alb = both(S, empty, (5, 4, 3), (0.0, 0.0, 0.0), 1.0, empty=123.0)
    assert bool((sdf == 123.0).all()) and bool((alb == 0.0).all())
    full = prims(3, MAXP)
    both(S, full, (17, 9, 13), (-8.0, 0.0, -8.0), 1.0)
    over = prims(4, MAXP + 1)
    with pytest.raises(S.SdfddgiError) as e:
        S.sdfddgi_bake_sdf(over.kind, over.center, over.half, over.albedo, (4, 4, 4),
                           (0.0, 0.0, 0.0), 1.0, noalloc=True)
    assert e.value.status == S.SDFDDGI_EINVAL
