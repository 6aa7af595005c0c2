"""GPU parity of the analytic-primitive SDF query of Sec. 3.3: the cluster-culled
distance, with and without the previous sample's bound, equals the minimum over
every primitive bit for bit, and so do the sphere traces built on it; culling
evaluates fewer primitives."""
import numpy as np
import pytest

import oracle
import scenegen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    from paper_2007_14394_amd import sdfddgi
    assert torch.cuda.is_available(), "GPU tests need a visible gfx950 device"
    sdfddgi.load_library()
    return sdfddgi


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def open_prims(n=400, seed=0):
    rng = np.random.default_rng(seed)
    return scenegen.open_scene_primitives(rng, n, (-32.0, 0.0, -32.0), (32.0, 16.0, 32.0))


@pytest.mark.parametrize("cluster_size", [2, 8, 64])
def test_culled_query_is_the_brute_force_minimum(S, cluster_size):
    print(f"[gpu] analytic query cluster_size={cluster_size}", flush=True)
    prims = open_prims()
    an = S.sdfddgi_analytic_create(prims.kind, prims.center, prims.half, cluster_size)
    rng = np.random.default_rng(1)
    pts = rng.uniform([-34, -2, -34], [34, 18, 34], (3000, 3)).astype(np.float32)
    pts[:200] = prims.center[:200] + rng.normal(0, 0.3, (200, 3))   # near and inside primitives
    ref = oracle.AnalyticScene(prims).sdf(pts)
    d0, e0 = S.sdfddgi_analytic_query(an, to_dev(pts), 0)
    d1, e1 = S.sdfddgi_analytic_query(an, to_dev(pts), 1)
    assert np.array_equal(to_host(d0).view(np.int32), ref.view(np.int32))
    assert np.array_equal(to_host(d1).view(np.int32), ref.view(np.int32))
    assert e0 == 3000 * 400 and (cluster_size == 400 or e1 < e0)


def test_culled_traces_match_the_checker_bit_for_bit(S):
    prims = open_prims()
    w = scenegen.config2(0, probes=8192, frames=1)
    origins = np.repeat(np.array([oracle.Checker(w).probe_position(p) for p in range(0, 8192, 97)],
                                 dtype=np.float32), 24, axis=0)
    dirs = np.tile(oracle.ray_directions(12345, 24).astype(np.float32), (origins.shape[0] // 24, 1))
    print(f"[gpu] analytic trace {origins.shape[0]} rays", flush=True)
    an = S.sdfddgi_analytic_create(prims.kind, prims.center, prims.half, 8)
    t_max = 64.0 * np.sqrt(3.0)
    ref_t, ref_s, ref_k = oracle.AnalyticScene(prims).trace(origins, dirs, t_max, 1e-3, 1.0, 64)
    evals = []
    for mode in (0, 1, 2):
        t, st, kd, ev = S.sdfddgi_analytic_trace(an, to_dev(origins), to_dev(dirs), t_max,
                                                 mode=mode)
        assert np.array_equal(to_host(t).view(np.int32), ref_t.view(np.int32)), mode
        assert np.array_equal(to_host(st), ref_s) and np.array_equal(to_host(kd), ref_k), mode
        evals.append(ev)
    assert evals[2] < evals[1] < evals[0]
    assert (ref_k == 2).any() and (ref_k == 0).any()


def test_analytic_errors(S):
    with pytest.raises(S.SdfddgiError):
        S.sdfddgi_analytic_create([0], [[0, 0, 0]], [[1, 1, 1]], 0)
    with pytest.raises(S.SdfddgiError):
        S.sdfddgi_analytic_create([2], [[0, 0, 0]], [[1, 1, 1]], 4)
    an = S.sdfddgi_analytic_create([0], [[0, 0, 0]], [[1, 1, 1]], 4)
    with pytest.raises(S.SdfddgiError):
        S.sdfddgi_analytic_query(an, to_dev(np.zeros((4, 3))), 2)
