"""GPU tests of the batched build's HIP graph, its autotuner and its timing:
a captured build replays bit-identically to the eager call (with eager work
and synchronisations between replays, inputs changed in place between
launches), every launch shape the autotuner can pick gives identical
results, and the per-call timing splits the build consistently."""
import numpy as np
import pytest

import kfsynth
import oracle

pytestmark = pytest.mark.gpu

PRIOR = oracle.DEFAULT_PRIOR
KEYS = ("n_cands", "hits", "n_hits", "n_holes", "chi2")


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.fixture(scope="module")
def kfx():
    from paper_2002_06295_amd import kfx as k
    return k


@pytest.fixture(scope="module")
def setup(dev, kfx):
    import torch
    ev = kfsynth.generate("batch256", n_events=6)
    ctx = kfx.Context(0)
    w = ev.workload
    ctx.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    hits = kfx.DeviceHits.from_events(ev, dev)
    seeds = torch.as_tensor(ev.seeds, device=dev)
    sev = torch.as_tensor(ev.trk_event.astype(np.int32), device=dev)
    kw = dict(chi2_cut=w.chi2_cut, max_cands=w.max_cands, max_holes=w.max_holes, max_steps=32, prior=PRIOR)
    return ev, ctx, hits, seeds, sev, kw


def snapshot(out):
    res = {k: out[k].cpu().numpy().copy() for k in KEYS}
    res["p"], res["C"] = out["state"].to_numpy()
    res["stats"] = out["stats"].cpu().numpy().copy()
    return res


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in KEYS + ("p", "C"))


def test_graph_replays_match_eager(dev, kfx, setup):
    import torch
    ev, ctx, hits, seeds, sev, kw = setup
    ref_out = ctx.build_tracks(hits, seeds, sev, **kw)
    torch.cuda.synchronize()
    ref = snapshot(ref_out)
    graph, gout = ctx.build_graph(hits, seeds, sev, **kw)
    try:
        for rep in range(3):
            gout["stats"].zero_()
            # eager work between replays, on other buffers
            other = ctx.build_tracks(hits, seeds, sev, **kw)
            torch.cuda.synchronize()
            graph.launch()
            torch.cuda.synchronize()
            got = snapshot(gout)
            assert same(got, ref), f"replay {rep}"
            assert np.array_equal(got["stats"][:3], ref["stats"][:3]), f"replay {rep} stats"
            assert same(snapshot(other), ref)
    finally:
        graph.close()


def test_graph_sees_inputs_changed_in_place(dev, kfx, setup):
    import torch
    ev, ctx, hits, seeds, sev, kw = setup
    s2 = seeds.clone()
    e2 = sev.clone()
    graph, gout = ctx.build_graph(hits, s2, e2, **kw)
    try:
        # new contents, same sizes: the seeds in reverse order
        s2.copy_(torch.flip(seeds, [0]))
        e2.copy_(torch.flip(sev, [0]))
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        ref = snapshot(ctx.build_tracks(hits, torch.flip(seeds, [0]).contiguous(),
                                        torch.flip(sev, [0]).contiguous(), **kw))
        assert same(snapshot(gout), ref)
    finally:
        graph.close()


def test_autotune_shapes_are_bit_identical(dev, kfx, setup):
    import torch
    ev, ctx, hits, seeds, sev, kw = setup
    ref = snapshot(ctx.build_tracks(hits, seeds, sev, **kw))
    choice = ctx.autotune_build(hits, seeds, sev, reps=1, **kw)
    assert choice["block_threads"] in (64, 128, 256)
    assert choice["lanes_per_seed"] in (6, 8, 16) and choice["scan_tile"] in (16, 32, 64, 128, 256)
    assert choice["blocks"] > 0 and choice["ms"] > 0
    assert 1 <= choice["seeds_per_wave"] <= 64 // choice["lanes_per_seed"]
    tuned = {k: v for k, v in choice.items() if k != "ms"}
    assert same(snapshot(ctx.build_tracks(hits, seeds, sev, **kw, **tuned)), ref)
    # the extreme shapes too
    for shape in (dict(block_threads=64, blocks=3, lanes_per_seed=16, scan_tile=1),
                  dict(block_threads=128, blocks=1000, lanes_per_seed=8, scan_tile=100000),
                  dict(block_threads=256, waves_per_simd=2, scan_tile=8),
                  dict(lanes_per_seed=8, seeds_per_wave=1, blocks=7),
                  dict(lanes_per_seed=16, seeds_per_wave=3, scan_tile=32),
                  # groups of 6 lanes: ten seeds a wavefront, lanes 60-63 idle
                  dict(lanes_per_seed=6),
                  dict(lanes_per_seed=6, waves_per_simd=2, block_threads=128, scan_tile=16),
                  dict(lanes_per_seed=6, seeds_per_wave=3, blocks=5, scan_tile=100000)):
        assert same(snapshot(ctx.build_tracks(hits, seeds, sev, **kw, **shape)), ref), shape


def test_twelve_lane_groups_bit_identical(dev, kfx, setup):
    """K = 10 on groups of 12 lanes (five seeds a wavefront, lanes 60-63
    idle, group minimum by lane shuffles) gives the same tracks as on groups
    of 16, at one and two wavefronts per SIMD."""
    ev, ctx, hits, seeds, sev, kw = setup
    kw10 = dict(kw, max_cands=10)
    ref = snapshot(ctx.build_tracks(hits, seeds, sev, **kw10, lanes_per_seed=16))
    assert ref["n_cands"].max() > 6
    for shape in (dict(lanes_per_seed=12), dict(lanes_per_seed=12, waves_per_simd=2, block_threads=128),
                  dict(lanes_per_seed=12, seeds_per_wave=2, scan_tile=16)):
        assert same(snapshot(ctx.build_tracks(hits, seeds, sev, **kw10, **shape)), ref), shape
    with pytest.raises(kfx.KfxError):
        ctx.build_tracks(hits, seeds, sev, **kw, lanes_per_seed=12)  # K = 6


def test_autotune_cache(dev, kfx, setup, tmp_path, monkeypatch):
    """A second autotuner call with the same device and workload signature
    returns the cached shape and time without building; another signature
    (another K) is tuned anew; with KFX_AUTOTUNE_CACHE set every new entry
    is appended to the file, and after the in-process cache is cleared the
    entries come back from the file."""
    import time
    ev, ctx, hits, seeds, sev, kw = setup
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("KFX_AUTOTUNE_CACHE", str(path))
    ctx.autotune_cache_clear()
    t0 = time.perf_counter()
    a = ctx.autotune_build(hits, seeds, sev, reps=1, **kw)
    t1 = time.perf_counter()
    b = ctx.autotune_build(hits, seeds, sev, reps=1, **kw)
    t2 = time.perf_counter()
    assert a == b
    assert (t2 - t1) < 0.2 * (t1 - t0), (t1 - t0, t2 - t1)
    c = ctx.autotune_build(hits, seeds, sev, reps=1, **dict(kw, max_cands=4))
    assert c["lanes_per_seed"] in (4, 8, 16)
    assert len(path.read_text().strip().splitlines()) == 2
    ctx.autotune_cache_clear()
    t3 = time.perf_counter()
    d = ctx.autotune_build(hits, seeds, sev, reps=1, **kw)
    t4 = time.perf_counter()
    assert d["block_threads"] == a["block_threads"] and d["blocks"] == a["blocks"]
    assert d["lanes_per_seed"] == a["lanes_per_seed"] and d["seeds_per_wave"] == a["seeds_per_wave"]
    assert d["scan_tile"] == a["scan_tile"] and d["waves_per_simd"] == a["waves_per_simd"]
    assert (t4 - t3) < 0.2 * (t1 - t0)
    ctx.autotune_cache_clear()
    monkeypatch.delenv("KFX_AUTOTUNE_CACHE")


def test_build_timing_split(dev, kfx, setup):
    import torch
    ev, ctx, hits, seeds, sev, kw = setup
    ctx.enable_timing(4)
    for _ in range(3):
        ctx.build_tracks(hits, seeds, sev, **kw)
    torch.cuda.synchronize()
    times = ctx.build_times(3)
    ctx.enable_timing(0)
    assert len(times) == 3
    for binning, search, building, total in times:
        assert 0 < search <= building <= total and 0 < binning <= total


def test_bad_launch_shapes_rejected(dev, kfx, setup):
    ev, ctx, hits, seeds, sev, kw = setup
    for bad in (dict(lanes_per_seed=4), dict(lanes_per_seed=12), dict(scan_tile=-1), dict(block_threads=96),
                dict(waves_per_simd=3), dict(seeds_per_wave=11), dict(lanes_per_seed=8, seeds_per_wave=9),
                dict(lanes_per_seed=16, seeds_per_wave=5),
                dict(lanes_per_seed=6, seeds_per_wave=11), dict(lanes_per_seed=5),
                dict(seeds_per_wave=-1)):
        with pytest.raises(kfx.KfxError):
            ctx.build_tracks(hits, seeds, sev, **kw, **bad)
