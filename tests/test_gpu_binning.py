"""GPU tests of the build's hit index made one workgroup per event (LDS
counters, per-event scan) against the counting sort over the whole batch:
the tracks built on either index are bit-identical, on a batch large enough
for the automatic choice to take the per-event kernel, on events with hits
that get no bin (non-finite coordinates, layer ids outside the geometry),
an empty event, a bin holding more hits than the 8-bit LDS counters can
count (the workgroup then counts its event again with global atomics), and
in a captured graph."""
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


def snapshot(out):
    res = {k: out[k].cpu().numpy().copy() for k in KEYS}
    res["p"], res["C"] = out["state"].to_numpy()
    res["stats"] = out["stats"].cpu().numpy().copy()
    return res


def same(a, b):
    return all(np.array_equal(a[k], b[k]) for k in KEYS + ("p", "C"))


def _context(kfx, ev):
    ctx = kfx.Context(0)
    w = ev.workload
    ctx.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    return ctx


def _kw(ev):
    w = ev.workload
    return dict(chi2_cut=w.chi2_cut, max_cands=w.max_cands, max_holes=w.max_holes, max_steps=32, prior=PRIOR)


def test_per_event_index_gives_identical_tracks(dev, kfx):
    import torch
    ev = kfsynth.generate("batch256", n_events=70)
    ctx = _context(kfx, ev)
    hits = kfx.DeviceHits.from_events(ev, dev)
    seeds = torch.as_tensor(ev.seeds, device=dev)
    sev = torch.as_tensor(ev.trk_event.astype(np.int32), device=dev)
    kw = _kw(ev)
    print(f"[binning] 70 events, {ev.n_hits} hits, {ev.n_tracks} seeds", flush=True)
    nk = ev.geometry.n_layers * ev.workload.n_eta_bins * ev.workload.n_phi_bins
    ref = snapshot(ctx.build_tracks(hits, seeds, sev, binning=1, **kw))
    assert ctx.index_keys_per_event() == nk
    assert ref["stats"][0] > 0
    for b in (0, 2):
        got = snapshot(ctx.build_tracks(hits, seeds, sev, binning=b, **kw))
        # 70 events: the automatic choice takes one workgroup per event too
        assert ctx.index_keys_per_event() == nk + 1, f"binning={b}"
        assert same(got, ref), f"binning={b}"
        assert np.array_equal(got["stats"][:3], ref["stats"][:3]), f"binning={b} stats"
    # the plain per-stage path on the per-event index
    got = snapshot(ctx.build_tracks(hits, seeds, sev, binning=2, mode=kfx.MODE_PLAIN, **kw))
    assert same(got, ref)
    # captured with the per-event binning, replayed between eager builds
    graph, gout = ctx.build_graph(hits, seeds, sev, binning=2, **kw)
    try:
        for rep in range(3):
            other = ctx.build_tracks(hits, seeds, sev, binning=1, **kw)
            torch.cuda.synchronize()
            graph.launch()
            torch.cuda.synchronize()
            assert same(snapshot(gout), ref), f"replay {rep}"
            assert same(snapshot(other), ref)
    finally:
        graph.close()


def _awkward_batch():
    """batch256-like events with, inserted at the end of some events: hits
    without a bin (NaN coordinates, layer -1, a layer id past the table),
    301 copies of one hit (a bin with more than 255 hits), and an empty
    event inserted after event 3.  Seeds are remapped to the new indices."""
    ev = kfsynth.generate("batch256", n_events=8)
    off = ev.event_offsets.astype(np.int64)
    x, y, z, lay = (np.asarray(a) for a in (ev.x, ev.y, ev.z, ev.layer))
    parts = {k: [] for k in "xyzl"}
    new_off = [0]
    shift = np.zeros(ev.n_events, np.int64)
    extra_total = 0
    for e in range(ev.n_events):
        lo, hi = int(off[e]), int(off[e + 1])
        ex = {k: [] for k in "xyzl"}

        def add(n, xv, yv, zv, lv):
            ex["x"] += [xv] * n
            ex["y"] += [yv] * n
            ex["z"] += [zv] * n
            ex["l"] += [lv] * n

        if e == 2:
            add(5, np.nan, y[lo], z[lo], 3)
            add(5, x[lo], y[lo], z[lo], -1)
            add(5, x[lo], y[lo], z[lo], 999)
        if e == 5:
            # the fifth hit of the event's first track with six or more
            t = next(t for t in range(ev.n_tracks)
                     if ev.trk_event[t] == 5 and ev.trk_offsets[t + 1] - ev.trk_offsets[t] >= 6)
            j = int(ev.trk_hits[ev.trk_offsets[t] + 4])
            add(301, x[j], y[j], z[j], lay[j])
        shift[e] = extra_total
        for k, a in zip("xyzl", (x, y, z, lay)):
            parts[k].append(a[lo:hi])
            parts[k].append(np.asarray(ex[k], dtype=a.dtype))
        extra_total += len(ex["x"])
        new_off.append(hi + extra_total)
        if e == 3:
            new_off.append(new_off[-1])  # an empty event
    cat = {k: np.concatenate(v) for k, v in parts.items()}
    seeds = ev.seeds.astype(np.int64)
    se = ev.trk_event.astype(np.int64)
    seeds = seeds + shift[se][:, None]
    se = se + (se >= 4)
    return ev, cat, np.asarray(new_off, np.int32), seeds.astype(np.int32), se.astype(np.int32)


def test_per_event_index_awkward_events(dev, kfx):
    import torch
    ev, cat, off, seeds_h, se_h = _awkward_batch()
    ctx = _context(kfx, ev)
    t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt), device=dev)
    hits = kfx.DeviceHits(t(cat["x"], np.float32), t(cat["y"], np.float32), t(cat["z"], np.float32),
                          t(cat["l"], np.int32), t(off, np.int32))
    seeds, sev = t(seeds_h, np.int32), t(se_h, np.int32)
    kw = _kw(ev)
    print(f"[binning] awkward batch: {hits.n_events} events, {hits.n_hits} hits", flush=True)
    ref = snapshot(ctx.build_tracks(hits, seeds, sev, binning=1, **kw))
    assert ref["stats"][0] > 0
    got = snapshot(ctx.build_tracks(hits, seeds, sev, binning=2, **kw))
    nk = ev.geometry.n_layers * ev.workload.n_eta_bins * ev.workload.n_phi_bins
    assert ctx.index_keys_per_event() == nk + 1
    assert same(got, ref)
    assert np.array_equal(got["stats"][:3], ref["stats"][:3])
    # the copies are found: some kept candidate holds one of them (event 5
    # is the 7th range, after the inserted empty event)
    h = got["hits"]
    assert ((h >= int(off[7]) - 301) & (h < int(off[7]))).any()


def test_binning_mode_validated(dev, kfx):
    import torch
    ev = kfsynth.generate("batch256", n_events=2)
    ctx = _context(kfx, ev)
    hits = kfx.DeviceHits.from_events(ev, dev)
    seeds = torch.as_tensor(ev.seeds, device=dev)
    sev = torch.as_tensor(ev.trk_event.astype(np.int32), device=dev)
    with pytest.raises(kfx.KfxError, match="binning"):
        ctx.build_tracks(hits, seeds, sev, binning=3, **_kw(ev))
