"""GPU parity of duplicate removal (kfx_find_duplicates) against the oracle
(oracle/duplicates.py; abstract and Sec. 3).  Every decision is integer or a
float32 comparison of the inputs, so the result must be identical."""
import json
import os

import numpy as np
import pytest

import kfsynth
import oracle
from oracle import duplicates as D

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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
def ctx(kfx, dev):
    return kfx.Context(0)


def _gpu(ctx, t, K, NH, num=1, den=2):
    import torch
    out = ctx.tracks_from_arrays(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], K)
    d = ctx.find_duplicates(out, NH, (num, den))
    torch.cuda.synchronize()
    return d.cpu().numpy()


def _oracle(t, K, NH, num=1, den=2, only=None):
    return D.find_duplicates(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], K, NH, num, den,
                             only=only)


@pytest.mark.parametrize("frac", ["1/2", "1/1", "1/100"])
def test_golden(ctx, frac):
    with open(os.path.join(HERE, "golden", "duplicates_small.json")) as f:
        d = json.load(f)
    num, den = map(int, frac.split("/"))
    t = {k: np.array(d[k]) for k in ("n_cands", "hits", "n_hits", "n_holes", "chi2")}
    print(f"golden {frac}", flush=True)
    assert _gpu(ctx, t, d["K"], d["n_hits_total"], num, den).tolist() == d["expected"][frac]


# (seeds, K, max_hits, hits in the batch, fraction, generator seed): sizes
# around the 64-track blocks, K at 1 and 16,
# list capacities 3 and 64, no hits at all, heavy sharing (few hits)
CASES = [
    (1, 1, 48, 10, 1, 2, 0), (63, 6, 48, 100, 1, 2, 1), (64, 6, 48, 100, 1, 3, 2), (65, 16, 48, 500, 2, 3, 3),
    (257, 1, 3, 50, 1, 2, 4), (1000, 6, 64, 4000, 1, 2, 5), (3000, 10, 48, 40, 1, 100, 6),
    (2000, 6, 48, 0, 1, 2, 7), (20000, 6, 48, 200000, 1, 2, 8), (5000, 6, 64, 20000, 1, 1, 9),
]


@pytest.mark.parametrize("S,K,H,NH,num,den,seed", CASES)
def test_parity_synthetic(ctx, S, K, H, NH, num, den, seed):
    print(f"dups S={S} K={K} H={H} NH={NH} frac={num}/{den} seed={seed}", flush=True)
    t = kfsynth.track_lists(S, K, H, NH, seed=seed, chi2_levels=1 + seed % 5)
    g = _gpu(ctx, t, K, NH, num, den)
    o = _oracle(t, K, NH, num, den)
    np.testing.assert_array_equal(g, o)


def test_parity_full_size_sampled(ctx):
    """100k seeds over 1.5M hits (the batched workload's scale): every seed's
    result is checked for validity, 3000 sampled seeds against the oracle."""
    S, K, NH = 100000, 6, 1500000
    print(f"dups full size S={S}", flush=True)
    t = kfsynth.track_lists(S, K, 48, NH, seed=21, seeds_per_truth=1.3)
    g = _gpu(ctx, t, K, NH)
    sample = np.random.default_rng(5).choice(S, 3000, replace=False)
    o = _oracle(t, K, NH, only=sample)
    np.testing.assert_array_equal(g[sample], o[sample])
    # validity everywhere: a flagged seed points to a seed with a track
    nc = t["n_cands"]
    assert ((g == -2) == (nc <= 0)).all()
    f = np.nonzero(g >= 0)[0]
    assert (nc[g[f]] > 0).all() and (g[f] != f).all()


def test_repeat_calls_and_shrinking_input(ctx):
    """Workspaces are reused: a large call, then a small one, then the large
    one again give the oracle's result each time."""
    big = kfsynth.track_lists(3000, 6, 48, 5000, seed=31)
    small = kfsynth.track_lists(100, 6, 48, 300, seed=32)
    for t, NH in ((big, 5000), (small, 300), (big, 5000)):
        np.testing.assert_array_equal(_gpu(ctx, t, 6, NH), _oracle(t, 6, NH))


def test_empty_and_errors(ctx, kfx):
    import torch
    t = kfsynth.track_lists(10, 6, 48, 100, seed=1)
    out = ctx.tracks_from_arrays(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], 6)
    assert ctx.find_duplicates(out, 100, n_seeds=0).numel() == 0
    for frac in ((0, 2), (3, 2), (-1, 1)):
        with pytest.raises(kfx.KfxError):
            ctx.find_duplicates(out, 100, frac)
    with pytest.raises(kfx.KfxError):
        ctx.find_duplicates(out, -1)
    bad = dict(out)
    bad["K"] = 17
    with pytest.raises(kfx.KfxError):
        ctx.find_duplicates(bad, 100)
    wide = kfsynth.track_lists(4, 1, 65, 100, seed=2)
    out = ctx.tracks_from_arrays(wide["n_cands"], wide["hits"], wide["n_hits"], wide["n_holes"], wide["chi2"], 1)
    with pytest.raises(kfx.KfxError):
        ctx.find_duplicates(out, 100)
    torch.cuda.synchronize()


def test_after_building_with_duplicate_seeds(kfx, dev):
    """End to end on the 5k-track event with a second seed for a quarter of
    the particles: GPU building + GPU duplicate removal against oracle
    building + oracle duplicate removal (the builds agree on nearly every
    best candidate; the duplicate decisions must agree as often), and the
    physics: extra seeds flagged as duplicates of their particle's track."""
    import torch
    ev = kfsynth.generate("build5k")
    seeds, seed_event, seed_track = kfsynth.duplicate_seeds(ev, 0.25, seed=0)
    S, T, K = seeds.shape[0], ev.n_tracks, 6
    print(f"dups after building S={S}", flush=True)
    ctx = kfx.Context(0)
    w = ev.workload
    ctx.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    hits = kfx.DeviceHits.from_events(ev, dev)
    out = ctx.build_tracks(hits, seeds, seed_event, chi2_cut=30.0, max_cands=K, max_holes=3, max_steps=32,
                           prior=oracle.DEFAULT_PRIOR, mode=kfx.MODE_FUSED)
    g = ctx.find_duplicates(out, ev.n_hits)
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    o_b = oracle.build_tracks(ev, seeds=seeds, seed_event=seed_event, prior=oracle.DEFAULT_PRIOR,
                              max_hits=out["hits"].shape[1])
    o = D.find_duplicates(o_b["n"], o_b["hits"].reshape(S * K, -1), o_b["nhits"].ravel(),
                          o_b["nholes"].ravel(), o_b["chi2"].ravel().astype(np.float32), K, ev.n_hits)
    agree = np.mean(g == o)
    assert agree >= 0.98, agree
    extra = np.arange(T, S)
    assert np.mean(g[extra] == seed_track[extra]) > 0.8
    # validity of every GPU decision on the GPU's own building output
    gh = out["hits"].cpu().numpy()
    nh = out["n_hits"].cpu().numpy()[::K]
    for b in np.nonzero(g >= 0)[0][:2000]:
        a = g[b]
        hb = set(gh[b * K][gh[b * K] >= 0].tolist())
        ha = set(gh[a * K][gh[a * K] >= 0].tolist())
        assert 2 * len(ha & hb) >= min(len(ha), len(hb)) and nh[a] >= nh[b]


# ------------------------------------------------------------ hit masking

def _gpu_mask(ctx, t, K, layer, dup=None, min_hits=8, cut=3.0, in_place=False):
    import torch
    out = ctx.tracks_from_arrays(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], K)
    lay = torch.as_tensor(np.ascontiguousarray(layer, dtype=np.int32), device=ctx.device)
    d = None if dup is None else torch.as_tensor(np.ascontiguousarray(dup, dtype=np.int32), device=ctx.device)
    res = ctx.mask_hits(out, lay, d, min_hits, cut, layer_out=lay if in_place else None)
    torch.cuda.synchronize()
    return res.cpu().numpy()


@pytest.mark.parametrize("cut", ["3.0", "1.0"])
def test_mask_golden(ctx, cut):
    with open(os.path.join(HERE, "golden", "duplicates_small.json")) as f:
        d = json.load(f)
    t = {k: np.array(d[k]) for k in ("n_cands", "hits", "n_hits", "n_holes", "chi2")}
    layer = (np.arange(d["n_hits_total"]) % 7).astype(np.int32)
    got = _gpu_mask(ctx, t, d["K"], layer, d["expected"]["1/2"], d["mask"]["min_hits"], float(cut))
    assert np.nonzero(got == -1)[0].tolist() == d["mask"]["expected_masked"][cut]


@pytest.mark.parametrize("S,K,H,NH,min_hits,cut,use_dup,in_place,seed", [
    (1, 1, 48, 10, 3, 3.0, True, False, 0), (300, 6, 48, 2000, 4, 1.0, True, False, 1),
    (5000, 16, 64, 30000, 6, 2.5, False, True, 2), (20000, 6, 48, 0, 3, 3.0, True, False, 3),
    (20000, 6, 3, 100000, 1, float("inf"), True, True, 4),
    # masking has no list-width limit (duplicate removal stops at 64)
    (500, 4, 100, 3000, 5, 2.0, False, False, 5)])
def test_mask_parity(ctx, S, K, H, NH, min_hits, cut, use_dup, in_place, seed):
    print(f"mask S={S} K={K} H={H} NH={NH} min_hits={min_hits} cut={cut} dup={use_dup} "
          f"in_place={in_place}", flush=True)
    t = kfsynth.track_lists(S, K, H, NH, seed=seed, chi2_levels=12)
    layer = np.random.default_rng(seed).integers(-1, 35, NH).astype(np.int32)
    dup = _oracle(t, K, NH) if use_dup else None
    got = _gpu_mask(ctx, t, K, layer, dup, min_hits, cut, in_place)
    exp = D.mask_hits(t["n_cands"], t["hits"], t["n_hits"], t["chi2"], K, layer, dup, min_hits, cut)
    np.testing.assert_array_equal(got, exp)


def test_mask_errors(ctx, kfx):
    import torch
    t = kfsynth.track_lists(10, 6, 48, 100, seed=1)
    out = ctx.tracks_from_arrays(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], 6)
    lay = torch.zeros(100, dtype=torch.int32, device=ctx.device)
    with pytest.raises(kfx.KfxError):
        ctx.mask_hits(out, lay, max_chi2_ndof=float("nan"))
    bad = dict(out)
    bad["K"] = 0
    with pytest.raises(kfx.KfxError):
        ctx.mask_hits(bad, lay)
    assert ctx.mask_hits(out, lay, n_seeds=0).cpu().numpy().tolist() == [0] * 100


def test_two_iterations(kfx, dev):
    """Iteration 1 builds from the first three hits of half of the particles
    (even ids); duplicate removal and masking take the good tracks' hits
    out; iteration 2 builds from a second seed (hits 1, 2, 4) of every
    particle whose seed hits are all still free (the other half).  The GPU's mask from its own iteration 1 agrees with the
    oracle's from the oracle's iteration 1 on nearly every hit; iteration 2
    on the oracle's mask and seeds agrees with the oracle's iteration 2 on
    nearly every best candidate, and searches fewer hits than without the
    mask."""
    import dataclasses
    import torch
    ev = kfsynth.generate("build5k", tracks_per_event=1500)
    K = 6
    print("two iterations", flush=True)
    ctx = kfx.Context(0)
    w = ev.workload
    ctx.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    hits = kfx.DeviceHits.from_events(ev, dev)
    kw = dict(chi2_cut=30.0, max_cands=K, max_holes=3, max_steps=32, prior=oracle.DEFAULT_PRIOR)
    half = np.arange(0, ev.n_tracks, 2)
    seeds1, sev1 = ev.seeds[half], ev.trk_event[half]
    out1 = ctx.build_tracks(hits, seeds1, sev1, **kw)
    dup1 = ctx.find_duplicates(out1, ev.n_hits)
    lay_g = ctx.mask_hits(out1, hits.layer, dup1, 8, 3.0).cpu().numpy()
    o1 = oracle.build_tracks(ev, seeds=seeds1, seed_event=sev1, prior=oracle.DEFAULT_PRIOR,
                             max_hits=out1["hits"].shape[1])
    S = half.shape[0]
    H = o1["hits"].shape[2]
    od = D.find_duplicates(o1["n"], o1["hits"].reshape(S * K, H), o1["nhits"].ravel(), o1["nholes"].ravel(),
                           o1["chi2"].ravel().astype(np.float32), K, ev.n_hits)
    lay_o = D.mask_hits(o1["n"], o1["hits"].reshape(S * K, H), o1["nhits"].ravel(),
                        o1["chi2"].ravel().astype(np.float32), K, ev.layer, od, 8, 3.0)
    assert np.mean(lay_g == lay_o) > 0.99
    masked = np.mean(lay_o == -1)
    assert 0.15 < masked < 0.6, masked
    # iteration 2 on the oracle's mask
    seeds2, sev2, strk2 = kfsynth.duplicate_seeds(ev, 1.0, seed=0)
    T = ev.n_tracks
    seeds2, sev2, strk2 = seeds2[T:], sev2[T:], strk2[T:]
    free = (lay_o[seeds2] >= 0).all(axis=1)
    seeds2, sev2 = seeds2[free], sev2[free]
    # the free second seeds are those of the particles iteration 1 skipped
    assert np.mean(strk2[free] % 2 == 1) > 0.95 and free.sum() > 0.4 * T
    ev2 = dataclasses.replace(ev, layer=lay_o.astype(np.int32))
    hits2 = kfx.DeviceHits.from_events(ev2, dev)
    ctx2 = kfx.Context(0)
    ctx2.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    out2 = ctx2.build_tracks(hits2, seeds2, sev2, **kw)
    torch.cuda.synchronize()
    o2 = oracle.build_tracks(ev2, seeds=seeds2, seed_event=sev2, prior=oracle.DEFAULT_PRIOR,
                             max_hits=out2["hits"].shape[1])
    g2 = out2["hits"].cpu().numpy()
    same = np.mean([np.array_equal(g2[s * K], o2["hits"][s, 0]) for s in range(seeds2.shape[0])])
    assert same >= 0.97, same
    # no masked hit is used by iteration 2
    used = g2[g2 >= 0]
    assert (lay_o[used] >= 0).all()
