"""kfx_fit_tracks_backward_noalloc (the fit's gradient with its scratch in a
fixed device array of the library, for callers that cannot allocate)
against kfx_fit_tracks_backward on the same inputs: identical gradients on
two calls in a row, the second with fewer tracks, with one weight and with
per-track weights; zero tracks give a zero gradient; a track count beyond
the scratch limit is refused before any work is queued."""
import numpy as np
import pytest

import kfsynth
import oracle

pytestmark = pytest.mark.gpu

PRIOR = oracle.DEFAULT_PRIOR


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
    ev = kfsynth.generate("align200k", tracks_per_event=3000)
    ctx = kfx.Context(0)
    w = ev.workload
    ctx.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    hits = kfx.DeviceHits.from_events(ev, dev)
    rng = np.random.default_rng(7)
    align = rng.normal(0.0, 50e-4, size=(ev.geometry.n_layers, 3)).astype(np.float32)
    return ev, ctx, hits, align


def grads(kfx, dev, ctx, hits, ev, n, align, per_track, no_alloc):
    import torch
    off = torch.as_tensor(ev.trk_offsets[:n + 1].copy(), device=dev)
    th = torch.as_tensor(ev.trk_hits[:int(ev.trk_offsets[n])].copy(), device=dev)
    al = torch.as_tensor(align.reshape(-1), device=dev)
    out = ctx.fit_tracks(hits, off, th, prior=PRIOR, align=al, field_scale=1.002, ckpt=True)
    if per_track:
        w = torch.as_tensor(np.linspace(0.5, 1.5, n).astype(np.float32), device=dev)
    else:
        w = torch.ones(1, device=dev)
    da, df = ctx.fit_tracks_backward(hits, off, th, out, w, prior=PRIOR, align=al, field_scale=1.002,
                                     no_alloc=no_alloc)
    torch.cuda.synchronize()
    return np.concatenate([da.cpu().numpy(), df.cpu().numpy()])


@pytest.mark.parametrize("per_track", [False, True])
def test_noalloc_matches_the_allocating_call(dev, kfx, setup, per_track):
    ev, ctx, hits, align = setup
    for n in (3000, 700):  # the second call with a smaller input
        print(f"[no_alloc] tracks {n} per_track {per_track}", flush=True)
        g_na = grads(kfx, dev, ctx, hits, ev, n, align, per_track, True)
        g_ref = grads(kfx, dev, ctx, hits, ev, n, align, per_track, False)
        assert np.abs(g_ref).max() > 0
        assert np.array_equal(g_na, g_ref), f"{n} tracks: max diff {np.abs(g_na - g_ref).max()}"


def test_noalloc_zero_tracks_and_limit(dev, kfx, setup):
    import torch
    ev, ctx, hits, align = setup
    off = torch.as_tensor(ev.trk_offsets[:11].copy(), device=dev)
    th = torch.as_tensor(ev.trk_hits[:int(ev.trk_offsets[10])].copy(), device=dev)
    out = ctx.fit_tracks(hits, off, th, prior=PRIOR, ckpt=True)
    z = torch.zeros(1, dtype=torch.int32, device=dev)
    da, df = ctx.fit_tracks_backward_noalloc(hits, z, th[:0], out, torch.ones(1, device=dev), prior=PRIOR)
    torch.cuda.synchronize()
    assert float(da.abs().sum()) == 0.0 and float(df.abs().sum()) == 0.0
    # 1.4M tracks need more than the 2^20 float64 of scratch with 17 barrel
    # layers: refused on the host (the arrays are never read)
    big = torch.zeros(1_400_001, dtype=torch.int32, device=dev)
    with pytest.raises(kfx.KfxError) as e:
        ctx.fit_tracks_backward_noalloc(hits, big, th, out, torch.ones(1, device=dev), prior=PRIOR)
    assert e.value.code == kfx.KFX_EOVERFLOW
    # the entry point still works after the refusal
    g_na = grads(kfx, dev, ctx, hits, ev, 500, align, False, True)
    g_ref = grads(kfx, dev, ctx, hits, ev, 500, align, False, False)
    assert np.array_equal(g_na, g_ref)
