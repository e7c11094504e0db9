"""GPU parity of the fit's adjoint (kfx_fit_tracks_backward and the
torch.autograd.Function around it) against the FP64 oracle: its own
reverse-mode adjoint, its forward-mode dual numbers, and central finite
differences of its chi2 (h = 1e-6) on 1000-track subsets.

Tolerance, per gradient component g against the reference g_ref:
  |g - g_ref| <= 1e-3 max(|g_ref|, 1e-3 max_j |g_ref_j|)
(components near zero are judged against the largest one: near an optimum
a gradient component is a sum of terms of both signs).
"""
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


def make_ctx(kfx, ev):
    ctx = kfx.Context(0)
    w = ev.workload
    ctx.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    return ctx


def mixed_err(g, ref):
    scale = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return np.abs(g - ref) / scale


def gpu_grad(kfx, dev, ev, align=None, fscale=1.0, dchi2=None):
    import torch
    ctx = make_ctx(kfx, ev)
    hits = kfx.DeviceHits.from_events(ev, dev)
    off = torch.as_tensor(ev.trk_offsets, device=dev)
    th = torch.as_tensor(ev.trk_hits, device=dev)
    al = None if align is None else torch.as_tensor(np.asarray(align, np.float32).reshape(-1), device=dev)
    out = ctx.fit_tracks(hits, off, th, prior=PRIOR, align=al, field_scale=fscale, ckpt=True)
    w = torch.ones(1, device=dev) if dchi2 is None else torch.as_tensor(dchi2, dtype=torch.float32, device=dev)
    da, df = ctx.fit_tracks_backward(hits, off, th, out, w, prior=PRIOR, align=al, field_scale=fscale)
    g = np.concatenate([da.cpu().numpy(), df.cpu().numpy()])
    st = out["status"].cpu().numpy()[:ev.n_tracks]
    return g, st, out["chi2"].cpu().numpy()[:ev.n_tracks]


@pytest.fixture(scope="module")
def ev_align():
    # a 1000-track subset of the alignment workload
    return kfsynth.generate("align200k", tracks_per_event=1000)


def test_grad_matches_oracle_adjoint_and_duals(dev, kfx, ev_align):
    ev = ev_align
    g, st, _ = gpu_grad(kfx, dev, ev)
    tot_r, gr = oracle.fit_grad(ev, mode="reverse", prior=PRIOR)
    tot_f, gf = oracle.fit_grad(ev, mode="forward", prior=PRIOR)
    assert np.allclose(gr, gf, rtol=1e-9, atol=1e-9 * np.abs(gr).max())
    nl = ev.geometry.n_layers
    assert np.abs(g).max() > 0 and np.count_nonzero(g[:3 * nl]) == 3 * nl  # barrel only
    err = mixed_err(g, gr)
    assert err.max() <= 1e-3, f"worst component {err.argmax()}: {g[err.argmax()]} vs {gr[err.argmax()]}"


def test_grad_matches_central_differences(dev, kfx, ev_align):
    ev = ev_align
    g, st, _ = gpu_grad(kfx, dev, ev)
    nl = ev.geometry.n_layers
    h = 1e-6
    rng = np.random.default_rng(7)
    comps = list(rng.choice(3 * nl, size=6, replace=False)) + [3 * nl]
    _, gr = oracle.fit_grad(ev, mode="reverse", prior=PRIOR)
    for j in comps:
        a_p = np.zeros(3 * nl)
        a_m = np.zeros(3 * nl)
        fs_p = fs_m = 1.0
        if j < 3 * nl:
            a_p[j] = h
            a_m[j] = -h
        else:
            fs_p, fs_m = 1.0 + h, 1.0 - h
        _, _, cp, _, okp = oracle.fit(ev, align=a_p, fscale=fs_p, prior=PRIOR)
        okp = okp.astype(bool)
        _, _, cm, _, okm = oracle.fit(ev, align=a_m, fscale=fs_m, prior=PRIOR)
        okm = okm.astype(bool)
        assert np.array_equal(okp, okm)
        fd = (cp[okp].sum() - cm[okm].sum()) / (2 * h)
        scale = max(abs(fd), 1e-3 * np.abs(gr).max())
        assert abs(g[j] - fd) <= 1e-3 * scale, f"component {j}: gpu {g[j]} fd {fd}"


def test_grad_away_from_zero(dev, kfx):
    # at the true alignment and field scale (float32-rounded for both sides)
    ev = kfsynth.generate("align200k", tracks_per_event=400, seed_offset=1)
    al = ev.align_true.astype(np.float32)
    fs = np.float32(1.002)
    g, st, _ = gpu_grad(kfx, dev, ev, align=al, fscale=float(fs))
    _, gr = oracle.fit_grad(ev, align=al.astype(np.float64), fscale=float(fs), mode="reverse", prior=PRIOR)
    err = mixed_err(g, gr)
    assert err.max() <= 1e-3, f"worst component {err.argmax()}: {g[err.argmax()]} vs {gr[err.argmax()]}"


def test_grad_full_geometry_with_disks(dev, kfx):
    ev = kfsynth.generate(kfsynth.workload("build5k", noise_per_event=0), tracks_per_event=500)
    g, st, _ = gpu_grad(kfx, dev, ev)
    _, gr = oracle.fit_grad(ev, mode="reverse", prior=PRIOR)
    geo = ev.geometry
    kinds = np.asarray(geo.as_records())[:, 0]
    disk_rows = np.concatenate([[3 * l, 3 * l + 1, 3 * l + 2] for l in np.nonzero(kinds == 1)[0]])
    assert np.all(g[disk_rows] == 0.0) and np.all(gr[disk_rows] == 0.0)
    err = mixed_err(g, gr)
    assert err.max() <= 1e-3, f"worst component {err.argmax()}: {g[err.argmax()]} vs {gr[err.argmax()]}"


def test_grad_weights_and_determinism(dev, kfx, ev_align):
    ev = ev_align
    g1, st, _ = gpu_grad(kfx, dev, ev)
    g1b, _, _ = gpu_grad(kfx, dev, ev)
    assert np.array_equal(g1, g1b)  # fixed-order reduction
    g2, _, _ = gpu_grad(kfx, dev, ev, dchi2=np.array([2.0], np.float32))
    assert np.array_equal(g2, 2.0 * g1)  # every step is linear in the weight
    # per-track weights: the two halves add up to the whole
    T = ev.n_tracks
    wa = np.zeros(T, np.float32)
    wa[: T // 2] = 1.0
    ga, _, _ = gpu_grad(kfx, dev, ev, dchi2=wa)
    gb, _, _ = gpu_grad(kfx, dev, ev, dchi2=1.0 - wa)
    assert np.allclose(ga + gb, g1, rtol=1e-12, atol=1e-12 * np.abs(g1).max())
    # one track alone against the oracle on that track
    t = int(np.nonzero(st == 1)[0][3])
    w1 = np.zeros(T, np.float32)
    w1[t] = 1.0
    gt, _, _ = gpu_grad(kfx, dev, ev, dchi2=w1)
    off = ev.trk_offsets
    _, gro = oracle.fit_grad(ev, trk_offsets=np.array([0, off[t + 1] - off[t]], np.int32),
                             trk_hits=ev.trk_hits[off[t]:off[t + 1]], mode="reverse", prior=PRIOR)
    err = mixed_err(gt, gro)
    assert err.max() <= 1e-3


def test_autograd_function(dev, kfx, ev_align):
    import torch
    from paper_2002_06295_amd import fit_chi2
    ev = ev_align
    ctx = make_ctx(kfx, ev)
    hits = kfx.DeviceHits.from_events(ev, dev)
    off = torch.as_tensor(ev.trk_offsets, device=dev)
    th = torch.as_tensor(ev.trk_hits, device=dev)
    nl = ev.geometry.n_layers
    align = torch.zeros(nl, 3, dtype=torch.float32, device=dev, requires_grad=True)
    fs = torch.ones(1, dtype=torch.float64, requires_grad=True)
    chi2 = fit_chi2(ctx, hits, off, th, align, fs, prior=PRIOR)
    total = chi2.double().sum()
    total.backward()
    tot_r, gr = oracle.fit_grad(ev, mode="reverse", prior=PRIOR)
    assert abs(total.item() - tot_r) <= 1e-6 * tot_r
    g = np.concatenate([align.grad.double().cpu().numpy().reshape(-1), fs.grad.numpy()])
    # float32 align.grad: rounding 6e-8 relative on top of the adjoint's error
    err = mixed_err(g, gr)
    assert err.max() <= 1e-3


def test_backward_bad_inputs(dev, kfx, ev_align):
    import torch
    ev = ev_align
    ctx = make_ctx(kfx, ev)
    hits = kfx.DeviceHits.from_events(ev, dev)
    out = ctx.fit_tracks(hits, ev.trk_offsets, ev.trk_hits, prior=PRIOR)  # no checkpoint
    with pytest.raises(kfx.KfxError):
        ctx.fit_tracks_backward(hits, ev.trk_offsets, ev.trk_hits, out, torch.ones(1, device=dev))
    out = ctx.fit_tracks(hits, ev.trk_offsets, ev.trk_hits, prior=PRIOR, ckpt=True)
    with pytest.raises(kfx.KfxError):  # weights of the wrong length
        ctx.fit_tracks_backward(hits, ev.trk_offsets, ev.trk_hits, out, torch.ones(5, device=dev))
    # zero tracks: zero gradient
    da, df = ctx.fit_tracks_backward(hits, np.zeros(1, np.int32), np.zeros(0, np.int32), out,
                                     torch.ones(1, device=dev))
    assert float(da.abs().sum()) == 0.0 and float(df.abs().sum()) == 0.0
