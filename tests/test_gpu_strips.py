"""GPU parity of strip clustering (kfx_cluster_strips) against the oracle
(oracle/strips.py; Sec. 4).  Every decision is integer or a float32 /
float64 operation taken in the same order, so the kept clusters must be
identical, barycentres included."""
import numpy as np
import pytest

import kfsynth
from oracle import strips as O
from test_oracle_strips import GOLDEN_PARAMS, expected_rows, golden_inputs, rows_of

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2002_06295_amd import kfx
    return kfx.Context(0)


def _gpu(ctx, digis, calib, capacity=None, **p):
    import torch
    dg, cb = ctx.strip_inputs(digis, calib)
    out = ctx.cluster_strips(dg, cb, capacity=capacity, **p)
    torch.cuda.synchronize()
    n = int(out["n"].cpu()[0])
    m = min(n, out["capacity"])
    r = {k: out[k][:m].cpu().numpy() for k in ("event", "module", "first", "size", "charge", "barycenter")}
    return n, r


@pytest.mark.parametrize("key", sorted(GOLDEN_PARAMS))
def test_golden(ctx, key):
    g, digis, calib = golden_inputs()
    print(f"strips golden {key}", flush=True)
    n, r = _gpu(ctx, digis, calib, **GOLDEN_PARAMS[key])
    assert rows_of(r) == expected_rows(g, key) and n == len(expected_rows(g, key))


# (modules, strips per module, events, particles, noise fraction, bad
# fraction, params, seed): tiny to a few 10^5 digis, gap limits 0-4 and 64,
# a charge cut, raised thresholds, dense noise, dense bad strips
CASES = [
    (4, 16, 1, 3, 0.1, 0.1, {}, 0),
    (50, 64, 3, 40, 0.05, 0.08, dict(max_gap=0), 1),
    (200, 128, 5, 300, 0.03, 0.05, dict(max_gap=2, min_charge=60), 2),
    (300, 256, 4, 800, 0.2, 0.05, dict(max_gap=4, seed_thr=6.0, chan_thr=2.5, clus_thr=7.0), 3),
    (3000, 768, 2, 4000, 0.01, 0.01, {}, 4),
    # the gap limit at its maximum over 40 % bad strips (clusters bridge
    # runs of several bad strips)
    (100, 256, 2, 400, 0.05, 0.45, dict(max_gap=64), 5),
]


@pytest.mark.parametrize("M,P,E,npart,nf,bf,params,seed", CASES)
def test_parity(ctx, M, P, E, npart, nf, bf, params, seed):
    print(f"strips M={M} P={P} E={E} particles={npart} noise={nf} bad={bf} {params}", flush=True)
    det = kfsynth.strip_detector(M, P, bad_frac=bf, seed=seed)
    ev = kfsynth.strip_events(det, E, particles_per_event=npart, noise_frac=nf, seed=seed)
    n, r = _gpu(ctx, ev, det, **params)
    o = O.cluster_strips(ev, det, params)
    assert n == o["charge"].shape[0]
    for k in o:
        np.testing.assert_array_equal(r[k], o[k], err_msg=k)


def test_full_size_sampled_modules(ctx):
    """16 events of the full detector (15,000 modules x 768 strips, 20,000
    particles per event; ~2.6M digis): every kept cluster of 150 sampled
    modules identical to the oracle's (modules are independent)."""
    det = kfsynth.strip_detector()
    ev = kfsynth.strip_events(det, 16, seed=7)
    print(f"strips full size: {ev['module'].shape[0]} digis", flush=True)
    n, r = _gpu(ctx, ev, det)
    mods = set(np.random.default_rng(3).choice(det["n_modules"], 150, replace=False).tolist())
    o = O.cluster_strips(ev, det, modules=mods)
    sel = np.isin(r["module"], list(mods))
    for k in o:
        np.testing.assert_array_equal(r[k][sel], o[k], err_msg=k)
    # order and event ranges everywhere
    key = r["event"].astype(np.int64) * 2**40 + r["module"].astype(np.int64) * 2**20 + r["first"]
    assert (np.diff(key) > 0).all() and n == r["charge"].shape[0]
    assert 0.8 * 16 * 20000 < n < 16 * 20000


def test_capacity_and_empty(ctx):
    import torch
    g, digis, calib = golden_inputs()
    n, r = _gpu(ctx, digis, calib, capacity=2)
    assert n == 4 and rows_of(r) == expected_rows(g, "gap1")[:2]
    empty = dict(module=np.zeros(0, np.int32), strip=np.zeros(0, np.int32), adc=np.zeros(0, np.uint16),
                 event_offsets=np.zeros(4, np.int32))
    n, r = _gpu(ctx, empty, calib)
    assert n == 0
    torch.cuda.synchronize()


def test_bad_arguments(ctx):
    from paper_2002_06295_amd import kfx
    g, digis, calib = golden_inputs()
    for p in (dict(seed_thr=float("nan")), dict(chan_thr=-1.0), dict(max_gap=65), dict(max_gap=-1)):
        with pytest.raises(kfx.KfxError):
            _gpu(ctx, digis, calib, **p)
    with pytest.raises(kfx.KfxError):
        _gpu(ctx, digis, dict(calib, n_modules=0))


def test_repeat_calls_shrinking(ctx):
    det = kfsynth.strip_detector(500, 256, seed=5)
    big = kfsynth.strip_events(det, 6, particles_per_event=1000, noise_frac=0.02, seed=5)
    small = kfsynth.strip_events(det, 1, particles_per_event=50, noise_frac=0.02, seed=6)
    for ev in (big, small, big):
        n, r = _gpu(ctx, ev, det)
        o = O.cluster_strips(ev, det)
        for k in o:
            np.testing.assert_array_equal(r[k], o[k], err_msg=k)


def test_digis_outside_the_events_are_ignored(ctx):
    """Digis before the first event's offset or after the last one's end
    are not clustered, even when the context's workspace still holds the
    codes of an earlier call over the same digis (they were cluster strips
    there); a moved boundary between two events moves digis between them."""
    det = kfsynth.strip_detector(400, 256, seed=8)
    ev = kfsynth.strip_events(det, 4, particles_per_event=800, noise_frac=0.03, seed=8)
    off = np.asarray(ev["event_offsets"]).copy()
    n, r = _gpu(ctx, ev, det)                      # fills the workspace
    cut = dict(ev)
    # event 0 starts late, event 3 ends early, and the boundary between
    # events 1 and 2 moves
    o2 = off.copy()
    o2[0] = off[0] + 50
    o2[2] = off[2] - 300
    o2[4] = off[4] - 120
    cut["event_offsets"] = o2
    print("strips outside events", o2.tolist(), flush=True)
    n2, r2 = _gpu(ctx, cut, det)
    o = O.cluster_strips(cut, det)
    assert n2 == o["charge"].shape[0]
    for k in o:
        np.testing.assert_array_equal(r2[k], o[k], err_msg=k)


@pytest.mark.parametrize("thr", [5.1, 4.3, 6.7])
def test_non_dyadic_quadrature_threshold(ctx, thr):
    """clus_thr crosses the boundary as a float64 and is squared in float64
    on both sides, so thresholds that float32 cannot hold give the same
    clusters as the oracle."""
    det = kfsynth.strip_detector(300, 256, seed=9)
    ev = kfsynth.strip_events(det, 3, particles_per_event=600, noise_frac=0.03, seed=9)
    n, r = _gpu(ctx, ev, det, clus_thr=thr)
    o = O.cluster_strips(ev, det, params=dict(clus_thr=thr))
    assert n == o["charge"].shape[0]
    for k in o:
        np.testing.assert_array_equal(r[k], o[k], err_msg=k)
