"""The seeded input generators of the steps after building (kfsynth): the
layouts and invariants both sides rely on.  They hold no arithmetic of the
method; these checks only guard the inputs."""
import numpy as np

import kfsynth


def test_strip_events_layout_and_determinism():
    det = kfsynth.strip_detector(300, 128, seed=3)
    a = kfsynth.strip_events(det, 3, particles_per_event=200, noise_frac=0.02, seed=4)
    b = kfsynth.strip_events(det, 3, particles_per_event=200, noise_frac=0.02, seed=4)
    for k in a:
        np.testing.assert_array_equal(a[k], b[k])
    off = a["event_offsets"]
    assert off[0] == 0 and off[-1] == a["module"].shape[0] and (np.diff(off) > 0).all()
    for e in range(off.shape[0] - 1):
        m, s = a["module"][off[e]:off[e + 1]], a["strip"][off[e]:off[e + 1]]
        key = m.astype(np.int64) * 128 + s
        assert (np.diff(key) > 0).all()          # sorted, one digi per strip
    assert (a["adc"] > 0).all() and (a["adc"] <= 1023).all()
    assert ((a["module"] >= 0) & (a["module"] < 300) & (a["strip"] >= 0) & (a["strip"] < 128)).all()
    assert det["noise"].dtype == np.float32 and (det["noise"] >= 1.0).all()
    assert 0.005 < det["bad"].mean() < 0.03


def test_duplicate_seeds():
    ev = kfsynth.generate("build5k", tracks_per_event=300)
    seeds, sev, strk = kfsynth.duplicate_seeds(ev, 0.5, seed=1)
    T = ev.n_tracks
    np.testing.assert_array_equal(seeds[:T], ev.seeds)
    extra = np.arange(T, seeds.shape[0])
    assert 0.3 * T < extra.size < 0.7 * T
    for k in extra[:50]:
        t = strk[k]
        h = ev.trk_hits[ev.trk_offsets[t]:ev.trk_offsets[t + 1]]
        np.testing.assert_array_equal(seeds[k], h[[0, 1, 3]])
        assert sev[k] == ev.trk_event[t]


def test_track_lists_layout():
    t = kfsynth.track_lists(500, 6, 48, 2000, seed=2)
    assert t["hits"].shape == (3000, 48) and t["n_cands"].shape == (500,)
    assert t["chi2"].dtype == np.float32 and np.isfinite(t["chi2"]).all()
    slot0 = t["hits"][::6]
    # slot 0 counts match its list; padding -3 after the entries
    assert (t["n_holes"][::6] == (slot0 == -1).sum(axis=1)).all()
    assert (t["n_hits"][::6] == (slot0 >= 0).sum(axis=1)).all()
    assert (t["n_cands"] == 0).any() and (t["n_cands"] <= 6).all()
