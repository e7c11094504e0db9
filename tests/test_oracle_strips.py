"""Pins of the strip-clustering oracle (Sec. 4: seed, cluster and
quadrature-sum thresholds and a gap rule tied to bad strips; the reading is
stated in oracle/strips.py).

Pinned by: a case worked out by hand (tests/golden/strips_small.json) at
three gap limits and with a minimum charge; properties any correct result
has (kept clusters hold a seed and pass the quadrature cut when recomputed
from the digis, clusters of one module never overlap, raising a threshold
never adds a cluster, events are independent, no digis give no clusters);
and the physics of the synthetic data (nearly every isolated particle
deposit yields one kept cluster, pure noise almost none).
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import kfsynth
from oracle import strips as O

HERE = os.path.dirname(os.path.abspath(__file__))


def golden_inputs():
    with open(os.path.join(HERE, "golden", "strips_small.json")) as f:
        g = json.load(f)
    M, P = g["n_modules"], g["strips_per_module"]
    noise = np.full(M * P, g["noise"], np.float32)
    bad = np.zeros(M * P, np.uint8)
    for m, s in g["bad"]:
        bad[m * P + s] = 1
    rows = [r for ev in g["events"] for r in ev]
    off = np.cumsum([0] + [len(ev) for ev in g["events"]]).astype(np.int32)
    digis = dict(module=np.array([r[0] for r in rows], np.int32), strip=np.array([r[1] for r in rows], np.int32),
                 adc=np.array([r[2] for r in rows], np.uint16), event_offsets=off)
    calib = dict(noise=noise, bad=bad, n_modules=M, strips_per_module=P)
    return g, digis, calib


GOLDEN_PARAMS = {"gap0": dict(max_gap=0), "gap1": dict(max_gap=1), "gap2": dict(max_gap=2),
                 "gap1_min_charge31": dict(max_gap=1, min_charge=31)}


def expected_rows(g, key):
    out = []
    for e, m, f, s, c, b in g["expected"][key]:
        out.append((e, m, f, s, c, float(np.float32(float(Fraction(b))))))
    return out


def rows_of(r):
    return list(zip(r["event"].tolist(), r["module"].tolist(), r["first"].tolist(), r["size"].tolist(),
                    r["charge"].tolist(), r["barycenter"].tolist()))


@pytest.mark.parametrize("key", sorted(GOLDEN_PARAMS))
def test_golden_hand_worked(key):
    g, digis, calib = golden_inputs()
    assert rows_of(O.cluster_strips(digis, calib, GOLDEN_PARAMS[key])) == expected_rows(g, key)


@pytest.fixture(scope="module")
def small():
    det = kfsynth.strip_detector(300, 128, bad_frac=0.03, seed=1)
    ev = kfsynth.strip_events(det, 3, particles_per_event=500, noise_frac=0.03, seed=1)
    return det, ev


def test_kept_clusters_recomputed_from_digis(small):
    det, ev = small
    r = O.cluster_strips(ev, det)
    assert r["charge"].shape[0] > 500
    P = det["strips_per_module"]
    off = ev["event_offsets"]
    for k in range(0, r["charge"].shape[0], 7):
        e, m, f, s = int(r["event"][k]), int(r["module"][k]), int(r["first"][k]), int(r["size"][k])
        a, b = off[e], off[e + 1]
        sel = (ev["module"][a:b] == m) & (ev["strip"][a:b] >= f) & (ev["strip"][a:b] < f + s)
        st, adc = ev["strip"][a:b][sel], ev["adc"][a:b][sel].astype(np.int64)
        nz = det["noise"][m * P + st].astype(np.float64)
        good = (det["bad"][m * P + st] == 0) & (adc > 2.0 * nz)
        # every strip of the span is a cluster strip or bad; charge and cuts
        assert good.sum() >= 1 and adc[good].sum() == r["charge"][k]
        assert (adc[good] > 3.0 * nz[good]).any()
        assert np.sqrt((adc[good] ** 2).sum()) > 5.0 * np.sqrt((nz[good] ** 2).sum())
        span = np.arange(f, f + s)
        assert all(det["bad"][m * P + t] or t in set(st[good].tolist()) for t in span)
        assert abs(r["barycenter"][k] - (st[good] * adc[good]).sum() / adc[good].sum()) < 1e-4


def test_clusters_do_not_overlap(small):
    det, ev = small
    r = O.cluster_strips(ev, det, dict(max_gap=3))
    key = r["event"].astype(np.int64) * 10**7 + r["module"].astype(np.int64) * 10**3
    for k in range(1, key.shape[0]):
        if key[k] == key[k - 1]:
            assert r["first"][k] > r["first"][k - 1] + r["size"][k - 1] - 1


@pytest.mark.parametrize("name,lo,hi", [("seed_thr", 3.0, 6.5), ("clus_thr", 5.0, 8.0), ("min_charge", 0, 80)])
def test_higher_threshold_never_adds(small, name, lo, hi):
    # (the 5-sigma quadrature cut implies a strip above 5 sigma when the
    # noise is uniform, so the seed threshold matters above 5)
    det, ev = small
    a = set(rows_of(O.cluster_strips(ev, det, {name: lo})))
    b = set(rows_of(O.cluster_strips(ev, det, {name: hi})))
    assert b <= a and len(b) < len(a)


def test_events_are_independent(small):
    det, ev = small
    r = O.cluster_strips(ev, det)
    off = ev["event_offsets"]
    for e in range(off.shape[0] - 1):
        one = {k: v[off[e]:off[e + 1]] for k, v in ev.items() if k != "event_offsets"}
        one["event_offsets"] = np.array([0, off[e + 1] - off[e]], np.int32)
        re = O.cluster_strips(one, det)
        sel = r["event"] == e
        assert rows_of(re) == [(0,) + t[1:] for t in rows_of({k: v[sel] for k, v in r.items()})]


def test_no_digis():
    det = kfsynth.strip_detector(10, 16, seed=0)
    ev = dict(module=np.zeros(0, np.int32), strip=np.zeros(0, np.int32), adc=np.zeros(0, np.uint16),
              event_offsets=np.zeros(3, np.int32))
    assert O.cluster_strips(ev, det)["charge"].shape[0] == 0


def test_physics_of_the_synthetic_data():
    det = kfsynth.strip_detector(2000, 768, seed=2)
    sig = kfsynth.strip_events(det, 1, particles_per_event=400, noise_frac=0.0, seed=2)
    noi = kfsynth.strip_events(det, 1, particles_per_event=0, noise_frac=0.01, seed=3)
    r_sig = O.cluster_strips(sig, det)
    r_noi = O.cluster_strips(noi, det)
    # sparse deposits: about one kept cluster each (a few fall on bad strips
    # or below threshold, a few pairs overlap)
    assert 0.85 * 400 < r_sig["charge"].shape[0] <= 400
    # ~15k noise digis over 1.5M strips: a handful of fakes at most
    assert r_noi["charge"].shape[0] < 0.01 * noi["module"].shape[0]
