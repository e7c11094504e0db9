"""Runs the oracle's entry points (and, with --hostsim, the host build of the
GPU library's device math) on small seeded inputs, for the sanitizer
builds of tests/test_sanitizers.py: every call path the tests use, once,
including the edge cases (non-finite hits, empty events, short tracks)."""
import ctypes
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import kfsynth  # noqa: E402
import oracle  # noqa: E402


def run_oracle():
    ev = kfsynth.generate("build5k", tracks_per_event=120)
    # a few non-finite hits and a hit without a layer
    ev.x = ev.x.copy()
    ev.layer = ev.layer.copy()
    ev.x[5] = np.nan
    ev.x[17] = np.inf
    ev.layer[23] = -1
    w = ev.workload
    oracle.bin_hits(ev.geometry, w.n_eta_bins, w.n_phi_bins, ev.x, ev.y, ev.z, ev.layer)
    p, C, c2, ok = oracle.seed_states(ev)
    o = oracle.build_tracks(ev, max_hits=48)
    oracle.build_tracks(ev, seeds=ev.seeds[:20], brute=True, max_hits=48)
    oracle.build_tracks(ev, seeds=ev.seeds[:0], max_hits=48)
    idx = np.nonzero(ok)[0][:10]
    for s in idx:
        oracle.step_compat(ev, 0, int(ev.layer[ev.seeds[s][2]]), p[s], C[s])
    evf = kfsynth.generate("fit1k", tracks_per_event=60)
    oracle.fit(evf)
    off = evf.trk_offsets.copy()
    oracle.fit(evf, trk_offsets=off[:3], trk_hits=evf.trk_hits[:off[2]])
    eva = kfsynth.generate("align200k", tracks_per_event=40)
    nl = eva.geometry.n_layers
    al = np.random.default_rng(1).normal(0, 50e-4, (nl, 3))
    oracle.fit_grad(eva, align=al, fscale=1.002, mode="reverse")
    oracle.fit_grad(eva, align=al, fscale=1.002, mode="forward")
    from oracle import duplicates as D
    from oracle import strips as OS
    t = kfsynth.track_lists(80, 6, 48, 600, seed=2)
    d = D.find_duplicates(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], 6, 600)
    D.mask_hits(t["n_cands"], t["hits"], t["n_hits"], t["chi2"], 6, np.zeros(600, np.int32), d, 4, 3.0)
    det = kfsynth.strip_detector(40, 64, seed=2)
    sev = kfsynth.strip_events(det, 2, particles_per_event=60, noise_frac=0.03, seed=2)
    OS.cluster_strips(sev, det)
    print("oracle ok", int(o["stats"][0]), flush=True)


def run_hostsim(path):
    hs = ctypes.CDLL(path)
    hs.hs_predict.restype = ctypes.c_float
    hs.hs_update.restype = ctypes.c_float
    hs.hs_pair_chi2.restype = ctypes.c_float
    hs.hs_fit_grad.restype = ctypes.c_double

    def P(a):
        return a.ctypes.data_as(ctypes.c_void_p)

    ev = kfsynth.generate("build5k", tracks_per_event=60)
    tab = np.ascontiguousarray(ev.geometry.as_records(), np.float64)
    nl = tab.shape[0]
    bz = ctypes.c_double(ev.bz)
    pr = np.asarray(oracle.DEFAULT_PRIOR, np.float32)
    x, y, z = (np.ascontiguousarray(a, np.float32) for a in (ev.x, ev.y, ev.z))
    lay = np.ascontiguousarray(ev.layer, np.int32)
    n = 0
    for s in range(ev.n_tracks):
        sh = np.ascontiguousarray(ev.seeds[s], np.int32)
        p = np.zeros(6)
        c = np.zeros(21, np.float32)
        c2 = np.zeros(1, np.float32)
        if not hs.hs_seed_state(P(tab), nl, bz, P(x), P(y), P(z), P(lay), ev.n_hits, P(sh), P(pr), P(p), P(c),
                                P(c2)):
            continue
        cur = int(lay[sh[2]])
        for _ in range(30):
            so = np.zeros(1)
            nxt = hs.hs_navigate(P(tab), nl, bz, cur, P(p), P(so))
            if nxt < 0:
                break
            p1 = np.zeros(6)
            c1 = np.zeros(21, np.float32)
            if hs.hs_predict(P(tab), nl, bz, int(nxt), P(p), P(c), P(p1), P(c1)) < 0:
                break
            w4 = np.zeros(4, np.int32)
            hs.hs_window(P(tab), nl, int(nxt), P(p1), P(c1), ctypes.c_float(30.0), P(w4))
            h3 = np.array([p1[0], p1[1], p1[2]], np.float32)
            hs.hs_pair_chi2(P(tab), nl, int(nxt), P(p1), P(c1), P(h3))
            m = h3.astype(np.float64)
            p2 = np.zeros(6)
            c2_ = np.zeros(21, np.float32)
            hs.hs_update(P(tab), nl, int(nxt), P(p1), P(c1), P(m), P(p2), P(c2_))
            p, c, cur = p2, c2_, int(nxt)
            n += 1
        hs.hs_hit_bin(P(tab), nl, cur, ctypes.c_float(float("nan")), ctypes.c_float(1.0), ctypes.c_float(1.0))
    evf = kfsynth.generate("fit1k", tracks_per_event=30)
    tf = np.ascontiguousarray(evf.geometry.as_records(), np.float64)
    nt = evf.n_tracks
    po = np.zeros(6 * nt)
    co = np.zeros(21 * nt, np.float32)
    c2 = np.zeros(nt, np.float32)
    nd = np.zeros(nt, np.int32)
    st = np.zeros(nt, np.int32)
    fx, fy, fz = (np.ascontiguousarray(a, np.float32) for a in (evf.x, evf.y, evf.z))
    fl = np.ascontiguousarray(evf.layer, np.int32)
    off = np.ascontiguousarray(evf.trk_offsets, np.int32)
    th = np.ascontiguousarray(evf.trk_hits, np.int32)
    hs.hs_fit(P(tf), tf.shape[0], ctypes.c_double(evf.bz), P(fx), P(fy), P(fz), P(fl), evf.n_hits, P(off), P(th), nt,
              P(pr), None, ctypes.c_float(1.0), P(po), P(co), P(c2), P(nd), P(st))
    print("hostsim ok", n, int(st.sum()), flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 2 and sys.argv[1] == "--hostsim":
        run_hostsim(sys.argv[2])
    else:
        run_oracle()
