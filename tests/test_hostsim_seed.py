"""CPU check of the GPU library's seed start (kfx_math.h seed_estimate and
the FP64 Kalman filter over the three seed hits, compiled for the host by
tests/hostsim) against the FP64 oracle's seed states: with the field, with
no field (a straight line along the chord from hit 1 to hit 3, k = 0), and
for three collinear points in a field (the same straight line)."""
import ctypes
import os
import shutil

import numpy as np
import pytest

import kfsynth
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
PRIOR = oracle.DEFAULT_PRIOR


@pytest.fixture(scope="module")
def hs():
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    import importlib.util
    spec = importlib.util.spec_from_file_location("hs_build", os.path.join(HERE, "hostsim", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return ctypes.CDLL(mod.build())


def P(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def device_seeds(hs, ev, seeds):
    tab = np.ascontiguousarray(ev.geometry.as_records(), np.float64)
    pr = np.asarray(PRIOR, np.float32)
    x, y, z = (np.ascontiguousarray(a, np.float32) for a in (ev.x, ev.y, ev.z))
    lay = np.ascontiguousarray(ev.layer, np.int32)
    p = np.zeros((len(seeds), 6))
    c = np.zeros((len(seeds), 21))
    c2 = np.zeros(len(seeds))
    for i, s in enumerate(seeds):
        sh = np.ascontiguousarray(s, np.int32)
        pi, ci, c2i = np.zeros(6), np.zeros(21), np.zeros(1)
        assert hs.hs_seed_state64(P(tab), tab.shape[0], ctypes.c_double(ev.bz), P(x), P(y), P(z), P(lay), P(sh),
                                  P(pr), P(pi), P(ci), P(c2i))
        p[i], c[i], c2[i] = pi, ci, c2i[0]
    return p, c, c2


def compare(hs, ev, seeds):
    pg, cg, c2g = device_seeds(hs, ev, seeds)
    po, Co, c2o, ok = oracle.seed_states(ev, seeds=seeds, prior=PRIOR)
    assert ok.all()
    d = pg - po
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    scale = np.maximum(np.abs(po), [1, 1, 1, 1e-3, 1, 1])
    assert np.max(np.abs(d) / scale) < 1e-9
    # the chi2 of an update from the wide prior cancels to ~1e-4 of its terms
    assert np.max(np.abs(c2g - c2o)) < 1e-6
    il = np.tril_indices(6)
    Cpo = Co[:, il[0], il[1]]
    assert np.max(np.abs(cg - Cpo) / (np.abs(Cpo).max(axis=1, keepdims=True))) < 1e-6
    return pg


def test_seed_states_in_field(hs):
    ev = kfsynth.generate("build5k", tracks_per_event=300)
    compare(hs, ev, ev.seeds)


def test_seed_states_without_field(hs):
    ev = kfsynth.generate(kfsynth.workload("build5k", bz=0.0, scatter=False), tracks_per_event=300)
    p = compare(hs, ev, ev.seeds)
    assert np.all(p[:, 3] == 0.0)


def test_collinear_seed_hits_in_field(hs):
    # three hits on one straight line through the origin, on the first
    # three barrel layers: the start is that line, k = 0
    ev = kfsynth.generate("build5k", tracks_per_event=50)
    g = ev.geometry.as_records()
    bar = [i for i in range(len(g)) if g[i][0] == 0][:3]
    # directions whose (x, y) are exactly proportional in float32: along
    # the axes and the diagonals (x = +-y)
    dirs = [(1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
    cots = [-0.75, 0.0, 0.5]
    n = len(dirs) * len(cots)
    xs, ys, zs, ls = [], [], [], []
    for ux, uy in dirs:
        for cot in cots:
            for li in bar:
                R = g[li][1]
                a = R / np.sqrt(2.0) if ux and uy else R
                xs.append(ux * a)
                ys.append(uy * a)
                zs.append(R * cot)
                ls.append(li)
    ev.x = np.asarray(xs, np.float32)
    ev.y = np.asarray(ys, np.float32)
    ev.z = np.asarray(zs, np.float32)
    ev.layer = np.asarray(ls, np.int32)
    seeds = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    # keep only triples that stay exactly collinear after rounding to float32
    x, y = ev.x.astype(np.float64), ev.y.astype(np.float64)
    cr = ((x[seeds[:, 1]] - x[seeds[:, 0]]) * (y[seeds[:, 2]] - y[seeds[:, 0]])
          - (y[seeds[:, 1]] - y[seeds[:, 0]]) * (x[seeds[:, 2]] - x[seeds[:, 0]]))
    seeds = seeds[cr == 0.0]
    if len(seeds) == 0:
        pytest.skip("no exactly collinear triple after rounding")
    p = compare(hs, ev, seeds)
    assert np.all(p[:, 3] == 0.0)
