"""Strip clustering, written out plainly (test infrastructure only, like the
rest of this package).

The paper (Sec. 4, towards an HLT implementation) describes the clustering
of silicon-strip data that it ports to GPUs: seed strips above three times
their expected noise; clusters grown from a seed by the strips above twice
their noise that are consecutive or separated by a small gap whose allowed
size depends on bad strips; a cluster kept when the quadrature sum of its
ADCs exceeds five times the quadrature sum of its noise and its total
charge reaches a minimum.  The reading implemented here:

* input per event: digis (module, strip, adc) sorted by (module, strip),
  one per strip at most; calibration per (module, strip): noise (float32)
  and a bad flag; digis outside the calibration table are ignored;
* a candidate strip is not bad and has adc > chan_thr * noise; a seed strip
  is a candidate with adc > seed_thr * noise (float32 products);
* two consecutive candidates a < b of the same module and event belong to
  one cluster when b - a - 1 <= max_gap and every strip strictly between
  them is bad (max_gap = 0: adjacent strips only);
* a cluster (a maximal chain of such candidates) is kept when it holds a
  seed, sum(adc^2) > clus_thr^2 * sum(noise^2) (noise^2 summed in float64
  in strip order, clus_thr^2 formed in float64) and sum(adc) >= min_charge;
* output per kept cluster, in (event, module, first strip) order: event,
  module, first strip, size (last - first + 1, bridged strips included),
  charge sum(adc), barycenter sum(strip * adc) / sum(adc) (float64 divide,
  stored as float32).

Every decision is integer or a float32 / float64 operation taken in the
same order, so the GPU result must match this one exactly.
"""
from __future__ import annotations

import numpy as np


def cluster_event(module, strip, adc, noise, bad, n_modules, spm, seed_thr=3.0, chan_thr=2.0,
                  clus_thr=5.0, max_gap=1, min_charge=0, event=0, modules=None):
    """Clusters of one event's digis; a list of tuples (event, module,
    first, size, charge, barycenter).  modules: optional set of modules to
    process (the others are skipped), for spot checks of large inputs."""
    f32 = np.float32
    st, ct = f32(seed_thr), f32(chan_thr)
    thr2 = float(clus_thr) * float(clus_thr)
    n = len(module)
    cand = []
    for i in range(n):
        m, s = int(module[i]), int(strip[i])
        if not (0 <= m < n_modules and 0 <= s < spm):
            continue
        if modules is not None and m not in modules:
            continue
        c = m * spm + s
        if bad[c]:
            continue
        a = f32(int(adc[i]))
        if a > ct * f32(noise[c]):
            cand.append((m, s, int(adc[i]), bool(a > st * f32(noise[c])), float(noise[c])))
    out = []
    k = 0
    while k < len(cand):
        run = [cand[k]]
        while k + 1 < len(cand):
            m0, s0 = run[-1][0], run[-1][1]
            m1, s1 = cand[k + 1][0], cand[k + 1][1]
            if m1 != m0 or s1 <= s0 or s1 - s0 - 1 > max_gap:
                break
            if not all(bad[m0 * spm + t] for t in range(s0 + 1, s1)):
                break
            run.append(cand[k + 1])
            k += 1
        k += 1
        charge = sum(r[2] for r in run)
        sq = sum(r[2] * r[2] for r in run)
        nsq = 0.0
        for r in run:
            nsq += float(np.float64(r[4]) * np.float64(r[4]))
        if any(r[3] for r in run) and float(sq) > thr2 * nsq and charge >= min_charge:
            bary = np.float32(float(sum(r[1] * r[2] for r in run)) / float(charge))
            out.append((event, run[0][0], run[0][1], run[-1][1] - run[0][1] + 1, charge, bary))
    return out


def cluster_strips(digis, calib, params=None, modules=None):
    """All events: digis = dict(module, strip, adc, event_offsets); calib =
    dict(noise, bad, n_modules, strips_per_module); params = dict(seed_thr,
    chan_thr, clus_thr, max_gap, min_charge).  Returns a dict of arrays
    (event, module, first, size, charge, barycenter)."""
    p = dict(seed_thr=3.0, chan_thr=2.0, clus_thr=5.0, max_gap=1, min_charge=0)
    if params:
        p.update(params)
    off = np.asarray(digis["event_offsets"])
    rows = []
    for e in range(off.shape[0] - 1):
        a, b = int(off[e]), int(off[e + 1])
        rows += cluster_event(digis["module"][a:b], digis["strip"][a:b], digis["adc"][a:b], calib["noise"],
                              calib["bad"], calib["n_modules"], calib["strips_per_module"], event=e,
                              modules=modules, **p)
    cols = list(zip(*rows)) if rows else [[]] * 6
    return dict(event=np.array(cols[0], np.int32), module=np.array(cols[1], np.int32),
                first=np.array(cols[2], np.int32), size=np.array(cols[3], np.int32),
                charge=np.array(cols[4], np.int32), barycenter=np.array(cols[5], np.float32))
