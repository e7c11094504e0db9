"""Seeded synthetic silicon-strip data: a module table with per-strip noise
and bad strips, and zero-suppressed digis of signal and noise (input
generator shared by the oracle and the GPU path; no clustering arithmetic).

Defaults follow the scale of a CMS-like strip tracker: 15,000 modules of 768
strips (11.5M strips), noise of 2.5-5 ADC counts, 1 % bad strips (some in
short runs); per event 20,000 particle crossings, each depositing a
Landau-like charge (a gamma distribution, mean ~ 120 ADC) over 1-4 strips,
and noise digis on ~1 % of the strips (Gaussian tail above 2 sigma).  ADCs
are clipped to 10 bits.
"""
from __future__ import annotations

import numpy as np


def strip_detector(n_modules=15000, strips_per_module=768, bad_frac=0.01, seed=0):
    """Calibration table: noise (float32) and bad flags (uint8) per strip."""
    rng = np.random.default_rng([21, seed])
    n = n_modules * strips_per_module
    base = rng.uniform(2.5, 5.0, n_modules).astype(np.float32)
    noise = np.repeat(base, strips_per_module) + rng.normal(0.0, 0.3, n).astype(np.float32)
    noise = np.maximum(noise, 1.0).astype(np.float32)
    bad = (rng.random(n) < bad_frac * 0.7).astype(np.uint8)
    # a few short runs of bad strips (2-3 in a row)
    starts = rng.integers(0, n - 3, int(n * bad_frac * 0.1))
    for k in range(3):
        bad[np.minimum(starts + k, n - 1)] = 1
    return dict(noise=noise, bad=bad, n_modules=n_modules, strips_per_module=strips_per_module)


def _event(rng, det, n_particles, noise_frac):
    M, P = det["n_modules"], det["strips_per_module"]
    n = M * P
    # particle crossings: centre strip, width 1-4, gamma charge
    mod = rng.integers(0, M, n_particles)
    width = rng.choice([1, 2, 3, 4], n_particles, p=[0.15, 0.45, 0.3, 0.1])
    first = rng.integers(0, P, n_particles) - (width - 1) // 2
    charge = rng.gamma(4.0, 30.0, n_particles)
    idx, val = [], []
    for w in (1, 2, 3, 4):
        sel = np.nonzero(width == w)[0]
        if sel.size == 0:
            continue
        share = rng.dirichlet(np.full(w, 3.0), sel.size)
        for j in range(w):
            s = first[sel] + j
            ok = (s >= 0) & (s < P)
            idx.append((mod[sel] * P + s)[ok])
            val.append((charge[sel] * share[:, j])[ok])
    sidx = np.concatenate(idx) if idx else np.zeros(0, np.int64)
    sval = np.concatenate(val) if val else np.zeros(0)
    # noise digis: strips whose noise fluctuation passed zero suppression
    k = rng.binomial(n, noise_frac)
    nidx = rng.choice(n, k, replace=False)
    tail = 2.0 + rng.exponential(0.45, k)
    nval = det["noise"][nidx] * tail
    allidx = np.concatenate([sidx, nidx])
    allval = np.concatenate([sval, nval])
    # strips hit by a signal also carry their noise
    allval[:sidx.size] += rng.normal(0.0, 1.0, sidx.size) * det["noise"][sidx]
    order = np.argsort(allidx, kind="stable")
    allidx, allval = allidx[order], allval[order]
    uniq, start = np.unique(allidx, return_index=True)
    summed = np.add.reduceat(allval, start) if allval.size else allval
    adc = np.clip(np.rint(summed), 0, 1023).astype(np.uint16)
    keep = adc > 0
    uniq, adc = uniq[keep], adc[keep]
    return (uniq // P).astype(np.int32), (uniq % P).astype(np.int32), adc


def strip_events(det, n_events, particles_per_event=20000, noise_frac=0.01, seed=0):
    """Digis of n_events events, sorted by (event, module, strip): dict of
    module, strip (int32), adc (uint16) and event_offsets (int32 [E+1])."""
    rng = np.random.default_rng([22, seed])
    ms, ss, aa, off = [], [], [], [0]
    for _ in range(n_events):
        m, s, a = _event(rng, det, particles_per_event, noise_frac)
        ms.append(m)
        ss.append(s)
        aa.append(a)
        off.append(off[-1] + m.shape[0])
    cat = lambda x, dt: np.concatenate(x).astype(dt) if x else np.zeros(0, dt)
    return dict(module=cat(ms, np.int32), strip=cat(ss, np.int32), adc=cat(aa, np.uint16),
                event_offsets=np.asarray(off, np.int32))
