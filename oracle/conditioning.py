"""Conditioning of building candidates (test and benchmark infrastructure,
part of the oracle).

The gain-form Kalman update C+ = C- - K H C- cancels: a variance that one
update reduces by a factor kappa comes out of the subtraction with the
relative rounding of its inputs multiplied by kappa.  A covariance kept in
FP32 (relative rounding 2^-24) between steps, as the GPU building keeps it,
therefore carries about 2^-24 kappa of relative error after such an update,
and the later gains and states inherit it.  These helpers compute kappa for
a building candidate from the oracle's own FP64 steps.
"""
from __future__ import annotations

import numpy as np

from . import navigate, predict, seed_states, update

BARREL = 0

# Conditioning above which an FP32 covariance cannot hold the parameters to
# 1e-4: 2^-24 kappa = 1e-4.
KAPPA_1E4 = 1e-4 * 2.0 ** 24


def _surface_T(p, kind):
    """5x6 map from (x, y, z, k, phi, theta) to the surface parameters
    (u, v, k, phi, theta): u along r phi, v along z (barrel) or r (disk)."""
    r = np.hypot(p[0], p[1])
    c, s = p[0] / r, p[1] / r
    T = np.zeros((5, 6))
    T[0, 0], T[0, 1] = -s, c
    if kind == BARREL:
        T[1, 2] = 1.0
    else:
        T[1, 0], T[1, 1] = c, s
    T[2, 3] = T[3, 4] = T[4, 5] = 1.0
    return T
def update_conditioning(geometry, bz, p, C, layer, p_upd, C_upd):
    """Variance reduction of one Kalman update on the five surface
    parameters (u, v, k, phi, theta): max_j C-_jj / C+_jj.  The gain-form
    update C+ = C- - K H C- cancels to that ratio, so a covariance stored
    with relative rounding e (2^-24 in FP32) comes out of it with a relative
    error of about e times the ratio."""
    T = _surface_T(p, geometry.kind[layer])
    a = np.einsum("ij,jk,ik->i", T, C, T)
    b = np.einsum("ij,jk,ik->i", T, C_upd, T)
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        return float(np.max(a / np.maximum(b, 1e-300)))


def candidate_conditioning(ev, seed_hits, entries, prior):
    """Largest update_conditioning along a building candidate, replayed
    with the oracle from its seed through its list of entries after the
    three seed hits (hit index, or -1 for a hole): navigate, predict,
    update where there is a hit.  A hit on the layer of the hit just before
    it (a recovered overlap hit) is a second update on that surface, with
    no navigation."""
    g = ev.geometry
    p, C, _, ok = seed_states(ev, seeds=np.asarray(seed_hits, np.int32)[None], prior=prior)
    if not ok[0]:
        return float("nan")
    p, C = p[0], C[0]
    cur = int(ev.layer[seed_hits[2]])
    kappa = 1.0
    last_hit_layer = -1
    for e in entries:
        if e >= 0 and int(ev.layer[e]) == last_hit_layer:
            m = np.array([ev.x[e], ev.y[e], ev.z[e]], np.float64)
            p2, C2, _ = update(g, cur, p, C, m)
            kappa = max(kappa, update_conditioning(g, ev.bz, p, C, cur, p2, C2))
            p, C = p2, C2
            last_hit_layer = -1
            continue
        nxt = navigate(g, ev.bz, cur, p)
        if nxt < 0:
            break
        p, C = predict(g, ev.bz, nxt, p, C)
        if p is None:
            return float("nan")
        if e >= 0:
            m = np.array([ev.x[e], ev.y[e], ev.z[e]], np.float64)
            p2, C2, _ = update(g, nxt, p, C, m)
            kappa = max(kappa, update_conditioning(g, ev.bz, p, C, nxt, p2, C2))
            p, C = p2, C2
        last_hit_layer = nxt if e >= 0 else -1
        cur = nxt
    return kappa

