"""Duplicate removal after building, and the hit masking between
iterations, written out plainly (test infrastructure only, like the rest of
this package).

The paper (abstract; Sec. 3) states that the building used to produce too
many duplicate tracks and that these are now removed in a separate step
after building, without giving the criterion.  The reading implemented
here:

* every seed with at least one candidate contributes one track, its best
  candidate (slot 0 of the building output);
* the hits of a track are the distinct entries of its hit list that are
  valid hit indices (0 <= h < n_hits_total); holes (-1) and padding are not
  hits;
* tracks a and b share s(a, b) = |hits(a) & hits(b)| hits;  b is a duplicate
  of a when s(a, b) >= 1, frac_den * s(a, b) >= frac_num * min(|hits(a)|,
  |hits(b)|), and a ranks above b;
* the rank is the building's order of candidates: more hits (the n_hits
  count), then fewer holes, then smaller total chi2 (compared as float32),
  then the smaller seed index;
* the judgement is pairwise (a track flagged as a duplicate still flags the
  tracks below it);  dup_of[b] is the highest-ranked track of which b is a
  duplicate, -1 for a kept track, -2 for a seed without a candidate.

Every decision is integer or a float32 comparison, so the GPU result must
match this one exactly.
"""
from __future__ import annotations

import numpy as np

NO_TRACK = -2
KEPT = -1


def track_hit_sets(n_cands, hits, K, n_hits_total):
    """Hit set of the best candidate of each seed (None for a seed without
    candidates).  hits: int32 [S*K, H] (row s*K is slot 0 of seed s)."""
    n_cands = np.asarray(n_cands)
    hits = np.asarray(hits)
    S = n_cands.shape[0]
    sets = []
    for s in range(S):
        if n_cands[s] <= 0:
            sets.append(None)
            continue
        row = hits[s * K]
        sets.append({int(h) for h in row if 0 <= int(h) < n_hits_total})
    return sets


def ranks_above(a, b, n_hits, n_holes, chi2):
    """True when the track of seed a ranks above the track of seed b
    (arrays indexed by seed)."""
    if n_hits[a] != n_hits[b]:
        return n_hits[a] > n_hits[b]
    if n_holes[a] != n_holes[b]:
        return n_holes[a] < n_holes[b]
    if chi2[a] != chi2[b]:
        return chi2[a] < chi2[b]
    return a < b


def find_duplicates(n_cands, hits, n_hits, n_holes, chi2, K, n_hits_total,
                    frac_num=1, frac_den=2, only=None):
    """dup_of[S] (int32) per the reading in the module docstring.

    n_hits, n_holes, chi2: per candidate entry [S*K] (entry s*K is the best
    candidate of seed s); chi2 is taken as float32 and must be finite.
    only: optional seeds to judge (the others are returned as -3), for
    spot checks of large inputs."""
    if not (0 < frac_num <= frac_den):
        raise ValueError("need 0 < frac_num <= frac_den")
    n_cands = np.asarray(n_cands)
    S = n_cands.shape[0]
    nh = np.asarray(n_hits)[::K][:S].astype(np.int64)
    ho = np.asarray(n_holes)[::K][:S].astype(np.int64)
    c2 = np.asarray(chi2, dtype=np.float32)[::K][:S]
    if not np.all(np.isfinite(c2[n_cands > 0])):
        raise ValueError("chi2 of a best candidate is not finite")
    sets = track_hit_sets(n_cands, hits, K, n_hits_total)

    # which tracks hold each hit: only pairs sharing a hit can be duplicates
    holders = {}
    for s, hs in enumerate(sets):
        if hs:
            for h in hs:
                holders.setdefault(h, []).append(s)

    dup_of = np.full(S, KEPT, dtype=np.int32)
    judge = range(S)
    if only is not None:
        dup_of[:] = -3
        judge = [int(b) for b in only]
    for b in judge:
        if sets[b] is None:
            dup_of[b] = NO_TRACK
            continue
        partners = set()
        for h in sets[b]:
            partners.update(holders[h])
        partners.discard(b)
        best = KEPT
        for a in sorted(partners):
            if not ranks_above(a, b, nh, ho, c2):
                continue
            shared = len(sets[a] & sets[b])
            shorter = min(len(sets[a]), len(sets[b]))
            if shared >= 1 and frac_den * shared >= frac_num * shorter:
                if best == KEPT or ranks_above(a, best, nh, ho, c2):
                    best = a
        dup_of[b] = best
    return dup_of


def mask_hits(n_cands, hits, n_hits, chi2, K, layer, dup_of=None, min_hits=8,
              max_chi2_ndof=3.0):
    """Hits of high-quality tracks masked for the next iteration (Sec. 3:
    later iterations run on the hits that the tracks of good quality found
    by earlier ones did not use).  Reading: a track (slot 0 of a seed with
    candidates) is good when it is kept by duplicate removal (dup_of == -1;
    every track when dup_of is None), has n_hits >= min_hits and chi2 <=
    max_chi2_ndof * (2 n_hits - 5), the product formed in float32.  Returns
    a copy of `layer` (int32 [n_hits_total]) with -1 at every valid hit of
    a good track."""
    n_cands = np.asarray(n_cands)
    hits = np.asarray(hits)
    out = np.array(layer, dtype=np.int32, copy=True)
    NH = out.shape[0]
    S = n_cands.shape[0]
    for s in range(S):
        if n_cands[s] <= 0:
            continue
        if dup_of is not None and int(dup_of[s]) != KEPT:
            continue
        nh = int(n_hits[s * K])
        if nh < min_hits:
            continue
        cut = np.float32(max_chi2_ndof) * np.float32(2 * nh - 5)
        if not (np.float32(chi2[s * K]) <= cut):
            continue
        for h in hits[s * K]:
            if 0 <= int(h) < NH:
                out[int(h)] = -1
    return out
