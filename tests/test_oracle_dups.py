"""Pins of the duplicate-removal and hit-masking oracle (abstract and
Sec. 3: duplicates left by building are removed in a step of their own, and
the hits of good tracks are masked before the next iteration; the criteria
are the readings in oracle/duplicates.py).

Pinned by: a small case worked out by hand (tests/golden), an independent
brute force (incidence-matrix product for the shared counts, lexsort for the
rank), properties that any correct result has (monotone in the fraction,
containment at fraction 1, relabelling), and the physics of the synthetic
events (a second seed of the same particle is flagged, the original kept).
The masking is pinned by a hand-worked case on the same fixture and by
monotonicity, idempotence and the set of masked hits.
"""
import json
import os

import numpy as np
import pytest

import kfsynth
from oracle import duplicates as D

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    with open(os.path.join(HERE, "golden", "duplicates_small.json")) as f:
        return json.load(f)


@pytest.mark.parametrize("frac", ["1/2", "1/1", "1/100"])
def test_golden_hand_worked(frac):
    d = _golden()
    num, den = map(int, frac.split("/"))
    got = D.find_duplicates(np.array(d["n_cands"]), np.array(d["hits"]), np.array(d["n_hits"]),
                            np.array(d["n_holes"]), np.array(d["chi2"]), d["K"], d["n_hits_total"],
                            num, den)
    assert got.tolist() == d["expected"][frac]


def _brute(t, K, NH, num, den):
    """Shared counts from the product of the track x hit incidence matrix
    with its transpose; rank positions from a lexsort."""
    nc = t["n_cands"]
    S = nc.shape[0]
    M = np.zeros((S, max(NH, 1)), dtype=np.int64)
    for s in range(S):
        if nc[s] > 0:
            r = t["hits"][s * K]
            r = r[(r >= 0) & (r < NH)]
            M[s, r] = 1
    shared = M @ M.T
    n = M.sum(axis=1)
    nh = t["n_hits"][::K][:S]
    ho = t["n_holes"][::K][:S]
    c2 = t["chi2"][::K][:S].astype(np.float32)
    order = np.lexsort((np.arange(S), c2, ho, -nh.astype(np.int64)))
    pos = np.empty(S, np.int64)
    pos[order] = np.arange(S)
    shorter = np.minimum(n[:, None], n[None, :])
    q = (shared >= 1) & (den * shared >= num * shorter) & (pos[:, None] < pos[None, :])
    has = nc > 0
    q &= has[:, None] & has[None, :]
    np.fill_diagonal(q, False)
    out = np.full(S, -1, np.int32)
    for b in range(S):
        a = np.nonzero(q[:, b])[0]
        if a.size:
            out[b] = a[np.argmin(pos[a])]
    out[~has] = -2
    return out


CASES = [(1, 6, 50, 1, 2, 0), (40, 6, 200, 1, 2, 1), (300, 10, 3000, 1, 3, 2), (500, 1, 40, 2, 3, 3),
         (800, 6, 5000, 1, 1, 4), (600, 16, 400, 1, 100, 5)]


@pytest.mark.parametrize("S,K,NH,num,den,seed", CASES)
def test_against_brute_force(S, K, NH, num, den, seed):
    t = kfsynth.track_lists(S, K, 48, NH, seed=seed, chi2_levels=2 + seed % 4)
    got = D.find_duplicates(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], K, NH, num, den)
    np.testing.assert_array_equal(got, _brute(t, K, NH, num, den))


def test_disjoint_tracks_are_all_kept():
    S, K, H = 50, 3, 12
    hits = np.full((S * K, H), -3, np.int32)
    for s in range(S):
        hits[s * K, :10] = np.arange(10 * s, 10 * s + 10)
    z = np.zeros(S * K, np.int32)
    got = D.find_duplicates(np.ones(S, np.int32), hits, z + 10, z, np.zeros(S * K, np.float32), K, 10 * S)
    assert (got == -1).all()


def test_identical_tracks_point_to_the_best():
    S, K, H = 7, 1, 6
    hits = np.tile(np.arange(6, dtype=np.int32), (S, 1))
    chi2 = np.array([5, 4, 9, 1, 1, 7, 3], np.float32)
    z = np.zeros(S, np.int32)
    got = D.find_duplicates(np.ones(S, np.int32), hits, z + 6, z, chi2, K, 6)
    # best: smallest chi2, then the lower index (seed 3 before seed 4)
    assert got.tolist() == [3, 3, 3, -1, 3, 3, 3]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_monotone_in_fraction(seed):
    t = kfsynth.track_lists(400, 6, 48, 800, seed=seed)
    flagged = [D.find_duplicates(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], 6, 800, n, d) >= 0
               for n, d in [(1, 100), (1, 3), (1, 2), (2, 3), (1, 1)]]
    for lo, hi in zip(flagged[:-1], flagged[1:]):
        assert not (hi & ~lo).any()
    assert flagged[0].sum() > flagged[-1].sum()


def test_fraction_one_means_containment():
    NH, K = 300, 4
    t = kfsynth.track_lists(300, K, 48, NH, seed=9, p_swap=0.02)
    got = D.find_duplicates(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], K, NH, 1, 1)
    sets = D.track_hit_sets(t["n_cands"], t["hits"], K, NH)
    assert (got >= 0).sum() > 10
    for b in np.nonzero(got >= 0)[0]:
        a = got[b]
        assert sets[b] <= sets[a] or sets[a] <= sets[b]


def test_relabelling():
    S, K, NH = 200, 2, 600
    t = kfsynth.track_lists(S, K, 48, NH, seed=4)
    # distinct chi2 so that the seed index never decides
    t["chi2"] = np.random.default_rng(0).permutation(S * K).astype(np.float32)
    got = D.find_duplicates(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], K, NH)
    perm = np.random.default_rng(1).permutation(S)
    rows = (perm[:, None] * K + np.arange(K)[None, :]).ravel()
    t2 = dict(n_cands=t["n_cands"][perm], hits=t["hits"][rows], n_hits=t["n_hits"][rows],
              n_holes=t["n_holes"][rows], chi2=t["chi2"][rows])
    got2 = D.find_duplicates(t2["n_cands"], t2["hits"], t2["n_hits"], t2["n_holes"], t2["chi2"], K, NH)
    inv = np.empty(S, np.int64)
    inv[perm] = np.arange(S)
    mapped = np.where(got[perm] >= 0, inv[np.maximum(got[perm], 0)], got[perm])
    np.testing.assert_array_equal(got2, mapped)


def test_rejects_bad_fraction():
    z = np.zeros(1, np.int32)
    with pytest.raises(ValueError):
        D.find_duplicates(z + 1, np.zeros((1, 3), np.int32), z, z, np.zeros(1, np.float32), 1, 3, 3, 2)


@pytest.mark.slow
def test_second_seed_of_a_particle_is_flagged():
    """Building from two seeds of one particle gives two tracks through the
    same hits: the later one (fewer hits: it skips the particle's third
    hit) is flagged as a duplicate of the original."""
    import oracle
    ev = kfsynth.generate("build5k", tracks_per_event=150)
    seeds, seed_event, seed_track = kfsynth.duplicate_seeds(ev, 0.5, seed=0)
    T = ev.n_tracks
    o = oracle.build_tracks(ev, seeds=seeds, seed_event=seed_event, max_hits=48)
    K = o["hits"].shape[1]
    S = seeds.shape[0]
    got = D.find_duplicates(o["n"], o["hits"].reshape(S * K, -1), o["nhits"].ravel(), o["nholes"].ravel(),
                            o["chi2"].ravel().astype(np.float32), K, ev.n_hits)
    extra = np.arange(T, S)
    assert extra.size > 30
    flagged_to_own = np.mean(got[extra] == seed_track[extra])
    kept_orig = np.mean(got[:T][np.isin(np.arange(T), seed_track[extra])] == -1)
    assert flagged_to_own > 0.8, flagged_to_own
    assert kept_orig > 0.8, kept_orig
    # tracks of particles seeded once are rarely flagged
    once = ~np.isin(np.arange(T), seed_track[extra])
    assert np.mean(got[:T][once] >= 0) < 0.1


# ------------------------------------------------------------ hit masking
# Sec. 3: the hits of good tracks are masked before the next iteration.

def _golden_mask_inputs():
    d = _golden()
    t = {k: np.array(d[k]) for k in ("n_cands", "hits", "n_hits", "n_holes", "chi2")}
    dup = np.array(d["expected"]["1/2"], np.int32)
    layer = (np.arange(d["n_hits_total"]) % 7).astype(np.int32)
    return d, t, dup, layer


@pytest.mark.parametrize("cut", ["3.0", "1.0"])
def test_mask_golden_hand_worked(cut):
    d, t, dup, layer = _golden_mask_inputs()
    out = D.mask_hits(t["n_cands"], t["hits"], t["n_hits"], t["chi2"], d["K"], layer, dup,
                      d["mask"]["min_hits"], float(cut))
    masked = np.nonzero(out == -1)[0].tolist()
    assert masked == d["mask"]["expected_masked"][cut]
    keep = out != -1
    np.testing.assert_array_equal(out[keep], layer[keep])


def test_mask_properties():
    NH, K = 2000, 6
    t = kfsynth.track_lists(500, K, 48, NH, seed=3, chi2_levels=8)
    layer = np.random.default_rng(0).integers(0, 35, NH).astype(np.int32)
    dup = D.find_duplicates(t["n_cands"], t["hits"], t["n_hits"], t["n_holes"], t["chi2"], K, NH)
    m = lambda **kw: D.mask_hits(t["n_cands"], t["hits"], t["n_hits"], t["chi2"], K, layer, **kw)
    a = m(dup_of=dup, min_hits=4, max_chi2_ndof=1.0)
    b = m(dup_of=dup, min_hits=4, max_chi2_ndof=2.0)
    # a looser chi2 cut masks a superset; never unmasks; masking is idempotent
    assert ((a == -1) <= (b == -1)).all() and (a == -1).sum() < (b == -1).sum()
    again = D.mask_hits(t["n_cands"], t["hits"], t["n_hits"], t["chi2"], K, a, dup, 4, 1.0)
    np.testing.assert_array_equal(again, a)
    # no duplicate list: every track counts as kept
    allk = np.where(t["n_cands"] > 0, -1, -2).astype(np.int32)
    np.testing.assert_array_equal(m(dup_of=None, min_hits=4, max_chi2_ndof=2.0),
                                  m(dup_of=allk, min_hits=4, max_chi2_ndof=2.0))
    # an unreachable hit count masks nothing
    np.testing.assert_array_equal(m(dup_of=dup, min_hits=10**6, max_chi2_ndof=1e9), layer)
    # masked hits all lie on tracks that pass the cut
    sets = D.track_hit_sets(t["n_cands"], t["hits"], K, NH)
    on_good = set()
    for s, hs in enumerate(sets):
        if hs is not None and dup[s] == -1 and t["n_hits"][s * K] >= 4 and \
                t["chi2"][s * K] <= np.float32(2.0) * np.float32(2 * t["n_hits"][s * K] - 5):
            on_good |= hs
    assert set(np.nonzero(b == -1)[0].tolist()) == on_good
