"""Pins of the oracle's alignment and field-scale reading (the differentiable
fit's geometry corrections) against the generator's hidden truth.

The generator moves each barrel layer by its true (dr, drphi, dz), records
hits in the nominal frame and uses the field 3.8 T x 1.002; it applies these
with its own arithmetic (kfsynth/events.py), independent of the oracle.  A
fit that applies the correct corrections must then see only the smearing and
scattering it models: chi2/ndof near 1 and pulls of unit width.  Without the
corrections, or with the sign of a correction reversed (what a sign mistake
in the oracle's aligned hit would compute), the fit must be clearly worse,
and the oracle's gradient at zero alignment must point away from the truth
(moving towards it lowers the chi2).

The fit's start estimate comes from the recorded, uncorrected hits (no
gradient flows through it), so this workload's curvature prior is 5 |k|
(kfsynth: fit_prior): with 0.5 |k|, offsets of 50 um at the innermost radii,
which can exceed a high-pT seed's sagitta, made the prior bias the fit
(chi2/ndof 1.11 at the true alignment, against 1.003 with the wider prior)."""
import math

import numpy as np
import pytest

import kfsynth
import oracle


@pytest.fixture(scope="module")
def ev():
    # tracks above 0.7 GeV: lower momenta cross the outer layers near their
    # turning point, where the linearised filter does not hold
    e = kfsynth.generate("align200k", tracks_per_event=3000)
    return e


def fit_stats(ev, align, fscale):
    p, C, c2, nd, ok = oracle.fit(ev, align=align, fscale=fscale, prior=ev.workload.fit_prior)
    pt = 1.0 / np.abs(ev.trk_vertex[:, 3])
    s = ok & (pt > 0.7)
    return p, C, c2, nd, s


def test_true_alignment_gives_unit_chi2_and_pulls(ev):
    p, C, c2, nd, s = fit_stats(ev, ev.align_true, 1.002)
    assert s.sum() > 2500
    assert c2[s].sum() / nd[s].sum() == pytest.approx(1.0, abs=0.03)
    last = ev.trk_offsets[1:] - 1
    tr = ev.trk_truth[last]
    d = p - tr
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    n = s.sum()
    for i in (3, 4, 5):
        pull = d[s, i] / np.sqrt(C[s, i, i])
        assert pull.std() == pytest.approx(1.0, abs=0.06)
        assert abs(pull.mean()) < 4.0 / math.sqrt(n)
    # the position along the layer (r phi) and z: the hit positions carry
    # the layer offsets, so these pulls test the corrections most directly
    r = np.hypot(p[s, 0], p[s, 1])
    u = np.stack([-p[s, 1] / r, p[s, 0] / r, np.zeros(n)], 1)
    v = np.tile([0.0, 0.0, 1.0], (n, 1))
    for ax in (u, v):
        du = np.einsum("ni,ni->n", ax, d[s, :3])
        var = np.einsum("ni,nij,nj->n", ax, C[s][:, :3, :3], ax)
        pull = du / np.sqrt(var)
        assert pull.std() == pytest.approx(1.0, abs=0.06)
        assert abs(pull.mean()) < 4.0 / math.sqrt(n)


def test_wrong_alignment_is_clearly_worse(ev):
    _, _, c2t, ndt, s = fit_stats(ev, ev.align_true, 1.002)
    best = c2t[s].sum() / ndt[s].sum()
    cases = {"none": (np.zeros_like(ev.align_true), 1.0)}
    for col, name in ((1, "drphi"), (2, "dz")):
        a = ev.align_true.copy()
        a[:, col] = -a[:, col]
        cases["reversed " + name] = (a, 1.002)
    for name, (a, fs) in cases.items():
        _, _, c2, nd, s2 = fit_stats(ev, a, fs)
        worse = c2[s2].sum() / nd[s2].sum()
        assert worse > best + 0.3, (name, worse, best)


def test_gradient_at_zero_points_away_from_truth(ev):
    sub = np.arange(0, ev.n_tracks, 3)
    toff = ev.trk_offsets
    lens = toff[sub + 1] - toff[sub]
    soff = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    shits = np.concatenate([ev.trk_hits[toff[i]:toff[i + 1]] for i in sub]).astype(np.int32)
    L = ev.geometry.n_layers
    pr = ev.workload.fit_prior
    tot0, g = oracle.fit_grad(ev, trk_offsets=soff, trk_hits=shits, align=np.zeros((L, 3)), fscale=1.0, prior=pr)
    step = np.concatenate([ev.align_true.reshape(-1), [0.002]])
    assert float(np.dot(g, step)) < 0.0
    # and the chi2 does fall along that direction
    tot1, _ = oracle.fit_grad(ev, trk_offsets=soff, trk_hits=shits, align=0.5 * ev.align_true, fscale=1.001,
                              prior=pr)
    assert tot1 < tot0
