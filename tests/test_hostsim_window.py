"""CPU check of the search window's superset property (the device's
window_bins, compiled for the host by tests/hostsim): for predictions on
barrel and disk layers -- narrow and very wide covariances, at the phi
wrap, near the layers' eta edges -- every point on the chi2 = cut ellipsoid
of the measurement frame lies in a bin inside the window, the bin taken as
the binning computes it for a hit (FP64, from FP32 coordinates).  A window
that missed such a bin would lose compatible hits; the compatible lists do
not depend on the window only if it is a superset."""
import ctypes
import os
import shutil

import numpy as np
import pytest

import kfsynth

HERE = os.path.dirname(os.path.abspath(__file__))
N_ETA, N_PHI = 20, 128


@pytest.fixture(scope="module")
def hs():
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    import importlib.util
    spec = importlib.util.spec_from_file_location("hs_build", os.path.join(HERE, "hostsim", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    lib = ctypes.CDLL(mod.build())
    vp, ci, cf = ctypes.c_void_p, ctypes.c_int, ctypes.c_float
    lib.hs_window.argtypes = [vp, ci, ci, vp, vp, cf, vp]
    lib.hs_hit_bin.argtypes = [vp, ci, ci, cf, cf, cf]
    lib.hs_hit_bin.restype = ci
    lib.hs_frame.argtypes = [vp, ci, ci, vp, vp, vp, vp]
    return lib


def P(a):
    return a.ctypes.data


def random_cov(rng, scale):
    # SPD position block of the given size (cm), small angles and curvature
    a = rng.normal(size=(6, 6)) * 0.3 + np.eye(6)
    d = np.array([scale, scale, scale, 1e-3, 1e-3 + 0.1 * scale, 1e-3 + 0.05 * scale])
    c = (a * d[:, None]) @ (a * d[:, None]).T
    return np.array([c[i, j] for i in range(6) for j in range(i + 1)], dtype=np.float32)


def check_case(hs, tab, layer, p, cov, cut, rng, n_dir=1500):
    w = np.zeros(4, np.int32)
    hs.hs_window(P(tab), tab.shape[0], layer, P(p), P(cov), ctypes.c_float(cut), P(w))
    eb0, eb1, pb0, npb = (int(v) for v in w)
    if npb == 0:
        return 0  # an empty window (non-finite input) has no points to check
    h = np.zeros(9)
    si = np.zeros(6)
    hs.hs_frame(P(tab), tab.shape[0], layer, P(p), P(cov), P(h), P(si))
    H = h.reshape(3, 3)
    S_inv = np.array([[si[0], si[1], si[3]], [si[1], si[2], si[4]], [si[3], si[4], si[5]]])
    d = rng.normal(size=(n_dir, 3))
    q = np.einsum("ni,ij,nj->n", d, S_inv, d)
    r = d * np.sqrt(cut / q)[:, None] * (1.0 - 1e-6)
    m = p[:3][None, :] + r @ H  # global point = x + H^T r
    bad = 0
    for x, y, z in m.astype(np.float32):
        b = hs.hs_hit_bin(P(tab), tab.shape[0], layer, float(x), float(y), float(z))
        eta, phi = b // N_PHI, b % N_PHI
        in_eta = eb0 <= eta <= eb1
        in_phi = (phi - pb0) % N_PHI < npb
        bad += not (in_eta and in_phi)
    return bad


def test_window_holds_the_chi2_ellipsoid(hs):
    ev = kfsynth.generate(kfsynth.workload("build5k", noise_per_event=0), tracks_per_event=10)
    tab = np.ascontiguousarray(ev.geometry.as_records(), dtype=np.float64)
    rng = np.random.default_rng(31)
    cut = 30.0
    checked = bad = 0
    for case in range(240):
        layer = int(rng.integers(0, tab.shape[0]))
        kind, pos, lo, hi = tab[layer, :4]
        if case % 6 == 0:
            phi = np.pi - rng.uniform(0, 0.02)  # at the phi wrap
        else:
            phi = rng.uniform(-np.pi, np.pi)
        if kind == 0:  # barrel: on the cylinder, z anywhere, near the edges too
            z = rng.uniform(lo, hi) if case % 5 else (hi - rng.uniform(0, 1.0)) * rng.choice([-1, 1])
            x, y = pos * np.cos(phi), pos * np.sin(phi)
        else:  # disk: on the plane, r anywhere in its band
            rr = rng.uniform(lo, hi) if case % 5 else lo + rng.uniform(0, 0.5)
            x, y, z = rr * np.cos(phi), rr * np.sin(phi), pos
        p = np.array([x, y, z, rng.choice([-1, 1]) / rng.uniform(0.5, 20), rng.uniform(-np.pi, np.pi),
                      rng.uniform(0.1, np.pi - 0.1)])
        scale = 10 ** rng.uniform(-3.5, 0.5)  # 3 um .. 3 cm in position
        cov = random_cov(rng, scale)
        bad += check_case(hs, tab, layer, p, cov, cut, rng)
        checked += 1
    assert checked == 240
    assert bad == 0, f"{bad} points of the chi2 ellipsoids fall outside their windows"


def test_device_binning_of_non_finite_hits(hs):
    """The device binning (host build) gives a hit with a NaN or infinite
    coordinate no bin, as the oracle does, on barrel and disk layers; finite
    hits agree with the oracle."""
    import oracle
    ev = kfsynth.generate("build5k", tracks_per_event=20)
    tab = np.ascontiguousarray(ev.geometry.as_records(), dtype=np.float64)
    nan, inf = float("nan"), float("inf")
    pts = [(nan, 1.0, 1.0), (1.0, nan, 1.0), (1.0, 1.0, nan), (inf, 1.0, 1.0), (1.0, -inf, 1.0),
           (1.0, 1.0, inf), (30.0, 4.0, 50.0), (-20.0, 50.0, 270.0)]
    for layer in (5, 20):
        for x, y, z in pts:
            b = hs.hs_hit_bin(P(tab), tab.shape[0], layer, x, y, z)
            bo = oracle.bin_hits(ev.geometry, N_ETA, N_PHI, np.array([x], np.float32), np.array([y], np.float32),
                                 np.array([z], np.float32), np.array([layer], np.int32))[0]
            assert b == bo, (layer, x, y, z, b, bo)
            assert (b == -1) == (not np.isfinite([x, y, z]).all())


def test_fast_binning_equals_fp64_binning(hs):
    """The binning kernel takes the bin from FP32 estimates of eta and phi
    when they lie clearly inside a bin and falls back to the FP64 formula
    otherwise: on every layer, for random points on and beyond the layer
    and for points a few float32 ulps around every eta and phi bin edge, the
    result equals the FP64 binning (itself equal to the oracle's)."""
    ev = kfsynth.generate("build5k", tracks_per_event=20)
    g = ev.geometry
    tab = np.ascontiguousarray(g.as_records(), dtype=np.float64)
    rng = np.random.default_rng(3)
    vp, ci = ctypes.c_void_p, ctypes.c_int
    hs.hs_hit_bin_fast_many.argtypes = [vp, ci, ci, vp, vp, vp, ci, vp, vp]
    hs.hs_hit_bin_fast_many.restype = None
    total = 0
    for layer in range(g.n_layers):
        kind, pos, lo, hi = tab[layer, :4]
        n = 4000
        phi = rng.uniform(-np.pi, np.pi, n)
        if kind == 0:
            r = np.full(n, pos)
            z = rng.uniform(1.3 * lo, 1.3 * hi, n)
            elo, ehi = np.arcsinh(lo / pos), np.arcsinh(hi / pos)
        else:
            r = rng.uniform(0.7 * lo, 1.3 * hi, n)
            z = np.full(n, pos)
            a, b = np.arcsinh(pos / hi), np.arcsinh(pos / lo)
            elo, ehi = min(a, b), max(a, b)
        pts = [np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)]
        # edges: every eta edge at random phi, every phi edge at random eta
        ee = elo + (ehi - elo) * np.arange(N_ETA + 1) / N_ETA
        pe = -np.pi + 2 * np.pi * np.arange(N_PHI + 1) / N_PHI
        for m in (-3, -1, 0, 1, 3):
            f = 1.0 + m * 2.0 ** -23
            ph = rng.uniform(-np.pi, np.pi, ee.size)
            if kind == 0:
                zz = pos * np.sinh(ee) * f
                pts.append(np.stack([pos * np.cos(ph), pos * np.sin(ph), zz], axis=1))
            else:
                rr = pos / np.sinh(ee) * f
                pts.append(np.stack([rr * np.cos(ph), rr * np.sin(ph), np.full(ee.size, pos)], axis=1))
            et = rng.uniform(elo, ehi, pe.size)
            pp = pe * f
            if kind == 0:
                pts.append(np.stack([pos * np.cos(pp), pos * np.sin(pp), pos * np.sinh(et)], axis=1))
            else:
                rr = pos / np.sinh(et)
                pts.append(np.stack([rr * np.cos(pp), rr * np.sin(pp), np.full(pe.size, pos)], axis=1))
        p = np.concatenate(pts).astype(np.float32)
        x, y, z = (np.ascontiguousarray(p[:, i]) for i in range(3))
        fast = np.zeros(len(p), np.int32)
        exact = np.zeros(len(p), np.int32)
        hs.hs_hit_bin_fast_many(P(tab), tab.shape[0], layer, P(x), P(y), P(z), len(p), P(fast), P(exact))
        bad = np.nonzero(fast != exact)[0]
        assert bad.size == 0, (layer, p[bad[:5]], fast[bad[:5]], exact[bad[:5]])
        total += len(p)
    assert total > 100000
