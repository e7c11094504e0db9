"""FP64 CPU oracle (test infrastructure only).

Only tests/, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It wraps the plain C++ reference in kfo.cpp through
ctypes (building, fit, adjoint); duplicates.py (duplicate removal, hit
masking) and strips.py (strip clustering) are plain Python;
conditioning.py computes the variance reduction of building candidates'
Kalman updates from the oracle's own steps (the parity bound of FP32
covariances).  It shares no code with the GPU library.

Covariances are exchanged as full row-major 6x6 float64 blocks.  Geometry is
the float64 layer table [L, 8] = (kind, pos, lo, hi, x0, su, sv, sn).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "kfo.cpp"), os.path.join(_HERE, "kfo_ad.h")]
_LIB = os.path.join(_HERE, "libkfo.so")
_lib = None

DEFAULT_PRIOR = (0.1, 0.5, 0.05, 0.05)   # sigma_pos [cm], sigma_k/|k|, sigma_phi, sigma_theta


def compile_lib(force: bool = False) -> str:
    """Compile the oracle with g++ (plain host code, -O2, FP64)."""
    newest = max(os.path.getmtime(s) for s in _SRC)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", tmp,
               os.path.join(_HERE, "kfo.cpp")]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    """The oracle library.  KFO_LIB names a prebuilt one to load instead
    (the tests' sanitizer build); otherwise libkfo.so is (re)built."""
    global _lib
    if _lib is None:
        path = os.environ.get("KFO_LIB")
        if not path:
            compile_lib()
            path = _LIB
        _lib = ctypes.CDLL(path)
        _lib.kfo_step_compat.restype = ctypes.c_long
        _lib.kfo_fit_grad.restype = ctypes.c_double
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _D(x):
    return ctypes.c_double(float(x))


def layer_table(geometry) -> np.ndarray:
    return _f64(geometry.as_records())


def bin_hits(geometry, n_eta, n_phi, x, y, z, layer):
    L = layer_table(geometry)
    x, y, z, layer = _f32(x), _f32(y), _f32(z), _i32(layer)
    out = np.empty(x.shape[0], dtype=np.int32)
    lib().kfo_bin_hits(_p(L), L.shape[0], int(n_eta), int(n_phi), _p(x), _p(y), _p(z),
                       _p(layer), x.shape[0], _p(out))
    return out


def helix(bz, p0, s, fscale=1.0):
    p0 = _f64(p0)
    out = np.empty(6)
    lib().kfo_helix(_D(bz), _p(p0), _D(s), _D(fscale), _p(out))
    return out


def path_to_cylinder(bz, p0, R, fscale=1.0):
    p0 = _f64(p0)
    s = ctypes.c_double(0.0)
    ok = lib().kfo_path_to_cylinder(_D(bz), _p(p0), _D(R), _D(fscale), ctypes.byref(s))
    return s.value if ok else None


def propagate(geometry, bz, layer, p0, fscale=1.0, dr=0.0):
    L = layer_table(geometry)
    p0 = _f64(p0)
    p1 = np.empty(6)
    J = np.empty((6, 6))
    ok = lib().kfo_propagate(_p(L), L.shape[0], _D(bz), int(layer), _p(p0), _D(fscale),
                             _D(dr), _p(p1), _p(J))
    return (p1, J) if ok else (None, None)


def material_noise(geometry, layer, p):
    L = layer_table(geometry)
    p = _f64(p)
    Q = np.empty((6, 6))
    lib().kfo_material_noise(_p(L), L.shape[0], int(layer), _p(p), _p(Q))
    return Q


def predict(geometry, bz, layer, p0, C0, fscale=1.0, dr=0.0):
    L = layer_table(geometry)
    p0, C0 = _f64(p0), _f64(C0)
    p1 = np.empty(6)
    C1 = np.empty((6, 6))
    ok = lib().kfo_predict(_p(L), L.shape[0], _D(bz), int(layer), _p(p0), _p(C0),
                           _D(fscale), _D(dr), _p(p1), _p(C1))
    return (p1, C1) if ok else (None, None)


def update(geometry, layer, p, C, m):
    L = layer_table(geometry)
    p, C, m = _f64(p).copy(), _f64(C).copy(), _f64(m)
    c2 = ctypes.c_double(0.0)
    ok = lib().kfo_update(_p(L), L.shape[0], int(layer), _p(p), _p(C), _p(m), ctypes.byref(c2))
    return (p, C, c2.value) if ok else (None, None, None)


def navigate(geometry, bz, cur, p, fscale=1.0):
    L = layer_table(geometry)
    p = _f64(p)
    return int(lib().kfo_navigate(_p(L), L.shape[0], _D(bz), int(cur), _p(p), _D(fscale)))


def seed_estimate(geometry, bz, m1, m2, m3):
    L = layer_table(geometry)
    out = np.empty(6)
    lib().kfo_seed_estimate(_p(L), L.shape[0], _D(bz), _p(_f64(m1)), _p(_f64(m2)),
                            _p(_f64(m3)), _p(out))
    return out


def seed_states(ev, seeds=None, prior=DEFAULT_PRIOR):
    """KF over the three seed hits from the prior: state at hit 3."""
    L = layer_table(ev.geometry)
    seeds = _i32(ev.seeds if seeds is None else seeds)
    ns = seeds.shape[0]
    p = np.zeros((ns, 6))
    C = np.zeros((ns, 6, 6))
    c2 = np.zeros(ns)
    ok = np.zeros(ns, dtype=np.int32)
    pr = _f64(prior)
    x, y, z, lay = _f32(ev.x), _f32(ev.y), _f32(ev.z), _i32(ev.layer)
    lib().kfo_seed_states(_p(L), L.shape[0], _D(ev.bz), _p(x), _p(y), _p(z), _p(lay),
                          x.shape[0], _p(seeds), ns, _p(pr), _p(p), _p(C), _p(c2), _p(ok))
    return p, C, c2, ok.astype(bool)


def step_compat(ev, event, cur_layer, p_in, C_in, chi2_cut=30.0, brute=False,
                n_eta=20, n_phi=128, max_pairs=None):
    """One building step on identical inputs: navigate, predict, list
    compatible hits.  Returns (next_layer, p1, C1, pair_off, pair_hit,
    pair_chi2)."""
    L = layer_table(ev.geometry)
    cur = _i32(cur_layer)
    n = cur.shape[0]
    p_in = _f64(p_in).reshape(n, 6)
    C_in = _f64(C_in).reshape(n, 6, 6)
    b, e = int(ev.event_offsets[event]), int(ev.event_offsets[event + 1])
    if max_pairs is None:
        max_pairs = max(1024, 64 * n)
    nxt = np.zeros(n, dtype=np.int32)
    p1 = np.zeros((n, 6))
    C1 = np.zeros((n, 6, 6))
    off = np.zeros(n + 1, dtype=np.int32)
    ph = np.zeros(max_pairs, dtype=np.int32)
    pc = np.zeros(max_pairs)
    x, y, z, lay = _f32(ev.x), _f32(ev.y), _f32(ev.z), _i32(ev.layer)
    cnt = lib().kfo_step_compat(_p(L), L.shape[0], _D(ev.bz), int(n_eta), int(n_phi),
                                _p(x), _p(y), _p(z), _p(lay), b, e, n, _p(cur), _p(p_in),
                                _p(C_in), _D(chi2_cut), int(bool(brute)), _p(nxt), _p(p1),
                                _p(C1), _p(off), _p(ph), _p(pc), ctypes.c_long(max_pairs))
    if cnt < 0:
        raise RuntimeError("pair buffer too small")
    return nxt, p1, C1, off, ph[:cnt].copy(), pc[:cnt].copy()


def build_tracks(ev, seeds=None, seed_event=None, chi2_cut=None, max_cands=None,
          max_holes=None, brute=False, prior=DEFAULT_PRIOR, max_hits=64, overlap=False, score=None):
    """Beam-search track building.  Returns a dict of arrays per seed x K.
    overlap: recover a second hit on the layer of every kept hit child.
    score: None (rank by hits, holes, chi2) or (w_hit, w_hole, w_chi2):
    rank by w_hit n_hits - w_hole n_holes - w_chi2 chi2, highest first."""
    w = ev.workload
    chi2_cut = w.chi2_cut if chi2_cut is None else chi2_cut
    K = w.max_cands if max_cands is None else max_cands
    max_holes = w.max_holes if max_holes is None else max_holes
    seeds = _i32(ev.seeds if seeds is None else seeds)
    ns = seeds.shape[0]
    if seed_event is None:
        seed_event = ev.trk_event if ns == ev.n_tracks else np.zeros(ns, np.int32)
    seed_event = _i32(seed_event)
    L = layer_table(ev.geometry)
    x, y, z, lay = _f32(ev.x), _f32(ev.y), _f32(ev.z), _i32(ev.layer)
    off = _i32(ev.event_offsets)
    out = dict(
        n=np.zeros(ns, np.int32), hits=np.zeros((ns, K, max_hits), np.int32),
        nhits=np.zeros((ns, K), np.int32), nholes=np.zeros((ns, K), np.int32),
        chi2=np.zeros((ns, K)), p=np.zeros((ns, K, 6)), C=np.zeros((ns, K, 6, 6)),
        stats=np.zeros(3, np.int64))
    pr = _f64(prior)
    sw = None if score is None else _f64(score)
    lib().kfo_build(_p(L), L.shape[0], _D(ev.bz), int(w.n_eta_bins), int(w.n_phi_bins),
                    _p(x), _p(y), _p(z), _p(lay), _p(off), int(off.shape[0] - 1), _p(seeds),
                    _p(seed_event), ns, _D(chi2_cut), int(K), int(max_holes), int(bool(brute)),
                    int(bool(overlap)), None if sw is None else _p(sw), _p(pr), int(max_hits), _p(out["n"]), _p(out["hits"]), _p(out["nhits"]),
                    _p(out["nholes"]), _p(out["chi2"]), _p(out["p"]), _p(out["C"]),
                    _p(out["stats"]))
    return out


def fit(ev, trk_offsets=None, trk_hits=None, align=None, fscale=1.0, prior=DEFAULT_PRIOR):
    """Forward Kalman fit over fixed hit lists.  Returns p, C, chi2, ndof, ok."""
    L = layer_table(ev.geometry)
    toff = _i32(ev.trk_offsets if trk_offsets is None else trk_offsets)
    th = _i32(ev.trk_hits if trk_hits is None else trk_hits)
    nt = toff.shape[0] - 1
    p = np.zeros((nt, 6))
    C = np.zeros((nt, 6, 6))
    c2 = np.zeros(nt)
    nd = np.zeros(nt, np.int32)
    ok = np.zeros(nt, np.int32)
    al = None if align is None else _f64(align).reshape(-1)
    x, y, z, lay = _f32(ev.x), _f32(ev.y), _f32(ev.z), _i32(ev.layer)
    pr = _f64(prior)
    lib().kfo_fit(_p(L), L.shape[0], _D(ev.bz), _p(x), _p(y), _p(z), _p(lay), _p(toff),
                  _p(th), nt, None if al is None else _p(al), _D(fscale), _p(pr), _p(p),
                  _p(C), _p(c2), _p(nd), _p(ok))
    return p, C, c2, nd, ok.astype(bool)


def fit_grad(ev, trk_offsets=None, trk_hits=None, align=None, fscale=1.0, mode="reverse",
             prior=DEFAULT_PRIOR):
    """d(total chi2)/d(alignment[3 L], field scale).  mode: 'forward' (dual
    numbers) or 'reverse' (tape).  Returns (total_chi2, grad[3 L + 1])."""
    L = layer_table(ev.geometry)
    toff = _i32(ev.trk_offsets if trk_offsets is None else trk_offsets)
    th = _i32(ev.trk_hits if trk_hits is None else trk_hits)
    nt = toff.shape[0] - 1
    g = np.zeros(3 * L.shape[0] + 1)
    al = None if align is None else _f64(align).reshape(-1)
    x, y, z, lay = _f32(ev.x), _f32(ev.y), _f32(ev.z), _i32(ev.layer)
    pr = _f64(prior)
    tot = lib().kfo_fit_grad(_p(L), L.shape[0], _D(ev.bz), _p(x), _p(y), _p(z), _p(lay),
                             _p(toff), _p(th), nt, None if al is None else _p(al), _D(fscale),
                             _p(pr), 0 if mode == "forward" else 1, _p(g))
    return tot, g


from .conditioning import KAPPA_1E4, candidate_conditioning, update_conditioning  # noqa: E402,F401
