"""CPU check of the GPU library's adjoint logic: the reverse sweep of
kfx_adjoint.h, compiled for the host (tests/hostsim), against the FP64
oracle's own reverse-mode gradient of the fit chi2.  The same comparison
runs on the GPU in test_gpu_grad.py."""
import ctypes
import os
import shutil

import numpy as np
import pytest

import kfsynth
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def hs():
    if not (shutil.which("hipcc") or os.path.exists("/opt/rocm/bin/hipcc")):
        pytest.skip("hipcc not available")
    import importlib.util
    spec = importlib.util.spec_from_file_location("hs_build", os.path.join(HERE, "hostsim", "build.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    lib = ctypes.CDLL(mod.build())
    lib.hs_fit_grad.restype = ctypes.c_double
    return lib


def P(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def host_grad(hs, ev, align=None, fscale=1.0, w=None):
    tab = np.ascontiguousarray(ev.geometry.as_records(), dtype=np.float64)
    nl = tab.shape[0]
    pr = np.array(oracle.DEFAULT_PRIOR, np.float32)
    g = np.zeros(3 * nl + 1)
    al = None if align is None else np.ascontiguousarray(align, np.float32).reshape(-1)
    wt = None if w is None else np.ascontiguousarray(w, np.float64)
    tot = hs.hs_fit_grad(P(tab), nl, ctypes.c_double(ev.bz), P(ev.x), P(ev.y), P(ev.z), P(ev.layer), ev.n_hits,
                         P(ev.trk_offsets), P(ev.trk_hits), ev.n_tracks, P(pr), None if al is None else P(al),
                         ctypes.c_float(fscale), None if wt is None else P(wt), P(g))
    return tot, g


def mixed_err(g, ref):
    return np.abs(g - ref) / np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())


@pytest.mark.parametrize("name,kw", [("align200k", dict(tracks_per_event=300)),
                                     ("build5k", dict(tracks_per_event=300, noise_per_event=0))])
def test_host_adjoint_matches_oracle(hs, name, kw):
    ev = kfsynth.generate(kfsynth.workload(name, **kw))
    tot, g = host_grad(hs, ev)
    tot_o, go = oracle.fit_grad(ev, mode="reverse")
    assert abs(tot - tot_o) <= 1e-6 * tot_o
    assert mixed_err(g, go).max() <= 1e-4


def test_host_adjoint_at_true_alignment(hs):
    ev = kfsynth.generate("align200k", tracks_per_event=200, seed_offset=2)
    al = ev.align_true.astype(np.float32)
    _, g = host_grad(hs, ev, align=al, fscale=float(np.float32(1.002)))
    _, go = oracle.fit_grad(ev, align=al.astype(np.float64), fscale=float(np.float32(1.002)), mode="reverse")
    assert mixed_err(g, go).max() <= 1e-4


def test_host_adjoint_planted_mistake_is_caught(hs):
    # the comparison is sharp enough to see a small error in the reference:
    # the oracle's gradient with a 1e-3 change in the field scale no longer
    # matches at the tolerance used above
    ev = kfsynth.generate("align200k", tracks_per_event=200)
    _, g = host_grad(hs, ev)
    _, go = oracle.fit_grad(ev, fscale=1.001, mode="reverse")
    assert mixed_err(g, go).max() > 1e-4
