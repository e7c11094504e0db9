"""Python binding of libkfx.so (C ABI in include/kfx.h).

Argument marshalling only: torch supplies device memory and the current
HIP stream; every step of the computation runs in the library's HIP
kernels.  Importing this module does not touch the GPU; creating a Context
loads the library and fails loudly if it is missing or no GPU is present.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkfx.so")

KFX_OK = 0
KFX_EINVAL = -1
KFX_EOVERFLOW = -2
KFX_EHIP = -3
KFX_ESTATE = -4
KFX_ENOMEM = -5
MODE_PLAIN = 0
MODE_FUSED = 1
MAX_CANDS = 16
MAX_STEPS = 40

EXPORTED = ["kfx_create", "kfx_destroy", "kfx_last_error", "kfx_load_layers", "kfx_bin_hits",
            "kfx_seed_states", "kfx_step_compat", "kfx_build_tracks", "kfx_fit_tracks",
            "kfx_fit_tracks_backward", "kfx_fit_tracks_backward_noalloc", "kfx_enable_timing", "kfx_build_times", "kfx_build_graph",
            "kfx_graph_launch", "kfx_graph_destroy", "kfx_autotune_build", "kfx_autotune_cache_clear", "kfx_find_duplicates", "kfx_mask_hits",
            "kfx_cluster_strips", "kfx_index_keys_per_event"]


class c_states(ctypes.Structure):
    _fields_ = [("par", ctypes.c_void_p), ("cov", ctypes.c_void_p), ("stride", ctypes.c_int64)]


class c_hits(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p),
                ("layer", ctypes.c_void_p), ("event_offsets", ctypes.c_void_p),
                ("n_hits", ctypes.c_int32), ("n_events", ctypes.c_int32)]


class c_prior(ctypes.Structure):
    _fields_ = [("spos", ctypes.c_float), ("sk_rel", ctypes.c_float), ("sphi", ctypes.c_float),
                ("stheta", ctypes.c_float)]


class c_build_params(ctypes.Structure):
    _fields_ = [("chi2_cut", ctypes.c_float), ("max_cands", ctypes.c_int32),
                ("max_holes", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("prior", c_prior), ("mode", ctypes.c_int32), ("block_threads", ctypes.c_int32),
                ("blocks", ctypes.c_int32), ("lanes_per_seed", ctypes.c_int32), ("scan_tile", ctypes.c_int32),
                ("waves_per_simd", ctypes.c_int32), ("seeds_per_wave", ctypes.c_int32),
                ("window_inflate", ctypes.c_float), ("overlap", ctypes.c_int32),
                ("score", ctypes.c_int32), ("score_hit", ctypes.c_float), ("score_hole", ctypes.c_float),
                ("score_chi2", ctypes.c_float), ("binning", ctypes.c_int32)]


class c_tracks(ctypes.Structure):
    _fields_ = [("n_cands", ctypes.c_void_p), ("hits", ctypes.c_void_p), ("n_hits", ctypes.c_void_p),
                ("n_holes", ctypes.c_void_p), ("chi2", ctypes.c_void_p), ("state", c_states),
                ("stats", ctypes.c_void_p), ("max_hits", ctypes.c_int32), ("capacity", ctypes.c_int64),
                ("needed", ctypes.c_int64)]


class c_digis(ctypes.Structure):
    _fields_ = [("module", ctypes.c_void_p), ("strip", ctypes.c_void_p), ("adc", ctypes.c_void_p),
                ("event_offsets", ctypes.c_void_p), ("n", ctypes.c_int32), ("n_events", ctypes.c_int32)]


class c_strip_calib(ctypes.Structure):
    _fields_ = [("noise", ctypes.c_void_p), ("bad", ctypes.c_void_p), ("n_modules", ctypes.c_int32),
                ("strips_per_module", ctypes.c_int32)]


class c_cluster_params(ctypes.Structure):
    _fields_ = [("seed_thr", ctypes.c_float), ("chan_thr", ctypes.c_float), ("clus_thr", ctypes.c_double),
                ("max_gap", ctypes.c_int32), ("min_charge", ctypes.c_int32)]


class c_clusters(ctypes.Structure):
    _fields_ = [("event", ctypes.c_void_p), ("module", ctypes.c_void_p), ("first", ctypes.c_void_p),
                ("size", ctypes.c_void_p), ("charge", ctypes.c_void_p), ("barycenter", ctypes.c_void_p),
                ("capacity", ctypes.c_int32), ("n_out", ctypes.c_void_p)]


_lib = None


def load_library():
    """Load libkfx.so (built by __graft_entry__.build()); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                           "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    lib.kfx_create.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_void_p)]
    lib.kfx_destroy.argtypes = [ctypes.c_void_p]
    lib.kfx_destroy.restype = None
    lib.kfx_last_error.argtypes = [ctypes.c_void_p]
    lib.kfx_last_error.restype = ctypes.c_char_p
    lib.kfx_load_layers.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_int, ctypes.c_int]
    lib.kfx_bin_hits.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.kfx_seed_states.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.POINTER(c_prior), ctypes.POINTER(c_states),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.kfx_step_compat.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p,
                                    ctypes.c_void_p, ctypes.POINTER(c_states), ctypes.c_int32,
                                    ctypes.c_float, ctypes.c_void_p, ctypes.POINTER(c_states),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p]
    lib.kfx_build_tracks.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(c_build_params),
                                     ctypes.POINTER(c_tracks), ctypes.c_void_p]
    lib.kfx_fit_tracks.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(c_prior),
                                   ctypes.c_void_p, ctypes.c_float, ctypes.POINTER(c_states),
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.POINTER(c_states), ctypes.c_void_p]
    lib.kfx_fit_tracks_backward.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(c_prior),
                                            ctypes.c_void_p, ctypes.c_float, ctypes.POINTER(c_states),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.kfx_fit_tracks_backward_noalloc.argtypes = lib.kfx_fit_tracks_backward.argtypes
    lib.kfx_build_graph.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.POINTER(c_build_params), ctypes.POINTER(c_tracks),
                                    ctypes.POINTER(ctypes.c_void_p)]
    lib.kfx_graph_launch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    lib.kfx_graph_destroy.argtypes = [ctypes.c_void_p]
    lib.kfx_graph_destroy.restype = None
    lib.kfx_autotune_cache_clear.argtypes = []
    lib.kfx_autotune_cache_clear.restype = None
    lib.kfx_autotune_build.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_hits), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int32, ctypes.POINTER(c_build_params), ctypes.POINTER(c_tracks),
                                       ctypes.c_int32, ctypes.POINTER(ctypes.c_float), ctypes.c_void_p]
    lib.kfx_find_duplicates.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_tracks), ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p]
    lib.kfx_mask_hits.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_tracks), ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_void_p, ctypes.c_int32, ctypes.c_float, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]
    lib.kfx_cluster_strips.argtypes = [ctypes.c_void_p, ctypes.POINTER(c_digis), ctypes.POINTER(c_strip_calib),
                                       ctypes.POINTER(c_cluster_params), ctypes.POINTER(c_clusters),
                                       ctypes.c_void_p]
    lib.kfx_enable_timing.argtypes = [ctypes.c_void_p, ctypes.c_int]
    lib.kfx_build_times.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
    for name in EXPORTED:
        if name not in ("kfx_destroy", "kfx_last_error", "kfx_graph_destroy"):
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class KfxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"kfx error {code}: {msg}")
        self.code = code


@dataclass
class States:
    """Device SoA states: par float64 [6, n] (x, y, z, k, phi, theta), cov
    float32 [21, n] (packed lower triangle)."""

    par: object
    cov: object

    @staticmethod
    def empty(n, device):
        import torch
        n = max(int(n), 1)
        return States(torch.zeros((6, n), dtype=torch.float64, device=device),
                      torch.zeros((21, n), dtype=torch.float32, device=device))

    @staticmethod
    def from_numpy(p, C, device):
        """p: [n, 6] (x, y, z, k, phi, theta); C: [n, 6, 6] or [n, 21]."""
        import torch
        p = np.asarray(p, dtype=np.float64)
        n = p.shape[0]
        C = np.asarray(C)
        if C.ndim == 3:
            C = pack_cov(C)
        return States(torch.as_tensor(np.ascontiguousarray(p.T), device=device),
                      torch.as_tensor(np.ascontiguousarray(C.T.astype(np.float32)), device=device))

    @property
    def n(self):
        return int(self.par.shape[1])

    def c(self):
        return c_states(self.par.data_ptr(), self.cov.data_ptr(), self.n)

    def to_numpy(self, n=None):
        """Returns p [n, 6] (float64) and C [n, 6, 6] (float64)."""
        par = self.par.cpu().numpy()
        cov = self.cov.cpu().numpy().astype(np.float64)
        n = par.shape[1] if n is None else n
        return par.T[:n].copy(), unpack_cov(cov.T[:n])


def pack_cov(C):
    idx = [(i, j) for i in range(6) for j in range(i + 1)]
    return np.stack([C[:, i, j] for i, j in idx], axis=1)


def unpack_cov(P):
    n = P.shape[0]
    C = np.zeros((n, 6, 6))
    q = 0
    for i in range(6):
        for j in range(i + 1):
            C[:, i, j] = P[:, q]
            C[:, j, i] = P[:, q]
            q += 1
    return C


class DeviceHits:
    """Hits resident in device memory (kept alive with the struct)."""

    def __init__(self, x, y, z, layer, event_offsets):
        self.x, self.y, self.z, self.layer, self.event_offsets = x, y, z, layer, event_offsets
        self.struct = c_hits(x.data_ptr(), y.data_ptr(), z.data_ptr(), layer.data_ptr(),
                             event_offsets.data_ptr(), int(x.shape[0]), int(event_offsets.shape[0] - 1))

    @staticmethod
    def from_events(ev, device):
        import torch
        t = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a, dtype=dt), device=device)
        return DeviceHits(t(ev.x, np.float32), t(ev.y, np.float32), t(ev.z, np.float32),
                          t(ev.layer, np.int32), t(ev.event_offsets, np.int32))

    @property
    def n_hits(self):
        return int(self.struct.n_hits)

    @property
    def n_events(self):
        return int(self.struct.n_events)


def prior_struct(prior):
    return c_prior(*[float(v) for v in prior])


class Graph:
    """A captured build (kfx_build_graph); launch() replays it on torch's
    current stream."""

    def __init__(self, ctx, handle, keep):
        self.ctx, self.h, self._keep = ctx, handle, keep

    def launch(self):
        self.ctx._check(self.ctx.lib.kfx_graph_launch(self.h, self.ctx._stream()))

    def close(self):
        if getattr(self, "h", None):
            self.ctx.lib.kfx_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """A kfx context on one HIP device."""

    def __init__(self, device=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("kfx needs a HIP GPU (torch.cuda.is_available() is False)")
        self.lib = load_library()
        h = ctypes.c_void_p()
        rc = self.lib.kfx_create(int(device), ctypes.byref(h))
        if rc != KFX_OK:
            raise KfxError(rc, f"kfx_create failed for device {device}")
        self.h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if getattr(self, "h", None):
            self.lib.kfx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != KFX_OK:
            raise KfxError(rc, self.lib.kfx_last_error(self.h).decode())

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    # ------------------------------------------------------------------
    def load_layers(self, table, bz, n_eta, n_phi):
        t = np.ascontiguousarray(table, dtype=np.float64)
        self._check(self.lib.kfx_load_layers(self.h, t.ctypes.data_as(ctypes.c_void_p), int(t.shape[0]),
                                             float(bz), int(n_eta), int(n_phi)))
        self.n_layers = int(t.shape[0])
        self.n_eta, self.n_phi = int(n_eta), int(n_phi)

    def bin_hits(self, hits: DeviceHits, want=True):
        import torch
        n_keys = hits.n_events * getattr(self, "n_layers", 0) * getattr(self, "n_eta", 0) * getattr(self, "n_phi", 0)
        d = self.device
        bins = torch.empty(max(hits.n_hits, 1), dtype=torch.int32, device=d) if want else None
        off = torch.empty(n_keys + 1, dtype=torch.int32, device=d) if want else None
        perm = torch.empty(max(hits.n_hits, 1), dtype=torch.int32, device=d) if want else None
        self._check(self.lib.kfx_bin_hits(self.h, ctypes.byref(hits.struct), _ptr(bins), _ptr(off), _ptr(perm),
                                          self._stream()))
        return bins, off, perm

    def seed_states(self, hits: DeviceHits, seeds, prior):
        import torch
        seeds = torch.as_tensor(np.ascontiguousarray(seeds, dtype=np.int32), device=self.device)
        n = int(seeds.shape[0])
        out = States.empty(n, self.device)
        chi2 = torch.zeros(max(n, 1), dtype=torch.float32, device=self.device)
        status = torch.zeros(max(n, 1), dtype=torch.int32, device=self.device)
        pr = prior_struct(prior)
        st = out.c()
        self._check(self.lib.kfx_seed_states(self.h, ctypes.byref(hits.struct), _ptr(seeds), n, ctypes.byref(pr),
                                             ctypes.byref(st), _ptr(chi2), _ptr(status), self._stream()))
        return out, chi2[:n], status[:n]

    def step_compat(self, hits: DeviceHits, cand_event, cand_layer, states: States, chi2_cut, max_pairs=64):
        import torch
        d = self.device
        ce = torch.as_tensor(np.ascontiguousarray(cand_event, dtype=np.int32), device=d)
        cl = torch.as_tensor(np.ascontiguousarray(cand_layer, dtype=np.int32), device=d)
        n = int(ce.shape[0])
        nxt = torch.zeros(max(n, 1), dtype=torch.int32, device=d)
        pred = States.empty(n, d)
        cnt = torch.zeros(max(n, 1), dtype=torch.int32, device=d)
        ph = torch.full((max(n, 1), max_pairs), -1, dtype=torch.int32, device=d)
        pc = torch.zeros((max(n, 1), max_pairs), dtype=torch.float32, device=d)
        si, sp = states.c(), pred.c()
        self._check(self.lib.kfx_step_compat(self.h, ctypes.byref(hits.struct), _ptr(ce), _ptr(cl), ctypes.byref(si),
                                             n, float(chi2_cut), _ptr(nxt), ctypes.byref(sp), _ptr(cnt), _ptr(ph),
                                             _ptr(pc), int(max_pairs), self._stream()))
        return nxt[:n], pred, cnt[:n], ph[:n], pc[:n]

    def _build_args(self, seeds, seed_event, chi2_cut=30.0, max_cands=6, max_holes=3, max_steps=32,
                    prior=(0.1, 0.5, 0.05, 0.05), mode=MODE_FUSED, block_threads=0, blocks=0, lanes_per_seed=0,
                    scan_tile=0, waves_per_simd=0, seeds_per_wave=0, max_hits=48, out=None, window_inflate=0.0,
                    overlap=False, score=None, binning=0):
        import torch
        d = self.device
        if not isinstance(seeds, torch.Tensor):
            seeds = torch.as_tensor(np.ascontiguousarray(seeds, dtype=np.int32), device=d)
        if not isinstance(seed_event, torch.Tensor):
            seed_event = torch.as_tensor(np.ascontiguousarray(seed_event, dtype=np.int32), device=d)
        S = int(seeds.shape[0])
        K = int(max_cands)
        if out is None:
            out = self.alloc_tracks(S, K, max_hits)
        p = c_build_params(float(chi2_cut), K, int(max_holes), int(max_steps), prior_struct(prior), int(mode),
                           int(block_threads), int(blocks), int(lanes_per_seed), int(scan_tile),
                           int(waves_per_simd), int(seeds_per_wave), float(window_inflate), int(bool(overlap)),
                           0 if score is None else 1, *(float(v) for v in (score or (0.0, 0.0, 0.0))),
                           int(binning))
        return seeds, seed_event, S, p, out

    def build_tracks(self, hits: DeviceHits, seeds, seed_event, **kw):
        """Returns a dict of device tensors (see kfx_tracks in kfx.h).
        Keywords: chi2_cut, max_cands, max_holes, max_steps, prior, mode,
        block_threads, blocks, lanes_per_seed, scan_tile, waves_per_simd, seeds_per_wave, max_hits,
        out, window_inflate, overlap (overlap recovery), score (None, or the weights (w_hit, w_hole,
        w_chi2) of the score ranking), binning (0 automatic, 1 global counting sort, 2 one workgroup
        per event)."""
        seeds, seed_event, S, p, out = self._build_args(seeds, seed_event, **kw)
        self._check(self.lib.kfx_build_tracks(self.h, ctypes.byref(hits.struct), _ptr(seeds), _ptr(seed_event), S,
                                              ctypes.byref(p), ctypes.byref(out["_struct"]), self._stream()))
        return out

    def build_graph(self, hits: DeviceHits, seeds, seed_event, **kw):
        """Capture one build into a HIP graph; returns (Graph, out).  The
        graph keeps references to the buffers it was captured with."""
        seeds, seed_event, S, p, out = self._build_args(seeds, seed_event, **kw)
        g = ctypes.c_void_p()
        self._check(self.lib.kfx_build_graph(self.h, ctypes.byref(hits.struct), _ptr(seeds), _ptr(seed_event), S,
                                             ctypes.byref(p), ctypes.byref(out["_struct"]), ctypes.byref(g)))
        return Graph(self, g, (hits, seeds, seed_event, out)), out

    def autotune_build(self, hits: DeviceHits, seeds, seed_event, reps=2, **kw):
        """Fastest launch shape of the fused kernel for this workload: a dict
        of block_threads, blocks, lanes_per_seed, scan_tile, waves_per_simd,
        seeds_per_wave (pass it back to build_tracks) and the time of one
        build in ms.  Cached per device and workload signature (see
        kfx_autotune_build); autotune_cache_clear() empties the cache."""
        kw = dict(kw)
        kw["mode"] = MODE_FUSED
        seeds, seed_event, S, p, out = self._build_args(seeds, seed_event, **kw)
        ms = ctypes.c_float(0.0)
        self._check(self.lib.kfx_autotune_build(self.h, ctypes.byref(hits.struct), _ptr(seeds), _ptr(seed_event), S,
                                                ctypes.byref(p), ctypes.byref(out["_struct"]), int(reps),
                                                ctypes.byref(ms), self._stream()))
        return dict(block_threads=p.block_threads, blocks=p.blocks, lanes_per_seed=p.lanes_per_seed,
                    scan_tile=p.scan_tile, waves_per_simd=p.waves_per_simd, seeds_per_wave=p.seeds_per_wave,
                    ms=float(ms.value))

    def autotune_cache_clear(self):
        self.lib.kfx_autotune_cache_clear()

    def index_keys_per_event(self):
        """Keys per event of the hit index the last bin/build call made:
        n_layers * n_bins (counting sort over the batch) or one more (one
        workgroup per event)."""
        k = ctypes.c_int64()
        self._check(self.lib.kfx_index_keys_per_event(self.h, ctypes.byref(k)))
        return int(k.value)

    def enable_timing(self, n_calls=64):
        self._check(self.lib.kfx_enable_timing(self.h, int(n_calls)))

    def build_times(self, n_calls):
        """[(binning, search kernel, building, total) in ms] of the last
        n_calls timed builds, oldest first."""
        ms = (ctypes.c_float * (4 * max(n_calls, 1)))()
        n = self.lib.kfx_build_times(self.h, ms, int(n_calls))
        if n < 0:
            self._check(n)
        return [tuple(ms[4 * i + k] for k in range(4)) for i in range(n)]

    def alloc_tracks(self, S, K, max_hits=48):
        import torch
        d = self.device
        n = max(S * K, 1)
        out = dict(n_cands=torch.zeros(max(S, 1), dtype=torch.int32, device=d),
                   hits=torch.zeros((n, max_hits), dtype=torch.int32, device=d),
                   n_hits=torch.zeros(n, dtype=torch.int32, device=d),
                   n_holes=torch.zeros(n, dtype=torch.int32, device=d),
                   chi2=torch.zeros(n, dtype=torch.float32, device=d),
                   state=States.empty(n, d),
                   stats=torch.zeros(4, dtype=torch.int64, device=d))
        out["_struct"] = c_tracks(out["n_cands"].data_ptr(), out["hits"].data_ptr(), out["n_hits"].data_ptr(),
                                  out["n_holes"].data_ptr(), out["chi2"].data_ptr(), out["state"].c(),
                                  out["stats"].data_ptr(), int(max_hits), n, 0)
        out["S"], out["K"] = S, K
        return out

    def tracks_from_arrays(self, n_cands, hits, n_hits, n_holes, chi2, K):
        """A building-output dict (as build_tracks returns) holding the given
        host arrays on the device: n_cands [S], hits [S*K, max_hits],
        n_hits, n_holes, chi2 [S*K].  The states are left unset."""
        import torch
        d = self.device
        hits = np.ascontiguousarray(hits, dtype=np.int32)
        S = int(np.asarray(n_cands).shape[0])
        out = dict(n_cands=torch.as_tensor(np.ascontiguousarray(n_cands, dtype=np.int32), device=d),
                   hits=torch.as_tensor(hits, device=d),
                   n_hits=torch.as_tensor(np.ascontiguousarray(n_hits, dtype=np.int32), device=d),
                   n_holes=torch.as_tensor(np.ascontiguousarray(n_holes, dtype=np.int32), device=d),
                   chi2=torch.as_tensor(np.ascontiguousarray(chi2, dtype=np.float32), device=d))
        out["_struct"] = c_tracks(out["n_cands"].data_ptr(), out["hits"].data_ptr(), out["n_hits"].data_ptr(),
                                  out["n_holes"].data_ptr(), out["chi2"].data_ptr(), c_states(None, None, 0),
                                  None, int(hits.shape[1]), int(hits.shape[0]), 0)
        out["S"], out["K"] = S, int(K)
        return out

    def find_duplicates(self, out, n_hits, frac=(1, 2), n_seeds=None, dup_of=None):
        """dup_of [S] (device int32) of a building output `out` (a dict from
        build_tracks or tracks_from_arrays): -2 no candidate, -1 kept, else
        the seed of the highest-ranked track it duplicates.  n_hits: hit
        count of the batch; frac = (num, den) shared-hit fraction."""
        import torch
        S = out["S"] if n_seeds is None else int(n_seeds)
        if dup_of is None:
            dup_of = torch.empty(max(S, 1), dtype=torch.int32, device=self.device)
        self._check(self.lib.kfx_find_duplicates(self.h, ctypes.byref(out["_struct"]), S, int(out["K"]),
                                                 int(n_hits), int(frac[0]), int(frac[1]), _ptr(dup_of),
                                                 self._stream()))
        return dup_of[:S]

    def mask_hits(self, out, layer, dup_of=None, min_hits=8, max_chi2_ndof=3.0, layer_out=None, n_seeds=None):
        """Layer array for the next iteration (device int32 [n_hits]): a copy
        of `layer` with -1 at the hits of the good tracks of the building
        output `out` (see kfx_mask_hits in kfx.h).  layer_out may be `layer`
        itself."""
        import torch
        S = out["S"] if n_seeds is None else int(n_seeds)
        if layer_out is None:
            layer_out = torch.empty_like(layer)
        self._check(self.lib.kfx_mask_hits(self.h, ctypes.byref(out["_struct"]), S, int(out["K"]),
                                           None if dup_of is None else _ptr(dup_of), int(min_hits),
                                           float(max_chi2_ndof), _ptr(layer), _ptr(layer_out),
                                           int(layer.numel()), self._stream()))
        return layer_out

    def strip_inputs(self, digis, calib):
        """Device copies of digis (dict: module, strip, adc, event_offsets) and
        of a calibration table (dict: noise, bad, n_modules,
        strips_per_module); tensors already on the device are kept."""
        import torch
        d = self.device

        def t(a, dt):
            if isinstance(a, torch.Tensor):
                return a
            return torch.as_tensor(np.ascontiguousarray(a, dtype=dt), device=d)
        dg = dict(module=t(digis["module"], np.int32), strip=t(digis["strip"], np.int32),
                  adc=t(np.asarray(digis["adc"]).astype(np.int16) if not isinstance(digis["adc"], torch.Tensor)
                        else digis["adc"], np.int16),
                  event_offsets=t(digis["event_offsets"], np.int32))
        cb = dict(noise=t(calib["noise"], np.float32), bad=t(calib["bad"], np.uint8),
                  n_modules=int(calib["n_modules"]), strips_per_module=int(calib["strips_per_module"]))
        return dg, cb

    def cluster_strips(self, digis, calib, seed_thr=3.0, chan_thr=2.0, clus_thr=5.0, max_gap=1, min_charge=0,
                       capacity=None, out=None):
        """Kept clusters of a batch of strip events (see kfx_cluster_strips):
        dict of device tensors event, module, first, size, charge,
        barycenter (the first n of each) and n (a device int32 [1]).  digis
        and calib as returned by strip_inputs; the adc tensor holds the
        16-bit ADCs."""
        import torch
        d = self.device
        n = int(digis["module"].numel())
        E = int(digis["event_offsets"].numel()) - 1
        if out is None:
            cap = max(n, 1) if capacity is None else int(capacity)
            out = dict(event=torch.empty(max(cap, 1), dtype=torch.int32, device=d),
                       module=torch.empty(max(cap, 1), dtype=torch.int32, device=d),
                       first=torch.empty(max(cap, 1), dtype=torch.int32, device=d),
                       size=torch.empty(max(cap, 1), dtype=torch.int32, device=d),
                       charge=torch.empty(max(cap, 1), dtype=torch.int32, device=d),
                       barycenter=torch.empty(max(cap, 1), dtype=torch.float32, device=d),
                       n=torch.zeros(1, dtype=torch.int32, device=d), capacity=cap)
        dg = c_digis(digis["module"].data_ptr(), digis["strip"].data_ptr(), digis["adc"].data_ptr(),
                     digis["event_offsets"].data_ptr(), n, E)
        cb = c_strip_calib(calib["noise"].data_ptr(), calib["bad"].data_ptr(), int(calib["n_modules"]),
                           int(calib["strips_per_module"]))
        pr = c_cluster_params(float(seed_thr), float(chan_thr), float(clus_thr), int(max_gap), int(min_charge))
        oc = c_clusters(out["event"].data_ptr(), out["module"].data_ptr(), out["first"].data_ptr(),
                        out["size"].data_ptr(), out["charge"].data_ptr(), out["barycenter"].data_ptr(),
                        int(out["capacity"]), out["n"].data_ptr())
        self._check(self.lib.kfx_cluster_strips(self.h, ctypes.byref(dg), ctypes.byref(cb), ctypes.byref(pr),
                                                ctypes.byref(oc), self._stream()))
        return out

    def fit_tracks(self, hits: DeviceHits, trk_off, trk_hits, prior=(0.1, 0.5, 0.05, 0.05), align=None,
                   field_scale=1.0, ckpt=False, out=None):
        import torch
        d = self.device
        if not isinstance(trk_off, torch.Tensor):
            trk_off = torch.as_tensor(np.ascontiguousarray(trk_off, dtype=np.int32), device=d)
        if not isinstance(trk_hits, torch.Tensor):
            trk_hits = torch.as_tensor(np.ascontiguousarray(trk_hits, dtype=np.int32), device=d)
        if align is not None and not isinstance(align, torch.Tensor):
            align = torch.as_tensor(np.ascontiguousarray(align, dtype=np.float32).reshape(-1), device=d)
        T = int(trk_off.shape[0] - 1)
        if out is None:
            out = dict(state=States.empty(T, d), chi2=torch.zeros(max(T, 1), dtype=torch.float32, device=d),
                       ndof=torch.zeros(max(T, 1), dtype=torch.int32, device=d),
                       status=torch.zeros(max(T, 1), dtype=torch.int32, device=d))
            if ckpt:
                lens = torch.diff(trk_off.to(torch.int64))
                longest = int(lens.max().item()) if T > 0 else 0
                out["ckpt"] = States.empty(max(T * longest, 1), d)
        pr = prior_struct(prior)
        so = out["state"].c()
        ck = out["ckpt"].c() if "ckpt" in out else None
        self._check(self.lib.kfx_fit_tracks(self.h, ctypes.byref(hits.struct), _ptr(trk_off), _ptr(trk_hits), T,
                                            ctypes.byref(pr), _ptr(align), float(field_scale), ctypes.byref(so),
                                            _ptr(out["chi2"]), _ptr(out["ndof"]), _ptr(out["status"]),
                                            ctypes.byref(ck) if ck is not None else None, self._stream()))
        return out

    def fit_tracks_backward(self, hits: DeviceHits, trk_off, trk_hits, fit_out, dchi2,
                            prior=(0.1, 0.5, 0.05, 0.05), align=None, field_scale=1.0, dalign=None, dfield=None,
                            no_alloc=False):
        """Gradient of sum_t dchi2[t] chi2_t (dchi2: a device float32 tensor of
        one element or of n_tracks) with respect to the alignment and the
        field scale, for the fit that wrote fit_out (made with ckpt=True and
        the same inputs).  Returns float64 device tensors (dalign [3 L],
        dfield [1]), written into the given ones if passed.  no_alloc=True
        calls kfx_fit_tracks_backward_noalloc (no device allocation in the
        library: its scratch is a fixed array per GPU)."""
        import torch
        d = self.device
        if "ckpt" not in fit_out:
            raise KfxError(KFX_EINVAL, "fit_tracks_backward needs a fit made with ckpt=True")
        if not isinstance(trk_off, torch.Tensor):
            trk_off = torch.as_tensor(np.ascontiguousarray(trk_off, dtype=np.int32), device=d)
        if not isinstance(trk_hits, torch.Tensor):
            trk_hits = torch.as_tensor(np.ascontiguousarray(trk_hits, dtype=np.int32), device=d)
        if align is not None and not isinstance(align, torch.Tensor):
            align = torch.as_tensor(np.ascontiguousarray(align, dtype=np.float32).reshape(-1), device=d)
        T = int(trk_off.shape[0] - 1)
        dchi2 = dchi2.to(device=d, dtype=torch.float32).contiguous().reshape(-1)
        per_track = 1 if dchi2.numel() > 1 else 0
        if per_track and dchi2.numel() != T:
            raise KfxError(KFX_EINVAL, f"dchi2 has {dchi2.numel()} entries for {T} tracks")
        n_layers = self.n_layers
        if dalign is None:
            dalign = torch.empty(3 * n_layers, dtype=torch.float64, device=d)
        if dfield is None:
            dfield = torch.empty(1, dtype=torch.float64, device=d)
        for t, n in ((dalign, 3 * n_layers), (dfield, 1)):
            if t.dtype != torch.float64 or t.numel() < n or not t.is_contiguous() or t.device != d:
                raise KfxError(KFX_EINVAL, "gradient outputs: contiguous float64 device tensors of 3 L and 1")
        pr = prior_struct(prior)
        ck = fit_out["ckpt"].c()
        fn = self.lib.kfx_fit_tracks_backward_noalloc if no_alloc else self.lib.kfx_fit_tracks_backward
        self._check(fn(
            self.h, ctypes.byref(hits.struct), _ptr(trk_off), _ptr(trk_hits), T, ctypes.byref(pr), _ptr(align),
            float(field_scale), ctypes.byref(ck), _ptr(fit_out["status"]), _ptr(dchi2), per_track, _ptr(dalign),
            _ptr(dfield), self._stream()))
        return dalign, dfield

    def fit_tracks_backward_noalloc(self, *args, **kw):
        """fit_tracks_backward through kfx_fit_tracks_backward_noalloc."""
        kw["no_alloc"] = True
        return self.fit_tracks_backward(*args, **kw)
