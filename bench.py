#!/usr/bin/env python
"""Benchmark of Kalman-filter track building on one MI355X.

One step = one pass of the building hot path over one batch of synthetic
events already resident in HBM: hit binning (counting sort into the
(eta, phi) index), seed start states, and the search -- navigate and
propagate every candidate, scan its window for compatible hits, keep the best
K children per seed, update them -- in the fused persistent kernel, replayed
from a HIP graph.  The default workload is the batched one: 256 events of
uneven size (about 767k seeds, 16M hits) in one persistent launch.

value = candidate-layer Kalman steps per second (candidate-surface pairs
propagated, counted by the kernel), for a run whose best candidates were
checked against the FP64 oracle on seeds sampled across the batch.

Prints one JSON line.  Extra objects: roofline (the building kernel, timed
with HIP events on its own stream), cpu_baseline (the FP64 oracle on the
host's cores, and on one, over the parity sample), parity, and secondary
measurements (the plain per-step path on the same input, the single-event
workload, the high-occupancy workload, the fit and fit + adjoint, duplicate
removal, hit masking, strip clustering).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "cand-layer Kalman steps/s at 1e-4 rel tol; fit+grad tracks/s vs plain path"

# Floating-point operations per unit of work, counted from the formulas as
# the kernels implement them (FMA = 2, transcendental calls = 1):
#   per step   navigation (closed-form cylinder crossing ~25, its z check
#              and the polar angle ~5, one disk check ~25) ~55, transport and
#              covariance J C J^T + Q with the tangent-plane projection ~540,
#              measurement frame and S^-1 ~195, window ~40
#   per pair   FP64 residual + 3x3 chi2 ~35
#   per update FP64 frame, gain, state and covariance update ~500
FLOP_PER_STEP = 830.0
FLOP_PER_PAIR = 35.0
FLOP_PER_UPDATE = 500.0
# The fit (FP64 throughout): per hit the surface crossing, J C J^T + Q and
# the projection, the update ~1700; its adjoint per hit (recompute of the
# step from its checkpoint and the reverse sweep) ~6000.
FIT_FLOP_PER_HIT = 1700.0
ADJ_FLOP_PER_HIT = 6000.0
# MI355X vector peaks: FP32 157.3 TFLOP/s (the published figure, which
# counts packed FP32: 256 CUs x 2.4 GHz x 256 FLOP/clk) and FP64 78.6
# TFLOP/s (128 FLOP/clk, the same issue rate as unpacked FP32).  These
# kernels are built without packed FP32, so 78.6 is the most they can
# issue; the roofline object reports against 157.3 and gives both.
FP32_PEAK_TFLOPS = 256 * 2.4e9 * 256 / 1e12
ALU_PEAK_TFLOPS = 256 * 2.4e9 * 128 / 1e12
# FP64 part of the per-unit counts: the crossing geometry (~55 per step),
# the residual (~10 per pair) and the whole update (500)
FP64_FLOP_PER_STEP = 55.0
FP64_FLOP_PER_PAIR = 10.0

WORKLOADS = {
    "build5k": "5000 seeded tracks, 17 barrel layers (R 3-110 cm) + 2x9 disks (|z| 30-270 cm, "
               "r 20-110 cm), eta U[-2.4,2.4], pT log-U[0.5,20] GeV, 1% inefficiency, 20k noise "
               "hits, 20x128 (eta, phi) bins, chi2 < 30, K = 6",
    "batch256": "256 events, tracks Poisson(3000) clipped [200, 12000], noise = 5x tracks, "
                "geometry as build5k, 5-26 hits per track, K = 6, one persistent kernel",
    "occ10k": "4 events x (10k tracks, pT log-U[0.3,50], eta U[-2.5,2.5], 10% displaced "
              "vertices r_xy < 5 cm, 300k noise hits), K = 10",
}


def source_sha256():
    """Hash of the HIP sources (names and contents), to tell whether stored
    profiler counters still describe the kernels that run."""
    import glob
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2002_06295_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.h")) + glob.glob(os.path.join(csrc, "*.hip"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(name="k_build_fused_batch256_traffic.json"):
    """HBM bytes per launch of the fused kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (calibrated against a copy of known
    size), or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    return t["hbm_bytes_per_launch"] if t.get("source_sha256") == source_sha256() else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_flops(stats):
    return stats[0] * FLOP_PER_STEP + stats[1] * FLOP_PER_PAIR + stats[2] * FLOP_PER_UPDATE


def fp64_flops(stats):
    return stats[0] * FP64_FLOP_PER_STEP + stats[1] * FP64_FLOP_PER_PAIR + stats[2] * FLOP_PER_UPDATE


def alu_roofline(stats, kernel_ms, kernel, traffic):
    """Roofline object of a building launch: algorithmic FLOP per launch
    over the kernel's mean launch time, against the FP32 vector peak."""
    flops = algorithmic_flops(stats)
    achieved = flops / (kernel_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, calibrated)",
            "peak_issue_without_packed_fp32": ALU_PEAK_TFLOPS,
            "frac_of_issue_peak": achieved / ALU_PEAK_TFLOPS,
            "fp64_flop_share": fp64_flops(stats) / flops if flops else None,
            "kernel": kernel, "avg_launch_ms": kernel_ms, "flop_per_launch": flops,
            "steps_per_launch": stats[0], "pairs_per_launch": stats[1], "updates_per_launch": stats[2],
            "flop_formula": f"{FLOP_PER_STEP:.0f} per step + {FLOP_PER_PAIR:.0f} per compatible pair + "
                            f"{FLOP_PER_UPDATE:.0f} per Kalman update"}


def build_kw(ev, mode):
    w = ev.workload
    return dict(chi2_cut=w.chi2_cut, max_cands=w.max_cands, max_holes=w.max_holes, max_steps=32, mode=mode)


def run_build(ctx, kfx, hits, ev, steps, warmup, mode, out=None, shape=None):
    """Warm up, then time `steps` build calls; returns (wall ms per step,
    per-call times (binning, search kernel, building, total), stats of one
    call, out)."""
    import torch
    seeds = torch.as_tensor(ev.seeds, device=ctx.device)
    sev = torch.as_tensor(ev.trk_event.astype(np.int32), device=ctx.device)
    kw = build_kw(ev, mode)
    kw.update(shape or {})
    for _ in range(warmup):
        out = ctx.build_tracks(hits, seeds, sev, out=out, **kw)
    torch.cuda.synchronize()
    out["stats"].zero_()
    ctx.enable_timing(max(steps, 1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = ctx.build_tracks(hits, seeds, sev, out=out, **kw)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    times = ctx.build_times(steps)
    ctx.enable_timing(0)
    stats = out["stats"].cpu().numpy().astype(np.float64) / max(steps, 1)
    return wall, times, stats, out


def parity_sample(ev, target=2560, max_events=32, seed=0):
    """Seeds sampled across the batch: about `target` seeds, drawn evenly
    from up to `max_events` events spread over it."""
    rng = np.random.default_rng(seed)
    E = ev.n_events
    evs = np.unique(np.linspace(0, E - 1, min(E, max_events)).round().astype(int))
    per = int(np.ceil(target / len(evs)))
    idx = []
    for e in evs:
        cand = np.nonzero(ev.trk_event == e)[0]
        idx.append(np.sort(rng.choice(cand, min(per, cand.size), replace=False)))
    return np.concatenate(idx)


def gather_rows(out, rows):
    """Host copies of the sampled output rows (gathered on the device)."""
    import torch
    r = torch.as_tensor(np.asarray(rows, dtype=np.int64), device=out["hits"].device)
    return {"hits": out["hits"].index_select(0, r).cpu().numpy(),
            "chi2": out["chi2"].index_select(0, r).cpu().numpy(),
            "n_hits": out["n_hits"].index_select(0, r).cpu().numpy(),
            "n_holes": out["n_holes"].index_select(0, r).cpu().numpy(),
            "p": out["state"].par.index_select(1, r).cpu().numpy().T}


def parity_check(ev, out, idx, ores, prior):
    """Best candidates of the sampled seeds against the oracle's (the
    oracle's building run of the CPU-baseline leg, same seeds).  Bars: best
    hit lists identical for >= 98 % of the seeds, candidate counts equal for
    >= 99 %, and for every identical best candidate the parameters within
    max(1e-4, 2^-24 kappa) (floors 1 cm, 1 rad; none for k) and, where
    kappa <= 2^24 * 1e-4, the chi2 sum within 1e-3.  kappa is the
    candidate's largest variance reduction in one Kalman update, from the
    oracle's own steps: the FP32 covariance of building carries about
    2^-24 kappa of relative error after such an update (see
    oracle/conditioning.py), so candidates above 2^24 * 1e-4 cannot be held
    to 1e-4 and are reported apart."""
    import oracle
    import torch
    K = ev.workload.max_cands
    g = gather_rows(out, idx * K)
    ncg = out["n_cands"].index_select(0, torch.as_tensor(idx, device=out["n_cands"].device)).cpu().numpy()
    same = 0
    rel, kap, dchi = [], [], []
    for j, s in enumerate(idx):
        gh = g["hits"][j]
        oh = ores["hits"][j, 0, :gh.shape[0]]
        if np.array_equal(gh, oh):
            same += 1
            po = ores["p"][j, 0]
            d = g["p"][j] - po
            d[4] = (d[4] + np.pi) % (2 * np.pi) - np.pi
            rel.append(float(np.max(np.abs(d) / np.maximum(np.abs(po), [1, 1, 1, 0, 1, 1]))))
            nh = int(ores["nhits"][j, 0] + ores["nholes"][j, 0])
            k = oracle.candidate_conditioning(ev, ev.seeds[s], ores["hits"][j, 0, 3:nh], prior)
            kap.append(np.inf if np.isnan(k) else k)
            dchi.append(abs(float(g["chi2"][j]) - float(ores["chi2"][j, 0])))
    n = len(idx)
    rel, kap, dchi = np.asarray(rel), np.asarray(kap), np.asarray(dchi)
    bound = np.maximum(1e-4, 2.0 ** -24 * kap)
    ill = kap > oracle.KAPPA_1E4
    well = ~ill
    above = rel > 1e-4
    counts_equal = int(np.sum(ncg == ores["n"]))
    res = dict(seeds_checked=int(n), events_sampled=int(np.unique(ev.trk_event[idx]).size),
               best_identical=int(same), n_cands_equal=counts_equal,
               well_conditioned=int(well.sum()), ill_conditioned=int(ill.sum()),
               params_rel_max_well=float(rel[well].max()) if well.any() else 0.0,
               params_rel_p99_well=float(np.percentile(rel[well], 99)) if well.any() else 0.0,
               chi2_abs_max_well=float(dchi[well].max()) if well.any() else 0.0,
               params_rel_max_ill=float(rel[ill].max()) if ill.any() else 0.0,
               params_rel_p99_ill=float(np.percentile(rel[ill], 99)) if ill.any() else 0.0,
               above_1e_4=int(above.sum()),
               above_1e_4_kappa=[float(k) for k in np.sort(kap[above])],
               within_conditioning_bound=bool(np.all(rel <= bound)),
               criterion="best hit lists identical for >= 98% and candidate counts equal for >= 99% of "
                         "the sampled seeds; every identical best candidate within max(1e-4, 2^-24 kappa) "
                         "in the parameters; chi2 sums within 1e-3 where kappa <= 2^24 * 1e-4")
    res["passed"] = bool(same >= 0.98 * n and counts_equal >= 0.99 * n and res["within_conditioning_bound"]
                         and np.all(dchi[well] <= 1e-3))
    return res


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def _event_view(ev, e):
    """The hits of event e alone, as the oracle reads them (its hit
    indices start at 0; the event's first hit in the batch is returned)."""
    from types import SimpleNamespace
    lo, hi = int(ev.event_offsets[e]), int(ev.event_offsets[e + 1])
    return SimpleNamespace(workload=ev.workload, geometry=ev.geometry, bz=ev.bz, x=ev.x[lo:hi], y=ev.y[lo:hi],
                           z=ev.z[lo:hi], layer=ev.layer[lo:hi],
                           event_offsets=np.array([0, hi - lo], dtype=np.int32)), lo


def cpu_baseline(ev, idx, prior, min_seconds=4.0):
    """The FP64 oracle (as it is) on the host's cores, building the sampled
    seeds: one task per sampled event, given that event's hits alone (the
    oracle bins every event it is given, and seeds are independent; the
    ctypes call releases the GIL), on up to 16 threads, repeated until
    min_seconds have passed; then on one thread over the tasks for about
    min_seconds.  Returns the baseline record and the oracle's results for
    the seeds (hit indices in the batch's numbering)."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    oracle.lib()
    threads = max(1, min(16, os.cpu_count() or 1))
    te = ev.trk_event[idx]
    events = list(np.unique(te))
    tasks = [(e, np.nonzero(te == e)[0]) for e in events]  # positions in idx, in idx order per event
    views = {e: _event_view(ev, e) for e in events}

    def run(task):
        e, pos = task
        view, lo = views[e]
        seeds = (ev.seeds[idx[pos]] - lo).astype(np.int32)
        q = oracle.build_tracks(view, seeds=seeds, seed_event=np.zeros(len(pos), np.int32), max_hits=48,
                                prior=prior)
        q["hits"] = np.where(q["hits"] >= 0, q["hits"] + lo, q["hits"])
        return pos, q

    steps = 0
    reps = 0
    parts = None
    nthr = min(threads, len(tasks))
    with ThreadPoolExecutor(nthr) as ex:
        t0 = time.perf_counter()
        while reps < 1 or time.perf_counter() - t0 < min_seconds:
            parts = list(ex.map(run, tasks))
            steps += sum(int(q["stats"][0]) for _, q in parts)
            reps += 1
        dt = time.perf_counter() - t0
    n = len(idx)
    res = {}
    for k in parts[0][1]:
        if k == "stats":
            continue
        first = parts[0][1][k]
        arr = np.zeros((n,) + first.shape[1:], dtype=first.dtype)
        for pos, q in parts:
            arr[pos] = q[k]
        res[k] = arr
    res["stats"] = sum(q["stats"] for _, q in parts)
    # one thread: the tasks in turn until min_seconds
    st1, sd1, t1 = 0, 0, time.perf_counter()
    for task in tasks:
        _, q = run(task)
        st1 += int(q["stats"][0])
        sd1 += len(task[1])
        if time.perf_counter() - t1 >= min_seconds:
            break
    dt1 = time.perf_counter() - t1
    rec = dict(value=steps / dt, unit="steps/s", cores=nthr, kind="oracle",
               tracks_per_s=reps * n / dt,
               single_thread_steps_per_s=st1 / dt1, single_thread_tracks_per_s=sd1 / dt1,
               sample=f"{n} seeds sampled over {len(events)} events of the {ev.workload.name} workload, one "
                      f"task per event with that event's hits (binned by the oracle in every task), x {reps}, "
                      f"FP64 building with the binned compatibility search, {nthr} threads on "
                      f"{host_cpu_model()}, {dt:.1f} s wall; one thread: {sd1} of the seeds, {dt1:.1f} s")
    return rec, res


HBM_PEAK_GBPS = 8000.0


def hbm_roofline(bytes_per_call, ms, what):
    """Roofline object of an HBM-bound step: algorithmic bytes per call
    over the measured time per call, against the 8 TB/s HBM peak."""
    gbps = bytes_per_call / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": gbps / HBM_PEAK_GBPS, "bytes_per_call": int(bytes_per_call), "bytes": what}


def dedup_bytes(out, n_hits):
    """Algorithmic bytes of one duplicate-removal call: per track its hit
    list row read twice (sort, then judging) and its sorted list written once
    (3 x 4 max_hits B), its counts and chi2 read (16 B), its key written
    and read (32 B) and its result written (4 B); per (track, hit) entry the
    exchange on the hit's head (8 B), the next link written and read (8 B)
    and the head read again (4 B); the heads cleared (4 B per hit)."""
    S, K = int(out["S"]), int(out["K"])
    h = out["hits"].reshape(-1, out["hits"].shape[-1])[::K][:S]
    has = (out["n_cands"][:S] > 0).reshape(-1, 1)
    entries = int((((h >= 0) & (h < n_hits)) & has).sum().item())
    H = int(h.shape[1])
    return S * (12 * H + 16 + 32 + 4) + entries * 20 + 4 * n_hits


def time_dedup(ctx, out, n_hits, reps=20):
    """Mean time (ms, torch events on the call's stream) of duplicate
    removal over a building output, and its result."""
    import torch
    d = ctx.find_duplicates(out, n_hits)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        d = ctx.find_duplicates(out, n_hits, dup_of=d)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps, d.cpu().numpy()


def setup_workload(kfx, name, dev):
    """Generate a workload, load its layers and upload its hits."""
    import torch

    import kfsynth
    t0 = time.perf_counter()
    ev = kfsynth.generate(name)
    log(f"[bench] generated {name}: {ev.n_events} events, {ev.n_hits} hits, {ev.n_tracks} seeds "
        f"in {time.perf_counter() - t0:.1f}s")
    ctx = kfx.Context(0)
    w = ev.workload
    torch.cuda.synchronize()
    t_ll = time.perf_counter()
    ctx.load_layers(ev.geometry.as_records(), ev.bz, w.n_eta_bins, w.n_phi_bins)
    torch.cuda.synchronize()
    load_layers_ms = (time.perf_counter() - t_ll) * 1e3
    t_h2d = time.perf_counter()
    hits = kfx.DeviceHits.from_events(ev, dev)
    torch.cuda.synchronize()
    h2d_ms = (time.perf_counter() - t_h2d) * 1e3
    seeds_d = torch.as_tensor(ev.seeds, device=dev)
    sev_d = torch.as_tensor(ev.trk_event.astype(np.int32), device=dev)
    return ev, ctx, hits, seeds_d, sev_d, load_layers_ms, h2d_ms


def tuned_shape(ctx, kfx, ev, hits, seeds_d, sev_d, shape_json="", reps=2):
    if shape_json:
        shape = {k: int(v) for k, v in json.loads(shape_json).items() if k != "ms"}
        log(f"[bench] launch shape given: {shape}")
        return shape
    t = time.perf_counter()
    shape = ctx.autotune_build(hits, seeds_d, sev_d, reps=reps, **build_kw(ev, kfx.MODE_FUSED))
    ms = shape.pop("ms")
    log(f"[bench] {ev.workload.name}: autotuned {shape} ({ms:.3f} ms) in {time.perf_counter() - t:.1f}s")
    return shape


def timed_graph(ctx, kfx, ev, hits, seeds_d, sev_d, shape, steps, warmup, out):
    """Time `steps` replays of the build captured as a HIP graph; returns
    (ms per step, identical to the eager output)."""
    import torch
    graph, gout = ctx.build_graph(hits, seeds_d, sev_d, **build_kw(ev, kfx.MODE_FUSED), **shape)
    for _ in range(warmup):
        graph.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.launch()
    torch.cuda.synchronize()
    gwall = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    same = all(torch.equal(gout[k], out[k]) for k in ("n_cands", "hits", "n_hits", "chi2"))
    graph.close()
    del gout
    return gwall, bool(same)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batch256", choices=sorted(WORKLOADS))
    ap.add_argument("--no-secondary", action="store_true", help="skip the secondary workloads")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle leg (and the parity gate)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed region, copy this many MiB device-to-device (a kernel of "
                         "known traffic for scaling the profiler's FETCH_SIZE/WRITE_SIZE)")
    ap.add_argument("--calib-flops-mi", type=int, default=0,
                    help="after the timed region, multiply two float32 and two float64 vectors of this "
                         "many Mi elements (kernels of known FLOP count for scaling the profiler's "
                         "VALU FLOP counters)")
    ap.add_argument("--shape", default="",
                    help="launch shape of the fused kernel as JSON (as the autotuner reports it); "
                         "skips the autotuner, e.g. to profile the tuned shape alone")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: every GPU box here has one, and the "
                                   "building shards by event with no exchange (see the design notes)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    import kfsynth
    from paper_2002_06295_amd import kfx

    dev = torch.device("cuda", 0)
    props = torch.cuda.get_device_properties(dev)
    ev, ctx, hits, seeds_d, sev_d, load_layers_ms, h2d_ms = setup_workload(kfx, args.workload, dev)
    # launch shape of the fused kernel for this workload (identical results
    # for every shape; only the time differs)
    shape = tuned_shape(ctx, kfx, ev, hits, seeds_d, sev_d, args.shape)
    wall, times, stats, out = run_build(ctx, kfx, hits, ev, args.steps, args.warmup, kfx.MODE_FUSED, shape=shape)
    search_ms = float(np.mean([t[1] for t in times]))
    kern_ms = float(np.mean([t[2] for t in times]))
    bin_ms = float(np.mean([t[0] for t in times]))
    log(f"[bench] fused eager: {wall:.3f} ms/step wall, fused kernel {search_ms:.3f} ms, building {kern_ms:.3f} ms, "
        f"binning {bin_ms:.3f} ms, steps {stats[0]:.0f} pairs {stats[1]:.0f} updates {stats[2]:.0f}")
    # the same build replayed from a HIP graph (the timed path)
    gwall, same_graph = timed_graph(ctx, kfx, ev, hits, seeds_d, sev_d, shape, args.steps, args.warmup, out)
    log(f"[bench] graph: {gwall:.3f} ms/step wall, identical to eager: {same_graph}")
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.calib_flops_mi > 0:
        n = args.calib_flops_mi * (1 << 20)
        for dt in (torch.float32, torch.float64):
            a = torch.ones(n, dtype=dt, device=dev)
            b = torch.full((n,), 1.5, dtype=dt, device=dev)
            torch.mul(a, b)
            torch.cuda.synchronize()
            del a, b

    value = stats[0] / (gwall * 1e-3)
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": gwall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}",
                   "events_per_step": ev.n_events, "seeds_per_step": ev.n_tracks, "hits_per_step": ev.n_hits,
                   "path": "fused persistent kernel replayed from a HIP graph", "launch_shape": shape,
                   "parallelism": "single GPU"},
        "roofline": alu_roofline(stats, search_ms, "k_build_fused",
                                 stored_traffic(f"k_build_fused_{args.workload}_traffic.json")),
        "tracks_per_s": ev.n_tracks / (gwall * 1e-3),
        "pairs_per_s": stats[1] / (gwall * 1e-3),
        "updates_per_s": stats[2] / (gwall * 1e-3),
        "binning_ms": bin_ms,
        "load_layers_ms": load_layers_ms,
        "hits_upload_ms": h2d_ms,
        "hits_upload_bytes": int(ev.n_hits * 16 + (ev.n_events + 1) * 4),
        "device": {"name": props.name, "compute_units": props.multi_processor_count,
                   "arch": getattr(props, "gcnArchName", ""), "clock": "not locked"},
        "building_ms": kern_ms,
        "eager_ms_per_step": wall,
        "graph_identical_to_eager": bool(same_graph),
    }

    if not args.no_cpu_baseline:
        idx = parity_sample(ev)
        cb, ores = cpu_baseline(ev, idx, oracle_prior())
        result["cpu_baseline"] = cb
        result["parity"] = parity_check(ev, out, idx, ores, oracle_prior())
        log(f"[bench] oracle {cb['value']:.3e} steps/s ({cb['cores']} threads), "
            f"{cb['single_thread_steps_per_s']:.3e} on one; parity {result['parity']}")
    dedup = None
    if not args.no_secondary:
        # duplicate removal on this workload's own output
        dms, dres = time_dedup(ctx, out, ev.n_hits)
        dedup = {"ms": dms, "tracks_per_s": ev.n_tracks / (dms * 1e-3), "flagged": int((dres >= 0).sum()),
                 "roofline": hbm_roofline(dedup_bytes(out, ev.n_hits), dms,
                                          "per track 12 max_hits + 52 B, per (track, hit) entry 20 B, 4 B per hit")}
        log(f"[bench] duplicate removal on {args.workload}: {dms * 1e3:.1f} us, {dedup['flagged']} flagged")
    del out
    torch.cuda.empty_cache()

    if not args.no_secondary:
        result["secondary"] = secondary(args, kfx, kfsynth, dev, ctx, hits, ev, shape)
        result["secondary"][f"duplicate_removal_{args.workload}"] = dedup
    print(json.dumps(result), flush=True)


def oracle_prior():
    import oracle
    return oracle.DEFAULT_PRIOR


def secondary(args, kfx, kfsynth, dev, ctx, hits, ev, shape):
    import torch
    sec = {}
    wall_p, times_p, stats_p, _ = run_build(ctx, kfx, hits, ev, 2, 1, kfx.MODE_PLAIN)
    sec["plain_path_same_input"] = {"steps_per_s": stats_p[0] / (wall_p * 1e-3), "ms_per_step": wall_p,
                                    "kernels_ms": float(np.mean([t[1] for t in times_p]))}
    log(f"[bench] plain path: {wall_p:.3f} ms/step")
    torch.cuda.empty_cache()
    # the other building workloads: their own graph replays and rooflines
    for name in ("build5k", "batch256", "occ10k"):
        if name == args.workload:
            continue
        ev2, ctx2, h2, s2, e2, _, _ = setup_workload(kfx, name, dev)
        sh2 = tuned_shape(ctx2, kfx, ev2, h2, s2, e2, reps=1)
        wf, tf, sf, o2 = run_build(ctx2, kfx, h2, ev2, 4, 1, kfx.MODE_FUSED, shape=sh2)
        gw, same2 = timed_graph(ctx2, kfx, ev2, h2, s2, e2, sh2, 5, 1, o2)
        dms2, dres2 = time_dedup(ctx2, o2, ev2.n_hits)
        dbytes2 = dedup_bytes(o2, ev2.n_hits)
        wp, tp, sp, o2 = run_build(ctx2, kfx, h2, ev2, 2, 1, kfx.MODE_PLAIN, out=o2)
        km = float(np.mean([t[1] for t in tf]))
        sec[name] = {"steps_per_s": sf[0] / (gw * 1e-3), "ms_per_step": gw, "graph_identical_to_eager": same2,
                     "eager_ms_per_step": wf, "fused_kernel_ms": km,
                     "binning_ms": float(np.mean([t[0] for t in tf])),
                     "building_ms": float(np.mean([t[2] for t in tf])),
                     "roofline": alu_roofline(sf, km, "k_build_fused",
                                              stored_traffic(f"k_build_fused_{name}_traffic.json")),
                     "launch_shape": sh2, "tracks_per_s": ev2.n_tracks / (gw * 1e-3),
                     "plain_steps_per_s": sp[0] / (wp * 1e-3), "steps_per_launch": sf[0],
                     "duplicate_removal_ms": dms2, "duplicates_flagged": int((dres2 >= 0).sum()),
                     "duplicate_removal_roofline": hbm_roofline(
                         dbytes2, dms2, "per track 12 max_hits + 52 B, per (track, hit) entry 20 B, 4 B per hit")}
        log(f"[bench] {name}: fused {sec[name]['steps_per_s']:.3e} steps/s "
            f"({sec[name]['roofline']['frac']:.4f} of FP32 peak), plain {sec[name]['plain_steps_per_s']:.3e}")
        del o2, h2, ctx2, ev2
        torch.cuda.empty_cache()
    # duplicate removal, hit masking and a second iteration on the single
    # event: the 5k-track event with a second seed (hits 1, 2, 4) for a
    # quarter of the particles
    ev5, ctx5, hits5, s5, e5, _, _ = setup_workload(kfx, "build5k", dev)
    shape5 = tuned_shape(ctx5, kfx, ev5, hits5, s5, e5, reps=1)
    dseeds, dsev, dtrk = kfsynth.duplicate_seeds(ev5, 0.25, seed=0)
    dout = ctx5.build_tracks(hits5, dseeds, dsev, **build_kw(ev5, kfx.MODE_FUSED), **shape5)
    dms, dres = time_dedup(ctx5, dout, ev5.n_hits)
    extra = np.arange(ev5.n_tracks, dseeds.shape[0])
    sec["duplicate_removal"] = {
        "workload": "build5k + a second seed for 25 % of the particles",
        "seeds": int(dseeds.shape[0]), "extra_seeds": int(extra.size), "ms": dms,
        "tracks_per_s": dseeds.shape[0] / (dms * 1e-3), "flagged": int((dres >= 0).sum()),
        "extra_flagged_to_own_particle": float(np.mean(dres[extra] == dtrk[extra])),
        "roofline": hbm_roofline(dedup_bytes(dout, ev5.n_hits), dms,
                                 "per track 12 max_hits + 52 B, per (track, hit) entry 20 B, 4 B per hit")}
    log(f"[bench] duplicate removal: {dms * 1e3:.1f} us, flagged {(dres >= 0).sum()} of "
        f"{extra.size} extra seeds")
    del dout
    sec["second_iteration"] = second_iteration(kfx, kfsynth, dev, ctx5, hits5, ev5, shape5)
    del hits5, ctx5
    sec["overlap5k"] = overlap_build(kfx, dev)
    sec["strip_clustering"] = strip_clustering(kfx, kfsynth, ctx)
    sec["align200k_fit"] = align_fit(kfx, kfsynth, dev)
    return sec


def overlap_build(kfx, dev):
    """The overlap workload (20 % of the crossings leave a second hit on
    the same layer) built with and without overlap recovery: graph-replayed
    time, steps/s, and the hits recovered in the best candidates."""
    import torch
    ev, ctx, hits, s, e, _, _ = setup_workload(kfx, "overlap5k", dev)
    res = {"workload": "build5k with 20 % of the crossings leaving a second hit on their layer (overlap5k)"}
    K = ev.workload.max_cands
    for on in (False, True):
        kw = dict(build_kw(ev, kfx.MODE_FUSED), overlap=on)
        shape = ctx.autotune_build(hits, s, e, reps=1, **kw)
        shape.pop("ms")
        out = ctx.build_tracks(hits, s, e, **kw, **shape)
        graph, gout = ctx.build_graph(hits, s, e, **kw, **shape)
        graph.launch()
        torch.cuda.synchronize()
        gout["stats"].zero_()
        n = 5
        t0 = time.perf_counter()
        for _ in range(n):
            graph.launch()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / n
        st = gout["stats"].cpu().numpy().astype(np.float64) / n
        best = gout["hits"].reshape(-1, gout["hits"].shape[-1])[::K][:ev.n_tracks].cpu().numpy()
        lay = ev.layer
        rec = 0
        for row in best:
            h = row[row >= 0]
            rec += int(np.sum(lay[h][1:] == lay[h][:-1]))
        tag = "recovery" if on else "no_recovery"
        res[tag] = {"ms_per_step": ms, "steps_per_s": st[0] / (ms * 1e-3), "updates_per_launch": st[2],
                    "recovered_hits_in_best_candidates": rec, "launch_shape": shape}
        graph.close()
        del gout, out
        log(f"[bench] overlap5k {tag}: {ms:.3f} ms/step, {rec} recovered hits")
    del hits, ctx
    torch.cuda.empty_cache()
    return res


def second_iteration(kfx, kfsynth, dev, ctx, hits, ev, shape):
    """Two iterations: the first from half of the particles (even ids); the
    hits of its good tracks (kept, >= 8 hits, chi2/ndof <= 3) masked; the
    second from a second seed (hits 1, 2, 4) of the particles whose seed
    hits are all free, with and without the mask."""
    import torch
    half = np.arange(0, ev.n_tracks, 2)
    out1 = ctx.build_tracks(hits, torch.as_tensor(ev.seeds[half], device=dev),
                            torch.as_tensor(ev.trk_event[half].astype(np.int32), device=dev),
                            **build_kw(ev, kfx.MODE_FUSED), **shape)
    dup1 = ctx.find_duplicates(out1, ev.n_hits)
    lay2 = ctx.mask_hits(out1, hits.layer, dup1, 8, 3.0)
    torch.cuda.synchronize()
    m0, m1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    m0.record()
    for _ in range(20):
        ctx.mask_hits(out1, hits.layer, dup1, 8, 3.0, layer_out=lay2)
    m1.record()
    torch.cuda.synchronize()
    mask_ms = m0.elapsed_time(m1) / 20
    lay2_h = lay2.cpu().numpy()
    s2, e2_, _ = kfsynth.duplicate_seeds(ev, 1.0, seed=0)
    s2, e2_ = s2[ev.n_tracks:], e2_[ev.n_tracks:]
    free = (lay2_h[s2] >= 0).all(axis=1)
    s2, e2_ = s2[free], e2_[free]
    n_s2 = int(s2.shape[0])
    s2 = torch.as_tensor(s2, device=dev)
    e2_ = torch.as_tensor(e2_, device=dev)
    hits_m = kfx.DeviceHits(hits.x, hits.y, hits.z, lay2, hits.event_offsets)
    it2 = {}
    for tag, hh in (("masked", hits_m), ("unmasked", hits)):
        o2i = ctx.build_tracks(hh, s2, e2_, **build_kw(ev, kfx.MODE_FUSED), **shape)
        st2 = o2i["stats"]
        st2.zero_()
        t2a, t2b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t2a.record()
        for _ in range(10):
            ctx.build_tracks(hh, s2, e2_, **build_kw(ev, kfx.MODE_FUSED), **shape, out=o2i)
        t2b.record()
        torch.cuda.synchronize()
        st = st2.cpu().numpy() / 10
        it2[tag] = {"ms": t2a.elapsed_time(t2b) / 10, "steps": float(st[0]), "pairs": float(st[1])}
        del o2i
    masked = int((lay2_h == -1).sum()) - int((ev.layer < 0).sum())
    res = {"workload": "build5k: iteration 1 from the first three hits of half of the particles; "
                       "iteration 2 from hits 1, 2, 4 of the particles whose seed hits the mask left free",
           "mask_ms": mask_ms, "hits_masked": masked,
           "mask_roofline": hbm_roofline(
               8 * ev.n_hits + int(out1["S"]) * (4 * int(out1["hits"].shape[1]) + 16) + 4 * masked, mask_ms,
               "layer array read and written (8 B per hit), per track its list row and 16 B, 4 B per masked hit"),
           "hits": ev.n_hits, "seeds_iteration2": n_s2, "iteration2": it2}
    log(f"[bench] second iteration: mask {mask_ms * 1e3:.1f} us, {masked} hits masked, {n_s2} seeds: "
        f"{it2['masked']['ms']:.3f} ms masked vs {it2['unmasked']['ms']:.3f} ms unmasked")
    return res


def strip_clustering(kfx, kfsynth, ctx):
    """16 events of the full strip detector in one call, and one event alone."""
    import torch
    sdet = kfsynth.strip_detector()
    sev = kfsynth.strip_events(sdet, 16, seed=7)
    sd16, scal = ctx.strip_inputs(sev, sdet)
    one = {k: v[:int(sev["event_offsets"][1])] for k, v in sev.items() if k != "event_offsets"}
    one["event_offsets"] = sev["event_offsets"][:2]
    sd1, _ = ctx.strip_inputs(one, sdet)
    strip = {"workload": "16 events of 15,000 modules x 768 strips, 20,000 particles and 1 % noise "
                         "digis per event", "digis": int(sev["module"].shape[0])}
    for tag, dg in (("batch16", sd16), ("one_event", sd1)):
        so = ctx.cluster_strips(dg, scal)
        torch.cuda.synchronize()
        c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        c0.record()
        for _ in range(20):
            ctx.cluster_strips(dg, scal, out=so)
        c1.record()
        torch.cuda.synchronize()
        ms_c = c0.elapsed_time(c1) / 20
        nd = int(dg["module"].numel())
        ncl = int(so["n"].cpu()[0])
        strip[tag] = {"ms": ms_c, "digis": nd, "digis_per_s": nd / (ms_c * 1e-3), "clusters": ncl,
                      "roofline": hbm_roofline(15 * nd + 24 * ncl, ms_c,
                                               "per digi 10 B read and 5 B of calibration, 24 B per kept "
                                               "cluster written")}
    log(f"[bench] strip clustering: 16 events {strip['batch16']['ms'] * 1e3:.0f} us "
        f"({strip['batch16']['digis_per_s']:.3e} digis/s), one event {strip['one_event']['ms'] * 1e3:.0f} us")
    return strip


def align_fit(kfx, kfsynth, dev):
    """The fit on the alignment workload: forward only, and forward with
    checkpoints + the adjoint (fit+grad)."""
    import torch
    evf = kfsynth.generate("align200k")
    ctxf = kfx.Context(0)
    ctxf.load_layers(evf.geometry.as_records(), evf.bz, 20, 128)
    hf = kfx.DeviceHits.from_events(evf, dev)
    toff = torch.as_tensor(evf.trk_offsets, device=dev)
    th = torch.as_tensor(evf.trk_hits, device=dev)
    ones = torch.ones(1, device=dev)
    pr = evf.workload.fit_prior
    fo = ctxf.fit_tracks(hf, toff, th, field_scale=1.0, prior=pr)
    fg = ctxf.fit_tracks(hf, toff, th, field_scale=1.0, ckpt=True, prior=pr)
    ctxf.fit_tracks_backward(hf, toff, th, fg, ones)
    torch.cuda.synchronize()
    e0, e1, e2, e3 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
    nrep = 5
    e0.record()
    for _ in range(nrep):
        fo = ctxf.fit_tracks(hf, toff, th, field_scale=1.0, out=fo, prior=pr)
    e1.record()
    for _ in range(nrep):
        fg = ctxf.fit_tracks(hf, toff, th, field_scale=1.0, ckpt=True, out=fg, prior=pr)
        ctxf.fit_tracks_backward(hf, toff, th, fg, ones)
    e2.record()
    for _ in range(nrep):
        ctxf.fit_tracks_backward(hf, toff, th, fg, ones)
    e3.record()
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1) / nrep
    gms = e1.elapsed_time(e2) / nrep
    bms = e2.elapsed_time(e3) / nrep
    nh = int(evf.trk_offsets[-1])
    res = {"fit_tracks_per_s": evf.n_tracks / (fms * 1e-3), "fit_ms": fms,
           "fit_grad_tracks_per_s": evf.n_tracks / (gms * 1e-3), "fit_grad_ms": gms,
           "backward_ms": bms,
           # the fit is the propagate + update chain alone (FP64)
           "fit_roofline": {"bound": "alu", "kernel": "k_fit", "flop_per_hit": FIT_FLOP_PER_HIT,
                            "achieved": nh * FIT_FLOP_PER_HIT / (fms * 1e-3) / 1e12, "unit": "TFLOP/s",
                            "peak": ALU_PEAK_TFLOPS, "peak_kind": "FP64 vector",
                            "frac": nh * FIT_FLOP_PER_HIT / (fms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS},
           "backward_roofline": {"bound": "alu", "kernel": "k_fit_backward", "flop_per_hit": ADJ_FLOP_PER_HIT,
                                 "achieved": nh * ADJ_FLOP_PER_HIT / (bms * 1e-3) / 1e12, "unit": "TFLOP/s",
                                 "peak": ALU_PEAK_TFLOPS, "peak_kind": "FP64 vector",
                                 "frac": nh * ADJ_FLOP_PER_HIT / (bms * 1e-3) / 1e12 / ALU_PEAK_TFLOPS},
           "tracks": evf.n_tracks, "hits": nh, "grad_params": 3 * evf.geometry.n_layers + 1,
           "prior": list(pr)}
    log(f"[bench] align200k: fit {fms:.3f} ms ({evf.n_tracks / (fms * 1e-3):.3e} tracks/s), "
        f"fit+grad {gms:.3f} ms ({evf.n_tracks / (gms * 1e-3):.3e} tracks/s)")
    return res


if __name__ == "__main__":
    main()
