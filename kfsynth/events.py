"""Seeded synthetic events for the Kalman track-building workloads.

This module is the detector simulation that feeds both the FP64 oracle and
the GPU path.  It holds none of the reconstruction arithmetic: no covariance
transport, no Jacobian, no chi2, no Kalman update, no hit binning.  It only
moves truth particles through a lightweight geometry (barrel cylinders at a
fixed radius, forward disks at a fixed z, as the paper's geometry collapses
layers, Sec. 2), applies multiple scattering, smears hits, drops a fraction
of them and adds uniform noise.

Particles move on helices in a uniform field along +z.  Crossings are found
by brute force over every surface with the closed-form intersection of the
particle's transverse circle with each cylinder (and a linear solve in z for
each disk).  The particle is followed to its earliest crossing; a crossing
beyond the turning point of its transverse circle (the point farthest from
the beam line) ends it: loopers are not followed back inward, and a particle
that leaves the tracker does not re-enter it after a whole loop.

Units: cm, GeV, T, rad.  All arithmetic is float64; the stored hit
coordinates are float32.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# p_T [GeV] = C_LIGHT * B [T] * rho [cm]
C_LIGHT = 0.299792458e-2

BARREL = 0
DISK = 1

MAX_CROSSINGS = 40


@dataclasses.dataclass
class Geometry:
    """Layer table.  kind: 0 barrel / 1 disk; pos: radius R (barrel) or z
    position Z (disk); lo/hi: z bounds (barrel) or r bounds (disk);
    x0: thickness in radiation lengths; su/sv/sn: hit resolution along the
    local axes (u = r*phi direction, v = z for barrel or r for disk,
    n = surface normal)."""

    kind: np.ndarray
    pos: np.ndarray
    lo: np.ndarray
    hi: np.ndarray
    x0: np.ndarray
    su: np.ndarray
    sv: np.ndarray
    sn: np.ndarray

    @property
    def n_layers(self) -> int:
        return int(self.kind.shape[0])

    def as_records(self) -> np.ndarray:
        """Packed float64 table [L, 8]: kind, pos, lo, hi, x0, su, sv, sn."""
        return np.stack([self.kind.astype(np.float64), self.pos, self.lo,
                         self.hi, self.x0, self.su, self.sv, self.sn], axis=1)


def make_geometry(n_barrel: int, r_in: float, r_out: float, half_z: float,
                  n_disk_side: int = 0, z_in: float = 0.0, z_out: float = 0.0,
                  disk_rmin: float = 0.0, disk_rmax: float = 0.0,
                  x0: float | None = None, sig_rphi: float = 20e-4,
                  sig_z: float = 50e-4, sig_r: float = 50e-4,
                  sig_n: float = 10e-4) -> Geometry:
    """Barrel layers evenly spaced in radius, then +z disks (increasing z),
    then -z disks (decreasing z).  x0=None ramps the thickness linearly
    from 0.02 to 0.05 radiation lengths with radius (barrel) or |z| (disks)."""
    kinds, pos, lo, hi, xx, su, sv, sn = [], [], [], [], [], [], [], []
    radii = np.linspace(r_in, r_out, n_barrel)
    for r in radii:
        kinds.append(BARREL)
        pos.append(r)
        lo.append(-half_z)
        hi.append(half_z)
        if x0 is None:
            f = 0.0 if n_barrel == 1 else (r - r_in) / (r_out - r_in)
            xx.append(0.02 + 0.03 * f)
        else:
            xx.append(x0)
        su.append(sig_rphi)
        sv.append(sig_z)
        sn.append(sig_n)
    if n_disk_side:
        zs = np.linspace(z_in, z_out, n_disk_side)
        for side in (1.0, -1.0):
            for z in zs:
                kinds.append(DISK)
                pos.append(side * z)
                lo.append(disk_rmin)
                hi.append(disk_rmax)
                if x0 is None:
                    f = 0.0 if n_disk_side == 1 else (z - z_in) / (z_out - z_in)
                    xx.append(0.02 + 0.03 * f)
                else:
                    xx.append(x0)
                su.append(sig_rphi)
                sv.append(sig_r)
                sn.append(sig_n)
    f64 = lambda a: np.asarray(a, dtype=np.float64)
    return Geometry(np.asarray(kinds, dtype=np.int32), f64(pos), f64(lo),
                    f64(hi), f64(xx), f64(su), f64(sv), f64(sn))


@dataclasses.dataclass
class Workload:
    """Parameters of one synthetic workload."""

    name: str
    geometry: Geometry
    bz: float
    n_events: int
    tracks_per_event: object          # int, or ("poisson", mean, lo, hi)
    pt_range: tuple
    eta_range: tuple
    noise_per_event: object           # int, or ("per_track", factor)
    ineff: float
    min_hits: int
    max_hits: int
    displaced_frac: float = 0.0
    displaced_rmax: float = 0.0
    field_scale_true: float = 1.0
    align_sigma: float = 0.0
    n_eta_bins: int = 20
    n_phi_bins: int = 128
    chi2_cut: float = 30.0
    max_cands: int = 6
    max_holes: int = 3
    seed_id: int = 1
    smear: bool = True
    # fraction of recorded crossings that leave a second hit on the same
    # layer (a module overlap): the same crossing point smeared again
    overlap_frac: float = 0.0
    scatter: bool = True
    # prior of the fit's start estimate: sigma_pos [cm], sigma_k / |k|,
    # sigma_phi, sigma_theta (a reconstruction setting carried with the
    # workload, like the chi2 cut)
    fit_prior: tuple = (0.1, 0.5, 0.05, 0.05)


def _geom_barrel10():
    return make_geometry(10, 4.0, 110.0, 120.0, x0=0.02)


def _geom_full():
    return make_geometry(17, 3.0, 110.0, 120.0, n_disk_side=9, z_in=30.0,
                         z_out=270.0, disk_rmin=20.0, disk_rmax=110.0)


def _geom_barrel17():
    return make_geometry(17, 3.0, 110.0, 120.0)


def workload(name: str, **overrides) -> Workload:
    """The named workloads.

    fit1k       1000 tracks, 10-layer barrel (R 4-110, |z|<120), no noise,
                pT log-U[0.5,10], eta U[-1,1], x/X0 = 0.02.  Fit only.
    build5k     5000 seeded tracks, 17 barrel layers (R 3-110) + 2x9 disks
                (|z| 30-270, r 20-110), eta U[-2.4,2.4], pT log-U[0.5,20],
                1% inefficiency, 20k noise hits, K = 6.
    batch256    256 events, tracks ~ Poisson(3000) clipped [200, 12000],
                noise = 5x tracks, geometry as build5k, 5-26 hits per track.
    align200k   200k tracks in the 17-layer barrel, eta U[-1,1],
                pT log-U[0.5,20], hidden per-layer offsets N(0, 50 um) and
                field scale 1.002.
    occ10k      10k tracks (pT log-U[0.3,50], eta U[-2.5,2.5], 10% from
                vertices with r_xy < 5 cm) + 300k noise hits per event,
                geometry as build5k, K = 10, 4 events.
    overlap5k   build5k with module overlaps: 20% of the recorded crossings
                leave a second hit on the same layer.
    """
    base = dict(
        fit1k=dict(geometry=_geom_barrel10(), bz=3.8, n_events=1,
                   tracks_per_event=1000, pt_range=(0.5, 10.0),
                   eta_range=(-1.0, 1.0), noise_per_event=0, ineff=0.0,
                   min_hits=3, max_hits=40, seed_id=1),
        build5k=dict(geometry=_geom_full(), bz=3.8, n_events=1,
                     tracks_per_event=5000, pt_range=(0.5, 20.0),
                     eta_range=(-2.4, 2.4), noise_per_event=20000, ineff=0.01,
                     min_hits=3, max_hits=40, max_cands=6, seed_id=2),
        batch256=dict(geometry=_geom_full(), bz=3.8, n_events=256,
                      tracks_per_event=("poisson", 3000, 200, 12000),
                      pt_range=(0.5, 20.0), eta_range=(-2.4, 2.4),
                      noise_per_event=("per_track", 5), ineff=0.01,
                      min_hits=5, max_hits=26, max_cands=6, seed_id=3),
        align200k=dict(geometry=_geom_barrel17(), bz=3.8, n_events=1,
                       tracks_per_event=200000, pt_range=(0.5, 20.0),
                       eta_range=(-1.0, 1.0), noise_per_event=0, ineff=0.0,
                       min_hits=3, max_hits=40, field_scale_true=1.002,
                       align_sigma=50e-4, seed_id=4,
                       # the start estimate comes from the recorded
                       # (uncorrected) hits; 50 um offsets at the innermost
                       # radii can exceed a high-pT seed's sagitta, so the
                       # curvature prior is widened to 5 |k|
                       fit_prior=(0.1, 5.0, 0.05, 0.05)),
        overlap5k=dict(geometry=_geom_full(), bz=3.8, n_events=1,
                       tracks_per_event=5000, pt_range=(0.5, 20.0),
                       eta_range=(-2.4, 2.4), noise_per_event=20000, ineff=0.01,
                       min_hits=3, max_hits=40, max_cands=6, seed_id=6,
                       overlap_frac=0.2),
        occ10k=dict(geometry=_geom_full(), bz=3.8, n_events=4,
                    tracks_per_event=10000, pt_range=(0.3, 50.0),
                    eta_range=(-2.5, 2.5), noise_per_event=300000,
                    ineff=0.01, min_hits=3, max_hits=40, displaced_frac=0.1,
                    displaced_rmax=5.0, max_cands=10, seed_id=5),
    )
    if name not in base:
        raise KeyError(f"unknown workload {name!r}; known: {sorted(base)}")
    kw = dict(base[name])
    kw.update(overrides)
    return Workload(name=name, **kw)


@dataclasses.dataclass
class Events:
    """A batch of events.  Hits of event e occupy [event_offsets[e],
    event_offsets[e+1]) of the hit arrays; hit indices are global."""

    workload: Workload
    geometry: Geometry
    bz: float
    x: np.ndarray                 # float32 [N]
    y: np.ndarray
    z: np.ndarray
    layer: np.ndarray             # int32 [N]
    sim: np.ndarray               # int32 [N] global truth track id, -1 noise
    event_offsets: np.ndarray     # int32 [E+1]
    trk_event: np.ndarray         # int32 [T]
    trk_offsets: np.ndarray       # int32 [T+1] into trk_hits
    trk_hits: np.ndarray          # int32 global hit indices, crossing order
    trk_truth: np.ndarray         # float64 [sum hits, 6] state after the
                                  # scatter at each recorded hit
    trk_vertex: np.ndarray        # float64 [T, 6] x, y, z, q/pT, phi, theta
    seeds: np.ndarray             # int32 [T, 3] first three hits
    align_true: np.ndarray        # float64 [L, 3] (dr, drphi, dz)

    @property
    def n_hits(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_tracks(self) -> int:
        return int(self.trk_event.shape[0])

    @property
    def n_events(self) -> int:
        return int(self.event_offsets.shape[0] - 1)


def _wrap(a):
    return np.mod(a + np.pi, 2.0 * np.pi) - np.pi


def _simulate(rng, w: Workload, n: int, align: np.ndarray):
    """Simulate n particles from their vertices.  Returns per-particle lists
    of crossings (recorded hits only) and vertex kinematics."""
    g = w.geometry
    bz_true = w.bz * w.field_scale_true
    lpt = rng.uniform(math.log(w.pt_range[0]), math.log(w.pt_range[1]), n)
    pt = np.exp(lpt)
    eta = rng.uniform(w.eta_range[0], w.eta_range[1], n)
    phi = rng.uniform(-np.pi, np.pi, n)
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    theta = 2.0 * np.arctan(np.exp(-eta))
    p = pt / np.sin(theta)
    x = np.zeros(n)
    y = np.zeros(n)
    zz = np.zeros(n)
    if w.displaced_frac > 0.0:
        disp = rng.random(n) < w.displaced_frac
        rv = rng.uniform(0.0, w.displaced_rmax, n)
        av = rng.uniform(-np.pi, np.pi, n)
        x = np.where(disp, rv * np.cos(av), 0.0)
        y = np.where(disp, rv * np.sin(av), 0.0)
    vertex = np.stack([x, y, zz, q / pt, phi, theta], axis=1)

    bar = np.nonzero(g.kind == BARREL)[0]
    dsk = np.nonzero(g.kind == DISK)[0]
    r_true = g.pos[bar] + align[bar, 0]          # true barrel radii
    z_disk = g.pos[dsk]

    hits_xyz = np.zeros((n, MAX_CROSSINGS, 3))
    hits_lay = np.full((n, MAX_CROSSINGS), -1, dtype=np.int32)
    truth = np.zeros((n, MAX_CROSSINGS, 6))
    nrec = np.zeros(n, dtype=np.int64)
    alive = np.ones(n, dtype=bool)
    last_surface = np.full(n, -1, dtype=np.int64)

    for _step in range(MAX_CROSSINGS):
        idx = np.nonzero(alive)[0]
        if idx.size == 0:
            break
        xi, yi, zi = x[idx], y[idx], zz[idx]
        ph, th, pi_, qi = phi[idx], theta[idx], p[idx], q[idx]
        pti = pi_ * np.sin(th)
        om = -C_LIGHT * bz_true * qi / pti          # dphi/ds (transverse s)
        cot = np.cos(th) / np.sin(th)
        m = idx.size
        best_s = np.full(m, np.inf)
        best_l = np.full(m, -1, dtype=np.int64)
        # path to the turning point (the point of the transverse circle
        # farthest from the beam line): a crossing beyond it is either
        # inward or, after a whole loop outside the tracker, outward again
        # far from where the particle left; both end the particle
        with np.errstate(divide="ignore", invalid="ignore"):
            om_t = np.where(np.abs(om) < 1e-12, 1e-12, om)
            ccx = xi - np.sin(ph) / om_t
            ccy = yi + np.cos(ph) / om_t
            dlt_t = np.mod(np.sign(om_t) * (np.arctan2(ccy, ccx) - np.arctan2(yi - ccy, xi - ccx)), 2.0 * np.pi)
            s_turn = np.where(np.abs(om) < 1e-12, np.inf, dlt_t / np.abs(om_t))

        # --- barrel: transverse circle vs cylinder, closed form
        if bar.size:
            straight = np.abs(om) < 1e-12
            oms = np.where(straight, 1e-12, om)
            rho = 1.0 / np.abs(oms)
            cx = xi - np.sin(ph) / oms
            cy = yi + np.cos(ph) / oms
            d = np.hypot(cx, cy)
            beta0 = np.arctan2(yi - cy, xi - cx)
            gam = np.arctan2(cy, cx)
            R = r_true[None, :]
            kap = (R * R - d[:, None] ** 2 - rho[:, None] ** 2) / (
                2.0 * rho[:, None] * d[:, None])
            ok = np.abs(kap) <= 1.0
            ac = np.arccos(np.clip(kap, -1.0, 1.0))
            sgn = np.sign(om)[:, None]
            s_b = np.full(kap.shape, np.inf)
            for branch in (1.0, -1.0):
                bc = gam[:, None] + branch * ac
                dlt = np.mod(sgn * (bc - beta0[:, None]), 2.0 * np.pi)
                dlt = np.where(dlt < 1e-9, dlt + 2.0 * np.pi, dlt)
                s = dlt * rho[:, None]
                s_b = np.where(ok & (s < s_b), s, s_b)
            # no field: straight line |P0 + s e|^2 = R^2, smallest s > 0
            if straight.any():
                D = (xi * np.cos(ph) + yi * np.sin(ph))[:, None]
                disc = D * D - ((xi * xi + yi * yi)[:, None] - R * R)
                sq = np.sqrt(np.maximum(disc, 0.0))
                s_lin = np.full(kap.shape, np.inf)
                for root in (-D - sq, -D + sq):
                    s_lin = np.where((disc >= 0) & (root > 1e-9) & (root < s_lin), root, s_lin)
                s_b = np.where(straight[:, None], s_lin, s_b)
            s_b = np.where(s_b < s_turn[:, None], s_b, np.inf)
            zc = zi[:, None] + s_b * cot[:, None]
            valid = np.isfinite(s_b) & (np.abs(zc) <= g.hi[bar][None, :])
            # a particle sitting on a cylinder does not re-cross it at s ~ 0
            s_b = np.where(valid, s_b, np.inf)
            j = np.argmin(s_b, axis=1)
            sj = s_b[np.arange(m), j]
            better = sj < best_s
            best_s = np.where(better, sj, best_s)
            best_l = np.where(better, bar[j], best_l)

        # --- disks: linear in z, then transverse position from the chord
        if dsk.size:
            with np.errstate(divide="ignore", invalid="ignore"):
                s_d = (z_disk[None, :] - zi[:, None]) / cot[:, None]
            s_d = np.where(np.isfinite(s_d) & (s_d > 1e-9) & (s_d < s_turn[:, None]), s_d, np.inf)
            a = 0.5 * om[:, None] * np.where(np.isfinite(s_d), s_d, 0.0)
            chord = np.where(np.abs(a) > 1e-12,
                             np.sin(a) / np.where(a == 0, 1.0, a), 1.0)
            chord = chord * np.where(np.isfinite(s_d), s_d, 0.0)
            xd = xi[:, None] + chord * np.cos(ph[:, None] + a)
            yd = yi[:, None] + chord * np.sin(ph[:, None] + a)
            rd = np.hypot(xd, yd)
            valid = (np.isfinite(s_d) & (rd >= g.lo[dsk][None, :])
                     & (rd <= g.hi[dsk][None, :]))
            s_d = np.where(valid, s_d, np.inf)
            j = np.argmin(s_d, axis=1)
            sj = s_d[np.arange(m), j]
            better = sj < best_s
            best_s = np.where(better, sj, best_s)
            best_l = np.where(better, dsk[j], best_l)

        moved = np.isfinite(best_s)
        alive[idx[~moved]] = False
        if not moved.any():
            continue
        sel = np.nonzero(moved)[0]
        gi = idx[sel]
        s = best_s[sel]
        lay = best_l[sel]
        om_s, ph_s = om[sel], ph[sel]
        a = 0.5 * om_s * s
        chord = np.where(np.abs(a) > 1e-12, np.sin(a) / np.where(a == 0, 1.0, a), 1.0) * s
        nx = xi[sel] + chord * np.cos(ph_s + a)
        ny = yi[sel] + chord * np.sin(ph_s + a)
        nz = zi[sel] + s * cot[sel]
        is_disk = g.kind[lay] == DISK
        nz = np.where(is_disk, g.pos[lay], nz)
        nphi = _wrap(ph_s + om_s * s)
        # radial velocity at the crossing: inward means the particle turned
        vr = nx * np.cos(nphi) + ny * np.sin(nphi)
        inward = vr < 0.0
        alive[gi[inward]] = False
        keep = ~inward
        gi, lay, nx, ny, nz, nphi = gi[keep], lay[keep], nx[keep], ny[keep], nz[keep], nphi[keep]
        is_disk = is_disk[keep]
        x[gi], y[gi], zz[gi], phi[gi] = nx, ny, nz, nphi
        last_surface[gi] = lay
        th_g, p_g, q_g = theta[gi], p[gi], q[gi]
        k = gi.size
        if k == 0:
            continue

        # --- record the hit (before the scatter at this surface)
        rec = rng.random(k) >= w.ineff
        su = g.su[lay]
        sv = g.sv[lay]
        e1 = rng.standard_normal(k) if w.smear else np.zeros(k)
        e2 = rng.standard_normal(k) if w.smear else np.zeros(k)
        rxy = np.hypot(nx, ny)
        phpos = np.arctan2(ny, nx)
        # barrel: recorded in nominal coordinates of a (possibly displaced)
        # true layer: rotate by -drphi/R, shift by -dz, place at nominal R
        Rn = g.pos[lay]
        ph_loc = phpos - np.where(is_disk, 0.0, align[lay, 1] / np.where(is_disk, 1.0, Rn))
        z_loc = nz - np.where(is_disk, 0.0, align[lay, 2])
        hb_phi = ph_loc + su * e1 / np.where(is_disk, rxy, Rn)
        hb_x = np.where(is_disk, (rxy + sv * e2) * np.cos(hb_phi), Rn * np.cos(hb_phi))
        hb_y = np.where(is_disk, (rxy + sv * e2) * np.sin(hb_phi), Rn * np.sin(hb_phi))
        hb_z = np.where(is_disk, g.pos[lay], z_loc + sv * e2)
        if w.overlap_frac > 0.0:
            # a second module over the same crossing: the point smeared again
            ov = rng.random(k) < w.overlap_frac
            e3 = rng.standard_normal(k) if w.smear else np.zeros(k)
            e4 = rng.standard_normal(k) if w.smear else np.zeros(k)
            ob_phi = ph_loc + su * e3 / np.where(is_disk, rxy, Rn)
            ob_x = np.where(is_disk, (rxy + sv * e4) * np.cos(ob_phi), Rn * np.cos(ob_phi))
            ob_y = np.where(is_disk, (rxy + sv * e4) * np.sin(ob_phi), Rn * np.sin(ob_phi))
            ob_z = np.where(is_disk, g.pos[lay], z_loc + sv * e4)
        else:
            ov = np.zeros(k, dtype=bool)

        # --- multiple scattering (Highland), momentum magnitude kept
        ct, st = np.cos(th_g), np.sin(th_g)
        tx, ty, tz = st * np.cos(nphi), st * np.sin(nphi), ct
        cos_inc = np.where(is_disk, np.abs(tz), np.abs((nx * tx + ny * ty) / rxy))
        cos_inc = np.maximum(cos_inc, 1e-3)
        t = g.x0[lay] / cos_inc
        tpos = np.where(t > 0.0, t, 1.0)
        th0 = np.where(t > 0.0, 0.0136 / p_g * np.sqrt(tpos) * (1.0 + 0.038 * np.log(tpos)), 0.0)
        if w.scatter:
            g1 = rng.standard_normal(k) * th0
            g2 = rng.standard_normal(k) * th0
        else:
            g1 = np.zeros(k)
            g2 = np.zeros(k)
        # e_theta, e_phi: unit vectors orthogonal to the direction
        ux = tx + g1 * ct * np.cos(nphi) - g2 * np.sin(nphi)
        uy = ty + g1 * ct * np.sin(nphi) + g2 * np.cos(nphi)
        uz = tz - g1 * st
        un = np.sqrt(ux * ux + uy * uy + uz * uz)
        ux, uy, uz = ux / un, uy / un, uz / un
        nth = np.arccos(np.clip(uz, -1.0, 1.0))
        nph = np.arctan2(uy, ux)
        theta[gi] = nth
        phi[gi] = nph

        slot = nrec[gi]
        can = rec & (slot < MAX_CROSSINGS)
        gi_r = gi[can]
        sl = slot[can]
        hits_xyz[gi_r, sl, 0] = hb_x[can]
        hits_xyz[gi_r, sl, 1] = hb_y[can]
        hits_xyz[gi_r, sl, 2] = hb_z[can]
        hits_lay[gi_r, sl] = lay[can]
        pt_new = p_g[can] * np.sin(nth[can])
        truth[gi_r, sl, 0] = nx[can]
        truth[gi_r, sl, 1] = ny[can]
        truth[gi_r, sl, 2] = nz[can]
        truth[gi_r, sl, 3] = q_g[can] / pt_new
        truth[gi_r, sl, 4] = nph[can]
        truth[gi_r, sl, 5] = nth[can]
        nrec[gi_r] += 1
        # the overlap hit follows its primary
        can2 = can & ov & (slot + 1 < MAX_CROSSINGS)
        if can2.any():
            gi2 = gi[can2]
            sl2 = slot[can2] + 1
            hits_xyz[gi2, sl2, 0] = ob_x[can2]
            hits_xyz[gi2, sl2, 1] = ob_y[can2]
            hits_xyz[gi2, sl2, 2] = ob_z[can2]
            hits_lay[gi2, sl2] = lay[can2]
            truth[gi2, sl2] = truth[gi2, sl2 - 1]
            nrec[gi2] += 1
    return hits_xyz, hits_lay, truth, nrec, vertex


_CHUNK = 16384


def _draw_chunk(args):
    seed, w, n, align = args
    return _draw_tracks(np.random.default_rng(seed), w, n, align)


def _draw_all(seed_base, w: Workload, n: int, align: np.ndarray):
    """Draw n particles in fixed chunks of _CHUNK, chunk i from its own
    random stream, so the result does not depend on the worker count."""
    jobs = []
    for i, start in enumerate(range(0, n, _CHUNK)):
        jobs.append((list(seed_base) + [1000 + i], w, min(_CHUNK, n - start), align))
    if len(jobs) > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        import os
        workers = max(1, min(len(jobs), (os.cpu_count() or 1), 16))
        with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("fork")) as ex:
            parts = list(ex.map(_draw_chunk, jobs))
    else:
        parts = [_draw_chunk(j) for j in jobs]
    return tuple(np.concatenate([p[i] for p in parts]) for i in range(5))


def _draw_tracks(rng, w: Workload, n: int, align: np.ndarray):
    """Draw n particles with min_hits <= recorded hits <= max_hits,
    regenerating the rest."""
    out = []
    need = n
    while need > 0:
        m = max(int(need * 1.3) + 16, 64)
        hx, hl, tr, nr, vx = _simulate(rng, w, m, align)
        # layers crossed with a hit (an overlap hit repeats its primary's
        # layer right after it)
        nlay = nr - np.sum((hl[:, 1:] == hl[:, :-1]) & (hl[:, 1:] >= 0), axis=1)
        good = np.nonzero((nlay >= w.min_hits) & (nr <= w.max_hits))[0][:need]
        out.append((hx[good], hl[good], tr[good], nr[good], vx[good]))
        need -= good.size
    cat = lambda i: np.concatenate([o[i] for o in out])
    return cat(0), cat(1), cat(2), cat(3), cat(4)


def _noise(rng, g: Geometry, count: int):
    """Uniform noise over the sensitive area, split over layers
    multinomially by area."""
    area = np.where(g.kind == BARREL, 2.0 * np.pi * g.pos * (g.hi - g.lo),
                    np.pi * (g.hi ** 2 - g.lo ** 2))
    per = rng.multinomial(count, area / area.sum())
    xs, ys, zs, ls = [], [], [], []
    for l, c in enumerate(per):
        if c == 0:
            continue
        ph = rng.uniform(-np.pi, np.pi, c)
        if g.kind[l] == BARREL:
            r = np.full(c, g.pos[l])
            z = rng.uniform(g.lo[l], g.hi[l], c)
        else:
            r = np.sqrt(rng.uniform(g.lo[l] ** 2, g.hi[l] ** 2, c))
            z = np.full(c, g.pos[l])
        xs.append(r * np.cos(ph))
        ys.append(r * np.sin(ph))
        zs.append(z)
        ls.append(np.full(c, l, dtype=np.int32))
    if not xs:
        e = np.zeros(0)
        return e, e, e, np.zeros(0, dtype=np.int32)
    return (np.concatenate(xs), np.concatenate(ys), np.concatenate(zs),
            np.concatenate(ls))


def generate(w: Workload | str, n_events: int | None = None,
             tracks_per_event: int | None = None, seed_offset: int = 0) -> Events:
    """Generate the events of a workload.  Deterministic in
    (workload.seed_id, seed_offset).  n_events / tracks_per_event shrink
    a workload for tests while keeping its distributions."""
    if isinstance(w, str):
        w = workload(w)
    if n_events is not None or tracks_per_event is not None:
        w = dataclasses.replace(
            w, n_events=n_events if n_events is not None else w.n_events,
            tracks_per_event=(tracks_per_event if tracks_per_event is not None
                              else w.tracks_per_event))
    rng = np.random.default_rng([1, w.seed_id, seed_offset])
    g = w.geometry
    L = g.n_layers
    align = np.zeros((L, 3))
    if w.align_sigma > 0.0:
        bar = g.kind == BARREL
        align[bar] = rng.normal(0.0, w.align_sigma, (int(bar.sum()), 3))

    tpe = w.tracks_per_event
    if isinstance(tpe, tuple):
        _, mean, lo, hi = tpe
        counts = np.clip(rng.poisson(mean, w.n_events), lo, hi)
    else:
        counts = np.full(w.n_events, int(tpe))
    total = int(counts.sum())
    hx, hl, tr, nr, vx = _draw_all([1, w.seed_id, seed_offset], w, total, align)

    xs, ys, zs, ls, sims = [], [], [], [], []
    ev_off = [0]
    trk_event = np.repeat(np.arange(w.n_events, dtype=np.int32), counts)
    trk_off = np.zeros(total + 1, dtype=np.int64)
    trk_off[1:] = np.cumsum(nr)
    trk_hits = np.zeros(int(trk_off[-1]), dtype=np.int32)
    trk_truth = np.zeros((int(trk_off[-1]), 6))
    t0 = 0
    for e in range(w.n_events):
        c = int(counts[e])
        tids = np.arange(t0, t0 + c)
        nrs = nr[tids]
        mask = np.arange(MAX_CROSSINGS)[None, :] < nrs[:, None]
        txyz = hx[tids][mask]
        tlay = hl[tids][mask]
        tsim = np.repeat(tids, nrs).astype(np.int32)
        nz = w.noise_per_event
        n_noise = int(nz[1] * c) if isinstance(nz, tuple) else int(nz)
        nxs, nys, nzs, nls = _noise(rng, g, n_noise)
        ex = np.concatenate([txyz[:, 0], nxs])
        ey = np.concatenate([txyz[:, 1], nys])
        ez = np.concatenate([txyz[:, 2], nzs])
        el = np.concatenate([tlay, nls]).astype(np.int32)
        es = np.concatenate([tsim, np.full(nxs.shape[0], -1, dtype=np.int32)])
        perm = rng.permutation(ex.shape[0])
        inv = np.empty_like(perm)
        inv[perm] = np.arange(perm.shape[0])
        base = ev_off[-1]
        # truth hit j of the event (in track order) lands at base + inv[j]
        ntr = txyz.shape[0]
        trk_hits[trk_off[t0]:trk_off[t0 + c]] = base + inv[:ntr]
        trk_truth[trk_off[t0]:trk_off[t0 + c]] = tr[tids][mask]
        xs.append(ex[perm])
        ys.append(ey[perm])
        zs.append(ez[perm])
        ls.append(el[perm])
        sims.append(es[perm])
        ev_off.append(base + ex.shape[0])
        t0 += c
    x = np.concatenate(xs).astype(np.float32)
    y = np.concatenate(ys).astype(np.float32)
    z = np.concatenate(zs).astype(np.float32)
    if w.overlap_frac > 0.0:
        seeds = _first_three_layers(trk_hits, trk_off, np.concatenate(ls))
    else:
        seeds = np.stack([trk_hits[trk_off[:-1] + i] for i in range(3)], axis=1)
    return Events(workload=w, geometry=g, bz=w.bz, x=x, y=y, z=z,
                  layer=np.concatenate(ls), sim=np.concatenate(sims),
                  event_offsets=np.asarray(ev_off, dtype=np.int32),
                  trk_event=trk_event, trk_offsets=trk_off.astype(np.int32),
                  trk_hits=trk_hits, trk_truth=trk_truth, trk_vertex=vx,
                  seeds=seeds.astype(np.int32), align_true=align)


def _first_three_layers(trk_hits, trk_off, layer):
    """Seeds when tracks carry overlap hits: the first three hits of each
    track on three different layers (an overlap hit repeats the layer of
    the hit before it)."""
    T = trk_off.shape[0] - 1
    seeds = np.zeros((T, 3), np.int64)
    for t in range(T):
        got, prev = 0, -1
        for j in range(trk_off[t], trk_off[t + 1]):
            h = trk_hits[j]
            if layer[h] != prev:
                seeds[t, got] = h
                got += 1
                prev = layer[h]
                if got == 3:
                    break
    return seeds


def duplicate_seeds(ev: Events, frac: float, seed: int = 0):
    """The event's seeds (first three hits of every track) plus, for a
    random fraction `frac` of the tracks with at least four hits, a second
    seed from hits 1, 2 and 4 of the same track, as when several hit
    triplets of one particle seed it.  Returns (seeds [S, 3], seed_event
    [S], seed_track [S]); the extra seeds follow the originals."""
    rng = np.random.default_rng([7, ev.workload.seed_id, seed])
    nrec = np.diff(ev.trk_offsets)
    cand = np.nonzero(nrec >= 4)[0]
    pick = np.sort(cand[rng.random(cand.shape[0]) < frac])
    o = ev.trk_offsets[pick]
    extra = np.stack([ev.trk_hits[o], ev.trk_hits[o + 1], ev.trk_hits[o + 3]], axis=1)
    seeds = np.concatenate([ev.seeds, extra]).astype(np.int32)
    seed_event = np.concatenate([ev.trk_event, ev.trk_event[pick]]).astype(np.int32)
    seed_track = np.concatenate([np.arange(ev.n_tracks), pick]).astype(np.int32)
    return seeds, seed_event, seed_track


def track_lists(n_seeds: int, K: int, max_hits: int, n_hits_total: int,
                seed: int = 0, seeds_per_truth: float = 2.0, p_hole: float = 0.1,
                p_swap: float = 0.15, chi2_levels: int = 6, p_empty: float = 0.03):
    """Synthetic building output (hit lists, counts, chi2 per seed and slot)
    with clusters of overlapping tracks, for the duplicate-removal step.

    Truth tracks are lists of distinct hit indices; each seed copies one
    truth track (popular truths are copied many times), turns entries into
    holes (-1) or other hits at random and may drop its tail; lists are
    padded with -3.  chi2 takes few distinct values so that ties in the
    ranking occur.  A few seeds have no candidate, a few lists repeat an
    entry or hold an index outside [0, n_hits_total).  Slots above 0 hold
    random hits.  Returns a dict of numpy arrays shaped like the building
    output: n_cands [S], hits [S*K, max_hits], n_hits, n_holes [S*K] int32,
    chi2 [S*K] float32."""
    rng = np.random.default_rng([11, seed])
    S = n_seeds
    n_truth = max(1, int(S / seeds_per_truth))
    L = max(1, min(max_hits, 26))
    truth_len = rng.integers(3, L + 1, n_truth)
    truth = [rng.choice(n_hits_total, size=min(int(n), n_hits_total), replace=False)
             if n_hits_total > 0 else np.zeros(0, np.int64) for n in truth_len]
    # popularity: a Zipf-like choice of truth track per seed
    w = 1.0 / np.arange(1, n_truth + 1) ** 0.8
    owner = rng.choice(n_truth, size=S, p=w / w.sum())
    hits = rng.integers(-1, max(n_hits_total, 1), (S * K, max_hits)).astype(np.int32)
    n_cands = rng.integers(1, K + 1, S).astype(np.int32)
    n_cands[rng.random(S) < p_empty] = 0
    n_hits = rng.integers(0, 30, S * K).astype(np.int32)
    n_holes = rng.integers(0, 4, S * K).astype(np.int32)
    chi2 = (rng.integers(0, chi2_levels, S * K) * 2.5).astype(np.float32)
    for s in range(S):
        t = truth[owner[s]].copy()
        if t.shape[0] > 3 and rng.random() < 0.3:
            t = t[:rng.integers(3, t.shape[0] + 1)]
        row = t.astype(np.int64)
        u = rng.random(row.shape[0])
        row[u < p_hole] = -1
        swap = (u >= p_hole) & (u < p_hole + p_swap)
        if n_hits_total > 0:
            row[swap] = rng.integers(0, n_hits_total, int(swap.sum()))
        r = rng.random()
        if r < 0.02 and row.shape[0] > 1:
            row[-1] = row[0]                      # a repeated entry
        elif r < 0.04 and row.shape[0] > 0:
            row[-1] = n_hits_total + 5            # not a hit index
        elif r < 0.05:
            row[:] = -1                           # no hit at all
        row = row[:max_hits]
        full = np.full(max_hits, -3, np.int64)
        full[:row.shape[0]] = row
        hits[s * K] = full.astype(np.int32)
        n_hits[s * K] = int((row >= 0).sum())
        n_holes[s * K] = int((row == -1).sum())
    return dict(n_cands=n_cands, hits=hits, n_hits=n_hits, n_holes=n_holes, chi2=chi2)
