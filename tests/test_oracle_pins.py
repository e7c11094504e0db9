"""Pins of the FP64 oracle against what the mathematics fixes independently
of it: the Lorentz-force equation of motion, closed-form circle
intersections, finite differences, Monte-Carlo scattering, exact recovery on
noise-free hits, the chi2 distribution on smeared hits, the least-squares
special case of the Kalman filter and brute-force hit search.

The paper (arXiv 2002.06295) defines the Kalman filter as propagate (with
material effects) then update (Sec. 1) over a lightweight barrel/disk
geometry (Sec. 2); the oracle's numerical readings of it are pinned here.
"""
import math

import numpy as np
import pytest

import kfsynth
import oracle

KC = 0.299792458e-2


def rk4_lorentz(p0, bz, s_target, n_steps=4000):
    """Integrate dr/dl = t, dt/dl = (kC q / p) t x B in 3D path length l with
    classical RK4 (independent of the closed-form helix)."""
    x, y, z, k, phi, th = p0
    q = np.sign(k) if k != 0 else 1.0
    pt = 1.0 / abs(k)
    p = pt / math.sin(th)
    y0 = np.array([x, y, z, math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
    B = np.array([0.0, 0.0, bz])
    c = KC * q / p

    def f(v):
        t = v[3:]
        return np.concatenate([t, c * np.cross(t, B)])

    L = s_target / math.sin(th)
    h = L / n_steps
    v = y0.copy()
    for _ in range(n_steps):
        k1 = f(v)
        k2 = f(v + 0.5 * h * k1)
        k3 = f(v + 0.5 * h * k2)
        k4 = f(v + h * k3)
        v = v + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return v


@pytest.mark.parametrize("p0", [
    [0.0, 0.0, 0.0, 1.0 / 0.6, 0.3, 1.1],        # positive, low pT
    [1.0, -2.0, 3.0, -1.0 / 2.5, -2.9, 0.7],     # negative
    [5.0, 1.0, -4.0, 1.0 / 40.0, 2.0, 2.2],      # high pT, backward
])
def test_helix_matches_rk4_lorentz(p0):
    s = 110.0
    ref = rk4_lorentz(p0, 3.8, s)
    got = oracle.helix(3.8, p0, s)
    assert np.max(np.abs(got[:3] - ref[:3])) < 1e-8
    # direction: phi(s) from the integrated tangent
    phi_ref = math.atan2(ref[4], ref[3])
    d = (got[4] - phi_ref + math.pi) % (2 * math.pi) - math.pi
    assert abs(d) < 1e-9


def test_helix_special_cases():
    # no field: a straight line
    p0 = np.array([1.0, 2.0, 3.0, 1.3, 0.4, 1.0])
    got = oracle.helix(0.0, p0, 50.0)
    exp = p0[:3] + 50.0 * np.array([math.cos(0.4), math.sin(0.4), math.cos(1.0) / math.sin(1.0)])
    assert np.allclose(got[:3], exp, atol=1e-12)
    # periodicity: back to the start after one full turn 2 pi rho
    k = 1.0 / 0.8
    rho = 0.8 / (KC * 3.8)
    p1 = np.array([0.5, -0.2, 0.0, k, 1.2, math.pi / 2])
    got = oracle.helix(3.8, p1, 2 * math.pi * rho)
    assert np.allclose(got[:2], p1[:2], atol=1e-10)
    # from the origin r(s) = 2 rho sin(s / 2 rho), so s(R) = 2 rho asin(R / 2 rho)
    for pt in (0.7, 3.0, 30.0):
        rho = pt / (KC * 3.8)
        p0 = np.array([0.0, 0.0, 0.0, 1.0 / pt, 0.1, 1.0])
        s = oracle.path_to_cylinder(3.8, p0, 50.0)
        assert s == pytest.approx(2 * rho * math.asin(50.0 / (2 * rho)), rel=1e-13)


def circle_intersection_s(p0, bz, R):
    """Closed form: transverse circle (centre c, radius rho) meets |P| = R;
    path length = turning angle * rho to the first crossing in the direction
    of motion."""
    x, y, _, k, phi, _ = p0
    om = -KC * bz * k
    rho = 1.0 / abs(om)
    cx, cy = x - math.sin(phi) / om, y + math.cos(phi) / om
    d = math.hypot(cx, cy)
    kap = (R * R - d * d - rho * rho) / (2 * rho * d)
    if abs(kap) > 1:
        return None
    gam = math.atan2(cy, cx)
    b0 = math.atan2(y - cy, x - cx)
    best = None
    for sgn in (1, -1):
        b = gam + sgn * math.acos(kap)
        dl = (math.copysign(1, om) * (b - b0)) % (2 * math.pi)
        s = dl * rho
        if best is None or s < best:
            best = s
    return best


def test_path_to_cylinder_matches_closed_form():
    rng = np.random.default_rng(7)
    n_ok = 0
    for _ in range(200):
        r0 = rng.uniform(2, 60)
        a = rng.uniform(-math.pi, math.pi)
        phi = a + rng.uniform(-1.2, 1.2)       # moving outward
        pt = math.exp(rng.uniform(math.log(0.4), math.log(50)))
        k = rng.choice([-1, 1]) / pt
        p0 = [r0 * math.cos(a), r0 * math.sin(a), 0.0, k, phi, 1.0]
        R = r0 + rng.uniform(1, 50)
        s = oracle.path_to_cylinder(3.8, p0, R)
        ref = circle_intersection_s(p0, 3.8, R)
        # the first crossing in the closed form may be the incoming one only
        # if the oracle reports none (track turns first)
        if s is None:
            # no outgoing crossing: the circle misses the cylinder, or the
            # first crossing is reached moving inward (after the turn)
            if ref is not None:
                q = oracle.helix(3.8, p0, ref)
                assert q[0] * math.cos(q[4]) + q[1] * math.sin(q[4]) <= 1e-9
            continue
        n_ok += 1
        assert s == pytest.approx(ref, rel=1e-10, abs=1e-10)
    assert n_ok > 100


def _geom():
    return kfsynth.workload("build5k").geometry


@pytest.mark.parametrize("layer,p0", [
    (8, [20.0, 5.0, 10.0, 1.0 / 1.5, 0.4, 1.2]),          # barrel
    (16, [60.0, -40.0, 30.0, -1.0 / 0.9, -0.7, 1.4]),     # barrel, low pT
    (20, [25.0, 10.0, 60.0, 1.0 / 3.0, 0.3, 0.45]),       # +z disk
    (28, [15.0, -20.0, -60.0, -1.0 / 2.0, -1.0, 2.6]),    # -z disk
])
def test_jacobian_matches_central_differences(layer, p0):
    g = _geom()
    p0 = np.array(p0)
    p1, J = oracle.propagate(g, 3.8, layer, p0)
    assert p1 is not None
    Jfd = np.zeros((6, 6))
    for j in range(6):
        h = 1e-6 * max(1.0, abs(p0[j]))
        a, b = p0.copy(), p0.copy()
        a[j] += h
        b[j] -= h
        pa, _ = oracle.propagate(g, 3.8, layer, a)
        pb, _ = oracle.propagate(g, 3.8, layer, b)
        Jfd[:, j] = (pa - pb) / (2 * h)
    scale = np.maximum(np.abs(J), 1.0)
    assert np.max(np.abs(J - Jfd) / scale) < 2e-6
    # the propagated position stays on the surface: n . J_pos = 0
    if g.kind[layer] == kfsynth.BARREL:
        n = np.array([p1[0], p1[1], 0.0]) / math.hypot(p1[0], p1[1])
    else:
        n = np.array([0.0, 0.0, 1.0])
    assert np.max(np.abs(n @ J[:3, :])) < 1e-9
    # the k and theta rows are unit rows
    assert np.allclose(J[3], np.eye(6)[3]) and np.allclose(J[5], np.eye(6)[5])


def highland(x0, p, cos_inc):
    t = x0 / cos_inc
    return 0.0136 / p * math.sqrt(t) * (1 + 0.038 * math.log(t))


@pytest.mark.parametrize("layer,th,phi", [(5, 1.0, 0.3), (12, 2.0, -2.0), (22, 0.4, 1.0)])
def test_material_noise_matches_monte_carlo(layer, th, phi):
    g = _geom()
    k = -1.0 / 0.8
    R = g.pos[layer]
    if g.kind[layer] == kfsynth.BARREL:
        x, y, z = R * math.cos(phi - 0.2), R * math.sin(phi - 0.2), 3.0
        cos_inc = abs(math.sin(th) * math.cos(0.2))
    else:
        x, y, z = 30 * math.cos(phi), 30 * math.sin(phi), g.pos[layer]
        cos_inc = abs(math.cos(th))
    p = np.array([x, y, z, k, phi, th])
    Q = oracle.material_noise(g, layer, p)
    pmom = 1.0 / (abs(k) * math.sin(th))
    t0 = highland(g.x0[layer], pmom, cos_inc)
    rng = np.random.default_rng(3)
    n = 400000
    g1, g2 = rng.standard_normal(n) * t0, rng.standard_normal(n) * t0
    t = np.array([math.sin(th) * math.cos(phi), math.sin(th) * math.sin(phi), math.cos(th)])
    e_th = np.array([math.cos(th) * math.cos(phi), math.cos(th) * math.sin(phi), -math.sin(th)])
    e_ph = np.array([-math.sin(phi), math.cos(phi), 0.0])
    d = t[None, :] + g1[:, None] * e_th[None, :] + g2[:, None] * e_ph[None, :]
    d /= np.linalg.norm(d, axis=1)[:, None]
    th2 = np.arccos(d[:, 2])
    ph2 = np.arctan2(d[:, 1], d[:, 0])
    k2 = np.sign(k) / (pmom * np.sin(th2))
    dphi = (ph2 - phi + np.pi) % (2 * np.pi) - np.pi
    X = np.stack([k2 - k, dphi, th2 - th], axis=1)
    Cmc = np.cov(X.T)
    Qs = Q[np.ix_([3, 4, 5], [3, 4, 5])]
    for (i, j) in [(0, 0), (1, 1), (2, 2), (0, 2)]:
        assert Qs[i, j] == pytest.approx(Cmc[i, j], rel=0.02, abs=1e-3 * math.sqrt(Qs[i, i] * Qs[j, j]))
    # no position noise, and no k noise at theta = pi/2
    assert np.all(Q[:3] == 0) and np.all(Q[:, :3] == 0)
    p90 = p.copy()
    p90[5] = math.pi / 2
    assert abs(oracle.material_noise(g, layer, p90)[3, 3]) < 1e-20


def test_seed_estimate_exact_on_helix_points():
    g = _geom()
    for pt, q, phi, th in [(0.9, 1, 0.3, 1.2), (7.0, -1, -2.5, 0.5), (2.0, 1, 3.0, 2.5)]:
        p0 = np.array([0.0, 0.0, 0.0, q / pt, phi, th])
        rho = pt / (KC * 3.8)
        pts = []
        for R in (4.0, 11.0, 19.0):
            s = 2 * rho * math.asin(R / (2 * rho))
            pts.append(oracle.helix(3.8, p0, s))
        est = oracle.seed_estimate(g, 3.8, pts[0][:3], pts[1][:3], pts[2][:3])
        assert est[3] == pytest.approx(q / pt, rel=1e-10)
        d = (est[4] - pts[0][4] + np.pi) % (2 * np.pi) - np.pi
        assert abs(d) < 1e-10
        assert est[5] == pytest.approx(th, abs=1e-10)


def test_noise_free_fit_recovers_truth():
    w = kfsynth.workload("fit1k", smear=False, scatter=False)
    ev = kfsynth.generate(w, tracks_per_event=200)
    p, C, c2, nd, ok = oracle.fit(ev)
    last = ev.trk_offsets[1:] - 1
    tr = ev.trk_truth[last]
    pt = 1 / np.abs(ev.trk_vertex[:, 3])
    s = ok & (pt > 0.7)
    assert s.sum() > 150
    d = p[s] - tr[s]
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    # residual error is the float32 rounding of the stored hits (~1e-6 cm)
    assert np.max(np.abs(d[:, :3])) < 2e-5
    assert np.max(np.abs(d[:, 3] / tr[s, 3])) < 2e-4
    assert np.max(np.abs(d[:, 4:])) < 2e-6
    assert np.max(c2[s] / nd[s]) < 1e-3


def test_fit_chi2_and_pulls_on_smeared_hits():
    ev = kfsynth.generate("fit1k")
    p, C, c2, nd, ok = oracle.fit(ev)
    pt = 1 / np.abs(ev.trk_vertex[:, 3])
    # tracks that cross the outer layers near their turning point break the
    # linearisation; they are excluded from the statistical pins
    s = ok & (pt > 0.7)
    assert s.sum() > 850
    assert c2[s].sum() / nd[s].sum() == pytest.approx(1.0, abs=0.03)
    from scipy.stats import chi2 as chi2d, kstest
    pv = chi2d.sf(c2[s], nd[s])
    assert kstest(pv, "uniform").pvalue > 1e-3
    last = ev.trk_offsets[1:] - 1
    tr = ev.trk_truth[last]
    d = p - tr
    d[:, 4] = (d[:, 4] + np.pi) % (2 * np.pi) - np.pi
    n = s.sum()
    for i in (3, 4, 5):
        pull = d[s, i] / np.sqrt(C[s, i, i])
        assert pull.std() == pytest.approx(1.0, abs=0.05)
        assert abs(pull.mean()) < 3.5 / math.sqrt(n)
    # position pulls in the local frame (u = r phi, v = z)
    r = np.hypot(p[s, 0], p[s, 1])
    u = np.stack([-p[s, 1] / r, p[s, 0] / r, np.zeros(n)], 1)
    v = np.tile([0.0, 0.0, 1.0], (n, 1))
    for ax in (u, v):
        du = np.einsum("ni,ni->n", ax, d[s, :3])
        var = np.einsum("ni,nij,nj->n", ax, C[s][:, :3, :3], ax)
        pull = du / np.sqrt(var)
        assert pull.std() == pytest.approx(1.0, abs=0.05)


def test_straight_line_kf_equals_least_squares():
    """B = 0 and no material: the Kalman filter is the recursive form of the
    weighted least-squares fit (Fruhwirth 1987), up to the linearisation of
    the measurement map (second order in the 20-50 um residuals).  The
    least-squares fit here is independent: a straight line with 4 parameters
    (azimuth and z of its point on the last cylinder, direction phi and
    theta), residuals in the local (u, v, n) frame of each crossing, the
    start estimate as a prior on the point and direction at hit 1, solved by
    Gauss-Newton with numerical derivatives."""
    g0 = kfsynth.make_geometry(10, 4.0, 110.0, 120.0, x0=0.0)
    w = kfsynth.workload("fit1k", geometry=g0, bz=0.0, scatter=False)
    ev = kfsynth.generate(w, tracks_per_event=20)
    # a weak prior, so that its linearisation at the start estimate (the
    # one place where the filter and the batch fit differ) is negligible
    prior = (2.0, 0.5, 0.5, 0.5)
    p, C, c2, nd, ok = oracle.fit(ev, prior=prior)
    sig = np.array([20e-4, 50e-4, 10e-4])
    for t in range(6):
        hits = ev.trk_hits[ev.trk_offsets[t]:ev.trk_offsets[t + 1]]
        m = np.stack([ev.x[hits], ev.y[hits], ev.z[hits]], 1).astype(np.float64)
        R = g0.pos[ev.layer[hits]]
        RN = R[-1]
        est = oracle.seed_estimate(g0, 0.0, m[0], m[1], m[2])

        def line_point(q, Ri):
            a0, z0, ph, th = q
            P = np.array([RN * math.cos(a0), RN * math.sin(a0), z0])
            d = np.array([math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
            A = d[0] ** 2 + d[1] ** 2
            B = 2 * (P[0] * d[0] + P[1] * d[1])
            Cq = P[0] ** 2 + P[1] ** 2 - Ri * Ri
            l = (-B + math.sqrt(B * B - 4 * A * Cq)) / (2 * A)   # outgoing crossing
            return P + l * d

        def residuals(q):
            out = []
            for i in range(len(hits)):
                P = line_point(q, R[i])
                r = math.hypot(P[0], P[1])
                dm = m[i] - P
                out += [(-P[1] * dm[0] + P[0] * dm[1]) / r / sig[0], dm[2] / sig[1],
                        (P[0] * dm[0] + P[1] * dm[1]) / r / sig[2]]
            P1 = line_point(q, R[0])
            out += list((P1 - est[:3]) / prior[0])
            out += [((q[2] - est[4] + math.pi) % (2 * math.pi) - math.pi) / prior[2],
                    (q[3] - est[5]) / prior[3]]
            return np.array(out)

        q = np.array([math.atan2(m[-1, 1], m[-1, 0]), m[-1, 2], est[4], est[5]])
        for _ in range(8):
            r0 = residuals(q)
            Jm = np.zeros((r0.size, 4))
            for j in range(4):
                h = 1e-7
                a, b = q.copy(), q.copy()
                a[j] += h
                b[j] -= h
                Jm[:, j] = (residuals(a) - residuals(b)) / (2 * h)
            q = q + np.linalg.lstsq(Jm, -r0, rcond=None)[0]
        cov = np.linalg.inv(Jm.T @ Jm)
        sd = np.sqrt(np.diag(cov))
        x, y = p[t, 0], p[t, 1]
        r = math.hypot(x, y)
        kf = np.array([math.atan2(y, x), p[t, 2], p[t, 4], p[t, 5]])
        T = np.zeros((4, 6))
        T[0, 0], T[0, 1] = -y / r ** 2, x / r ** 2
        T[1, 2] = T[2, 4] = T[3, 5] = 1.0
        kcov = T @ C[t] @ T.T
        # the extended filter evaluates each transport Jacobian at its own
        # filtered state, the batch fit at the final estimate.  Across the
        # early states theta moves by ~5e-4 rad, changing dz/dtheta by ~1e-3
        # relative, applied to corrections ~20 final sigmas: a ~2e-2 sigma
        # difference.  A wrong or missing term would show at O(1) sigma.
        assert np.all(np.abs(kf - q) < 5e-2 * sd), (kf - q) / sd
        assert np.allclose(np.diag(kcov), np.diag(cov), rtol=1e-2)
        assert c2[t] == pytest.approx(np.sum(residuals(q) ** 2), rel=1e-2, abs=1e-2)


def test_information_form_update():
    """C+ from the gain form equals (C-^-1 + H^T V^-1 H)^-1 on the measured
    subspace (the two textbook forms of the update)."""
    g = _geom()
    layer = 9
    R = g.pos[layer]
    p = np.array([R * math.cos(0.7), R * math.sin(0.7), 12.0, 0.5, 0.75, 1.1])
    A = np.random.default_rng(1).standard_normal((6, 6)) * 0.01
    C = A @ A.T + np.diag([1e-4, 1e-4, 1e-4, 1e-4, 1e-5, 1e-5])
    m = p[:3] + np.array([-math.sin(0.7), math.cos(0.7), 0]) * 0.003 + np.array([0, 0, 0.004])
    p1, C1, c2 = oracle.update(g, layer, p, C, m)
    H3 = np.array([[-math.sin(0.7), math.cos(0.7), 0], [0, 0, 1], [math.cos(0.7), math.sin(0.7), 0]])
    H = np.zeros((3, 6))
    H[:, :3] = H3
    V = np.diag([g.su[layer] ** 2, g.sv[layer] ** 2, g.sn[layer] ** 2])
    Cinf = np.linalg.inv(np.linalg.inv(C) + H.T @ np.linalg.inv(V) @ H)
    assert np.allclose(C1, Cinf, rtol=1e-8, atol=1e-14)
    pinf = p + Cinf @ H.T @ np.linalg.inv(V) @ (H3 @ (m - p[:3]))
    assert np.allclose(p1, pinf, rtol=1e-10, atol=1e-12)


def test_hit_bins_contain_their_hits():
    ev = kfsynth.generate("build5k")
    g = ev.geometry
    b = oracle.bin_hits(g, 20, 128, ev.x, ev.y, ev.z, ev.layer)
    eb, pb = b // 128, b % 128
    x, y, z = ev.x.astype(np.float64), ev.y.astype(np.float64), ev.z.astype(np.float64)
    phi = np.arctan2(y, x)
    lo_phi = -np.pi + pb * (2 * np.pi / 128)
    assert np.all(phi >= lo_phi - 1e-12) and np.all(phi < lo_phi + 2 * np.pi / 128 + 1e-12)
    L = ev.layer
    bar = g.kind[L] == kfsynth.BARREL
    eta = np.where(bar, np.arcsinh(z / g.pos[L]), np.arcsinh(g.pos[L] / np.hypot(x, y)))
    e0 = np.where(bar, np.arcsinh(g.lo[L] / g.pos[L]),
                  np.minimum(np.arcsinh(g.pos[L] / g.hi[L]), np.arcsinh(g.pos[L] / g.lo[L])))
    e1 = np.where(bar, np.arcsinh(g.hi[L] / g.pos[L]),
                  np.maximum(np.arcsinh(g.pos[L] / g.hi[L]), np.arcsinh(g.pos[L] / g.lo[L])))
    w = (e1 - e0) / 20
    inside = (eta >= e0) & (eta <= e1)
    assert np.all(eta[inside] >= e0[inside] + eb[inside] * w[inside] - 1e-12)
    assert np.all(eta[inside] <= e0[inside] + (eb[inside] + 1) * w[inside] + 1e-12)
    assert np.all(eb[eta < e0] == 0) and np.all(eb[eta > e1] == 19)
    # every bin of the layer histogram adds up to the layer's hit count
    assert np.bincount(L, minlength=g.n_layers).sum() == b.size


def test_hit_bin_edge_cases():
    g = kfsynth.make_geometry(1, 10.0, 10.0, 100.0)
    # phi = pi wraps to bin 0; phi = -pi is bin 0; edges go to the upper bin
    x = np.array([-10.0, -10.0, 10.0, 0.0, 10.0], np.float32)
    y = np.array([0.0, -0.0, 0.0, 10.0, 0.0], np.float32)
    z = np.array([0.0, 0.0, 1e9, 0.0, -1e9], np.float32)
    b = oracle.bin_hits(g, 20, 128, x, y, z, np.zeros(5, np.int32))
    assert b[0] % 128 == 0                     # atan2(+0, -10) = pi -> wraps
    assert b[1] % 128 == 0                     # atan2(-0, -10) = -pi
    assert b[2] // 128 == 19 and b[4] // 128 == 0   # clamped in eta
    assert b[3] % 128 == 96                    # phi = pi/2: edge -> upper bin
    assert b[0] // 128 == 10                   # eta = 0 is the edge of bin 10
    # out-of-range layer id
    assert oracle.bin_hits(g, 20, 128, x[:1], y[:1], z[:1], np.array([5], np.int32))[0] == -1


@pytest.fixture(scope="module")
def build_event():
    return kfsynth.generate("build5k")


def _truth_cands(ev, n, step):
    """Candidate states taken from truth after the scatter at hit `step`,
    with a covariance typical of a track a few hits in."""
    sel = [t for t in range(ev.n_tracks) if ev.trk_offsets[t + 1] - ev.trk_offsets[t] > step + 1][:n]
    idx = ev.trk_offsets[sel] + step
    p = ev.trk_truth[idx].copy()
    lay = ev.layer[ev.trk_hits[idx]]
    C = np.zeros((len(sel), 6, 6))
    C[:, 0, 0] = C[:, 1, 1] = C[:, 2, 2] = (30e-4) ** 2
    C[:, 3, 3] = (0.02 * p[:, 3]) ** 2
    C[:, 4, 4] = C[:, 5, 5] = (2e-3) ** 2
    return np.asarray(sel), lay, p, C


def test_binned_compatibility_equals_brute_force(build_event):
    ev = build_event
    for step in (2, 5, 9):
        sel, lay, p, C = _truth_cands(ev, 300, step)
        a = oracle.step_compat(ev, 0, lay, p, C, brute=True)
        b = oracle.step_compat(ev, 0, lay, p, C, brute=False)
        assert np.array_equal(a[0], b[0])
        assert np.array_equal(a[3], b[3]) and np.array_equal(a[4], b[4])
        assert np.allclose(a[5], b[5], rtol=0, atol=0)
        assert a[4].size > 200


def test_navigation_matches_brute_force_crossings():
    """The two-candidate rule (next barrel outward, next disk ahead) reaches
    the surface that the generator found by brute force over every surface."""
    w = kfsynth.workload("build5k", ineff=0.0, noise_per_event=0, smear=False)
    ev = kfsynth.generate(w, tracks_per_event=400)
    g = ev.geometry
    n_checked = 0
    for t in range(ev.n_tracks):
        a, b = ev.trk_offsets[t], ev.trk_offsets[t + 1]
        hits = ev.trk_hits[a:b]
        for i in range(b - a - 1):
            st = ev.trk_truth[a + i]
            nxt = oracle.navigate(g, ev.bz, ev.layer[hits[i]], st)
            assert nxt == ev.layer[hits[i + 1]], (t, i)
            n_checked += 1
    assert n_checked > 4000


def test_gradient_reverse_equals_forward_and_finite_differences():
    w = kfsynth.workload("align200k")
    ev = kfsynth.generate(w, tracks_per_event=40)
    L = ev.geometry.n_layers
    al = np.zeros((L, 3))
    tot_f, g_f = oracle.fit_grad(ev, align=al, mode="forward")
    tot_r, g_r = oracle.fit_grad(ev, align=al, mode="reverse")
    assert tot_f == pytest.approx(tot_r, rel=1e-12)
    assert np.allclose(g_f, g_r, rtol=1e-9, atol=1e-9 * np.max(np.abs(g_f)))
    h = 1e-6
    base = al.reshape(-1)
    fd = np.zeros_like(g_f)
    for j in list(range(0, 3 * L, 4)) + [3 * L]:
        a, b = base.copy(), base.copy()
        fa = fb = 1.0
        if j < 3 * L:
            a[j] += h
            b[j] -= h
        else:
            fa, fb = 1 + h, 1 - h
        ca = oracle.fit(ev, align=a, fscale=fa)[2].sum()
        cb = oracle.fit(ev, align=b, fscale=fb)[2].sum()
        fd[j] = (ca - cb) / (2 * h)
        assert fd[j] == pytest.approx(g_r[j], rel=1e-4, abs=1e-4 * np.max(np.abs(g_r)))


def test_building_recovers_truth_on_clean_event():
    w = kfsynth.workload("build5k", ineff=0.0, noise_per_event=0)
    ev = kfsynth.generate(w, tracks_per_event=300)
    out = oracle.build_tracks(ev)
    n_ok = 0
    for t in range(ev.n_tracks):
        truth = list(ev.trk_hits[ev.trk_offsets[t]:ev.trk_offsets[t + 1]])
        best = [h for h in out["hits"][t, 0] if h != -3]
        found = [h for h in best if h >= 0]
        n_ok += found == truth
    assert n_ok / ev.n_tracks > 0.97


def test_building_efficiency_on_build5k(build_event):
    ev = build_event
    n = 400
    out = oracle.build_tracks(ev, seeds=ev.seeds[:n], seed_event=np.zeros(n, np.int32))
    eff = 0
    for t in range(n):
        best = out["hits"][t, 0]
        found = best[best >= 0]
        sim = ev.sim[found]
        # matched: more than 75% of the reconstructed hits from this track
        eff += np.mean(sim == t) > 0.75
    assert eff / n > 0.97
    st = out["stats"]
    assert st[0] > 10 * n and st[1] > 0 and st[2] > 0


def _truncated_event():
    """A noise-free build5k-like event in which 20 particles lose every hit
    after their sixth (those hits' layers set to -1: ignored)."""
    import dataclasses
    w = kfsynth.workload("build5k", noise_per_event=0, tracks_per_event=200, ineff=0.0)
    ev = kfsynth.generate(w)
    nrec = np.diff(ev.trk_offsets)
    cut = np.nonzero(nrec >= 12)[0][::3][:20]
    lay = ev.layer.copy()
    for t in cut:
        lay[ev.trk_hits[ev.trk_offsets[t] + 6: ev.trk_offsets[t + 1]]] = -1
    return ev, dataclasses.replace(ev, layer=lay), cut


def test_short_candidates_are_preserved():
    """Abstract and Sec. 3: short candidates are kept rather than extended
    over many layers.  Reading 11's stop child: a candidate that reaches
    the hole limit keeps its state and stays in the seed's top-K.  A track
    cut after six hits must come out as its six hits and max_holes holes,
    not be dropped or replaced by a longer fake."""
    ev, ev2, cut = _truncated_event()
    o = oracle.build_tracks(ev2, max_hits=48)
    exact = 0
    for t in cut:
        truth = ev.trk_hits[ev.trk_offsets[t]: ev.trk_offsets[t] + 6]
        row = o["hits"][t, 0]
        assert o["n"][t] >= 1
        np.testing.assert_array_equal(row[:6], truth)
        exact += (o["nhits"][t, 0] == 6 and row[6:9].tolist() == [-1, -1, -1] and (row[9:] == -3).all())
    # the rest picked up a hit of another particle after a hole or two
    assert exact >= 0.9 * len(cut), exact


def test_non_finite_hits_are_not_indexed():
    """A hit with a NaN or infinite coordinate has no place on its layer:
    no bin, never compatible, a seed that uses it gives no candidate, a fit
    that uses it fails; every other result is unchanged."""
    g = kfsynth.make_geometry(1, 10.0, 10.0, 100.0)
    nan, inf = np.float32("nan"), np.float32("inf")
    x = np.array([nan, 1.0, 10.0, -inf, 10.0], np.float32)
    y = np.array([0.0, inf, 0.0, 0.0, 0.0], np.float32)
    z = np.array([0.0, 0.0, nan, 0.0, 0.0], np.float32)
    b = oracle.bin_hits(g, 20, 128, x, y, z, np.zeros(5, np.int32))
    assert list(b[:4]) == [-1, -1, -1, -1] and b[4] >= 0
    ev = kfsynth.generate("build5k", tracks_per_event=300)
    ref = oracle.build_tracks(ev, max_hits=48)
    bad = ev.trk_hits[ev.trk_offsets[5] + 4]          # a hit of track 5 after its seed
    seedhit = ev.seeds[7, 1]                          # a seed hit of track 7
    noise = np.nonzero(ev.sim < 0)[0][:50]            # some noise hits
    ev.x = ev.x.copy()
    ev.y = ev.y.copy()
    ev.x[[bad, seedhit]] = np.nan
    ev.y[noise] = np.inf
    out = oracle.build_tracks(ev, max_hits=48)
    assert out["n"][7] == 0
    used = out["hits"][out["hits"] >= 0]
    assert not np.isin(used, [bad, seedhit, *noise]).any()
    # seeds whose candidates never met a changed hit are untouched
    touched = np.isin(ref["hits"], [bad, seedhit, *noise]).any(axis=(1, 2))
    same = ~touched
    same[7] = False
    assert np.array_equal(out["hits"][same], ref["hits"][same])
    p, C, c2, nd, ok = oracle.fit(ev)
    assert not ok[5] and not ok[7] and ok.sum() >= ev.n_tracks - 2 - 10


def _python_recover(ev, layer, p, C, h1, cut):
    """Reading 18 written out: the hits of the layer with an index above h1
    whose chi2 against the updated state (p, C) is below the cut, by brute
    force over the layer's hits (the update's chi2 is that of its pair);
    the best by (chi2, index), or None."""
    best = None
    for h in np.nonzero(ev.layer == layer)[0]:
        if h <= h1:
            continue
        m = np.array([ev.x[h], ev.y[h], ev.z[h]], np.float64)
        _, _, x2 = oracle.update(ev.geometry, layer, p, C, m)
        if x2 is not None and x2 < cut and (best is None or (x2, h) < best):
            best = (x2, int(h))
    return best


def _python_beam(ev, seed, K, max_holes, cut, prior, overlap=False, score=None):
    """Reading 11 written out in Python over the oracle's per-step
    primitives (step_compat: navigation, prediction and the compatible hits;
    update: the Kalman update): every child of every candidate is listed,
    and the K best are taken by a heap selection on the ranking key (hits
    desc, holes asc, chi2 asc, parent asc, hit index asc with holes and
    stops last), independent of the oracle's own sort-and-truncate."""
    import heapq
    p, C, c2, ok = oracle.seed_states(ev, seeds=np.asarray([seed], np.int32), prior=prior)
    if not ok[0]:
        return []
    beam = [dict(p=p[0], C=C[0], chi2=c2[0], layer=int(ev.layer[seed[2]]), nh=3, nho=0, consec=0,
                 done=False, hits=[int(h) for h in seed])]
    for _ in range(64):
        if all(c["done"] for c in beam):
            break
        kids, pred = [], {}
        for slot, c in enumerate(beam):
            stop = (slot, -2, c["nh"], c["nho"], c["chi2"])
            if c["done"]:
                kids.append(stop)
                continue
            nl, p1, C1, off, ph, pc = oracle.step_compat(ev, 0, [c["layer"]], c["p"][None], c["C"][None],
                                                         chi2_cut=cut)
            if nl[0] < 0:
                kids.append(stop)
                continue
            pred[slot] = (int(nl[0]), p1[0], C1[0])
            n0 = len(kids)
            for h, x2 in zip(ph[off[0]:off[1]], pc[off[0]:off[1]]):
                kids.append((slot, int(h), c["nh"] + 1, c["nho"], c["chi2"] + x2))
            if c["consec"] < max_holes:
                kids.append((slot, -1, c["nh"], c["nho"] + 1, c["chi2"]))
            if len(kids) == n0:
                kids.append(stop)
        if score is None:
            best = heapq.nsmallest(K, kids, key=lambda k: (-k[2], k[3], k[4], k[0], k[1] % (1 << 32)))
        else:
            wh, wm, wc = score
            best = heapq.nsmallest(K, kids, key=lambda k: (-(wh * k[2] - wm * k[3] - wc * k[4]), k[0],
                                                           k[1] % (1 << 32)))
        nb = []
        for parent, hit, nh, nho, x2 in best:
            c = dict(beam[parent])
            c["hits"] = list(c["hits"])
            if hit == -2:
                c["done"] = True
            else:
                nl, p1, C1 = pred[parent]
                c["layer"] = nl
                if hit >= 0:
                    m = np.array([ev.x[hit], ev.y[hit], ev.z[hit]], np.float64)
                    c["p"], c["C"], _ = oracle.update(ev.geometry, nl, p1, C1, m)
                    c.update(nh=nh, consec=0, chi2=x2)
                    c["hits"].append(hit)
                    rec = _python_recover(ev, nl, c["p"], c["C"], hit, cut) if overlap else None
                    if rec is not None:
                        m2 = np.array([ev.x[rec[1]], ev.y[rec[1]], ev.z[rec[1]]], np.float64)
                        c["p"], c["C"], _ = oracle.update(ev.geometry, nl, c["p"], c["C"], m2)
                        c.update(nh=c["nh"] + 1, chi2=c["chi2"] + rec[0])
                        c["hits"].append(rec[1])
                else:
                    c.update(p=p1, C=C1, nho=nho, consec=c["consec"] + 1)
                    c["hits"].append(-1)
            nb.append(c)
        beam = nb
    return beam


def _beam_event(ineff, dup):
    """A small build5k-like event (60 tracks, 3000 noise hits); with dup,
    exact copies of 40 hits of the first tracks (not their seed hits)
    appended, so that children of one parent tie in chi2 (broken by hit
    index) and twin candidates make children of different parents tie
    (broken by parent slot)."""
    import dataclasses
    w = kfsynth.workload("build5k", tracks_per_event=60, noise_per_event=3000, ineff=ineff)
    ev = kfsynth.generate(w)
    if dup:
        src = np.concatenate([ev.trk_hits[ev.trk_offsets[t] + 3:ev.trk_offsets[t + 1]] for t in range(12)])[:40]
        cat = lambda a: np.concatenate([a, a[src]])  # noqa: E731
        ev = dataclasses.replace(ev, x=cat(ev.x), y=cat(ev.y), z=cat(ev.z), layer=cat(ev.layer), sim=cat(ev.sim),
                                 event_offsets=np.array([0, ev.n_hits + len(src)], np.int32))
    return ev


@pytest.mark.parametrize("K,ineff,max_holes,dup", [(1, 0.01, 3, False), (3, 0.01, 3, False), (6, 0.01, 3, False),
                                                   (40, 0.01, 3, False), (6, 0.3, 1, False), (4, 0.3, 2, True),
                                                   (6, 0.01, 3, True)])
def test_beam_search_matches_heap_selection(K, ineff, max_holes, dup):
    """The oracle's building (sort of all children, truncate to K) against
    the Python beam of _python_beam: the same candidates, in the same order,
    with the same hit lists, counts, chi2 and states, for K from 1 (greedy)
    to 40 (no child dropped on these seeds), with many holes against a low
    hole limit, and with exact ties (duplicated hits)."""
    ev = _beam_event(ineff, dup)
    w = ev.workload
    prior = oracle.DEFAULT_PRIOR
    seeds = ev.seeds[:12]
    o = oracle.build_tracks(ev, seeds=seeds, seed_event=np.zeros(len(seeds), np.int32), max_cands=K,
                            max_holes=max_holes, max_hits=64, prior=prior)
    for i, s in enumerate(seeds):
        ref = _python_beam(ev, s, K, max_holes, w.chi2_cut, prior)
        assert o["n"][i] == len(ref)
        for j, c in enumerate(ref):
            row = o["hits"][i, j]
            assert row[:len(c["hits"])].tolist() == c["hits"] and (row[len(c["hits"]):] == -3).all()
            assert o["nhits"][i, j] == c["nh"] and o["nholes"][i, j] == c["nho"]
            assert abs(o["chi2"][i, j] - c["chi2"]) <= 1e-9 * max(1.0, abs(c["chi2"]))
            np.testing.assert_allclose(o["p"][i, j], c["p"], rtol=1e-12, atol=1e-12)


def _overlap_event(frac, noise, tracks=60):
    w = kfsynth.workload("overlap5k", tracks_per_event=tracks, noise_per_event=noise, overlap_frac=frac)
    return kfsynth.generate(w)


@pytest.mark.parametrize("K", [2, 6])
def test_overlap_recovery_matches_python_beam(K):
    """Reading 18 (overlap recovery) in the oracle against the Python beam
    with the recovery written out by brute force over the layer's hits:
    the same candidates, hit lists (the recovered hit right after the one it
    joins), counts, chi2 and states."""
    ev = _overlap_event(0.5, 2000)
    w = ev.workload
    prior = oracle.DEFAULT_PRIOR
    seeds = ev.seeds[:10]
    o = oracle.build_tracks(ev, seeds=seeds, seed_event=np.zeros(len(seeds), np.int32), max_cands=K,
                            max_hits=64, prior=prior, overlap=True)
    recovered = 0
    for i, s in enumerate(seeds):
        ref = _python_beam(ev, s, K, w.max_holes, w.chi2_cut, prior, overlap=True)
        assert o["n"][i] == len(ref)
        for j, c in enumerate(ref):
            row = o["hits"][i, j]
            assert row[:len(c["hits"])].tolist() == c["hits"] and (row[len(c["hits"]):] == -3).all()
            assert o["nhits"][i, j] == c["nh"] and o["nholes"][i, j] == c["nho"]
            assert abs(o["chi2"][i, j] - c["chi2"]) <= 1e-9 * max(1.0, abs(c["chi2"]))
            np.testing.assert_allclose(o["p"][i, j], c["p"], rtol=1e-12, atol=1e-12)
        hl = o["hits"][i, 0]
        hl = hl[hl >= 0]
        recovered += int(np.sum(ev.layer[hl][1:] == ev.layer[hl][:-1]))
    assert recovered > 10  # the recovery did take hits


def test_overlap_recovery_finds_the_second_hits():
    """On a noise-free event where every crossing leaves two hits, the best
    candidate of a seed holds both hits of almost every layer of its
    particle after the seed layers (a seed is three hits on three layers;
    recovery follows the search); without the recovery it holds one per
    layer."""
    ev = _overlap_event(1.0, 0, tracks=200)
    n = ev.n_tracks
    on = oracle.build_tracks(ev, max_hits=64, overlap=True)
    off = oracle.build_tracks(ev, max_hits=64, overlap=False)
    full = 0
    for t in range(n):
        seed_layers = set(ev.layer[ev.seeds[t]].tolist())
        truth = set(h for h in ev.trk_hits[ev.trk_offsets[t]:ev.trk_offsets[t + 1]].tolist()
                    if ev.layer[h] not in seed_layers or h in ev.seeds[t])
        got = on["hits"][t, 0]
        got = set(got[got >= 0].tolist())
        full += got == truth
        one = off["hits"][t, 0]
        one = one[one >= 0]
        assert len(set(ev.layer[one].tolist())) == len(one)  # one hit per layer
    assert full >= 0.9 * n, full
    assert on["nhits"][:, 0].sum() > 1.8 * off["nhits"][:, 0].sum()


@pytest.mark.parametrize("score", [(10.0, 10.0, 1.0), (10.0, 2.0, 0.5)])
def test_score_ranking_matches_python_beam(score):
    """Reading 19 (score ranking) in the oracle against the Python beam whose
    heap selection ranks by the score written out: same candidates, order,
    lists, counts, chi2 and states."""
    w = kfsynth.workload("build5k", tracks_per_event=60, noise_per_event=6000, ineff=0.1)
    ev = kfsynth.generate(w)
    prior = oracle.DEFAULT_PRIOR
    seeds = ev.seeds[:12]
    o = oracle.build_tracks(ev, seeds=seeds, seed_event=np.zeros(len(seeds), np.int32), max_hits=64, prior=prior,
                            score=score)
    for i, s in enumerate(seeds):
        ref = _python_beam(ev, s, w.max_cands, w.max_holes, w.chi2_cut, prior, score=score)
        assert o["n"][i] == len(ref)
        for j, c in enumerate(ref):
            row = o["hits"][i, j]
            assert row[:len(c["hits"])].tolist() == c["hits"] and (row[len(c["hits"]):] == -3).all()
            assert o["nhits"][i, j] == c["nh"] and o["nholes"][i, j] == c["nho"]
            np.testing.assert_allclose(o["p"][i, j], c["p"], rtol=1e-12, atol=1e-12)


def _truncated_noisy_event(noise):
    """A build5k-like event with `noise` noise hits in which 80 particles
    lose every hit after their sixth (their layers set to -1)."""
    import dataclasses
    w = kfsynth.workload("build5k", tracks_per_event=600, noise_per_event=noise)
    ev = kfsynth.generate(w)
    nrec = np.diff(ev.trk_offsets)
    cut = np.nonzero(nrec >= 12)[0][::4][:80]
    lay = ev.layer.copy()
    for t in cut:
        lay[ev.trk_hits[ev.trk_offsets[t] + 6: ev.trk_offsets[t + 1]]] = -1
    return ev, dataclasses.replace(ev, layer=lay), cut


def short_track_scores(ev, o, cut):
    """Fraction of the cut particles whose best candidate is exactly their
    six hits (then holes), and the matched fraction (> 75 % of the hits
    from the particle) of the other particles."""
    exact = 0
    for t in cut:
        truth = ev.trk_hits[ev.trk_offsets[t]: ev.trk_offsets[t] + 6]
        row = o["hits"][t, 0]
        exact += bool(np.array_equal(row[:6], truth) and (row[6:] < 0).all() and o["nhits"][t, 0] == 6)
    others = np.setdiff1d(np.arange(ev.n_tracks), cut)
    matched = 0
    for t in others:
        b = o["hits"][t, 0]
        f = b[b >= 0]
        matched += bool(f.size and np.mean(ev.sim[f] == t) > 0.75)
    return exact / len(cut), matched / len(others)


def test_score_ranking_keeps_short_tracks_in_dense_events():
    """Sec. 3: re-tuning the score recovered short tracks.  In an event with
    300k noise hits, particles cut after six hits come out exactly as their
    six hits far more often under the score ranking (10 per hit, 10 per
    hole, 1 per chi2 unit: a noise hit of chi2 above 10 lowers a
    candidate's score, so a finished short track beats its fake
    continuations) than under the key ranking (hits first), and the other
    particles are found no less often."""
    ev, ev2, cut = _truncated_noisy_event(300000)
    o_key = oracle.build_tracks(ev2, max_hits=48)
    o_sc = oracle.build_tracks(ev2, max_hits=48, score=(10.0, 10.0, 1.0))
    ek, mk = short_track_scores(ev, o_key, cut)
    es, ms = short_track_scores(ev, o_sc, cut)
    print(f"short exact: key {ek:.3f}, score {es:.3f}; others matched: key {mk:.4f}, score {ms:.4f}")
    assert es >= ek + 0.08
    assert ms >= mk
