// Device math of the Kalman step for gfx950: helix transport, surface
// crossing, surface-constrained transport Jacobian, multiple-scattering
// noise, 3x3 chi2 and the Kalman update.
//
// Paper: arXiv 2002.06295.  Sec. 1 defines the Kalman filter as a
// propagation of the track state (parameters and uncertainties) to the next
// layer, material effects included, followed by an update with the hit's
// position; Sec. 2 collapses barrel layers to a radius and forward layers to
// a z position and works with 3D hit positions.  Numerical readings (state
// parameters, field direction, local measurement frame, Highland noise)
// follow the Kalman filter of Fruhwirth (1987), the paper's KF reference.
//
// Precision plan.  The covariance algebra, the Jacobian and the chi2 run in
// FP32 with the covariance packed (21 floats, lower triangle).  The state's
// position and azimuth are carried in FP64, and the few operations that
// decide where a track meets a surface and how far a hit lies from it (the
// crossing equation, the displacement sum, the residual) run in FP64: on
// CDNA the FP64 vector rate equals the unpacked FP32 rate, so these ~40
// operations per step cost what 40 FP32 operations would, while an FP32
// position at 100 cm (ulp 7.6e-6 cm) would already be ~2e-3 of the 20 um hit
// resolution.
//
// Units: cm, GeV, T, rad.  State p = (x, y, z, k = q/pT, phi, theta).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define KFX_HD __host__ __device__ inline

namespace kfx {

constexpr double kPi = 3.14159265358979323846;
constexpr double kHcD = 0.299792458e-2;  // pT [GeV] = kHc * B [T] * rho [cm]
constexpr float kHc = (float)kHcD;
constexpr int kBarrel = 0;
constexpr int kDisk = 1;
constexpr int kMaxLayers = 64;
constexpr int kNavGrid = 256;  // cells of the navigation lookup grids

// Packed symmetric 6x6: element (i, j), i >= j, lives at i(i+1)/2 + j.
KFX_HD constexpr int sidx(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

struct Layer {
  int kind;        // kBarrel / kDisk
  int side;        // disks: +1 / -1 (z sign); barrel: 0
  double pos;      // R (barrel) or Z (disk)
  double lo, hi;   // z bounds (barrel) or r bounds (disk)
  double eta_lo, eta_hi;  // pseudorapidity range of the layer's hit bins
  float eta_scale;        // eta bins per unit of eta (n_eta / range)
  float x0;        // thickness in radiation lengths
  float v_u, v_v, v_n;    // hit variances along the local u, v, n axes
};

// Geometry as one device block: layers plus the navigation order.
struct Geometry {
  Layer L[kMaxLayers];
  int n_layers;
  int n_barrel, n_dpos, n_dneg;
  int barrel[kMaxLayers];   // barrel ids, increasing radius
  int dpos[kMaxLayers];     // +z disks, increasing z
  int dneg[kMaxLayers];     // -z disks, decreasing z
  int next_barrel[kMaxLayers];  // for a barrel layer: the next one out (-1)
  int brank[kMaxLayers];        // rank of a barrel layer by radius (disks: -1)
  int drank[kMaxLayers];        // rank of a disk within its side (barrel: -1)
  double bz;
  int n_eta, n_phi;
  // navigation tables (filled by nav_tables from the lists above): barrel
  // radii by rank, |Z| of the disks of each side (0: +z, 1: -z) by rank, and
  // for each a coarse grid giving, per cell of width 1 / ginv, the number of
  // entries at or below the cell's start (a first guess for nav_count)
  double bR[kMaxLayers];
  double dA[2][kMaxLayers];
  float ginv[3];
  unsigned char grid[3][kNavGrid];
};

// The lookup tables of the navigation, from the sorted barrel and disk
// lists (host side, once per geometry).
inline void nav_tables(Geometry& G) {
  const int n[3] = {G.n_barrel, G.n_dpos, G.n_dneg};
  for (int i = 0; i < kMaxLayers; ++i) G.drank[i] = -1;
  for (int i = 0; i < G.n_barrel; ++i) G.bR[i] = G.L[G.barrel[i]].pos;
  for (int i = 0; i < G.n_dpos; ++i) {
    G.dA[0][i] = G.L[G.dpos[i]].pos;
    G.drank[G.dpos[i]] = i;
  }
  for (int i = 0; i < G.n_dneg; ++i) {
    G.dA[1][i] = -G.L[G.dneg[i]].pos;
    G.drank[G.dneg[i]] = i;
  }
  for (int t = 0; t < 3; ++t) {
    const double* a = t == 0 ? G.bR : G.dA[t - 1];
    const double top = n[t] > 0 ? a[n[t] - 1] : 1.0;
    G.ginv[t] = (float)((kNavGrid - 1) / (top > 0.0 ? 1.01 * top : 1.0));
    for (int b = 0; b < kNavGrid; ++b) {
      const double w = b / (double)G.ginv[t];
      int c = 0;
      while (c < n[t] && a[c] <= w) ++c;
      G.grid[t][b] = (unsigned char)c;
    }
  }
}

// Number of entries of the ascending table a[0..n) that are <= w, exactly:
// the grid cell gives a first guess, which is then moved up or down.
KFX_HD int nav_count(const Geometry& G, int t, const double* a, int n, double w) {
  const float f = (float)w * G.ginv[t];
  const int b = f > 0.0f ? (f < (float)(kNavGrid - 1) ? (int)f : kNavGrid - 1) : 0;
  int c = G.grid[t][b];
  c = c < n ? c : n;
  while (c < n && a[c] <= w) ++c;
  while (c > 0 && a[c - 1] > w) --c;
  return c;
}

// Track parameters in FP64, covariance in R (FP32 on the hot path).
template <class R>
struct StateT {
  double x, y, z, k, phi, th;
  R C[21];  // covariance of (x, y, z, k, phi, theta), packed
};
using State = StateT<float>;

template <class A, class B>
KFX_HD void convert_state(const StateT<A>& a, StateT<B>& b) {
  b.x = a.x; b.y = a.y; b.z = a.z; b.k = a.k; b.phi = a.phi; b.th = a.th;
#pragma unroll
  for (int i = 0; i < 21; ++i) b.C[i] = (B)a.C[i];
}

// scalar math for float and double
KFX_HD float msqrt(float x) { return sqrtf(x); }
KFX_HD double msqrt(double x) { return sqrt(x); }
KFX_HD float mabs(float x) { return fabsf(x); }
KFX_HD double mabs(double x) { return fabs(x); }
KFX_HD float mlog(float x) { return logf(x); }
KFX_HD double mlog(double x) { return log(x); }
KFX_HD float mmax(float a, float b) { return fmaxf(a, b); }
KFX_HD double mmax(double a, double b) { return fmax(a, b); }

// sin and cos of an FP64 angle (the azimuth, the polar angle and the
// turning angle of a step are all below 8 in magnitude).  Cody-Waite
// reduction by pi/2 with a two-part constant: the fma rounds x - q pi/2_hi
// once, and the constant's missing part (~1e-33 q) stays far below FP64
// rounding of the reduced argument for |x| < 1e9.  Then the Taylor series of
// sin and cos on [-pi/4, pi/4] to the terms r^17 and r^16, whose truncation
// error (< 1e-17) is below FP64 rounding.  A non-finite argument gives NaN.
KFX_HD void sincos_d(double x, double& s, double& c) {
  constexpr double kPio2Hi = 1.5707963267948966;      // nearest double to pi/2
  constexpr double kPio2Lo = 6.123233995736766e-17;   // pi/2 - kPio2Hi
  constexpr double k2Opi = 0.6366197723675814;        // 2/pi
  const double q = rint(x * k2Opi);
  const double r = fma(-q, kPio2Lo, fma(-q, kPio2Hi, x));
  const double y = r * r, y2 = y * y, y4 = y2 * y2;
  // sin r = r + r y P(y), P(y) = -1/3! + y/5! - ... + y^7/17!; cos r = 1 +
  // y Q(y), Q(y) = -1/2! + y/4! - ... + y^7/16!.  Both evaluated by
  // Estrin's scheme (pairs, then pairs of pairs) rather than Horner's: a
  // dependent chain of about four multiply-adds instead of eight, which is
  // what the step's latency sees.
  const double ps = fma(y4, fma(y2, fma(y, 1.0 / 355687428096000.0, -1.0 / 1307674368000.0),
                                fma(y, 1.0 / 6227020800.0, -1.0 / 39916800.0)),
                        fma(y2, fma(y, 1.0 / 362880.0, -1.0 / 5040.0), fma(y, 1.0 / 120.0, -1.0 / 6.0)));
  const double sr = fma(ps * y, r, r);
  const double pc = fma(y4, fma(y2, fma(y, 1.0 / 20922789888000.0, -1.0 / 87178291200.0),
                                fma(y, 1.0 / 479001600.0, -1.0 / 3628800.0)),
                        fma(y2, fma(y, 1.0 / 40320.0, -1.0 / 720.0), fma(y, 1.0 / 24.0, -0.5)));
  const double cr = fma(pc, y, 1.0);
  // quadrant q mod 4 (|q| < 2^31 here, two's complement): odd quadrants
  // swap sine and cosine, quadrants 2 and 3 negate the sine, 1 and 2 the
  // cosine; selects rather than branches
  const int qi = (int)q & 3;
  const double a = (qi & 1) ? cr : sr, b = (qi & 1) ? sr : cr;
  s = (qi & 2) ? -a : a;
  c = ((qi + 1) & 2) ? -b : b;
}

KFX_HD double wrap_pi(double a) {  // to (-pi, pi]
  if (a > kPi) a -= 2.0 * kPi;
  if (a <= -kPi) a += 2.0 * kPi;
  return a;
}

// sin(a)/a and its derivative (cos a - sin(a)/a)/a, with series near 0.
template <class R>
KFX_HD void sinc_d(R a, R sa, R ca, R& sinc, R& dsinc) {
  if (mabs(a) < (R)1e-3) {
    const R a2 = a * a;
    sinc = (R)1 - a2 * (R)(1.0 / 6.0) + a2 * a2 * (R)(1.0 / 120.0);
    dsinc = a * ((R)(-1.0 / 3.0) + a2 * (R)(1.0 / 30.0));
  } else {
    const R ia = (R)1 / a;
    sinc = sa * ia;
    dsinc = (ca - sinc) * ia;
  }
}

// Half turning angle a = omega s / 2 of a step with its sine, cosine, sinc
// and sinc derivative in R (the Jacobian's precision).
template <class R>
struct ChordT {
  R a, sa, ca, sinc, dsinc;
  double dx, dy;
};

// Displacement after a transverse path s on a helix that starts with
// direction (cphi, sphi) and turns at omega = d(phi)/ds: a chord of length
// s sinc(a) at angle phi0 + a, a = omega s / 2, stable at omega -> 0; in
// FP64 with the direction at the end.  The crossing point and the residuals
// are computed from it.
struct ChordD {
  double a, sa, ca;   // half turning angle and its sine/cosine
  double dx, dy;      // displacement
  double c1, s1;      // direction (cos, sin) at the end
};

KFX_HD ChordD chord_d(double s, double omega, double cphi, double sphi) {
  ChordD c;
  c.a = 0.5 * omega * s;
  sincos_d(c.a, c.sa, c.ca);
  double sinc;
  if (fabs(c.a) < 1e-4) {
    const double a2 = c.a * c.a;
    sinc = 1.0 - a2 * (1.0 / 6.0) + a2 * a2 * (1.0 / 120.0);
  } else {
    sinc = c.sa / c.a;
  }
  const double L = s * sinc;
  const double dpar = L * c.ca, dperp = L * c.sa;
  c.dx = cphi * dpar - sphi * dperp;
  c.dy = sphi * dpar + cphi * dperp;
  const double c2a = 1.0 - 2.0 * c.sa * c.sa, s2a = 2.0 * c.sa * c.ca;
  c.c1 = cphi * c2a - sphi * s2a;
  c.s1 = sphi * c2a + cphi * s2a;
  return c;
}

// Outgoing crossing of the cylinder of radius Rc in closed form (FP64).
// With the half turning angle a = omega s / 2, the helix point is
// P(a) = P0 + (2 sin a / omega) (cos(phi0 + a), sin(phi0 + a)); writing
// t = tan a = k tau with k = omega / 2 turns |P|^2 = Rc^2 into
//   alpha tau^2 + 2 D tau + c0 = 0,
//   c0 = |P0|^2 - Rc^2 < 0, D = P0 . u, E = P0 . u_perp,
//   alpha = 1 + 2 k E + k^2 c0,
// (u the start direction, u_perp it turned by +90 degrees; alpha = 1 is the
// straight line).  The crossing on the outgoing arc, before the turning
// point, is the smallest positive root, tau = c0 / (-D - sqrt(D^2 -
// alpha c0)) in cancellation-free form, and s = atan(k tau) / k.  |a| stays
// below pi/2 on that arc, so a single branch of atan covers it.  Returns
// the transverse path, or a negative value when the track moves inward or
// never reaches the cylinder.
template <class R>
KFX_HD double path_to_cylinder(const StateT<R>& st, double cphi, double sphi, double omega, double Rc) {
  const double c0 = fma(st.x, st.x, fma(st.y, st.y, -Rc * Rc));
  const double D = st.x * cphi + st.y * sphi;
  if (!(c0 < 0.0) || !(D >= 0.0)) return -1.0;
  const double E = st.y * cphi - st.x * sphi;
  const double k = 0.5 * omega;
  const double alpha = fma(k, fma(k, c0, 2.0 * E), 1.0);
  const double disc = fma(D, D, -alpha * c0);
  if (!(disc >= 0.0)) return -1.0;
  const double tau = c0 / (-D - sqrt(disc));
  const double x = k * tau;
  double s;
  if (fabs(x) < 0.25) {
    // atan(x)/x = sum (-1)^n x^2n / (2n + 1), to the x^24 term: the
    // truncation (< 1e-17 for |x| < 0.25) is below FP64 rounding
    // (Estrin's scheme over u = x^2: pairs of terms, then pairs of pairs)
    const double u = x * x, u2 = u * u, u4 = u2 * u2, u8 = u4 * u4;
    const double b0 = fma(u2, fma(u, -1.0 / 7.0, 1.0 / 5.0), fma(u, -1.0 / 3.0, 1.0));       // u^0..3
    const double b1 = fma(u2, fma(u, -1.0 / 15.0, 1.0 / 13.0), fma(u, -1.0 / 11.0, 1.0 / 9.0));  // u^4..7
    const double b2 = fma(u2, fma(u, -1.0 / 23.0, 1.0 / 21.0), fma(u, -1.0 / 19.0, 1.0 / 17.0));  // u^8..11
    const double p = fma(u8, fma(u4, 1.0 / 25.0, b2), fma(u4, b1, b0));
    s = tau * p;
  } else {
    s = atan(x) / k;
  }
  return s > 0.0 ? s : -1.0;
}

// Plane z = Z: s = (Z - z0) tan(theta), ahead of the track (FP64).
template <class R>
KFX_HD double path_to_disk(const StateT<R>& st, double Z, double sth, double cth) {
  if (fabs(cth) < 1e-12) return -1.0;
  const double s = (Z - st.z) * (sth / cth);
  return s > 1e-12 ? s : -1.0;
}

template <class R>
KFX_HD double path_to_disk(const StateT<R>& st, double Z) {
  double sth, cth;
  sincos_d(st.th, sth, cth);
  return path_to_disk(st, Z, sth, cth);
}

// Path to the surface of a layer (barrel radius r_surf, possibly aligned).
template <class R>
KFX_HD double path_to_layer(const StateT<R>& st, const Layer& Ld, double r_surf, double cphi, double sphi,
                            double omega_d) {
  return Ld.kind == kBarrel ? path_to_cylinder(st, cphi, sphi, omega_d, r_surf) : path_to_disk(st, Ld.pos);
}

// Navigation: the next surface is the nearer of the next barrel layer
// outward (when its outgoing crossing lies within |z| <= zmax) and the
// first disk ahead in z whose crossing lies within [rmin, rmax] while the
// track still moves outward.  Returns the layer id (or -1) and its path.
KFX_HD int navigate(const Geometry& G, int cur, const State& st, double cphi, double sphi, double sth,
                    double cth, double omega_d, double& s_out) {
  double best = 3.0e38;
  int bl = -1;
  int nb = -1;
  s_out = best;
  // a state that is not finite goes nowhere (comparisons with NaN are false)
  if (!__builtin_isfinite(st.x) || !__builtin_isfinite(st.y) || !__builtin_isfinite(st.z) || !__builtin_isfinite(st.phi) || !__builtin_isfinite(st.th) ||
      !__builtin_isfinite(st.k) || !__builtin_isfinite(omega_d))
    return -1;
  const Layer& Lc = G.L[cur];
  if (Lc.kind == kBarrel) {
    nb = G.next_barrel[cur];
  } else {
    // the first barrel layer with a radius above the state's
    const double r = sqrt(st.x * st.x + st.y * st.y);
    const int rk = nav_count(G, 0, G.bR, G.n_barrel, r);
    nb = rk < G.n_barrel ? G.barrel[rk] : -1;
  }
  if (nb >= 0) {
    const double s = path_to_cylinder(st, cphi, sphi, omega_d, G.L[nb].pos);
    if (s > 0.0) {
      const double z = st.z + s * (cth / sth);
      if (fabs(z) <= G.L[nb].hi) {
        best = s;
        bl = nb;
      }
    }
  }
  if (fabs(cth) > 1e-12) {
    const bool fwd = cth > 0.0;
    const int n = fwd ? G.n_dpos : G.n_dneg;
    const int* dl = fwd ? G.dpos : G.dneg;
    const double* dA = G.dA[fwd ? 0 : 1];
    const double tanth = sth / cth;
    // the disks of this side ordered along the motion; the ones at or
    // behind the state's z are skipped at once, and so is the current disk
    const int crank = (Lc.kind == kDisk && (Lc.pos > 0.0) == fwd) ? G.drank[cur] : -1;
    for (int i = nav_count(G, fwd ? 1 : 2, dA, n, fwd ? st.z : -st.z); i < n; ++i) {
      if (i == crank) continue;
      const double Z = fwd ? dA[i] : -dA[i];
      const double s = (Z - st.z) * tanth;  // as path_to_disk
      if (!(s > 1e-12)) continue;
      // the disks ahead come in order of path length: once one is no nearer
      // than the barrel crossing, none after it can be either
      if (!(s < best)) break;
      const int id = dl[i];
      const float lo = (float)G.L[id].lo, hi = (float)G.L[id].hi;
      {
        // FP32 estimate of the crossing: a disk that the track clearly
        // leaves radially, or clearly passes inside of while still moving
        // outward, is decided without the FP64 chord; anything within the
        // margin (far above the FP32 error) takes the exact path below
        const float s32 = (float)s;
        const float a32 = 0.5f * (float)omega_d * s32;
        if (fabsf(a32) < 0.5f) {
          // Taylor series on |a| < 0.5 (truncation below 1e-8)
          const float a2 = a32 * a32;
          const float sinc = 1.0f + a2 * (-1.0f / 6.0f + a2 * (1.0f / 120.0f + a2 * (-1.0f / 5040.0f)));
          const float sa = a32 * sinc;
          const float ca = 1.0f + a2 * (-0.5f + a2 * (1.0f / 24.0f + a2 * (-1.0f / 720.0f + a2 * (1.0f / 40320.0f))));
          const float L = s32 * sinc;
          const float cp = (float)cphi, sp = (float)sphi;
          const float cps = cp * ca - sp * sa, sps = sp * ca + cp * sa;
          const float x = (float)st.x + L * cps, y = (float)st.y + L * sps;
          const float c1 = cps * ca - sps * sa, s1 = sps * ca + cps * sa;
          const float r = sqrtf(x * x + y * y);
          const float tol = 1e-3f * s32 + 1e-2f;
          if (r > hi + tol) break;                                         // left radially
          if (r < lo - tol && x * c1 + y * s1 > tol * (r + 1.0f)) continue;  // passes inside
        }
      }
      const ChordD c = chord_d(s, omega_d, cphi, sphi);
      const double x = st.x + c.dx, y = st.y + c.dy;
      if (x * c.c1 + y * c.s1 < 0.0) break;  // turned before reaching it
      const double r = sqrt(x * x + y * y);
      if (r > G.L[id].hi) break;          // left radially
      if (r < G.L[id].lo) continue;       // passes inside the disk
      if (s < best) {
        best = s;
        bl = id;
      }
      break;
    }
  }
  s_out = best;
  return bl;
}

// The same with sin and cos of the polar angle computed here.
KFX_HD int navigate(const Geometry& G, int cur, const State& st, double cphi, double sphi, double omega_d,
                    double& s_out) {
  double sth, cth;
  sincos_d(st.th, sth, cth);
  return navigate(G, cur, st, cphi, sphi, sth, cth, omega_d, s_out);
}

// Multiple scattering at a layer for a state on it (Highland, beta = 1,
// no energy loss): var(theta) = th0^2, var(phi) = th0^2 / sin^2(theta),
// and k = q/(|p| sin theta) follows theta at fixed |p|.
template <class R>
KFX_HD void add_noise(StateT<R>& st, const Layer& Ld, R sth, R cth, R cinc) {
  if (!(Ld.x0 > 0.0f)) return;
  cinc = mmax(cinc, (R)1e-3);
  const R t = (R)Ld.x0 / cinc;
  const R k = (R)st.k;
  const R th0 = (R)0.0136 * mabs(k) * sth * msqrt(t) * ((R)1 + (R)0.038 * mlog(t));
  const R var = th0 * th0;
  const R isth = (R)1 / sth;
  const R cot = cth * isth;
  st.C[sidx(4, 4)] += var * (isth * isth);
  st.C[sidx(5, 5)] += var;
  st.C[sidx(3, 3)] += k * k * cot * cot * var;
  st.C[sidx(5, 3)] += -k * cot * var;
}

// Unit vector along (x, y) in the precision of R: for FP32 from the
// coordinates rounded to FP32 (a result that is rounded to FP32 anyway
// needs no FP64 square root and division, which are long dependent chains
// on the GPU), for FP64 in FP64.
KFX_HD void unit_xy(double x, double y, float& c, float& s) {
  const float xf = (float)x, yf = (float)y;
  const float ir = 1.0f / sqrtf(xf * xf + yf * yf);
  c = xf * ir;
  s = yf * ir;
}
KFX_HD void unit_xy(double x, double y, double& c, double& s) {
  const double ir = 1.0 / sqrt(x * x + y * y);
  c = x * ir;
  s = y * ir;
}

// Transport (p, C) over transverse path s to the surface of layer Ld
// (barrel radius possibly aligned): new parameters, C- = J C J^T + Q with
// the surface-constrained Jacobian J = A + b c^T, where A = dF/dp at fixed
// s, b = dF/ds and c = ds/dp from the surface equation.  Written as
// C- = A C A^T + b u^T + u b^T + sigma b b^T, u = A C c, sigma = c^T C c,
// which exploits the unit rows of A (k and theta) and needs no branch
// between barrel and disk except in c.
template <class R>
KFX_HD void transport(const StateT<R>& in, const Layer& Ld, double cphi, double sphi, double sth_d, double cth_d,
                      double s_d, double kappa_d, StateT<R>& out) {
  const double omega_d = kappa_d * in.k;
  const ChordD cd = chord_d(s_d, omega_d, cphi, sphi);
  const bool disk = Ld.kind == kDisk;
  out.x = in.x + cd.dx;
  out.y = in.y + cd.dy;
  out.z = disk ? Ld.pos : in.z + s_d * (cth_d / sth_d);
  out.phi = wrap_pi(in.phi + 2.0 * cd.a);
  out.k = in.k;
  out.th = in.th;
  // Jacobian and noise in R from the rounded geometry
  const R s = (R)s_d, kappa = (R)kappa_d, omega = (R)omega_d;
  const R sth = (R)sth_d, cth = (R)cth_d;
  const R isth = (R)1 / sth;
  const R cot = cth * isth;
  ChordT<R> c;
  c.a = (R)cd.a;
  c.sa = (R)cd.sa;
  c.ca = (R)cd.ca;
  sinc_d(c.a, c.sa, c.ca, c.sinc, c.dsinc);
  // direction at the middle of the chord (psi) and at the end (phi1)
  const R cpsi = (R)(cphi * cd.ca - sphi * cd.sa);
  const R spsi = (R)(sphi * cd.ca + cphi * cd.sa);
  const R c1 = (R)cd.c1, s1 = (R)cd.s1;
  const R dxf = (R)cd.dx, dyf = (R)cd.dy;
  // A: free-helix partials at fixed s
  const R hs2 = (R)0.5 * kappa * s * s;
  const R Axk = hs2 * (c.dsinc * cpsi - c.sinc * spsi);
  const R Ayk = hs2 * (c.dsinc * spsi + c.sinc * cpsi);
  const R Axp = -dyf, Ayp = dxf;
  const R Azt = -s * (isth * isth);
  const R Apk = kappa * s;
  // c = ds/dp from the surface equation
  R cv[6];
  if (disk) {
    cv[0] = (R)0; cv[1] = (R)0; cv[3] = (R)0; cv[4] = (R)0;
    const R icth = (R)1 / cth;
    cv[2] = -sth * icth;
    cv[5] = s * (isth * icth);
  } else {
    const R x1 = (R)out.x, y1 = (R)out.y;
    const R iDn = (R)-1 / (x1 * c1 + y1 * s1);
    cv[0] = x1 * iDn;
    cv[1] = y1 * iDn;
    cv[2] = (R)0;
    cv[3] = (x1 * Axk + y1 * Ayk) * iDn;
    cv[4] = (x1 * Axp + y1 * Ayp) * iDn;
    cv[5] = (R)0;
  }
  const R* C = in.C;
  // v = C c
  R v[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    R acc = (R)0;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += C[sidx(i, j)] * cv[j];
    v[i] = acc;
  }
  R sig = (R)0;
#pragma unroll
  for (int i = 0; i < 6; ++i) sig += cv[i] * v[i];
  // u = A v
  R u[6];
  u[0] = v[0] + Axk * v[3] + Axp * v[4];
  u[1] = v[1] + Ayk * v[3] + Ayp * v[4];
  u[2] = v[2] + Azt * v[5];
  u[3] = v[3];
  u[4] = v[4] + Apk * v[3];
  u[5] = v[5];
  // M = C A^T (column j = C a_j)
  R M[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const R ck = C[sidx(i, 3)], cp = C[sidx(i, 4)], ct = C[sidx(i, 5)];
    M[i][0] = C[sidx(i, 0)] + Axk * ck + Axp * cp;
    M[i][1] = C[sidx(i, 1)] + Ayk * ck + Ayp * cp;
    M[i][2] = C[sidx(i, 2)] + Azt * ct;
    M[i][3] = ck;
    M[i][4] = cp + Apk * ck;
    M[i][5] = ct;
  }
  // N = A M, then the rank terms
  R N[6][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    N[0][j] = M[0][j] + Axk * M[3][j] + Axp * M[4][j];
    N[1][j] = M[1][j] + Ayk * M[3][j] + Ayp * M[4][j];
    N[2][j] = M[2][j] + Azt * M[5][j];
    N[3][j] = M[3][j];
    N[4][j] = M[4][j] + Apk * M[3][j];
    N[5][j] = M[5][j];
  }
  const R bv[6] = {c1, s1, cot, (R)0, omega, (R)0};
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      out.C[sidx(i, j)] = N[i][j] + bv[i] * u[j] + u[i] * bv[j] + sig * bv[i] * bv[j];
  // unit radius vector at the destination (barrel: the surface normal)
  R e0_n = (R)0, e1_n = (R)0;
  if (disk) {
    // the z row of J is identically zero on a plane
#pragma unroll
    for (int j = 0; j < 6; ++j) out.C[sidx(2, j)] = (R)0;
  } else {
    // n^T J_pos = 0 on the cylinder, so C- has no variance along the normal
    // e = (x, y, 0)/r.  Rounding leaves some; at a steep crossing it rivals
    // sigma_n^2 in S.  Apply P C P^T with P = I - e e^T (an identity in exact
    // arithmetic): C' = C - e w^T - w e^T + (e^T C e) e e^T, w = C e.
    R e0, e1;
    unit_xy(out.x, out.y, e0, e1);
    e0_n = e0;
    e1_n = e1;
    R w[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) w[j] = e0 * out.C[sidx(0, j)] + e1 * out.C[sidx(1, j)];
    const R sg = e0 * w[0] + e1 * w[1];
    const R ev[6] = {e0, e1, (R)0, (R)0, (R)0, (R)0};
#pragma unroll
    for (int i = 0; i < 6; ++i)
#pragma unroll
      for (int j = 0; j <= i; ++j)
        if (i < 2 || j < 2) out.C[sidx(i, j)] += -ev[i] * w[j] - w[i] * ev[j] + sg * ev[i] * ev[j];
  }
  // multiple scattering at the destination
  R cinc;
  if (disk) {
    cinc = mabs(cth);
  } else {
    // cosine of the incidence angle: sin(theta) times the transverse
    // direction's component along the radius (e0, e1)
    cinc = mabs(sth * (e0_n * c1 + e1_n * s1));
  }
  add_noise(out, Ld, sth, cth, cinc);
}

// The same with sin and cos of the polar angle computed here.
template <class R>
KFX_HD void transport(const StateT<R>& in, const Layer& Ld, double cphi, double sphi, double s_d, double kappa_d,
                      StateT<R>& out) {
  double sth_d, cth_d;
  sincos_d(in.th, sth_d, cth_d);
  transport(in, Ld, cphi, sphi, sth_d, cth_d, s_d, kappa_d, out);
}

// Measurement frame at a predicted state: rows u, v, n of H (acting on the
// position), H C and S^-1 for S = H C H^T + V (packed 3x3).
template <class R>
struct FrameT {
  R h[3][3];
  R Si[6];   // (0,0) (1,0) (1,1) (2,0) (2,1) (2,2)
  R S[6];
  R HC[3][6];
};
using Frame = FrameT<float>;

template <class R>
KFX_HD void make_frame(const StateT<R>& st, const Layer& Ld, FrameT<R>& F) {
  R c, s;
  unit_xy(st.x, st.y, c, s);
  const bool disk = Ld.kind == kDisk;
  const R z0 = (R)0, o1 = (R)1;
  F.h[0][0] = -s; F.h[0][1] = c; F.h[0][2] = z0;
  F.h[1][0] = disk ? c : z0; F.h[1][1] = disk ? s : z0; F.h[1][2] = disk ? z0 : o1;
  F.h[2][0] = disk ? z0 : c; F.h[2][1] = disk ? z0 : s; F.h[2][2] = disk ? o1 : z0;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      F.HC[a][j] = F.h[a][0] * st.C[sidx(0, j)] + F.h[a][1] * st.C[sidx(1, j)] + F.h[a][2] * st.C[sidx(2, j)];
  const R V[3] = {(R)Ld.v_u, (R)Ld.v_v, (R)Ld.v_n};
  R S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      const R acc = F.HC[a][0] * F.h[b][0] + F.HC[a][1] * F.h[b][1] + F.HC[a][2] * F.h[b][2];
      S[a][b] = acc + (a == b ? V[a] : z0);
      S[b][a] = S[a][b];
    }
  F.S[0] = S[0][0]; F.S[1] = S[1][0]; F.S[2] = S[1][1];
  F.S[3] = S[2][0]; F.S[4] = S[2][1]; F.S[5] = S[2][2];
  const R c00 = S[1][1] * S[2][2] - S[1][2] * S[2][1];
  const R c01 = S[1][2] * S[2][0] - S[1][0] * S[2][2];
  const R c02 = S[1][0] * S[2][1] - S[1][1] * S[2][0];
  const R id = o1 / (S[0][0] * c00 + S[0][1] * c01 + S[0][2] * c02);
  F.Si[0] = c00 * id;
  F.Si[1] = c01 * id;
  F.Si[2] = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) * id;
  F.Si[3] = c02 * id;
  F.Si[4] = (S[0][1] * S[2][0] - S[0][0] * S[2][1]) * id;
  F.Si[5] = (S[0][0] * S[1][1] - S[0][1] * S[1][0]) * id;
}

// Residual r = H (m - x) with the difference taken in FP64.
template <class R>
KFX_HD void residual(const StateT<R>& st, const FrameT<R>& F, double mx, double my, double mz, R r[3]) {
  const R dx = (R)(mx - st.x), dy = (R)(my - st.y), dz = (R)(mz - st.z);
#pragma unroll
  for (int a = 0; a < 3; ++a) r[a] = F.h[a][0] * dx + F.h[a][1] * dy + F.h[a][2] * dz;
}

template <class R>
KFX_HD R chi2_of(const FrameT<R>& F, const R r[3]) {
  return r[0] * r[0] * F.Si[0] + r[1] * r[1] * F.Si[2] + r[2] * r[2] * F.Si[5] +
         (R)2 * (r[0] * r[1] * F.Si[1] + r[0] * r[2] * F.Si[3] + r[1] * r[2] * F.Si[4]);
}

// Kalman update (gain form): K = C H^T S^-1, p += K r, C -= K H C.
template <class R>
KFX_HD R kf_update(StateT<R>& st, const FrameT<R>& F, double mx, double my, double mz) {
  R r[3];
  residual(st, F, mx, my, mz, r);
  const R chi2 = chi2_of(F, r);
  const R Si[3][3] = {{F.Si[0], F.Si[1], F.Si[3]}, {F.Si[1], F.Si[2], F.Si[4]}, {F.Si[3], F.Si[4], F.Si[5]}};
  R K[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) K[i][b] = F.HC[0][i] * Si[0][b] + F.HC[1][i] * Si[1][b] + F.HC[2][i] * Si[2][b];
  R dp[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) dp[i] = K[i][0] * r[0] + K[i][1] * r[1] + K[i][2] * r[2];
  st.x += (double)dp[0];
  st.y += (double)dp[1];
  st.z += (double)dp[2];
  st.k += (double)dp[3];
  st.phi = wrap_pi(st.phi + (double)dp[4]);
  st.th += (double)dp[5];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      st.C[sidx(i, j)] -= K[i][0] * F.HC[0][j] + K[i][1] * F.HC[1][j] + K[i][2] * F.HC[2][j];
  return chi2;
}

// The update of an FP32 state carried out in FP64.  C+ = C - K H C keeps
// the fraction V/(H C H^T + V) of the predicted variance along the measured
// directions; at a steep crossing that ratio reaches 1e-4 or less, and the
// FP32 subtraction would keep only a few correct digits.  H C, S^-1, the
// gain and C+ are formed in FP64 from the FP32 covariance and rounded once;
// the gain is formed one row at a time so that it is never held whole.
KFX_HD float kf_update_fp64(State& st, const Layer& Ld, double mx, double my, double mz) {
  const double r = sqrt(st.x * st.x + st.y * st.y);
  const double c = st.x / r, s = st.y / r;
  const bool disk = Ld.kind == kDisk;
  // rows of H: u = (-s, c, 0); v = (0, 0, 1) or (c, s, 0); n = (c, s, 0) or (0, 0, 1)
  double HC[3][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const double cx = st.C[sidx(0, j)], cy = st.C[sidx(1, j)], cz = st.C[sidx(2, j)];
    const double rad = c * cx + s * cy;
    HC[0][j] = -s * cx + c * cy;
    HC[1][j] = disk ? rad : cz;
    HC[2][j] = disk ? cz : rad;
  }
  // S = H C H^T + V: (H C H^T)[a][b] = HC[a] . h_b
  const double S00 = -s * HC[0][0] + c * HC[0][1] + (double)Ld.v_u;
  const double S10 = -s * HC[1][0] + c * HC[1][1];
  const double S20 = -s * HC[2][0] + c * HC[2][1];
  const double S11 = (disk ? c * HC[1][0] + s * HC[1][1] : HC[1][2]) + (double)Ld.v_v;
  const double S21 = disk ? c * HC[2][0] + s * HC[2][1] : HC[2][2];
  const double S22 = (disk ? HC[2][2] : c * HC[2][0] + s * HC[2][1]) + (double)Ld.v_n;
  const double c00 = S11 * S22 - S21 * S21;
  const double c01 = S21 * S20 - S10 * S22;
  const double c02 = S10 * S21 - S11 * S20;
  const double id = 1.0 / (S00 * c00 + S10 * c01 + S20 * c02);
  const double Si00 = c00 * id, Si10 = c01 * id, Si20 = c02 * id;
  const double Si11 = (S00 * S22 - S20 * S20) * id;
  const double Si21 = (S10 * S20 - S00 * S21) * id;
  const double Si22 = (S00 * S11 - S10 * S10) * id;
  // residual
  const double dx = mx - st.x, dy = my - st.y, dz = mz - st.z;
  const double ru = -s * dx + c * dy;
  const double rrad = c * dx + s * dy;
  const double rv = disk ? rrad : dz, rn = disk ? dz : rrad;
  const double w0 = Si00 * ru + Si10 * rv + Si20 * rn;
  const double w1 = Si10 * ru + Si11 * rv + Si21 * rn;
  const double w2 = Si20 * ru + Si21 * rv + Si22 * rn;
  const double chi2 = ru * w0 + rv * w1 + rn * w2;
  // K[i] = HC[.][i]^T S^-1; p_i += K[i] . r; C[i][j] -= K[i] . HC[.][j]
  double dp[6];
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    const double k0 = HC[0][i] * Si00 + HC[1][i] * Si10 + HC[2][i] * Si20;
    const double k1 = HC[0][i] * Si10 + HC[1][i] * Si11 + HC[2][i] * Si21;
    const double k2 = HC[0][i] * Si20 + HC[1][i] * Si21 + HC[2][i] * Si22;
    dp[i] = k0 * ru + k1 * rv + k2 * rn;
#pragma unroll
    for (int j = 0; j <= i; ++j)
      st.C[sidx(i, j)] = (float)((double)st.C[sidx(i, j)] - (k0 * HC[0][j] + k1 * HC[1][j] + k2 * HC[2][j]));
  }
  st.x += dp[0];
  st.y += dp[1];
  st.z += dp[2];
  st.k += dp[3];
  st.phi = wrap_pi(st.phi + dp[4]);
  st.th += dp[5];
  return (float)chi2;
}

// Prior covariance of the start estimate: diagonal (sigma_pos^2 x3,
// (sk_rel |k|)^2, sigma_phi^2, sigma_theta^2).
struct Prior {
  float spos, sk_rel, sphi, stheta;
};

template <class R>
KFX_HD void prior_cov(const Prior& pr, StateT<R>& st) {
#pragma unroll
  for (int i = 0; i < 21; ++i) st.C[i] = (R)0;
  st.C[sidx(0, 0)] = st.C[sidx(1, 1)] = st.C[sidx(2, 2)] = (R)pr.spos * (R)pr.spos;
  const R sk = (R)pr.sk_rel * (R)fabs(st.k);
  st.C[sidx(3, 3)] = sk * sk;
  st.C[sidx(4, 4)] = (R)pr.sphi * (R)pr.sphi;
  st.C[sidx(5, 5)] = (R)pr.stheta * (R)pr.stheta;
}

// Material noise of a layer added to a state sitting on it (the first hit,
// where there is no transport).
template <class R>
KFX_HD void add_material(StateT<R>& st, const Layer& Ld) {
  double sth_d, cth_d, sphi_d, cphi_d;
  sincos_d(st.th, sth_d, cth_d);
  sincos_d(st.phi, sphi_d, cphi_d);
  const R sth = (R)sth_d, cth = (R)cth_d;
  R cinc;
  if (Ld.kind == kDisk) {
    cinc = mabs(cth);
  } else {
    const double r = sqrt(st.x * st.x + st.y * st.y);
    cinc = mabs(sth * (R)((st.x * cphi_d + st.y * sphi_d) / r));
  }
  add_noise(st, Ld, sth, cth, cinc);
}

// Start estimate from three hits (FP64): signed curvature of the circle
// through the transverse points (omega = 2 cross / product of the sides),
// phi = tangent at hit 1 = chord direction minus half the turning angle,
// cot(theta) = dz / arc(1 -> 3).  Position = hit 1.  Without a field, or
// for three points on one line, the start is the straight line along the
// chord 1 -> 3 with k = 0.
template <class R>
KFX_HD void seed_estimate(double bz, const double m1[3], const double m2[3], const double m3[3],
                          StateT<R>& st) {
  const double ax = m2[0] - m1[0], ay = m2[1] - m1[1];
  const double bx = m3[0] - m1[0], by = m3[1] - m1[1];
  const double cx = m3[0] - m2[0], cy = m3[1] - m2[1];
  const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by), lc = sqrt(cx * cx + cy * cy);
  const double cr = ax * by - ay * bx;
  st.x = m1[0];
  st.y = m1[1];
  st.z = m1[2];
  if (bz == 0.0 || fabs(2.0 * cr) < 1e-300) {
    st.k = 0.0;
    st.phi = atan2(by, bx);
    st.th = atan2(lb, m3[2] - m1[2]);
    return;
  }
  const double omega = 2.0 * cr / (la * lb * lc);
  st.k = bz == 0.0 ? 0.0 : -omega / (kHcD * bz);
  // turning angle over the chord 1->2 is 2 asin(omega |P2-P1| / 2)
  const double half12 = asin(fmin(1.0, fmax(-1.0, 0.5 * omega * la)));
  st.phi = wrap_pi(atan2(ay, ax) - half12);
  const double half13 = asin(fmin(1.0, fmax(-1.0, 0.5 * omega * lb)));
  const double s13 = fabs(omega) > 0.0 ? 2.0 * half13 / omega : lb;
  st.th = atan2(s13, m3[2] - m1[2]);
}

}  // namespace kfx
