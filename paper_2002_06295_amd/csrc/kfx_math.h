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
constexpr float kHc = 0.299792458e-2f;  // pT [GeV] = kHc * B [T] * rho [cm]
constexpr int kBarrel = 0;
constexpr int kDisk = 1;
constexpr int kMaxLayers = 64;

// Packed symmetric 6x6: element (i, j), i >= j, lives at i(i+1)/2 + j.
KFX_HD constexpr int sidx(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

struct Layer {
  int kind;        // kBarrel / kDisk
  int side;        // disks: +1 / -1 (z sign); barrel: 0
  double pos;      // R (barrel) or Z (disk)
  double lo, hi;   // z bounds (barrel) or r bounds (disk)
  double eta_lo, eta_hi;  // pseudorapidity range of the layer's hit bins
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
  double bz;
  int n_eta, n_phi;
};

struct State {
  double x, y, z, phi;
  float k, th;
  float C[21];
};

KFX_HD double wrap_pi(double a) {  // to (-pi, pi]
  if (a > kPi) a -= 2.0 * kPi;
  if (a <= -kPi) a += 2.0 * kPi;
  return a;
}

// sin(a)/a and its derivative (cos a - sin(a)/a)/a, with series near 0.
KFX_HD void sinc_d(float a, float sa, float ca, float& sinc, float& dsinc) {
  if (fabsf(a) < 1e-3f) {
    float a2 = a * a;
    sinc = 1.0f - a2 * (1.0f / 6.0f) + a2 * a2 * (1.0f / 120.0f);
    dsinc = a * (-1.0f / 3.0f + a2 * (1.0f / 30.0f));
  } else {
    float ia = 1.0f / a;
    sinc = sa * ia;
    dsinc = (ca - sinc) * ia;
  }
}

// Displacement after a transverse path s on a helix that starts with
// direction (cphi, sphi) and turns at omega = d(phi)/ds: a chord of length
// s sinc(a) at angle phi0 + a, a = omega s / 2.  Stable at omega -> 0.
struct Chord {
  float a, sa, ca, sinc, dsinc;
  double dx, dy;
};

KFX_HD Chord chord(float s, float omega, double cphi, double sphi) {
  Chord c;
  c.a = 0.5f * omega * s;
  c.sa = sinf(c.a);
  c.ca = cosf(c.a);
  sinc_d(c.a, c.sa, c.ca, c.sinc, c.dsinc);
  float L = s * c.sinc;
  double dpar = (double)(L * c.ca), dperp = (double)(L * c.sa);
  c.dx = cphi * dpar - sphi * dperp;
  c.dy = sphi * dpar + cphi * dperp;
  return c;
}

// Outgoing crossing of the cylinder of radius R.  The start must lie inside
// it and move outward.  Newton on g(s) = |P(s)|^2 - R^2, with g evaluated
// relative to the start in FP64, from the straight-line root.  Returns the
// transverse path, or a negative value when there is no outgoing crossing.
KFX_HD float path_to_cylinder(const State& st, double cphi, double sphi, float omega, double R) {
  double c0 = st.x * st.x + st.y * st.y - R * R;
  double Dd = st.x * cphi + st.y * sphi;
  if (!(c0 < 0.0) || Dd < 0.0) return -1.0f;
  float D = (float)Dd;
  float s = (float)(-c0) / (D + sqrtf(D * D - (float)c0));
  bool conv = false;
  for (int it = 0; it < 12; ++it) {
    Chord c = chord(s, omega, cphi, sphi);
    double g = c0 + 2.0 * (st.x * c.dx + st.y * c.dy) + (c.dx * c.dx + c.dy * c.dy);
    // direction at s: phi0 + 2a
    float c2a = c.ca * c.ca - c.sa * c.sa, s2a = 2.0f * c.sa * c.ca;
    double c1 = cphi * c2a - sphi * s2a, s1 = sphi * c2a + cphi * s2a;
    float gp = 2.0f * (float)((st.x + c.dx) * c1 + (st.y + c.dy) * s1);
    if (!(gp > 0.0f)) return -1.0f;
    float ds = (float)g / gp;
    s -= ds;
    if (fabsf(ds) <= 2e-7f * fabsf(s) + 1e-9f) {
      conv = true;
      break;
    }
  }
  if (!conv || !(s > 0.0f)) return -1.0f;
  // moving outward at the crossing
  Chord c = chord(s, omega, cphi, sphi);
  float c2a = c.ca * c.ca - c.sa * c.sa, s2a = 2.0f * c.sa * c.ca;
  double c1 = cphi * c2a - sphi * s2a, s1 = sphi * c2a + cphi * s2a;
  if ((st.x + c.dx) * c1 + (st.y + c.dy) * s1 < 0.0) return -1.0f;
  return s;
}

// Plane z = Z: s = (Z - z0) tan(theta), ahead of the track.
KFX_HD float path_to_disk(const State& st, double Z) {
  float sth = sinf(st.th), cth = cosf(st.th);
  if (fabsf(cth) < 1e-12f) return -1.0f;
  float s = (float)(Z - st.z) * (sth / cth);
  return s > 1e-12f ? s : -1.0f;
}

// Navigation: the next surface is the nearer of the next barrel layer
// outward (when its outgoing crossing lies within |z| <= zmax) and the
// first disk ahead in z whose crossing lies within [rmin, rmax] while the
// track still moves outward.  Returns the layer id (or -1) and its path.
KFX_HD int navigate(const Geometry& G, int cur, const State& st, double cphi, double sphi,
                    float omega, float& s_out) {
  float best = 3.0e38f;
  int bl = -1;
  int nb = -1;
  const Layer& Lc = G.L[cur];
  if (Lc.kind == kBarrel) {
    nb = G.next_barrel[cur];
  } else {
    double r = sqrt(st.x * st.x + st.y * st.y);
    for (int i = 0; i < G.n_barrel; ++i)
      if (G.L[G.barrel[i]].pos > r) {
        nb = G.barrel[i];
        break;
      }
  }
  if (nb >= 0) {
    float s = path_to_cylinder(st, cphi, sphi, omega, G.L[nb].pos);
    if (s > 0.0f) {
      double z = st.z + (double)(s * (cosf(st.th) / sinf(st.th)));
      if (fabs(z) <= G.L[nb].hi) {
        best = s;
        bl = nb;
      }
    }
  }
  float cth = cosf(st.th);
  if (fabsf(cth) > 1e-12f) {
    bool fwd = cth > 0.0f;
    int n = fwd ? G.n_dpos : G.n_dneg;
    const int* dl = fwd ? G.dpos : G.dneg;
    for (int i = 0; i < n; ++i) {
      int id = dl[i];
      if (id == cur) continue;
      double Z = G.L[id].pos;
      if (fwd ? (Z <= st.z) : (Z >= st.z)) continue;
      float s = path_to_disk(st, Z);
      if (!(s > 0.0f)) continue;
      Chord c = chord(s, omega, cphi, sphi);
      double x = st.x + c.dx, y = st.y + c.dy;
      float c2a = c.ca * c.ca - c.sa * c.sa, s2a = 2.0f * c.sa * c.ca;
      double c1 = cphi * c2a - sphi * s2a, s1 = sphi * c2a + cphi * s2a;
      if (x * c1 + y * s1 < 0.0) break;  // turned before reaching it
      double r = sqrt(x * x + y * y);
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

// Transport (p, C) over transverse path s to the surface of layer Ld
// (barrel radius Rsurf, possibly aligned): new parameters, C- = J C J^T + Q
// with the surface-constrained Jacobian J = A + b c^T, where A = dF/dp at
// fixed s, b = dF/ds and c = ds/dp from the surface equation.  Written as
// C- = A C A^T + b u^T + u b^T + sigma b b^T, u = A C c, sigma = c^T C c,
// which exploits the unit rows of A (k and theta) and needs no branch
// between barrel and disk except in c.
KFX_HD void transport(const State& in, const Layer& Ld, double cphi, double sphi, float s,
                      float kappa, State& out) {
  const float k = in.k, th = in.th;
  const float omega = kappa * k;
  Chord c = chord(s, omega, cphi, sphi);
  const float sth = sinf(th), cth = cosf(th);
  const float cot = cth / sth;
  const bool disk = Ld.kind == kDisk;
  out.x = in.x + c.dx;
  out.y = in.y + c.dy;
  out.z = disk ? Ld.pos : in.z + (double)(s * cot);
  out.phi = wrap_pi(in.phi + (double)(2.0f * c.a));
  out.k = k;
  out.th = th;
  // direction at the middle of the chord (psi) and at the end (phi1)
  const float cpsi = (float)(cphi * c.ca - sphi * c.sa), spsi = (float)(sphi * c.ca + cphi * c.sa);
  const float c2a = c.ca * c.ca - c.sa * c.sa, s2a = 2.0f * c.sa * c.ca;
  const float c1 = (float)(cphi * c2a - sphi * s2a), s1 = (float)(sphi * c2a + cphi * s2a);
  const float dxf = (float)c.dx, dyf = (float)c.dy;
  // A: free-helix partials at fixed s
  const float hs2 = 0.5f * kappa * s * s;
  const float Axk = hs2 * (c.dsinc * cpsi - c.sinc * spsi);
  const float Ayk = hs2 * (c.dsinc * spsi + c.sinc * cpsi);
  const float Axp = -dyf, Ayp = dxf;
  const float Azt = -s / (sth * sth);
  const float Apk = kappa * s;
  // b = dF/ds
  const float b0 = c1, b1 = s1, b2 = cot, b4 = omega;
  // c = ds/dp from the surface equation
  float cv[6];
  if (disk) {
    cv[0] = 0.0f; cv[1] = 0.0f; cv[3] = 0.0f; cv[4] = 0.0f;
    cv[2] = -sth / cth;
    cv[5] = s / (sth * cth);
  } else {
    const float x1 = (float)out.x, y1 = (float)out.y;
    const float iDn = -1.0f / (x1 * c1 + y1 * s1);
    cv[0] = x1 * iDn;
    cv[1] = y1 * iDn;
    cv[2] = 0.0f;
    cv[3] = (x1 * Axk + y1 * Ayk) * iDn;
    cv[4] = (x1 * Axp + y1 * Ayp) * iDn;
    cv[5] = 0.0f;
  }
  const float* C = in.C;
  // v = C c
  float v[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += C[sidx(i, j)] * cv[j];
    v[i] = acc;
  }
  float sig = 0.0f;
#pragma unroll
  for (int i = 0; i < 6; ++i) sig += cv[i] * v[i];
  // u = A v
  float u[6];
  u[0] = v[0] + Axk * v[3] + Axp * v[4];
  u[1] = v[1] + Ayk * v[3] + Ayp * v[4];
  u[2] = v[2] + Azt * v[5];
  u[3] = v[3];
  u[4] = v[4] + Apk * v[3];
  u[5] = v[5];
  // M = C A^T (column j = C a_j), full 6x6
  float M[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    const float ck = C[sidx(i, 3)], cp = C[sidx(i, 4)], ct = C[sidx(i, 5)];
    M[i][0] = C[sidx(i, 0)] + Axk * ck + Axp * cp;
    M[i][1] = C[sidx(i, 1)] + Ayk * ck + Ayp * cp;
    M[i][2] = C[sidx(i, 2)] + Azt * ct;
    M[i][3] = ck;
    M[i][4] = cp + Apk * ck;
    M[i][5] = ct;
  }
  // N = A M (lower triangle), then the rank terms and Q
  float N[6][6];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    N[0][j] = M[0][j] + Axk * M[3][j] + Axp * M[4][j];
    N[1][j] = M[1][j] + Ayk * M[3][j] + Ayp * M[4][j];
    N[2][j] = M[2][j] + Azt * M[5][j];
    N[3][j] = M[3][j];
    N[4][j] = M[4][j] + Apk * M[3][j];
    N[5][j] = M[5][j];
  }
  const float bv[6] = {b0, b1, b2, 0.0f, b4, 0.0f};
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      out.C[sidx(i, j)] = N[i][j] + bv[i] * u[j] + u[i] * bv[j] + sig * bv[i] * bv[j];
  if (disk) {
    // the z row of J is identically zero on a plane
#pragma unroll
    for (int j = 0; j < 6; ++j) out.C[sidx(2, j)] = 0.0f;
  }
  // multiple scattering at the destination (Highland, beta = 1)
  if (Ld.x0 > 0.0f) {
    float cinc;
    if (disk) {
      cinc = fabsf(cth);
    } else {
      const float x1 = (float)out.x, y1 = (float)out.y;
      cinc = fabsf(sth * (x1 * c1 + y1 * s1) * rsqrtf(x1 * x1 + y1 * y1));
    }
    cinc = fmaxf(cinc, 1e-3f);
    const float t = Ld.x0 / cinc;
    const float th0 = 0.0136f * fabsf(k) * sth * sqrtf(t) * (1.0f + 0.038f * logf(t));
    const float var = th0 * th0;
    out.C[sidx(4, 4)] += var / (sth * sth);
    out.C[sidx(5, 5)] += var;
    out.C[sidx(3, 3)] += k * k * cot * cot * var;
    out.C[sidx(5, 3)] += -k * cot * var;
  }
}

// Measurement frame at a predicted state: rows u, v, n of H (acting on the
// position), and S^-1 for S = H C H^T + V (packed 3x3).
struct Frame {
  float h[3][3];
  float Si[6];   // (0,0) (1,0) (1,1) (2,0) (2,1) (2,2)
  float S[6];
  float HC[3][6];
};

KFX_HD void make_frame(const State& st, const Layer& Ld, Frame& F) {
  const double r = sqrt(st.x * st.x + st.y * st.y);
  const float c = (float)(st.x / r), s = (float)(st.y / r);
  const bool disk = Ld.kind == kDisk;
  F.h[0][0] = -s; F.h[0][1] = c; F.h[0][2] = 0.0f;
  F.h[1][0] = disk ? c : 0.0f; F.h[1][1] = disk ? s : 0.0f; F.h[1][2] = disk ? 0.0f : 1.0f;
  F.h[2][0] = disk ? 0.0f : c; F.h[2][1] = disk ? 0.0f : s; F.h[2][2] = disk ? 1.0f : 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      F.HC[a][j] = F.h[a][0] * st.C[sidx(0, j)] + F.h[a][1] * st.C[sidx(1, j)] + F.h[a][2] * st.C[sidx(2, j)];
  const float V[3] = {Ld.v_u, Ld.v_v, Ld.v_n};
  float S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b <= a; ++b) {
      float acc = F.HC[a][0] * F.h[b][0] + F.HC[a][1] * F.h[b][1] + F.HC[a][2] * F.h[b][2];
      S[a][b] = acc + (a == b ? V[a] : 0.0f);
      S[b][a] = S[a][b];
    }
  F.S[0] = S[0][0]; F.S[1] = S[1][0]; F.S[2] = S[1][1];
  F.S[3] = S[2][0]; F.S[4] = S[2][1]; F.S[5] = S[2][2];
  const float c00 = S[1][1] * S[2][2] - S[1][2] * S[2][1];
  const float c01 = S[1][2] * S[2][0] - S[1][0] * S[2][2];
  const float c02 = S[1][0] * S[2][1] - S[1][1] * S[2][0];
  const float id = 1.0f / (S[0][0] * c00 + S[0][1] * c01 + S[0][2] * c02);
  F.Si[0] = c00 * id;
  F.Si[1] = c01 * id;
  F.Si[2] = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) * id;
  F.Si[3] = c02 * id;
  F.Si[4] = (S[0][1] * S[2][0] - S[0][0] * S[2][1]) * id;
  F.Si[5] = (S[0][0] * S[1][1] - S[0][1] * S[1][0]) * id;
}

// Residual r = H (m - x) with the difference taken in FP64.
KFX_HD void residual(const State& st, const Frame& F, double mx, double my, double mz, float r[3]) {
  const float dx = (float)(mx - st.x), dy = (float)(my - st.y), dz = (float)(mz - st.z);
#pragma unroll
  for (int a = 0; a < 3; ++a) r[a] = F.h[a][0] * dx + F.h[a][1] * dy + F.h[a][2] * dz;
}

KFX_HD float chi2_of(const Frame& F, const float r[3]) {
  return r[0] * r[0] * F.Si[0] + r[1] * r[1] * F.Si[2] + r[2] * r[2] * F.Si[5] +
         2.0f * (r[0] * r[1] * F.Si[1] + r[0] * r[2] * F.Si[3] + r[1] * r[2] * F.Si[4]);
}

// Kalman update (gain form): K = C H^T S^-1, p += K r, C -= K H C.
KFX_HD float kf_update(State& st, const Frame& F, double mx, double my, double mz) {
  float r[3];
  residual(st, F, mx, my, mz, r);
  const float chi2 = chi2_of(F, r);
  const float Si[3][3] = {{F.Si[0], F.Si[1], F.Si[3]}, {F.Si[1], F.Si[2], F.Si[4]}, {F.Si[3], F.Si[4], F.Si[5]}};
  float K[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int b = 0; b < 3; ++b) K[i][b] = F.HC[0][i] * Si[0][b] + F.HC[1][i] * Si[1][b] + F.HC[2][i] * Si[2][b];
  float dp[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) dp[i] = K[i][0] * r[0] + K[i][1] * r[1] + K[i][2] * r[2];
  st.x += (double)dp[0];
  st.y += (double)dp[1];
  st.z += (double)dp[2];
  st.k += dp[3];
  st.phi = wrap_pi(st.phi + (double)dp[4]);
  st.th += dp[5];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j)
      st.C[sidx(i, j)] -= K[i][0] * F.HC[0][j] + K[i][1] * F.HC[1][j] + K[i][2] * F.HC[2][j];
  return chi2;
}

// Prior covariance of the start estimate: diagonal (sigma_pos^2 x3,
// (sk_rel |k|)^2, sigma_phi^2, sigma_theta^2).
struct Prior {
  float spos, sk_rel, sphi, stheta;
};

KFX_HD void prior_cov(const Prior& pr, State& st) {
#pragma unroll
  for (int i = 0; i < 21; ++i) st.C[i] = 0.0f;
  st.C[sidx(0, 0)] = st.C[sidx(1, 1)] = st.C[sidx(2, 2)] = pr.spos * pr.spos;
  const float sk = pr.sk_rel * fabsf(st.k);
  st.C[sidx(3, 3)] = sk * sk;
  st.C[sidx(4, 4)] = pr.sphi * pr.sphi;
  st.C[sidx(5, 5)] = pr.stheta * pr.stheta;
}

// Add the material noise of a layer to a state sitting on it (used at the
// first hit, where there is no transport).
KFX_HD void add_material(State& st, const Layer& Ld) {
  if (!(Ld.x0 > 0.0f)) return;
  const float sth = sinf(st.th), cth = cosf(st.th), cot = cth / sth;
  float cinc;
  if (Ld.kind == kDisk) {
    cinc = fabsf(cth);
  } else {
    const double r = sqrt(st.x * st.x + st.y * st.y);
    cinc = fabsf(sth * (float)((st.x * cos(st.phi) + st.y * sin(st.phi)) / r));
  }
  cinc = fmaxf(cinc, 1e-3f);
  const float t = Ld.x0 / cinc;
  const float th0 = 0.0136f * fabsf(st.k) * sth * sqrtf(t) * (1.0f + 0.038f * logf(t));
  const float var = th0 * th0;
  st.C[sidx(4, 4)] += var / (sth * sth);
  st.C[sidx(5, 5)] += var;
  st.C[sidx(3, 3)] += st.k * st.k * cot * cot * var;
  st.C[sidx(5, 3)] += -st.k * cot * var;
}

// Start estimate from three hits (FP64): signed curvature of the circle
// through the transverse points (omega = 2 cross / product of the sides),
// phi = tangent at hit 1 = chord direction minus half the turning angle,
// cot(theta) = dz / arc(1 -> 3).  Position = hit 1.
KFX_HD void seed_estimate(double bz, const double m1[3], const double m2[3], const double m3[3],
                          State& st) {
  const double ax = m2[0] - m1[0], ay = m2[1] - m1[1];
  const double bx = m3[0] - m1[0], by = m3[1] - m1[1];
  const double cx = m3[0] - m2[0], cy = m3[1] - m2[1];
  const double la = sqrt(ax * ax + ay * ay), lb = sqrt(bx * bx + by * by), lc = sqrt(cx * cx + cy * cy);
  const double cr = ax * by - ay * bx;
  double omega = 2.0 * cr / (la * lb * lc);
  if (bz == 0.0) omega = 0.0;
  st.x = m1[0];
  st.y = m1[1];
  st.z = m1[2];
  st.k = bz == 0.0 ? 0.0f : (float)(-omega / ((double)kHc * bz));
  // turning angle over the chord 1->2 is 2 asin(omega |P2-P1| / 2)
  const double half12 = asin(fmin(1.0, fmax(-1.0, 0.5 * omega * la)));
  st.phi = wrap_pi(atan2(ay, ax) - half12);
  const double half13 = asin(fmin(1.0, fmax(-1.0, 0.5 * omega * lb)));
  const double s13 = fabs(omega) > 0.0 ? 2.0 * half13 / omega : lb;
  st.th = (float)atan2(s13, m3[2] - m1[2]);
}

}  // namespace kfx
