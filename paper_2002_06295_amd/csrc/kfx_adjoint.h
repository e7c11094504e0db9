// Reverse-mode adjoint of the fit: gradient of the weighted total chi2 with
// respect to the barrel-layer alignment (dr, drphi, dz) and the field scale.
//
// The forward fit (kfx_work.h: fit_track) stores the filtered state after
// every hit.  The reverse sweep walks each track backwards; at hit i it
// recomputes the step i-1 -> i in FP64 from the stored state after hit i-1
// (transport, material noise, update), then pulls the adjoint of the state
// after hit i back through it:
//
//   update   p+ = p- + P z,  C+ = C- - P W P^T,  chi2 = r^T z
//            with P = C- H^T, S = H C- H^T + V, W = S^-1, z = W r,
//            r = H (m - x-) and H the local frame at x- (rows u, v, n)
//   noise    C- += Q(k, theta, direction at the crossing)      (Highland)
//   cov      C- = J C J^T with J = A + b c^T                    (c = ds/dp)
//   helix    p- = F(p, s, omega) along the chord form of the helix
//   path     s from the surface equation (implicit-function derivative)
//
// The adjoint of a symmetric matrix C is the symmetric G with dL =
// sum_ij G_ij dC_ij, stored packed like C.  J = A + b c^T with A the unit
// matrix plus six entries, so J^T G J and the parts of the adjoint of J
// that matter (its entries in A, J_bar c and J_bar^T b) reduce to products
// of packed symmetric matrices with vectors; no 6x6 temporary is formed.
// The tangent-plane projection that the forward transport applies is an
// identity on the values that exact arithmetic produces, so its derivative
// is the identity and the sweep leaves it out; on a disk the z row of J is
// identically zero and is treated as the constant it is.
//
// Paper: arXiv 2002.06295, Sec. 1 (the Kalman filter: propagation with
// material effects, then the update with the hit position; the fit applies
// it over the hits found by building).  The paper has no alignment or field
// fit; the parametrisation of the alignment follows the fit of kfx_work.h.
#pragma once

#include "kfx_work.h"

namespace kfx {

// sin(a)/a and its first two derivatives, series near 0.
KFX_HD void sinc_dd(double a, double sa, double ca, double& f, double& f1, double& f2) {
  if (fabs(a) < 1e-2) {
    const double a2 = a * a;
    f = 1.0 + a2 * (-1.0 / 6.0 + a2 * (1.0 / 120.0 + a2 * (-1.0 / 5040.0)));
    f1 = a * (-1.0 / 3.0 + a2 * (1.0 / 30.0 + a2 * (-1.0 / 840.0)));
    f2 = -1.0 / 3.0 + a2 * (1.0 / 10.0 + a2 * (-1.0 / 168.0));
  } else {
    const double ia = 1.0 / a;
    f = sa * ia;
    f1 = (ca - f) * ia;
    f2 = -f - 2.0 * f1 * ia;
  }
}

// y = C x for a packed symmetric 6x6 C
KFX_HD void symv6(const double* C, const double x[6], double y[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) acc += C[sidx(i, j)] * x[j];
    y[i] = acc;
  }
}

// What the reverse sweep of one step needs from its forward recompute.
struct StepTape {
  bool disk;
  double R;                       // surface radius (barrel) or z (disk)
  double kappa, omega, s;
  double f, f1, f2;               // sinc and its derivatives at a = omega s / 2
  double cpsi, spsi;              // direction at the middle of the chord
  double dx, dy, Dx, Dy;          // chord and d(chord)/d(omega)
  double c1, s1;                  // direction at the crossing
  double sth, cth;
  double x1, y1, Dn;              // crossing point, (x1, y1) . (c1, s1)
  double A[6];                    // Axk Ayk Axp Ayp Azt Apk (the entries of A beyond the unit matrix)
  double cv[6];                   // c = ds/dp
  double be[6];                   // b = dF/ds as used in J (z entry 0 on a disk)
  double d22;                     // A_zz: 1, or 0 on a disk
  // noise
  bool noise, clamped;
  double cinc, t, th0, var;
  // update
  double p1[6];
  double hc, hs, r1;              // frame: (cos, sin) of the crossing's azimuth
  double d[3], r[3], P[6][3], W[6], z[3];  // W = S^-1 packed (00 10 11 20 21 22)
  double chi2;
};

KFX_HD int s3(int a, int b) { return a >= b ? a * (a + 1) / 2 + b : b * (b + 1) / 2 + a; }

// rows u, v, n of the measurement frame
KFX_HD void frame_rows(const StepTape& T, double H[3][3]) {
  H[0][0] = -T.hs; H[0][1] = T.hc; H[0][2] = 0.0;
  H[1][0] = T.disk ? T.hc : 0.0; H[1][1] = T.disk ? T.hs : 0.0; H[1][2] = T.disk ? 0.0 : 1.0;
  H[2][0] = T.disk ? 0.0 : T.hc; H[2][1] = T.disk ? 0.0 : T.hs; H[2][2] = T.disk ? 1.0 : 0.0;
}

// y = A x and y = A^T x (A: unit matrix, z diagonal d22, plus six entries)
KFX_HD void amul(const StepTape& T, const double x[6], double y[6]) {
  y[0] = x[0] + T.A[0] * x[3] + T.A[2] * x[4];
  y[1] = x[1] + T.A[1] * x[3] + T.A[3] * x[4];
  y[2] = T.d22 * x[2] + T.d22 * T.A[4] * x[5];
  y[3] = x[3];
  y[4] = x[4] + T.A[5] * x[3];
  y[5] = x[5];
}
KFX_HD void atmul(const StepTape& T, const double x[6], double y[6]) {
  y[0] = x[0];
  y[1] = x[1];
  y[2] = T.d22 * x[2];
  y[3] = x[3] + T.A[0] * x[0] + T.A[1] * x[1] + T.A[5] * x[4];
  y[4] = x[4] + T.A[2] * x[0] + T.A[3] * x[1];
  y[5] = x[5] + T.d22 * T.A[4] * x[2];
}
// y = J x and y = J^T x, J = A + b c^T
KFX_HD void jmul(const StepTape& T, const double x[6], double y[6]) {
  amul(T, x, y);
  double cx = 0.0;
#pragma unroll
  for (int j = 0; j < 6; ++j) cx += T.cv[j] * x[j];
#pragma unroll
  for (int i = 0; i < 6; ++i) y[i] += T.be[i] * cx;
}
KFX_HD void jtmul(const StepTape& T, const double x[6], double y[6]) {
  atmul(T, x, y);
  double bx = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) bx += T.be[i] * x[i];
#pragma unroll
  for (int j = 0; j < 6; ++j) y[j] += T.cv[j] * bx;
}

// Multiple-scattering noise at a crossing, with what its adjoint needs.
KFX_HD void tape_noise(StepTape& T, const Layer& Ld, double k, double sth, double cth, double cinc_raw, double* C1) {
  T.noise = Ld.x0 > 0.0f;
  if (!T.noise) return;
  T.clamped = !(cinc_raw > 1e-3);
  T.cinc = T.clamped ? 1e-3 : cinc_raw;
  T.t = (double)Ld.x0 / T.cinc;
  T.th0 = 0.0136 * fabs(k) * sth * sqrt(T.t) * (1.0 + 0.038 * log(T.t));
  T.var = T.th0 * T.th0;
  const double cot = cth / sth;
  C1[sidx(4, 4)] += T.var / (sth * sth);
  C1[sidx(5, 5)] += T.var;
  C1[sidx(3, 3)] += k * k * cot * cot * T.var;
  C1[sidx(5, 3)] += -k * cot * T.var;
}

// Update at hit m of the state (T.p1, C1); fills the update part of T.
KFX_HD void tape_update(StepTape& T, const Layer& Ld, const double* C1, const double m[3]) {
  T.r1 = sqrt(T.p1[0] * T.p1[0] + T.p1[1] * T.p1[1]);
  T.hc = T.p1[0] / T.r1;
  T.hs = T.p1[1] / T.r1;
  T.disk = Ld.kind == kDisk;
  double H[3][3];
  frame_rows(T, H);
#pragma unroll
  for (int j = 0; j < 3; ++j) T.d[j] = m[j] - T.p1[j];
#pragma unroll
  for (int a = 0; a < 3; ++a) T.r[a] = H[a][0] * T.d[0] + H[a][1] * T.d[1] + H[a][2] * T.d[2];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      T.P[i][a] = C1[sidx(i, 0)] * H[a][0] + C1[sidx(i, 1)] * H[a][1] + C1[sidx(i, 2)] * H[a][2];
  const double V[3] = {(double)Ld.v_u, (double)Ld.v_v, (double)Ld.v_n};
  double S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      S[a][b] = H[a][0] * T.P[0][b] + H[a][1] * T.P[1][b] + H[a][2] * T.P[2][b] + (a == b ? V[a] : 0.0);
  // symmetric 3x3 inverse by cofactors
  const double c00 = S[1][1] * S[2][2] - S[1][2] * S[2][1];
  const double c01 = S[1][2] * S[2][0] - S[1][0] * S[2][2];
  const double c02 = S[1][0] * S[2][1] - S[1][1] * S[2][0];
  const double id = 1.0 / (S[0][0] * c00 + S[0][1] * c01 + S[0][2] * c02);
  T.W[s3(0, 0)] = c00 * id;
  T.W[s3(1, 0)] = c01 * id;
  T.W[s3(2, 0)] = c02 * id;
  T.W[s3(1, 1)] = (S[0][0] * S[2][2] - S[0][2] * S[2][0]) * id;
  T.W[s3(2, 1)] = (S[0][1] * S[2][0] - S[0][0] * S[2][1]) * id;
  T.W[s3(2, 2)] = (S[0][0] * S[1][1] - S[0][1] * S[1][0]) * id;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    T.z[a] = T.W[s3(a, 0)] * T.r[0] + T.W[s3(a, 1)] * T.r[1] + T.W[s3(a, 2)] * T.r[2];
  T.chi2 = T.r[0] * T.z[0] + T.r[1] * T.z[1] + T.r[2] * T.z[2];
}

// Forward recompute of the transport from (p0, C0) onto layer Ld (barrel
// radius R, or the disk's z), the noise there and the update at m.  Returns
// false where the forward fit failed (no crossing).
KFX_HD bool tape_step(StepTape& T, const StateT<double>& st0, const Layer& Ld, double R, double kappa,
                      const double m[3]) {
  T.disk = Ld.kind == kDisk;
  T.R = T.disk ? (double)Ld.pos : R;
  T.kappa = kappa;
  T.omega = kappa * st0.k;
  double cphi, sphi;
  sincos_d(st0.phi, sphi, cphi);
  T.s = path_to_layer(st0, Ld, R, cphi, sphi, T.omega);
  if (!(T.s > 0.0)) return false;
  const double s = T.s;
  const double a = 0.5 * T.omega * s;
  double sa, ca;
  sincos_d(a, sa, ca);
  sinc_dd(a, sa, ca, T.f, T.f1, T.f2);
  T.cpsi = cphi * ca - sphi * sa;
  T.spsi = sphi * ca + cphi * sa;
  const double L = s * T.f;
  T.dx = L * T.cpsi;
  T.dy = L * T.spsi;
  const double hs2 = 0.5 * s * s;
  T.Dx = hs2 * (T.f1 * T.cpsi - T.f * T.spsi);
  T.Dy = hs2 * (T.f1 * T.spsi + T.f * T.cpsi);
  T.c1 = T.cpsi * ca - T.spsi * sa;
  T.s1 = T.spsi * ca + T.cpsi * sa;
  sincos_d(st0.th, T.sth, T.cth);
  const double cot = T.cth / T.sth;
  T.x1 = st0.x + T.dx;
  T.y1 = st0.y + T.dy;
  T.p1[0] = T.x1;
  T.p1[1] = T.y1;
  T.p1[2] = T.disk ? (double)Ld.pos : st0.z + s * cot;
  T.p1[3] = st0.k;
  T.p1[4] = wrap_pi(st0.phi + 2.0 * a);
  T.p1[5] = st0.th;
  T.A[0] = kappa * T.Dx;
  T.A[1] = kappa * T.Dy;
  T.A[2] = -T.dy;
  T.A[3] = T.dx;
  T.A[4] = -s / (T.sth * T.sth);
  T.A[5] = kappa * s;
  T.d22 = T.disk ? 0.0 : 1.0;
  T.Dn = T.x1 * T.c1 + T.y1 * T.s1;
  if (T.disk) {
    T.cv[0] = T.cv[1] = T.cv[3] = T.cv[4] = 0.0;
    T.cv[2] = -T.sth / T.cth;
    T.cv[5] = s / (T.sth * T.cth);
  } else {
    const double iDn = -1.0 / T.Dn;
    T.cv[0] = T.x1 * iDn;
    T.cv[1] = T.y1 * iDn;
    T.cv[2] = 0.0;
    T.cv[3] = (T.x1 * T.A[0] + T.y1 * T.A[1]) * iDn;
    T.cv[4] = (T.x1 * T.A[2] + T.y1 * T.A[3]) * iDn;
    T.cv[5] = 0.0;
  }
  T.be[0] = T.c1;
  T.be[1] = T.s1;
  T.be[2] = T.disk ? 0.0 : cot;
  T.be[3] = 0.0;
  T.be[4] = T.omega;
  T.be[5] = 0.0;
  // C1 = J C0 J^T, one column at a time: column j is J (C0 J^T e_j)
  double C1[21];
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    double e[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    e[j] = 1.0;
    double rj[6], zj[6], wj[6];
    jtmul(T, e, rj);
    symv6(st0.C, rj, zj);
    jmul(T, zj, wj);
#pragma unroll
    for (int i = j; i < 6; ++i) C1[sidx(i, j)] = wj[i];
  }
  const double cinc_raw = T.disk ? fabs(T.cth) : fabs(T.sth * T.Dn / sqrt(T.x1 * T.x1 + T.y1 * T.y1));
  tape_noise(T, Ld, st0.k, T.sth, T.cth, cinc_raw, C1);
  tape_update(T, Ld, C1, m);
  return true;
}

// Adjoint of the update.  In: pb (adjoint of p+), G (adjoint of C+,
// packed), w (the weight of this step's chi2).  Out: pb and G become the
// adjoints of p- and C- (the frame's dependence on x- included), mb the
// adjoint of the measurement.
KFX_HD void adj_update(const StepTape& T, double pb[6], double* G, double w, double mb[3]) {
  double H[3][3];
  frame_rows(T, H);
  // p+ = p- + P z:  zb = P^T pb
  double zb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) acc += T.P[i][a] * pb[i];
    zb[a] = acc;
  }
  // GP = G P
  double GP[6][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double pa[6] = {T.P[0][a], T.P[1][a], T.P[2][a], T.P[3][a], T.P[4][a], T.P[5][a]};
    double y[6];
    symv6(G, pa, y);
#pragma unroll
    for (int i = 0; i < 6; ++i) GP[i][a] = y[i];
  }
  // C+ = C- - P W P^T:  Pb = pb z^T - 2 G P W;  Wb = -P^T G P + w r r^T + zb r^T
  double Pb[6][3], Wb[3][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      Pb[i][a] = pb[i] * T.z[a] -
                 2.0 * (GP[i][0] * T.W[s3(0, a)] + GP[i][1] * T.W[s3(1, a)] + GP[i][2] * T.W[s3(2, a)]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) acc += T.P[i][a] * GP[i][b];
      Wb[a][b] = -acc + w * T.r[a] * T.r[b] + zb[a] * T.r[b];
    }
  // chi2 = r^T z, z = W r:  rb = 2 w z + W zb
  double rb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    rb[a] = 2.0 * w * T.z[a] + T.W[s3(a, 0)] * zb[0] + T.W[s3(a, 1)] * zb[1] + T.W[s3(a, 2)] * zb[2];
  // W = S^-1:  Sb = -W Wb W, symmetrised
  double WW[3][3], Sb[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      WW[a][b] = Wb[a][0] * T.W[s3(0, b)] + Wb[a][1] * T.W[s3(1, b)] + Wb[a][2] * T.W[s3(2, b)];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
      Sb[a][b] = -(T.W[s3(a, 0)] * WW[0][b] + T.W[s3(a, 1)] * WW[1][b] + T.W[s3(a, 2)] * WW[2][b]);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < a; ++b) Sb[a][b] = Sb[b][a] = 0.5 * (Sb[a][b] + Sb[b][a]);
  // the position columns of C-: CP = P H (H is orthonormal)
  double CP[6][3];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) CP[i][j] = T.P[i][0] * H[0][j] + T.P[i][1] * H[1][j] + T.P[i][2] * H[2][j];
  // S = H C_pp H^T + V and P = C[:, pos] H^T:  the adjoint of C- gains
  // H^T Sb H on the position block and Pb H on the position columns; H gains
  // 2 Sb H C_pp + Pb^T C[:, pos] + rb d^T
  double SbH[3][3], PbH[6][3], Hb[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) SbH[a][j] = Sb[a][0] * H[0][j] + Sb[a][1] * H[1][j] + Sb[a][2] * H[2][j];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) PbH[i][j] = Pb[i][0] * H[0][j] + Pb[i][1] * H[1][j] + Pb[i][2] * H[2][j];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      double acc = rb[a] * T.d[j];
#pragma unroll
      for (int q = 0; q < 3; ++q) acc += 2.0 * SbH[a][q] * CP[q][j];
#pragma unroll
      for (int i = 0; i < 6; ++i) acc += Pb[i][a] * CP[i][j];
      Hb[a][j] = acc;
    }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      double add = 0.0;
      if (i < 3) add += H[0][i] * SbH[0][j] + H[1][i] * SbH[1][j] + H[2][i] * SbH[2][j];  // j <= i < 3
      if (j < 3) add += 0.5 * PbH[i][j];
      if (i < 3) add += 0.5 * PbH[j][i];
      G[sidx(i, j)] += add;
    }
  // d = m - x-:  mb = H^T rb, pb_pos -= mb
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    mb[j] = H[0][j] * rb[0] + H[1][j] * rb[1] + H[2][j] * rb[2];
    pb[j] -= mb[j];
  }
  // frame: H from (hc, hs) = (x, y) / r
  double hcb, hsb;
  if (T.disk) {
    hcb = Hb[0][1] + Hb[1][0];
    hsb = -Hb[0][0] + Hb[1][1];
  } else {
    hcb = Hb[0][1] + Hb[2][0];
    hsb = -Hb[0][0] + Hb[2][1];
  }
  const double ir = 1.0 / T.r1;
  pb[0] += (hcb * T.hs * T.hs - hsb * T.hc * T.hs) * ir;
  pb[1] += (-hcb * T.hc * T.hs + hsb * T.hc * T.hc) * ir;
}

// Adjoint of the transport + noise.  In: pb, G = adjoints of (p-, C-) after
// the noise (G packed); C0 the covariance the step started from (packed).
// Out: pb, G become the adjoints of (p0, C0); Rb and kb the adjoints of the
// surface radius and of kappa.
KFX_HD void adj_transport(const StepTape& T, const double* C0, double pb[6], double* G, double& Rb, double& kb) {
  const double s = T.s, sth = T.sth, cth = T.cth;
  const double cot = cth / sth;
  const double k0 = T.p1[3];
  double x1b = pb[0], y1b = pb[1];
  double sb = 0.0, ob = 0.0, thb = pb[5], kb0 = pb[3], phb1 = pb[4];
  double sthb = 0.0, cthb = 0.0, cotb = 0.0, c1b = 0.0, s1b = 0.0, Dnb = 0.0;
  kb = 0.0;
  Rb = 0.0;
  // ---- noise
  if (T.noise) {
    const double G33 = G[sidx(3, 3)], G44 = G[sidx(4, 4)], G55 = G[sidx(5, 5)], G53 = G[sidx(5, 3)];
    const double vb = G44 / (sth * sth) + G55 + G33 * k0 * k0 * cot * cot - 2.0 * G53 * k0 * cot;
    kb0 += G33 * 2.0 * k0 * cot * cot * T.var - 2.0 * G53 * cot * T.var;
    cotb += G33 * k0 * k0 * 2.0 * cot * T.var - 2.0 * G53 * k0 * T.var;
    sthb += -2.0 * G44 * T.var / (sth * sth * sth);
    const double th0b = 2.0 * T.th0 * vb;
    if (k0 != 0.0) kb0 += th0b * T.th0 / k0;
    sthb += th0b * T.th0 / sth;
    if (!T.clamped) {
      const double sq = sqrt(T.t), lg = 1.0 + 0.038 * log(T.t);
      const double tb = th0b * 0.0136 * fabs(k0) * sth * (lg / (2.0 * sq) + sq * 0.038 / T.t);
      const double cincb = -tb * T.t / T.cinc;
      if (T.disk) {
        cthb += (cth >= 0.0 ? 1.0 : -1.0) * cincb;
      } else {
        const double r1 = sqrt(T.x1 * T.x1 + T.y1 * T.y1);
        const double q = sth * T.Dn / r1;
        const double sg = q >= 0.0 ? 1.0 : -1.0;
        sthb += sg * cincb * T.Dn / r1;
        Dnb += sg * cincb * sth / r1;
        const double r1b = -sg * cincb * q / r1;
        x1b += r1b * T.x1 / r1;
        y1b += r1b * T.y1 / r1;
      }
    }
  }
  // ---- covariance C- = J C0 J^T with J = A + b c^T.
  // The parts of J_bar = 2 G J C0 that reach the parameters:
  //   J_bar c = 2 G J (C0 c),   J_bar^T b = 2 C0 J^T (G b),
  //   its entries in A (columns 3, 4, 5: 2 G J (C0 e_j)).
  double u[6];
  symv6(G, T.be, u);
  double bb[6], cb[6], Ab[6];
  {
    double v[6], jv[6];
    symv6(C0, T.cv, v);
    jmul(T, v, jv);
    symv6(G, jv, bb);
#pragma unroll
    for (int i = 0; i < 6; ++i) bb[i] *= 2.0;
    double jtu[6];
    jtmul(T, u, jtu);
    symv6(C0, jtu, cb);
#pragma unroll
    for (int i = 0; i < 6; ++i) cb[i] *= 2.0;
    double col[6], y[6], gy[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) col[q] = C0[sidx(q, 3)];
    jmul(T, col, y);
    symv6(G, y, gy);
    Ab[0] = 2.0 * gy[0];
    Ab[1] = 2.0 * gy[1];
    Ab[5] = 2.0 * gy[4];
#pragma unroll
    for (int q = 0; q < 6; ++q) col[q] = C0[sidx(q, 4)];
    jmul(T, col, y);
    symv6(G, y, gy);
    Ab[2] = 2.0 * gy[0];
    Ab[3] = 2.0 * gy[1];
#pragma unroll
    for (int q = 0; q < 6; ++q) col[q] = C0[sidx(q, 5)];
    jmul(T, col, y);
    symv6(G, y, gy);
    Ab[4] = T.disk ? 0.0 : 2.0 * gy[2];
  }
  // G0 = J^T G J = A^T G A + w c^T + c w^T + sigma c c^T, w = A^T G b,
  // sigma = b^T G b; A^T G A column by column
  {
    double wv[6];
    atmul(T, u, wv);
    double sig = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) sig += T.be[i] * u[i];
    double G0[21];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double e[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      e[j] = 1.0;
      double aj[6], nj[6], mj[6];
      amul(T, e, aj);
      symv6(G, aj, nj);
      atmul(T, nj, mj);
#pragma unroll
      for (int i = j; i < 6; ++i)
        G0[sidx(i, j)] = mj[i] + wv[i] * T.cv[j] + T.cv[i] * wv[j] + sig * T.cv[i] * T.cv[j];
    }
#pragma unroll
    for (int q = 0; q < 21; ++q) G[q] = G0[q];
  }
  // b = (c1, s1, cot, 0, omega, 0); on a disk the z entry is the constant 0
  c1b += bb[0];
  s1b += bb[1];
  if (!T.disk) cotb += bb[2];
  ob += bb[4];
  // c
  if (T.disk) {
    thb += -cb[2] / (cth * cth);
    sb += cb[5] / (sth * cth);
    thb += -cb[5] * s * (cth * cth - sth * sth) / (sth * sth * cth * cth);
  } else {
    const double N[6] = {T.x1, T.y1, 0.0, T.x1 * T.A[0] + T.y1 * T.A[1], T.x1 * T.A[2] + T.y1 * T.A[3], 0.0};
    const double iDn = 1.0 / T.Dn;
    double Nb[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) Nb[j] = -cb[j] * iDn;
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j) t += cb[j] * N[j];
    Dnb += t * iDn * iDn;
    x1b += Nb[0] + Nb[3] * T.A[0] + Nb[4] * T.A[2];
    y1b += Nb[1] + Nb[3] * T.A[1] + Nb[4] * T.A[3];
    Ab[0] += Nb[3] * T.x1;
    Ab[1] += Nb[3] * T.y1;
    Ab[2] += Nb[4] * T.x1;
    Ab[3] += Nb[4] * T.y1;
  }
  // Dn = x1 c1 + y1 s1
  x1b += Dnb * T.c1;
  y1b += Dnb * T.s1;
  c1b += Dnb * T.x1;
  s1b += Dnb * T.y1;
  // A entries
  double dxb = Ab[3], dyb = -Ab[2];
  sb += -Ab[4] / (sth * sth);
  sthb += Ab[4] * 2.0 * s / (sth * sth * sth);
  sb += Ab[5] * T.kappa;
  kb += Ab[5] * s;
  const double Dxb = T.kappa * Ab[0], Dyb = T.kappa * Ab[1];
  kb += Ab[0] * T.Dx + Ab[1] * T.Dy;
  // ---- parameters p- = F(p0, s, omega)
  double pb0[6] = {x1b, y1b, 0.0, kb0, 0.0, thb};
  dxb += x1b;
  dyb += y1b;
  if (!T.disk) {
    pb0[2] = pb[2];
    sb += pb[2] * cot;
    cotb += pb[2] * s;
  }
  // direction at the crossing: phi1 = phi0 + omega s
  phb1 += -T.s1 * c1b + T.c1 * s1b;
  // chord d = s f(a) e^{i psi}, psi = phi0 + a, a = omega s / 2
  double phb0 = -dxb * T.dy + dyb * T.dx;
  sb += dxb * T.c1 + dyb * T.s1;
  ob += dxb * T.Dx + dyb * T.Dy;
  // D = (s^2/2) e^{i psi} (f1 + i f)
  phb0 += -Dxb * T.Dy + Dyb * T.Dx;
  {
    const double hs2 = 0.5 * s * s;
    // s e^{i psi} (f1 + i f)
    const double ex = s * (T.f1 * T.cpsi - T.f * T.spsi), ey = s * (T.f1 * T.spsi + T.f * T.cpsi);
    sb += Dxb * ex + Dyb * ey;
    // d/da: (s^2/2) e^{i psi} ((f2 + i f1) + i (f1 + i f)) = (s^2/2) e^{i psi} ((f2 - f) + 2 i f1)
    const double gr = T.f2 - T.f, gi = 2.0 * T.f1;
    const double ax = hs2 * (gr * T.cpsi - gi * T.spsi), ay = hs2 * (gr * T.spsi + gi * T.cpsi);
    const double ab = Dxb * ax + Dyb * ay;
    sb += ab * 0.5 * T.omega;
    ob += ab * 0.5 * s;
  }
  phb0 += phb1;
  sb += phb1 * T.omega;
  ob += phb1 * s;
  // ---- path s(p0, omega, R): implicit derivative of the surface equation
  if (T.disk) {
    // s = (Z - z0) tan(theta)
    pb0[2] += -sb * (sth / cth);
    thb += sb * s / (sth * cth);
  } else {
    // ds = c . dp0 (x0, y0, phi0) + ds/domega domega + R/Dn dR
    pb0[0] += sb * T.cv[0];
    pb0[1] += sb * T.cv[1];
    phb0 += sb * T.cv[4];
    ob += -sb * (T.x1 * T.Dx + T.y1 * T.Dy) / T.Dn;
    Rb += sb * T.R / T.Dn;
  }
  // theta trig
  thb += sthb * cth - cthb * sth - cotb / (sth * sth);
  pb0[5] = thb;
  pb0[4] = phb0;
  // omega = kappa k0
  pb0[3] += ob * T.kappa;
  kb += ob * k0;
#pragma unroll
  for (int i = 0; i < 6; ++i) pb[i] = pb0[i];
}

}  // namespace kfx

namespace kfx {

// Adjoint of the aligned hit position and of the surface radius with
// respect to (dr, drphi, dz) of a barrel layer; m is the aligned hit.
template <class Acc>
KFX_HD void hit_grad(const Layer& Ld, int l, const double m[3], const double mb[3], double Rb, Acc& acc) {
  if (Ld.kind != kBarrel) return;
  const double rr = sqrt(m[0] * m[0] + m[1] * m[1]);  // R + dr
  acc.add(l, 0, (mb[0] * m[0] + mb[1] * m[1]) / rr + Rb);
  acc.add(l, 1, (-mb[0] * m[1] + mb[1] * m[0]) / (double)Ld.pos);
  acc.add(l, 2, mb[2]);
}

// Reverse sweep of one fitted track: adds w * d(chi2 of the track) /
// d(alignment, field scale) to acc.  ckpt holds the filtered state after
// each hit (as written by fit_track: hit i of track t at i * n_tracks + t).  Returns false for a track that the
// forward fit did not fit.
template <class Acc>
KFX_HD bool fit_track_backward(const Geometry& G, const HitsView& H, const int* trk_off, const int* trk_hits, int t,
                               const Prior& pr, const float* align, float fscale, const StateSoA& ckpt,
                               int n_tracks, double w,
                               Acc& acc) {
  const int b = trk_off[t], n = trk_off[t + 1] - trk_off[t];
  if (n < 3) return false;
  const double kappa0 = -kHcD * G.bz;
  const double kappa = kappa0 * (double)fscale;
  double pb[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double Gb[21];
#pragma unroll
  for (int q = 0; q < 21; ++q) Gb[q] = 0.0;
  double fb = 0.0;
  for (int i = n - 1; i >= 0; --i) {
    const int h = trk_hits[b + i];
    const int l = H.layer[h];
    const Layer& Ld = G.L[l];
    const float* a = align ? align + 3 * l : nullptr;
    double m[3];
    aligned_hit(Ld, H.x[h], H.y[h], H.z[h], a, m);
    StepTape T;
    double mb[3], Rb = 0.0;
    if (i > 0) {
      const double r_surf = Ld.pos + ((a && Ld.kind == kBarrel) ? (double)a[0] : 0.0);
      State c;
      load_state(ckpt, (long)(i - 1) * n_tracks + t, c);
      StateT<double> s0;
      convert_state(c, s0);
      if (!tape_step(T, s0, Ld, r_surf, kappa, m)) return false;
      adj_update(T, pb, Gb, w, mb);
      double kb = 0.0;
      adj_transport(T, s0.C, pb, Gb, Rb, kb);
      fb += kb * kappa0;
    } else {
      // the start estimate from the first three hits as recorded, with the
      // prior covariance and this layer's noise: no gradient flows into it
      double m0[3][3];
      for (int q = 0; q < 3; ++q) {
        const int hq = trk_hits[b + q];
        m0[q][0] = H.x[hq];
        m0[q][1] = H.y[hq];
        m0[q][2] = H.z[hq];
      }
      StateT<double> sd;
      seed_estimate(G.bz, m0[0], m0[1], m0[2], sd);
      prior_cov(pr, sd);
      add_material(sd, Ld);
      T.p1[0] = sd.x; T.p1[1] = sd.y; T.p1[2] = sd.z; T.p1[3] = sd.k; T.p1[4] = sd.phi; T.p1[5] = sd.th;
      tape_update(T, Ld, sd.C, m);
      adj_update(T, pb, Gb, w, mb);
    }
    hit_grad(Ld, l, m, mb, Rb, acc);
  }
  acc.field(fb);
  return true;
}

}  // namespace kfx
