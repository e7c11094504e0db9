// FP64 CPU oracle for Kalman-filter track building and fitting.
//
// TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the
// CPU-baseline leg of the benchmark may load this library.  It shares no
// code, header, table or constant with the GPU library; the two meet only
// through the seeded synthetic inputs.
//
// What it computes (paper: arXiv 2002.06295, with the Kalman filter of
// Fruhwirth 1987, the paper's reference for the KF):
//   * Sec. 1: the KF is propagate-then-update.  The track state (parameters
//     and their uncertainties) is propagated from one layer to the next,
//     material effects included, then updated with the hit's position.
//     Track building is a combinatorial search for the hits of a track,
//     started from a seed in the innermost layers and proceeding outward;
//     fitting applies the same KF to the hits that building found.
//   * Sec. 2: lightweight geometry -- barrel layers collapsed to a radius,
//     forward layers to a z position, hits known by their 3D position -- and
//     at most K candidates kept per seed at each layer, the highest-ranked
//     of its children.
//   * Sec. 3: missing hits are counted consistently and enter the score that
//     ranks candidates.
// The paper gives no formulas for propagation, material, update, score or
// hit indexing; every numerical choice below is a stated reading (listed with
// the design notes of the repository).  The oracle is written as the plain
// definition: full 6x6 matrices, no packing, no fusion, double precision.
//
// Units: cm, GeV, T, rad.  State p = (x, y, z, k = q/pT, phi, theta);
// (x, y, z) lies on the current surface; phi and theta give the momentum
// direction there.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <numeric>
#include <vector>

#include "kfo_ad.h"

namespace kfo {

Tape& tape() {
  static thread_local Tape t;
  return t;
}

constexpr double kC = 0.299792458e-2;  // GeV / (T cm)
constexpr double kPi = 3.14159265358979323846;

enum { BARREL = 0, DISK = 1 };

struct Layer {
  int kind;
  double pos, lo, hi, x0, su, sv, sn;
};

struct Geom {
  std::vector<Layer> L;
  double bz = 0.0;
  int neta = 20, nphi = 128;
  std::vector<int> barrel;    // barrel ids by increasing radius
  std::vector<int> dpos;      // +z disks by increasing z
  std::vector<int> dneg;      // -z disks by decreasing z
  void index() {
    barrel.clear(); dpos.clear(); dneg.clear();
    for (int i = 0; i < (int)L.size(); ++i) {
      if (L[i].kind == BARREL) barrel.push_back(i);
      else if (L[i].pos > 0) dpos.push_back(i);
      else dneg.push_back(i);
    }
    std::sort(barrel.begin(), barrel.end(), [&](int a, int b) { return L[a].pos < L[b].pos; });
    std::sort(dpos.begin(), dpos.end(), [&](int a, int b) { return L[a].pos < L[b].pos; });
    std::sort(dneg.begin(), dneg.end(), [&](int a, int b) { return L[a].pos > L[b].pos; });
  }
};

static Geom make_geom(const double* rec, int nl, double bz, int neta, int nphi) {
  Geom g;
  g.bz = bz; g.neta = neta; g.nphi = nphi;
  for (int i = 0; i < nl; ++i) {
    const double* r = rec + 8 * i;
    g.L.push_back(Layer{(int)r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7]});
  }
  g.index();
  return g;
}

static double wrap_pi(double a) {  // to (-pi, pi]
  while (a > kPi) a -= 2 * kPi;
  while (a <= -kPi) a += 2 * kPi;
  return a;
}

// ------------------------------------------------------------------------
// Helix in a uniform field B*scale along +z.  s is the transverse path
// length; omega = d(phi)/ds = -kC * B * scale * k (a positive charge turns
// clockwise in +Bz, as the Lorentz force requires).
//   x(s) = x0 + s [cos(phi0) S(a) - sin(phi0) C(a)]
//   y(s) = y0 + s [sin(phi0) S(a) + cos(phi0) C(a)]
//   z(s) = z0 + s cot(theta),  phi(s) = phi0 + a,  a = omega s,
// S(a) = sin(a)/a, C(a) = (1 - cos a)/a (series near a = 0).
template <class T>
void helix(const T p0[6], const T& s, const T& omega, T out[6]) {
  using std::cos; using std::sin; using std::fabs;
  T a = omega * s;
  T S, C;
  if (fabs(val(a)) < 1e-4) {
    T a2 = a * a;
    S = 1.0 - a2 / 6.0 + a2 * a2 / 120.0;
    C = a * (0.5 - a2 / 24.0 + a2 * a2 / 720.0);
  } else {
    S = sin(a) / a;
    C = (1.0 - cos(a)) / a;
  }
  T c0 = cos(p0[4]), s0 = sin(p0[4]);
  out[0] = p0[0] + s * (c0 * S - s0 * C);
  out[1] = p0[1] + s * (s0 * S + c0 * C);
  out[2] = p0[2] + s * cos(p0[5]) / sin(p0[5]);
  out[3] = p0[3];
  out[4] = p0[4] + a;
  out[5] = p0[5];
}

template <class T>
T omega_of(const Geom& g, const T& k, const T& fscale) {
  return -kC * g.bz * fscale * k;
}

// Outgoing intersection with the cylinder of radius R.  The track must be
// moving outward (r increasing) at its start; the root is bracketed between
// the start and the turning point (maximum radius of the transverse circle),
// found by bisection, then polished by two Newton steps carried out in T so
// that derivatives flow through the implicit-function relation.
template <class T>
bool path_to_cylinder(const Geom& g, const T p0[6], const T& fscale, const T& R, T& s_out) {
  using std::cos; using std::sin;
  double x = val(p0[0]), y = val(p0[1]), ph = val(p0[4]);
  double RR = val(R);
  double om = -kC * g.bz * val(fscale) * val(p0[3]);
  double D = x * std::cos(ph) + y * std::sin(ph);
  double r0sq = x * x + y * y;
  if (!(r0sq < RR * RR) || D < 0.0) return false;
  double s_lo = 0.0, s_hi;
  if (std::fabs(om) < 1e-12) {
    s_hi = -D + std::sqrt(D * D + RR * RR - r0sq) + 1.0;
  } else {
    double rho = 1.0 / std::fabs(om);
    double cx = x - std::sin(ph) / om, cy = y + std::cos(ph) / om;
    double d = std::hypot(cx, cy);
    if (d + rho < RR) return false;
    double b0 = std::atan2(y - cy, x - cx), gam = std::atan2(cy, cx);
    double db = std::fmod((gam - b0) * (om > 0 ? 1.0 : -1.0), 2 * kPi);
    if (db < 0) db += 2 * kPi;
    s_hi = db * rho;
  }
  auto gfun = [&](double s) {
    double q[6], pp[6];
    for (int i = 0; i < 6; ++i) pp[i] = val(p0[i]);
    helix<double>(pp, s, om, q);
    return q[0] * q[0] + q[1] * q[1] - RR * RR;
  };
  if (gfun(s_hi) < 0.0) return false;
  for (int it = 0; it < 200 && s_hi - s_lo > 1e-14 * (1.0 + s_hi); ++it) {
    double m = 0.5 * (s_lo + s_hi);
    if (gfun(m) < 0.0) s_lo = m; else s_hi = m;
  }
  T s = T(0.5 * (s_lo + s_hi));
  T omT = omega_of(g, p0[3], fscale);
  for (int it = 0; it < 2; ++it) {
    T q[6];
    helix<T>(p0, s, omT, q);
    T gv = q[0] * q[0] + q[1] * q[1] - R * R;
    T gp = 2.0 * (q[0] * cos(q[4]) + q[1] * sin(q[4]));
    s = s - gv / gp;
  }
  if (!(val(s) > 0.0)) return false;
  s_out = s;
  return true;
}

// Disk at z = Z: s = (Z - z0) tan(theta); must be ahead of the track.
template <class T>
bool path_to_disk(const T p0[6], double Z, T& s_out) {
  using std::cos; using std::sin;
  double ct = std::cos(val(p0[5]));
  if (std::fabs(ct) < 1e-12) return false;
  T s = (Z - p0[2]) * sin(p0[5]) / cos(p0[5]);
  if (!(val(s) > 1e-12)) return false;
  s_out = s;
  return true;
}

// Surface alignment of a barrel layer (used by the fit): the true cylinder
// sits at radius R + dr.  Disks are not aligned.
template <class T>
bool propagate_state(const Geom& g, int layer, const T p0[6], const T& fscale,
                     const T& dr, T p1[6]) {
  const Layer& Lr = g.L[layer];
  T s;
  if (Lr.kind == BARREL) {
    T R = Lr.pos + dr;
    if (!path_to_cylinder<T>(g, p0, fscale, R, s)) return false;
  } else {
    if (!path_to_disk<T>(p0, Lr.pos, s)) return false;
  }
  helix<T>(p0, s, omega_of(g, p0[3], fscale), p1);
  if (Lr.kind == BARREL) {
    // moving outward at the crossing
    using std::cos; using std::sin;
    if (val(p1[0]) * std::cos(val(p1[4])) + val(p1[1]) * std::sin(val(p1[4])) < 0.0) return false;
  }
  return true;
}

// Transport Jacobian J = d p1 / d p0 of the map "move to the surface",
// including the dependence of the path length on p0 (the surface
// constraint), by forward differentiation in 6 directions.
template <class T>
bool propagate_with_jacobian(const Geom& g, int layer, const T p0[6], const T& fscale,
                             const T& dr, T p1[6], T J[6][6]) {
  using D6 = Dual<T, 6>;
  D6 q0[6], q1[6];
  for (int i = 0; i < 6; ++i) q0[i] = D6::make(p0[i], i);
  D6 fs = D6::make(fscale, -1), drr = D6::make(dr, -1);
  if (!propagate_state<D6>(g, layer, q0, fs, drr, q1)) return false;
  for (int i = 0; i < 6; ++i) {
    p1[i] = q1[i].v;
    for (int j = 0; j < 6; ++j) J[i][j] = q1[i].d[j];
  }
  return true;
}

// Multiple-scattering noise at a layer (Highland formula, beta = 1, no
// energy loss), for the state p on the layer.  The two projected angles
// each have variance theta0^2: var(theta) = theta0^2,
// var(phi) = theta0^2 / sin^2(theta).  At fixed |p|, k = q/(|p| sin theta)
// changes with theta: dk = -k cot(theta) dtheta.
template <class T>
void material_noise(const Layer& Lr, const T p[6], T Q[6][6]) {
  using std::cos; using std::sin; using std::sqrt; using std::log; using std::fabs;
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) Q[i][j] = T(0.0);
  if (!(Lr.x0 > 0.0)) return;  // no material
  T st = sin(p[5]), ct = cos(p[5]);
  T cinc;
  if (Lr.kind == BARREL) {
    T r = sqrt(p[0] * p[0] + p[1] * p[1]);
    cinc = fabs(st * (p[0] * cos(p[4]) + p[1] * sin(p[4])) / r);
  } else {
    cinc = fabs(ct);
  }
  if (val(cinc) < 1e-3) cinc = T(1e-3);
  T t = Lr.x0 / cinc;
  T inv_p = fabs(p[3]) * st;  // 1/|p|
  T th0 = 0.0136 * inv_p * sqrt(t) * (1.0 + 0.038 * log(t));
  T v = th0 * th0;
  T cot = ct / st;
  Q[4][4] = v / (st * st);
  Q[5][5] = v;
  Q[3][3] = p[3] * p[3] * cot * cot * v;
  Q[3][5] = -p[3] * cot * v;
  Q[5][3] = Q[3][5];
}

// Local measurement frame at the position of p: rows u, v, n of H acting
// on (x, y, z).  Barrel: u = phi-hat, v = z-hat, n = r-hat.  Disk:
// u = phi-hat, v = r-hat, n = z-hat.
template <class T>
void local_frame(const Layer& Lr, const T p[6], T H[3][3]) {
  using std::sqrt;
  T r = sqrt(p[0] * p[0] + p[1] * p[1]);
  T c = p[0] / r, s = p[1] / r;
  H[0][0] = -s; H[0][1] = c; H[0][2] = T(0.0);
  if (Lr.kind == BARREL) {
    H[1][0] = T(0.0); H[1][1] = T(0.0); H[1][2] = T(1.0);
    H[2][0] = c; H[2][1] = s; H[2][2] = T(0.0);
  } else {
    H[1][0] = c; H[1][1] = s; H[1][2] = T(0.0);
    H[2][0] = T(0.0); H[2][1] = T(0.0); H[2][2] = T(1.0);
  }
}

template <class T>
bool inverse3(const T A[3][3], T B[3][3]) {
  T c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  T c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  T c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  T det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
  if (!(std::fabs(val(det)) > 0.0)) return false;
  T id = 1.0 / det;
  B[0][0] = c00 * id;
  B[1][0] = c01 * id;
  B[2][0] = c02 * id;
  B[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
  B[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
  B[2][1] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
  B[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
  B[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
  B[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
  return true;
}

// chi2 of hit m against the predicted state (p, C) on layer Lr:
// r = H (m - x),  S = H C H^T + V,  chi2 = r^T S^-1 r   (3x3).
template <class T>
bool chi2_of(const Layer& Lr, const T p[6], const T C[6][6], const T m[3], T& chi2) {
  T H[3][3], res[3], S[3][3], Si[3][3];
  local_frame<T>(Lr, p, H);
  T dm[3] = {m[0] - p[0], m[1] - p[1], m[2] - p[2]};
  for (int a = 0; a < 3; ++a) res[a] = H[a][0] * dm[0] + H[a][1] * dm[1] + H[a][2] * dm[2];
  double V[3] = {Lr.su * Lr.su, Lr.sv * Lr.sv, Lr.sn * Lr.sn};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      T acc = T(0.0);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) acc += H[a][i] * C[i][j] * H[b][j];
      S[a][b] = acc + (a == b ? V[a] : 0.0);
    }
  if (!inverse3<T>(S, Si)) return false;
  T c = T(0.0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) c += res[a] * Si[a][b] * res[b];
  chi2 = c;
  return true;
}

// Kalman update (gain form): K = C H^T S^-1, p+ = p + K r, C+ = C - K H C.
template <class T>
bool kf_update(const Layer& Lr, T p[6], T C[6][6], const T m[3], T& chi2) {
  T H[3][3], res[3], S[3][3], Si[3][3];
  local_frame<T>(Lr, p, H);
  T dm[3] = {m[0] - p[0], m[1] - p[1], m[2] - p[2]};
  for (int a = 0; a < 3; ++a) res[a] = H[a][0] * dm[0] + H[a][1] * dm[1] + H[a][2] * dm[2];
  double V[3] = {Lr.su * Lr.su, Lr.sv * Lr.sv, Lr.sn * Lr.sn};
  // HC[a][j] = sum_i H[a][i] C[i][j]   (H acts on the position block)
  T HC[3][6];
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 6; ++j) {
      T acc = T(0.0);
      for (int i = 0; i < 3; ++i) acc += H[a][i] * C[i][j];
      HC[a][j] = acc;
    }
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      T acc = T(0.0);
      for (int j = 0; j < 3; ++j) acc += HC[a][j] * H[b][j];
      S[a][b] = acc + (a == b ? V[a] : 0.0);
    }
  if (!inverse3<T>(S, Si)) return false;
  T c = T(0.0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) c += res[a] * Si[a][b] * res[b];
  chi2 = c;
  T K[6][3];
  for (int i = 0; i < 6; ++i)
    for (int b = 0; b < 3; ++b) {
      T acc = T(0.0);
      for (int a = 0; a < 3; ++a) acc += HC[a][i] * Si[a][b];  // (C H^T)[i][a] = HC[a][i]
      K[i][b] = acc;
    }
  for (int i = 0; i < 6; ++i) {
    T acc = T(0.0);
    for (int b = 0; b < 3; ++b) acc += K[i][b] * res[b];
    p[i] = p[i] + acc;
  }
  // C+ = C - K H C is symmetric by definition; the product is formed in
  // full and its two triangles averaged, so that rounding cannot seed an
  // antisymmetric part (the transport would amplify it layer after layer).
  T KHC[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T acc = T(0.0);
      for (int b = 0; b < 3; ++b) acc += K[i][b] * HC[b][j];
      KHC[i][j] = acc;
    }
  T Cn[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) Cn[i][j] = 0.5 * ((C[i][j] - KHC[i][j]) + (C[j][i] - KHC[j][i]));
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C[i][j] = Cn[i][j];
  // keep phi in (-pi, pi]; a constant shift does not change derivatives
  double ph = val(p[4]);
  double w = wrap_pi(ph);
  if (w != ph) p[4] = p[4] + (w - ph);
  return true;
}

// C- = J C J^T + Q
template <class T>
void transport_cov(const T J[6][6], const T C[6][6], const T Q[6][6], T out[6][6]) {
  T JC[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T acc = T(0.0);
      for (int l = 0; l < 6; ++l) acc += J[i][l] * C[l][j];
      JC[i][j] = acc;
    }
  T M[6][6];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) {
      T acc = T(0.0);
      for (int l = 0; l < 6; ++l) acc += JC[i][l] * J[j][l];
      M[i][j] = acc;
    }
  // symmetric by definition: average the two triangles (see kf_update)
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) out[i][j] = 0.5 * (M[i][j] + M[j][i]) + Q[i][j];
}

// One full predict step to a given layer: propagate, transport the
// covariance, add material noise at the destination.
template <class T>
bool predict(const Geom& g, int layer, const T p0[6], const T C0[6][6], const T& fscale,
             const T& dr, T p1[6], T C1[6][6]) {
  T J[6][6], Q[6][6];
  if (!propagate_with_jacobian<T>(g, layer, p0, fscale, dr, p1, J)) return false;
  material_noise<T>(g.L[layer], p1, Q);
  transport_cov<T>(J, C0, Q, C1);
  return true;
}

// ------------------------------------------------------------------------
// Seed estimate from three hits: circle through the transverse points
// (centre from the perpendicular bisectors), charge sign from the sense of
// rotation, phi = tangent direction at hit 1, cot(theta) = dz / arc(1 -> 3).
// Position = hit 1.
static void seed_estimate(const Geom& g, const double m1[3], const double m2[3],
                          const double m3[3], double p[6]) {
  double ax = m2[0] - m1[0], ay = m2[1] - m1[1];
  double bx = m3[0] - m1[0], by = m3[1] - m1[1];
  double d = 2.0 * (ax * by - ay * bx);
  p[0] = m1[0]; p[1] = m1[1]; p[2] = m1[2];
  double a2 = ax * ax + ay * ay, b2 = bx * bx + by * by;
  if (std::fabs(d) < 1e-300 || g.bz == 0.0) {
    p[3] = 0.0;
    p[4] = std::atan2(by, bx);
    double s13 = std::sqrt(b2);
    p[5] = std::atan2(s13, m3[2] - m1[2]);
    return;
  }
  double cx = m1[0] + (by * a2 - ay * b2) / d;
  double cy = m1[1] + (ax * b2 - bx * a2) / d;
  double rho = std::hypot(m1[0] - cx, m1[1] - cy);
  // cross(P2-P1, P3-P2) > 0: counter-clockwise, omega > 0
  double cr = ax * (m3[1] - m2[1]) - ay * (m3[0] - m2[0]);
  double sg = cr > 0 ? 1.0 : -1.0;
  double om = sg / rho;
  p[3] = -om / (kC * g.bz);
  double tx = -sg * (m1[1] - cy), ty = sg * (m1[0] - cx);
  p[4] = std::atan2(ty, tx);
  double b1 = std::atan2(m1[1] - cy, m1[0] - cx);
  double b3 = std::atan2(m3[1] - cy, m3[0] - cx);
  double turn = std::fmod(sg * (b3 - b1), 2 * kPi);
  if (turn < 0) turn += 2 * kPi;
  double s13 = turn * rho;
  p[5] = std::atan2(s13, m3[2] - m1[2]);
}

struct Prior {
  double spos = 0.1, sk_rel = 0.5, sphi = 0.05, stheta = 0.05;
};

static void prior_cov(const Prior& pr, const double p[6], double C[6][6]) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) C[i][j] = 0.0;
  C[0][0] = C[1][1] = C[2][2] = pr.spos * pr.spos;
  double sk = pr.sk_rel * std::fabs(p[3]);
  C[3][3] = sk * sk;
  C[4][4] = pr.sphi * pr.sphi;
  C[5][5] = pr.stheta * pr.stheta;
}

// ------------------------------------------------------------------------
// Hit binning: per layer, n_eta equal bins in pseudorapidity over the
// layer's own eta range and n_phi equal bins in phi over [-pi, pi).
// Barrel: eta = asinh(z / R), range +-asinh(zmax / R).  Disk:
// eta = asinh(Z / r), r over [rmin, rmax].  Points on an edge go to the
// upper bin, phi = pi wraps to bin 0, eta outside the range is clamped.
static void eta_range(const Layer& Lr, double& lo, double& hi) {
  if (Lr.kind == BARREL) {
    lo = std::asinh(Lr.lo / Lr.pos);
    hi = std::asinh(Lr.hi / Lr.pos);
  } else {
    double a = std::asinh(Lr.pos / Lr.hi), b = std::asinh(Lr.pos / Lr.lo);
    lo = std::min(a, b);
    hi = std::max(a, b);
  }
}

static int eta_bin_of(const Geom& g, const Layer& Lr, double eta) {
  double lo, hi;
  eta_range(Lr, lo, hi);
  double f = std::floor((eta - lo) / (hi - lo) * g.neta);
  if (f < 0) f = 0;
  if (f > g.neta - 1) f = g.neta - 1;
  return (int)f;
}

static int phi_bin_of(const Geom& g, double phi) {
  int b = (int)std::floor((phi + kPi) / (2 * kPi) * g.nphi);
  if (b >= g.nphi) b -= g.nphi;
  if (b < 0) b += g.nphi;
  return b;
}

static double hit_eta(const Layer& Lr, double x, double y, double z) {
  if (Lr.kind == BARREL) return std::asinh(z / Lr.pos);
  return std::asinh(Lr.pos / std::sqrt(x * x + y * y));  // r of a float32 hit
}

static bool finite3(double x, double y, double z) {
  return std::isfinite(x) && std::isfinite(y) && std::isfinite(z);
}

// A hit with a coordinate that is not finite has no place on its layer: it
// gets no bin (-1) and is not indexed, like a hit without a layer.
static int hit_bin(const Geom& g, int layer, double x, double y, double z) {
  if (!finite3(x, y, z)) return -1;
  const Layer& Lr = g.L[layer];
  int eb = eta_bin_of(g, Lr, hit_eta(Lr, x, y, z));
  int pb = phi_bin_of(g, std::atan2(y, x));
  return eb * g.nphi + pb;
}

// ------------------------------------------------------------------------
// Event view used by building.
struct EventHits {
  const float *x, *y, *z;
  const int* layer;
  int begin, end;                          // global hit index range
  std::vector<std::vector<int>> by_layer;  // ascending global index
  // binned index: per layer, per bin, ascending global index
  std::vector<std::vector<std::vector<int>>> bins;
};

static void index_event(const Geom& g, EventHits& ev) {
  int nl = (int)g.L.size();
  ev.by_layer.assign(nl, {});
  ev.bins.assign(nl, std::vector<std::vector<int>>(g.neta * g.nphi));
  for (int h = ev.begin; h < ev.end; ++h) {
    int l = ev.layer[h];
    if (l < 0 || l >= nl) continue;
    const int b = hit_bin(g, l, ev.x[h], ev.y[h], ev.z[h]);
    if (b < 0) continue;
    ev.by_layer[l].push_back(h);
    ev.bins[l][b].push_back(h);
  }
}

struct Pair {
  int hit;
  double chi2;
};

// Every hit of the layer with chi2 < cut, ascending hit index (brute force).
static std::vector<Pair> compat_brute(const Geom& g, const EventHits& ev, int layer,
                                      const double p[6], const double C[6][6], double cut) {
  std::vector<Pair> out;
  for (int h : ev.by_layer[layer]) {
    double m[3] = {ev.x[h], ev.y[h], ev.z[h]}, c2;
    if (chi2_of<double>(g.L[layer], p, C, m, c2) && c2 < cut) out.push_back({h, c2});
  }
  return out;
}

// The same list through the binned index: the bounding box of the chi2
// ellipsoid (|r_u| <= sqrt(cut S_uu), |r_v| <= sqrt(cut S_vv)) mapped to
// phi and eta ranges, every hit of the covered bins tested.
static std::vector<Pair> compat_binned(const Geom& g, const EventHits& ev, int layer,
                                       const double p[6], const double C[6][6], double cut) {
  const Layer& Lr = g.L[layer];
  double H[3][3];
  local_frame<double>(Lr, p, H);
  double Suu = Lr.su * Lr.su, Svv = Lr.sv * Lr.sv;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Suu += H[0][i] * C[i][j] * H[0][j];
      Svv += H[1][i] * C[i][j] * H[1][j];
    }
  double Snn = Lr.sn * Lr.sn;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Snn += H[2][i] * C[i][j] * H[2][j];
  double wu = std::sqrt(cut * Suu) * (1 + 1e-9) + 1e-9;
  double wv = std::sqrt(cut * Svv) * (1 + 1e-9) + 1e-9;
  double wn = std::sqrt(cut * Snn) * (1 + 1e-9) + 1e-9;
  double rp = std::hypot(p[0], p[1]);
  double php = std::atan2(p[1], p[0]);
  double dphi, elo, ehi;
  if (Lr.kind == BARREL) {
    // r_u = r_h sin(dphi) and r_n = r_h cos(dphi) - r_p: a compatible hit has
    // r_h cos(dphi) >= r_p - w_n > 0 (so |dphi| < pi/2) and
    // |sin(dphi)| <= w_u / r_h <= w_u / (r_p - w_n)
    double rmin = rp - wn;
    dphi = (rmin <= 0 || wu >= rmin) ? kPi : std::asin(wu / rmin);
    elo = std::asinh((p[2] - wv) / Lr.pos);
    ehi = std::asinh((p[2] + wv) / Lr.pos);
  } else {
    double rmin = rp - wv;
    double rmax = std::sqrt(wu * wu + (rp + wv) * (rp + wv));
    dphi = (rmin <= 0 || wu >= rmin) ? kPi : std::asin(wu / rmin);
    double a = std::asinh(Lr.pos / rmax);
    double b = rmin > 0 ? std::asinh(Lr.pos / rmin) : (Lr.pos > 0 ? 1e300 : -1e300);
    elo = std::min(a, b);
    ehi = std::max(a, b);
  }
  double lo, hi;
  eta_range(Lr, lo, hi);
  int eb0 = eta_bin_of(g, Lr, elo), eb1 = eta_bin_of(g, Lr, ehi);
  std::vector<int> phib;
  if (dphi >= kPi * 0.5) {
    for (int b = 0; b < g.nphi; ++b) phib.push_back(b);
  } else {
    double bw = 2 * kPi / g.nphi;
    int b0 = (int)std::floor((php - dphi + kPi) / bw);
    int b1 = (int)std::floor((php + dphi + kPi) / bw);
    for (int b = b0; b <= b1; ++b) phib.push_back(((b % g.nphi) + g.nphi) % g.nphi);
    std::sort(phib.begin(), phib.end());
    phib.erase(std::unique(phib.begin(), phib.end()), phib.end());
  }
  std::vector<Pair> out;
  for (int eb = eb0; eb <= eb1; ++eb)
    for (int pb : phib)
      for (int h : ev.bins[layer][eb * g.nphi + pb]) {
        double m[3] = {ev.x[h], ev.y[h], ev.z[h]}, c2;
        if (chi2_of<double>(Lr, p, C, m, c2) && c2 < cut) out.push_back({h, c2});
      }
  std::sort(out.begin(), out.end(), [](const Pair& a, const Pair& b) { return a.hit < b.hit; });
  return out;
}

// ------------------------------------------------------------------------
// Navigation: from the current layer, the next surface is the candidate
// with the smaller positive path length among
//   * the next barrel layer outward (by index when on a barrel layer, else
//     the first with R > r), valid if its outgoing crossing has |z| <= zmax;
//   * the next disks in the direction of motion, the first whose crossing
//     has r within [rmin, rmax] while the track still moves outward.
// Returns -1 when there is none.
static int navigate(const Geom& g, int cur, const double p[6], double fscale) {
  double best = 1e300;
  int bl = -1;
  const Layer& C = g.L[cur];
  // barrel candidate
  int nb = -1;
  if (C.kind == BARREL) {
    for (size_t i = 0; i < g.barrel.size(); ++i)
      if (g.barrel[i] == cur && i + 1 < g.barrel.size()) nb = g.barrel[i + 1];
  } else {
    double r = std::hypot(p[0], p[1]);
    for (int id : g.barrel)
      if (g.L[id].pos > r) { nb = id; break; }
  }
  if (nb >= 0) {
    double s;
    if (path_to_cylinder<double>(g, p, fscale, g.L[nb].pos, s)) {
      double q[6];
      helix<double>(p, s, omega_of<double>(g, p[3], fscale), q);
      if (std::fabs(q[2]) <= g.L[nb].hi && s < best) { best = s; bl = nb; }
    }
  }
  // disk candidate
  double ct = std::cos(p[5]);
  const std::vector<int>& dl = ct > 0 ? g.dpos : g.dneg;
  if (std::fabs(ct) > 1e-12) {
    for (int id : dl) {
      double Z = g.L[id].pos;
      if (id == cur) continue;
      if ((ct > 0 && Z <= p[2]) || (ct < 0 && Z >= p[2])) continue;
      double s;
      if (!path_to_disk<double>(p, Z, s)) continue;
      double q[6];
      helix<double>(p, s, omega_of<double>(g, p[3], fscale), q);
      if (q[0] * std::cos(q[4]) + q[1] * std::sin(q[4]) < 0.0) break;  // turned
      double r = std::hypot(q[0], q[1]);
      if (r > g.L[id].hi) break;                    // left radially
      if (r < g.L[id].lo) continue;                 // passes inside the disk
      if (s < best) { best = s; bl = id; }
      break;
    }
  }
  return bl;
}

// ------------------------------------------------------------------------
// Track building (Sec. 1, 2, 3 of the paper): beam search over layers.
struct Cand {
  double p[6];
  double C[6][6];
  int layer;
  int nhits, nholes, consec;
  double chi2;
  bool done;
  std::vector<int> hits;  // seed hits, then one entry per step (-1 hole)
};

struct Child {
  int parent;
  int hit;    // >= 0 hit, -1 hole, -2 stop (candidate finished)
  int nhits, nholes;
  double chi2;
  double pair_chi2;
};

// Ranking key: more hits first, then fewer holes, then smaller total chi2,
// then parent slot, then hit index (holes after hits).
static bool child_less(const Child& a, const Child& b) {
  if (a.nhits != b.nhits) return a.nhits > b.nhits;
  if (a.nholes != b.nholes) return a.nholes < b.nholes;
  if (a.chi2 != b.chi2) return a.chi2 < b.chi2;
  if (a.parent != b.parent) return a.parent < b.parent;
  unsigned ha = (unsigned)a.hit, hb = (unsigned)b.hit;  // -1, -2 sort last
  return ha < hb;
}

// Score ranking (Sec. 3 re-tunes the score that decides which candidates
// are best, for short tracks; the paper gives no formula, the reading is
// ours): score = w_hit n_hits - w_hole n_holes - w_chi2 chi2, higher first,
// then parent slot, then hit index (holes after hits).
struct ScoreLess {
  double wh, wm, wc;
  double score(const Child& c) const { return wh * c.nhits - wm * c.nholes - wc * c.chi2; }
  bool operator()(const Child& a, const Child& b) const {
    const double sa = score(a), sb = score(b);
    if (sa != sb) return sa > sb;
    if (a.parent != b.parent) return a.parent < b.parent;
    return (unsigned)a.hit < (unsigned)b.hit;
  }
};

struct BuildParams {
  double chi2_cut = 30.0;
  int max_cands = 6;
  int max_holes = 3;
  int max_steps = 64;
  int brute = 0;
  int overlap = 0;  // recover a second hit on the layer of a kept hit child
  int score = 0;    // rank by ScoreLess with these weights (0: child_less)
  double w_hit = 0.0, w_hole = 0.0, w_chi2 = 0.0;
};

struct SeedResult {
  std::vector<Cand> cands;
  long steps = 0;      // (candidate, surface) pairs propagated
  long pairs = 0;      // compatible pairs found
  long updates = 0;    // KF updates of kept children
};

static bool seed_state(const Geom& g, const EventHits& ev, const int sh[3], const Prior& pr,
                       double p[6], double C[6][6], double& chi2) {
  double m[3][3];
  for (int i = 0; i < 3; ++i) {
    m[i][0] = ev.x[sh[i]]; m[i][1] = ev.y[sh[i]]; m[i][2] = ev.z[sh[i]];
    if (!finite3(m[i][0], m[i][1], m[i][2])) return false;  // a seed needs three real points
  }
  seed_estimate(g, m[0], m[1], m[2], p);
  prior_cov(pr, p, C);
  chi2 = 0.0;
  for (int i = 0; i < 3; ++i) {
    int l = ev.layer[sh[i]];
    if (i > 0) {
      double p1[6], C1[6][6];
      if (!predict<double>(g, l, p, C, 1.0, 0.0, p1, C1)) return false;
      std::memcpy(p, p1, sizeof(p1));
      std::memcpy(C, C1, sizeof(C1));
    } else {
      double Q[6][6];
      material_noise<double>(g.L[l], p, Q);
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) C[a][b] += Q[a][b];
    }
    double c2;
    if (!kf_update<double>(g.L[l], p, C, m[i], c2)) return false;
    chi2 += c2;
  }
  return true;
}

static SeedResult build_seed(const Geom& g, const EventHits& ev, const int sh[3],
                             const BuildParams& bp, const Prior& pr) {
  SeedResult R;
  Cand c0;
  if (!seed_state(g, ev, sh, pr, c0.p, c0.C, c0.chi2)) return R;
  c0.layer = ev.layer[sh[2]];
  c0.nhits = 3; c0.nholes = 0; c0.consec = 0; c0.done = false;
  c0.hits = {sh[0], sh[1], sh[2]};
  std::vector<Cand> beam{c0};
  for (int step = 0; step < bp.max_steps; ++step) {
    bool any = false;
    for (auto& c : beam) any |= !c.done;
    if (!any) break;
    std::vector<Child> kids;
    std::vector<Cand> pred(beam.size());
    std::vector<int> next(beam.size(), -1);
    for (int slot = 0; slot < (int)beam.size(); ++slot) {
      Cand& c = beam[slot];
      Child stop{slot, -2, c.nhits, c.nholes, c.chi2, 0.0};
      if (c.done) { kids.push_back(stop); continue; }
      int nl = navigate(g, c.layer, c.p, 1.0);
      if (nl >= 0) {
        Cand& q = pred[slot];
        if (!predict<double>(g, nl, c.p, c.C, 1.0, 0.0, q.p, q.C)) nl = -1;
      }
      if (nl < 0) { kids.push_back(stop); continue; }
      next[slot] = nl;
      R.steps++;
      std::vector<Pair> comp = bp.brute ? compat_brute(g, ev, nl, pred[slot].p, pred[slot].C, bp.chi2_cut)
                                        : compat_binned(g, ev, nl, pred[slot].p, pred[slot].C, bp.chi2_cut);
      R.pairs += (long)comp.size();
      int n0 = (int)kids.size();
      for (auto& pr2 : comp)
        kids.push_back(Child{slot, pr2.hit, c.nhits + 1, c.nholes, c.chi2 + pr2.chi2, pr2.chi2});
      if (c.consec < bp.max_holes)
        kids.push_back(Child{slot, -1, c.nhits, c.nholes + 1, c.chi2, 0.0});
      if ((int)kids.size() == n0) kids.push_back(stop);
    }
    if (bp.score)
      std::sort(kids.begin(), kids.end(), ScoreLess{bp.w_hit, bp.w_hole, bp.w_chi2});
    else
      std::sort(kids.begin(), kids.end(), child_less);
    if ((int)kids.size() > bp.max_cands) kids.resize(bp.max_cands);
    std::vector<Cand> nb;
    for (const Child& k : kids) {
      const Cand& par = beam[k.parent];
      Cand c = par;
      if (k.hit == -2) {
        c.done = true;
      } else {
        const Cand& q = pred[k.parent];
        std::memcpy(c.p, q.p, sizeof(c.p));
        std::memcpy(c.C, q.C, sizeof(c.C));
        c.layer = next[k.parent];
        if (k.hit >= 0) {
          double m[3] = {ev.x[k.hit], ev.y[k.hit], ev.z[k.hit]}, c2;
          kf_update<double>(g.L[c.layer], c.p, c.C, m, c2);
          R.updates++;
          c.nhits++; c.consec = 0; c.chi2 = k.chi2;
          c.hits.push_back(k.hit);
          if (bp.overlap) {
            // overlap recovery (Sec. 3 names it as planned work; the reading
            // is ours): on the state just updated with k.hit, the hits of the
            // same layer with a larger index and chi2 < cut are compatible;
            // the best of them by (chi2, index) becomes a second hit of this
            // layer.  The index condition keeps two children of one parent
            // that took the two hits of one overlap from recovering each
            // other's hit and becoming one candidate twice.
            std::vector<Pair> comp = bp.brute ? compat_brute(g, ev, c.layer, c.p, c.C, bp.chi2_cut)
                                              : compat_binned(g, ev, c.layer, c.p, c.C, bp.chi2_cut);
            int h2 = -1;
            double x2 = 0.0;
            for (const Pair& q : comp) {
              if (q.hit <= k.hit) continue;
              if (h2 < 0 || q.chi2 < x2 || (q.chi2 == x2 && q.hit < h2)) { h2 = q.hit; x2 = q.chi2; }
            }
            if (h2 >= 0) {
              double m2[3] = {ev.x[h2], ev.y[h2], ev.z[h2]}, c2b;
              kf_update<double>(g.L[c.layer], c.p, c.C, m2, c2b);
              R.updates++;
              c.nhits++; c.chi2 += x2;
              c.hits.push_back(h2);
            }
          }
        } else {
          c.nholes++; c.consec++;
          c.hits.push_back(-1);
        }
      }
      nb.push_back(std::move(c));
    }
    beam = std::move(nb);
  }
  R.cands = std::move(beam);
  return R;
}

// ------------------------------------------------------------------------
// Fit (Sec. 1): start at hit 1 from the three-hit estimate with the prior
// covariance, update at hit 1, then predict and update through hit N.
// Alignment a_L = (dr, drphi, dz) of barrel layer L: the hit recorded in the
// nominal frame is moved to ((R+dr) cos(phi + drphi/R), (R+dr) sin(...),
// z + dz) and the track is propagated to the cylinder R + dr; the field is
// B * fscale.  Returns the total chi2.
template <class T>
bool fit_track(const Geom& g, const float* hx, const float* hy, const float* hz,
               const int* hl, const int* hits, int n, const T* align, const T& fscale,
               const Prior& pr, T pout[6], T Cout[6][6], T& chi2_tot) {
  using std::cos; using std::sin;
  if (n < 3) return false;
  // every hit must be a real point
  for (int i = 0; i < n; ++i)
    if (!finite3(hx[hits[i]], hy[hits[i]], hz[hits[i]])) return false;
  double m0[3][3];
  for (int i = 0; i < 3; ++i) {
    m0[i][0] = hx[hits[i]]; m0[i][1] = hy[hits[i]]; m0[i][2] = hz[hits[i]];
  }
  double ps[6], Cs[6][6];
  seed_estimate(g, m0[0], m0[1], m0[2], ps);  // starting point: no gradient
  prior_cov(pr, ps, Cs);
  T p[6], C[6][6];
  for (int i = 0; i < 6; ++i) {
    p[i] = T(ps[i]);
    for (int j = 0; j < 6; ++j) C[i][j] = T(Cs[i][j]);
  }
  chi2_tot = T(0.0);
  for (int i = 0; i < n; ++i) {
    int h = hits[i];
    int l = hl[h];
    const Layer& Lr = g.L[l];
    T m[3];
    T dr = T(0.0);
    if (Lr.kind == BARREL) {
      dr = align ? align[3 * l + 0] : T(0.0);
      T drphi = align ? align[3 * l + 1] : T(0.0);
      T dz = align ? align[3 * l + 2] : T(0.0);
      double phl = std::atan2((double)hy[h], (double)hx[h]);
      T ang = phl + drphi / Lr.pos;
      T rr = Lr.pos + dr;
      m[0] = rr * cos(ang);
      m[1] = rr * sin(ang);
      m[2] = (double)hz[h] + dz;
    } else {
      m[0] = T((double)hx[h]); m[1] = T((double)hy[h]); m[2] = T((double)hz[h]);
    }
    if (i == 0) {
      // the estimate starts on hit 1 as recorded
      T Q[6][6];
      material_noise<T>(Lr, p, Q);
      for (int a = 0; a < 6; ++a)
        for (int b = 0; b < 6; ++b) C[a][b] += Q[a][b];
    } else {
      T p1[6], C1[6][6];
      if (!predict<T>(g, l, p, C, fscale, dr, p1, C1)) return false;
      for (int a = 0; a < 6; ++a) {
        p[a] = p1[a];
        for (int b = 0; b < 6; ++b) C[a][b] = C1[a][b];
      }
    }
    T c2;
    if (!kf_update<T>(Lr, p, C, m, c2)) return false;
    chi2_tot = chi2_tot + c2;
  }
  for (int a = 0; a < 6; ++a) {
    pout[a] = p[a];
    for (int b = 0; b < 6; ++b) Cout[a][b] = C[a][b];
  }
  return true;
}

}  // namespace kfo

// ==========================================================================
// C interface for the test harness (ctypes).  Layer table rows are
// (kind, pos, lo, hi, x0, su, sv, sn) in float64.  Covariances cross this
// interface as full row-major 6x6 float64 blocks.
using namespace kfo;

extern "C" {

int kfo_version() { return 1; }

// bins[i] = eta_bin * n_phi + phi_bin of hit i on its layer (-1 if the layer
// id is out of range).
void kfo_bin_hits(const double* layers, int nl, int neta, int nphi, const float* x,
                  const float* y, const float* z, const int* layer, int n, int* bins) {
  Geom g = make_geom(layers, nl, 0.0, neta, nphi);
  for (int i = 0; i < n; ++i) {
    int l = layer[i];
    bins[i] = (l < 0 || l >= nl) ? -1 : hit_bin(g, l, x[i], y[i], z[i]);
  }
}

// Helix position at transverse path s (for the analytic pins).
void kfo_helix(double bz, const double* p0, double s, double fscale, double* out) {
  Geom g;
  g.bz = bz;
  helix<double>(p0, s, omega_of<double>(g, p0[3], fscale), out);
}

// Path length to a cylinder of radius R (outgoing root); returns 0 if none.
int kfo_path_to_cylinder(double bz, const double* p0, double R, double fscale, double* s) {
  Geom g;
  g.bz = bz;
  return path_to_cylinder<double>(g, p0, fscale, R, *s) ? 1 : 0;
}

// Propagate state + Jacobian to a layer (no covariance); returns 1 if ok.
int kfo_propagate(const double* layers, int nl, double bz, int layer, const double* p0,
                  double fscale, double dr, double* p1, double* J) {
  Geom g = make_geom(layers, nl, bz, 20, 128);
  double JJ[6][6];
  if (!propagate_with_jacobian<double>(g, layer, p0, fscale, dr, p1, JJ)) return 0;
  std::memcpy(J, JJ, sizeof(JJ));
  return 1;
}

void kfo_material_noise(const double* layers, int nl, int layer, const double* p, double* Q) {
  Geom g = make_geom(layers, nl, 0.0, 20, 128);
  double QQ[6][6];
  material_noise<double>(g.L[layer], p, QQ);
  std::memcpy(Q, QQ, sizeof(QQ));
}

// Predict (propagate + J C J^T + Q) to a given layer.
int kfo_predict(const double* layers, int nl, double bz, int layer, const double* p0,
                const double* C0, double fscale, double dr, double* p1, double* C1) {
  Geom g = make_geom(layers, nl, bz, 20, 128);
  double c0[6][6], c1[6][6];
  std::memcpy(c0, C0, sizeof(c0));
  if (!predict<double>(g, layer, p0, c0, fscale, dr, p1, c1)) return 0;
  std::memcpy(C1, c1, sizeof(c1));
  return 1;
}

// Kalman update with hit m on a layer; p, C in place; chi2 out.
int kfo_update(const double* layers, int nl, int layer, double* p, double* C, const double* m,
               double* chi2) {
  Geom g = make_geom(layers, nl, 0.0, 20, 128);
  double cc[6][6];
  std::memcpy(cc, C, sizeof(cc));
  double c2;
  if (!kf_update<double>(g.L[layer], p, cc, m, c2)) return 0;
  std::memcpy(C, cc, sizeof(cc));
  *chi2 = c2;
  return 1;
}

int kfo_navigate(const double* layers, int nl, double bz, int cur, const double* p,
                 double fscale) {
  Geom g = make_geom(layers, nl, bz, 20, 128);
  return navigate(g, cur, p, fscale);
}

void kfo_seed_estimate(const double* layers, int nl, double bz, const double* m1,
                       const double* m2, const double* m3, double* p) {
  Geom g = make_geom(layers, nl, bz, 20, 128);
  seed_estimate(g, m1, m2, m3, p);
}

// Seed states (KF over the three seed hits from the prior) -> state at hit 3.
// ok[i] = 1 on success.
void kfo_seed_states(const double* layers, int nl, double bz, const float* x, const float* y,
                     const float* z, const int* layer, int nhits, const int* seeds, int ns,
                     const double* prior, double* p_out, double* C_out, double* chi2,
                     int* ok) {
  Geom g = make_geom(layers, nl, bz, 20, 128);
  EventHits ev{x, y, z, layer, 0, nhits, {}, {}};
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  for (int i = 0; i < ns; ++i) {
    double p[6] = {0, 0, 0, 0, 0, 0}, C[6][6] = {}, c2 = 0;
    ok[i] = seed_state(g, ev, seeds + 3 * i, pr, p, C, c2) ? 1 : 0;
    if (!ok[i]) {
      std::memset(p, 0, sizeof(p));
      std::memset(C, 0, sizeof(C));
      c2 = 0;
    }
    std::memcpy(p_out + 6 * i, p, sizeof(p));
    std::memcpy(C_out + 36 * i, C, sizeof(C));
    chi2[i] = c2;
  }
}

// One building step for a set of candidate states on given layers, on
// identical inputs: navigate, predict, then list every compatible hit of the
// event (brute force when brute != 0, else through the oracle's own binned
// index).  Outputs: next layer (-1 none), predicted p/C, and the pairs in CSR
// form (pair_off[n+1]; pair_hit/pair_chi2 sized by the caller with
// max_pairs, count returned; -1 when max_pairs is too small).
long kfo_step_compat(const double* layers, int nl, double bz, int neta, int nphi,
                     const float* x, const float* y, const float* z, const int* layer,
                     int ev_begin, int ev_end, int n, const int* cur_layer, const double* p_in,
                     const double* C_in, double chi2_cut, int brute, int* next_layer,
                     double* p_out, double* C_out, int* pair_off, int* pair_hit,
                     double* pair_chi2, long max_pairs) {
  Geom g = make_geom(layers, nl, bz, neta, nphi);
  EventHits ev{x, y, z, layer, ev_begin, ev_end, {}, {}};
  index_event(g, ev);
  long np = 0;
  pair_off[0] = 0;
  for (int i = 0; i < n; ++i) {
    double p[6], C[6][6];
    std::memcpy(p, p_in + 6 * i, sizeof(p));
    std::memcpy(C, C_in + 36 * i, sizeof(C));
    int nlay = navigate(g, cur_layer[i], p, 1.0);
    double p1[6], C1[6][6];
    if (nlay >= 0 && !predict<double>(g, nlay, p, C, 1.0, 0.0, p1, C1)) nlay = -1;
    next_layer[i] = nlay;
    if (nlay >= 0) {
      std::memcpy(p_out + 6 * i, p1, sizeof(p1));
      std::memcpy(C_out + 36 * i, C1, sizeof(C1));
      std::vector<Pair> comp = brute ? compat_brute(g, ev, nlay, p1, C1, chi2_cut)
                                     : compat_binned(g, ev, nlay, p1, C1, chi2_cut);
      for (auto& q : comp) {
        if (np >= max_pairs) return -1;
        pair_hit[np] = q.hit;
        pair_chi2[np] = q.chi2;
        ++np;
      }
    } else {
      std::fill(p_out + 6 * i, p_out + 6 * i + 6, 0.0);
      std::fill(C_out + 36 * i, C_out + 36 * i + 36, 0.0);
    }
    pair_off[i + 1] = (int)np;
  }
  return np;
}

// Build tracks for the seeds of one or more events.  seed_event[i] selects
// the event (hits [ev_off[e], ev_off[e+1])).  Output per seed: up to K
// candidates (best first), slots beyond the count are zero.
//   out_n[s]                     number of candidates
//   out_hits[(s*K + j)*maxh + t] hit list (-1 hole, -3 unused)
//   out_nhits, out_nholes, out_chi2 per candidate; out_p (6), out_C (36)
//   stats[3] += steps, pairs, updates
void kfo_build(const double* layers, int nl, double bz, int neta, int nphi, const float* x,
               const float* y, const float* z, const int* layer, const int* ev_off, int nev,
               const int* seeds, const int* seed_event, int ns, double chi2_cut, int K,
               int max_holes, int brute, int overlap, const double* score_w, const double* prior, int maxh,
               int* out_n,
               int* out_hits, int* out_nhits, int* out_nholes, double* out_chi2,
               double* out_p, double* out_C, long* stats) {
  Geom g = make_geom(layers, nl, bz, neta, nphi);
  BuildParams bp;
  bp.chi2_cut = chi2_cut; bp.max_cands = K; bp.max_holes = max_holes; bp.brute = brute;
  bp.overlap = overlap;
  if (score_w) {
    bp.score = 1;
    bp.w_hit = score_w[0]; bp.w_hole = score_w[1]; bp.w_chi2 = score_w[2];
  }
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  std::vector<EventHits> evs(nev);
  for (int e = 0; e < nev; ++e) {
    evs[e] = EventHits{x, y, z, layer, ev_off[e], ev_off[e + 1], {}, {}};
    index_event(g, evs[e]);
  }
  for (int s = 0; s < ns; ++s) {
    SeedResult R = build_seed(g, evs[seed_event[s]], seeds + 3 * s, bp, pr);
    stats[0] += R.steps; stats[1] += R.pairs; stats[2] += R.updates;
    out_n[s] = (int)R.cands.size();
    for (int j = 0; j < K; ++j) {
      long o = (long)s * K + j;
      int* hl = out_hits + o * maxh;
      for (int t = 0; t < maxh; ++t) hl[t] = -3;
      if (j >= (int)R.cands.size()) {
        out_nhits[o] = 0; out_nholes[o] = 0; out_chi2[o] = 0;
        std::fill(out_p + 6 * o, out_p + 6 * o + 6, 0.0);
        std::fill(out_C + 36 * o, out_C + 36 * o + 36, 0.0);
        continue;
      }
      const Cand& c = R.cands[j];
      for (int t = 0; t < (int)c.hits.size() && t < maxh; ++t) hl[t] = c.hits[t];
      out_nhits[o] = c.nhits; out_nholes[o] = c.nholes; out_chi2[o] = c.chi2;
      std::memcpy(out_p + 6 * o, c.p, sizeof(c.p));
      std::memcpy(out_C + 36 * o, c.C, sizeof(c.C));
    }
  }
}

// Fit tracks (CSR hit lists).  align: nullable float64[3 L].
void kfo_fit(const double* layers, int nl, double bz, const float* x, const float* y,
             const float* z, const int* layer, const int* trk_off, const int* trk_hits, int nt,
             const double* align, double fscale, const double* prior, double* p_out,
             double* C_out, double* chi2, int* ndof, int* ok) {
  Geom g = make_geom(layers, nl, bz, 20, 128);
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  for (int t = 0; t < nt; ++t) {
    int n = trk_off[t + 1] - trk_off[t];
    double p[6], C[6][6], c2 = 0;
    ok[t] = fit_track<double>(g, x, y, z, layer, trk_hits + trk_off[t], n, align, fscale, pr, p, C, c2) ? 1 : 0;
    std::memcpy(p_out + 6 * t, p, sizeof(p));
    std::memcpy(C_out + 36 * t, C, sizeof(C));
    chi2[t] = ok[t] ? c2 : 0.0;
    ndof[t] = 2 * n - 5;
  }
}

// Gradient of the total chi2 (sum over the tracks that fit) with respect to
// the 3 L alignment values and the field scale, written to grad[3 L + 1].
// mode 0: forward mode (dual numbers, all 3 L + 1 directions);
// mode 1: reverse mode (tape), the oracle's own adjoint.
// Returns the total chi2.
double kfo_fit_grad(const double* layers, int nl, double bz, const float* x, const float* y,
                    const float* z, const int* layer, const int* trk_off, const int* trk_hits,
                    int nt, const double* align, double fscale, const double* prior, int mode,
                    double* grad) {
  Geom g = make_geom(layers, nl, bz, 20, 128);
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  int np = 3 * nl + 1;
  for (int i = 0; i < np; ++i) grad[i] = 0.0;
  double total = 0.0;
  if (mode == 0) {
    constexpr int NB = 8;  // directions per pass
    using DN = Dual<double, NB>;
    for (int base = 0; base < np; base += NB) {
      std::vector<DN> a(3 * nl);
      for (int i = 0; i < 3 * nl; ++i) a[i] = DN::make(align ? align[i] : 0.0, (i >= base && i < base + NB) ? i - base : -1);
      DN fs = DN::make(fscale, (3 * nl >= base && 3 * nl < base + NB) ? 3 * nl - base : -1);
      double tot = 0.0;
      for (int t = 0; t < nt; ++t) {
        DN p[6], C[6][6], c2;
        int n = trk_off[t + 1] - trk_off[t];
        if (!fit_track<DN>(g, x, y, z, layer, trk_hits + trk_off[t], n, a.data(), fs, pr, p, C, c2)) continue;
        tot += c2.v;
        for (int d = 0; d < NB && base + d < np; ++d) grad[base + d] += c2.d[d];
      }
      total = tot;
    }
  } else {
    for (int t = 0; t < nt; ++t) {
      tape().clear();
      std::vector<Rv> a(3 * nl);
      for (int i = 0; i < 3 * nl; ++i) a[i] = Rv::input(align ? align[i] : 0.0);
      Rv fs = Rv::input(fscale);
      Rv p[6], C[6][6], c2;
      int n = trk_off[t + 1] - trk_off[t];
      if (!fit_track<Rv>(g, x, y, z, layer, trk_hits + trk_off[t], n, a.data(), fs, pr, p, C, c2)) continue;
      total += c2.v;
      std::vector<double> adj = tape().backward(c2.id);
      for (int i = 0; i < 3 * nl; ++i) grad[i] += adj[a[i].id];
      grad[3 * nl] += adj[fs.id];
    }
    tape().clear();
  }
  return total;
}

}  // extern "C"
