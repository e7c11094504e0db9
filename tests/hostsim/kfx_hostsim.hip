// Test-only host build of the GPU library's device math (kfx_math.h,
// kfx_work.h): the same __host__ __device__ functions, called on the CPU so
// that their logic can be checked against the oracle without a GPU.  The
// library never loads this; only tests/ do.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../paper_2002_06295_amd/csrc/kfx_work.h"

using namespace kfx;

namespace {
Geometry make_geo(const double* table, int nl, double bz) {
  Geometry G{};
  G.n_layers = nl;
  G.bz = bz;
  G.n_eta = 20;
  G.n_phi = 128;
  for (int i = 0; i < nl; ++i) {
    const double* r = table + 8 * i;
    Layer& L = G.L[i];
    L.kind = (int)r[0];
    L.pos = r[1];
    L.lo = r[2];
    L.hi = r[3];
    L.x0 = (float)r[4];
    L.v_u = (float)(r[5] * r[5]);
    L.v_v = (float)(r[6] * r[6]);
    L.v_n = (float)(r[7] * r[7]);
    // the pseudorapidity range of the layer's bins, as the library sets it
    if (L.kind == kBarrel) {
      L.eta_lo = asinh(L.lo / L.pos);
      L.eta_hi = asinh(L.hi / L.pos);
    } else {
      const double a = asinh(L.pos / L.hi), b = asinh(L.pos / L.lo);
      L.eta_lo = a < b ? a : b;
      L.eta_hi = a < b ? b : a;
    }
    L.eta_scale = (float)(G.n_eta / (L.eta_hi - L.eta_lo));
  }
  return G;
}

void to_state(const double* p, const float* cov21, State& s) {
  s.x = p[0]; s.y = p[1]; s.z = p[2]; s.k = p[3]; s.phi = p[4]; s.th = p[5];
  for (int i = 0; i < 21; ++i) s.C[i] = cov21[i];
}

void from_state(const State& s, double* p, float* cov21) {
  p[0] = s.x; p[1] = s.y; p[2] = s.z; p[3] = s.k; p[4] = s.phi; p[5] = s.th;
  for (int i = 0; i < 21; ++i) cov21[i] = s.C[i];
}
}  // namespace

extern "C" {

// transport to a layer along path s found by the device navigation rules
// of that surface kind; returns s (< 0 if not reached)
float hs_predict(const double* table, int nl, double bz, int layer, const double* p, const float* cov,
                 double* p_out, float* cov_out) {
  Geometry G = make_geo(table, nl, bz);
  State st, out;
  to_state(p, cov, st);
  const double cphi = cos(st.phi), sphi = sin(st.phi);
  const double kappa = -kHcD * bz;
  const Layer& L = G.L[layer];
  const double s = path_to_layer(st, L, L.pos, cphi, sphi, kappa * st.k);
  if (!(s > 0.0)) return -1.0f;
  transport(st, L, cphi, sphi, s, kappa, out);
  from_state(out, p_out, cov_out);
  return (float)s;
}

float hs_update(const double* table, int nl, int layer, const double* p, const float* cov, const double* m,
                double* p_out, float* cov_out) {
  Geometry G = make_geo(table, nl, 0.0);
  State st;
  to_state(p, cov, st);
  const float c2 = kf_update_fp64(st, G.L[layer], m[0], m[1], m[2]);
  from_state(st, p_out, cov_out);
  return c2;
}

}  // extern "C"

extern "C" {

// seed state (start estimate + KF over the three seed hits)
int hs_seed_state(const double* table, int nl, double bz, const float* x, const float* y, const float* z,
                  const int* layer, int nhits, const int* sh, const float* prior, double* p_out, float* cov_out,
                  float* chi2) {
  Geometry G = make_geo(table, nl, bz);
  G.n_layers = nl;
  HitsView H{x, y, z, layer, nullptr, nhits, 1};
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  State st;
  float c2 = 0.0f;
  const bool ok = seed_state(G, H, sh, pr, st, c2);
  from_state(st, p_out, cov_out);
  *chi2 = c2;
  return ok ? 1 : 0;
}

// fit of tracks (CSR hit lists), results per track
void hs_fit(const double* table, int nl, double bz, const float* x, const float* y, const float* z,
            const int* layer, int nhits, const int* trk_off, const int* trk_hits, int nt, const float* prior,
            const float* align, float fscale, double* p_out, float* cov_out, float* chi2, int* ndof, int* status) {
  Geometry G = make_geo(table, nl, bz);
  HitsView H{x, y, z, layer, nullptr, nhits, 1};
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  std::vector<double> par(6 * (size_t)nt);
  std::vector<float> cov(21 * (size_t)nt);
  FitOut o;
  o.state = StateSoA{par.data(), cov.data(), nt};
  o.chi2 = chi2;
  o.ndof = ndof;
  o.status = status;
  o.ckpt = StateSoA{nullptr, nullptr, 0};
  o.n_tracks = nt;
  for (int t = 0; t < nt; ++t) {
    fit_track(G, H, trk_off, trk_hits, t, pr, align, fscale, o);
    State s;
    load_state(o.state, t, s);
    from_state(s, p_out + 6 * t, cov_out + 21 * t);
  }
}

}  // extern "C"

// navigation from layer `cur`: next layer (-1 none) and its path
extern "C" int hs_navigate(const double* table, int nl, double bz, int cur, const double* p, double* s_out) {
  Geometry G = make_geo(table, nl, bz);
  std::vector<int> bar, dp, dn;
  for (int i = 0; i < nl; ++i) {
    if (G.L[i].kind == kBarrel) bar.push_back(i);
    else if (G.L[i].pos > 0) dp.push_back(i);
    else dn.push_back(i);
  }
  std::sort(bar.begin(), bar.end(), [&](int a, int b) { return G.L[a].pos < G.L[b].pos; });
  std::sort(dp.begin(), dp.end(), [&](int a, int b) { return G.L[a].pos < G.L[b].pos; });
  std::sort(dn.begin(), dn.end(), [&](int a, int b) { return G.L[a].pos > G.L[b].pos; });
  G.n_barrel = (int)bar.size();
  G.n_dpos = (int)dp.size();
  G.n_dneg = (int)dn.size();
  for (int i = 0; i < kMaxLayers; ++i) G.next_barrel[i] = -1;
  for (size_t i = 0; i < bar.size(); ++i) {
    G.barrel[i] = bar[i];
    G.next_barrel[bar[i]] = (i + 1 < bar.size()) ? bar[i + 1] : -1;
  }
  for (size_t i = 0; i < dp.size(); ++i) G.dpos[i] = dp[i];
  for (size_t i = 0; i < dn.size(); ++i) G.dneg[i] = dn[i];
  nav_tables(G);
  State st;
  float c[21] = {0};
  to_state(p, c, st);
  double cphi, sphi;
  sincos_d(st.phi, sphi, cphi);
  return navigate(G, cur, st, cphi, sphi, -kHcD * bz * st.k, *s_out);
}

extern "C" double hs_path_cylinder(const double* p, double bz, double Rc) {
  State st;
  float c[21] = {0};
  to_state(p, c, st);
  const double cphi = cos(st.phi), sphi = sin(st.phi);
  return path_to_cylinder(st, cphi, sphi, -kHcD * bz * st.k, Rc);
}

#include "../../paper_2002_06295_amd/csrc/kfx_adjoint.h"

namespace {
struct HostAcc {
  double* g;
  int nl;
  KFX_HD void add(int l, int c, double v) { g[3 * l + c] += v; }
  KFX_HD void field(double v) { g[3 * nl] += v; }
};
}  // namespace

extern "C" {

// forward fit with checkpoints, then the reverse sweep of every track that
// fitted; grad[3 nl + 1] = d(sum_t w_t chi2_t)/d(align, fscale)
double hs_fit_grad(const double* table, int nl, double bz, const float* x, const float* y, const float* z,
                   const int* layer, int nhits, const int* trk_off, const int* trk_hits, int nt,
                   const float* prior, const float* align, float fscale, const double* w, double* grad) {
  Geometry G = make_geo(table, nl, bz);
  HitsView H{x, y, z, layer, nullptr, nhits, 1};
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  long longest = 0;
  for (int t = 0; t < nt; ++t) longest = std::max<long>(longest, trk_off[t + 1] - trk_off[t]);
  const long ns = std::max<long>((long)nt * longest, 1);
  std::vector<double> par(6 * (size_t)nt), cpar(6 * (size_t)ns);
  std::vector<float> cov(21 * (size_t)nt), ccov(21 * (size_t)ns), c2(nt);
  std::vector<int> ndof(nt), status(nt);
  FitOut o;
  o.state = StateSoA{par.data(), cov.data(), nt};
  o.chi2 = c2.data();
  o.ndof = ndof.data();
  o.status = status.data();
  o.ckpt = StateSoA{cpar.data(), ccov.data(), ns};
  o.n_tracks = nt;
  for (int i = 0; i < 3 * nl + 1; ++i) grad[i] = 0.0;
  HostAcc acc{grad, nl};
  double tot = 0.0;
  for (int t = 0; t < nt; ++t) {
    fit_track(G, H, trk_off, trk_hits, t, pr, align, fscale, o);
    if (status[t] != 1) continue;
    tot += c2[t];
    fit_track_backward(G, H, trk_off, trk_hits, t, pr, align, fscale, o.ckpt, nt, w ? w[t] : 1.0, acc);
  }
  return tot;
}

}  // extern "C"

// search window of a prediction on `layer` (the device's window_bins) and
// the bin of a point on that layer (the binning's hit_bin): eta rows
// [eb0, eb1], phi bins pb0 .. pb0 + npb - 1 modulo n_phi
extern "C" void hs_window(const double* table, int nl, int layer, const double* p, const float* cov, float cut,
                          int* out4) {
  Geometry G = make_geo(table, nl, 0.0);
  State st;
  to_state(p, cov, st);
  Frame F;
  make_frame(st, G.L[layer], F);
  const Window w = window_bins(G, G.L[layer], st, F, cut);
  out4[0] = w.eb0;
  out4[1] = w.eb1;
  out4[2] = w.pb0;
  out4[3] = w.npb;
}

extern "C" int hs_hit_bin(const double* table, int nl, int layer, float x, float y, float z) {
  Geometry G = make_geo(table, nl, 0.0);
  return hit_bin(G, layer, x, y, z);
}

// the frame's rows (u, v, n) and S^-1 of a prediction, for placing points
// on its chi2 ellipse
extern "C" void hs_frame(const double* table, int nl, int layer, const double* p, const float* cov, double* h9,
                         double* si6) {
  Geometry G = make_geo(table, nl, 0.0);
  State st;
  to_state(p, cov, st);
  Frame F;
  make_frame(st, G.L[layer], F);
  for (int a = 0; a < 3; ++a)
    for (int j = 0; j < 3; ++j) h9[3 * a + j] = F.h[a][j];
  for (int i = 0; i < 6; ++i) si6[i] = F.Si[i];
}

// the building's chi2 of a candidate-hit pair on `layer` (FP32 frame and
// S^-1 of the prediction, FP64 difference of the positions)
extern "C" float hs_pair_chi2(const double* table, int nl, int layer, const double* p, const float* cov,
                              const float* hit3) {
  Geometry G = make_geo(table, nl, 0.0);
  State st;
  to_state(p, cov, st);
  Frame F;
  make_frame(st, G.L[layer], F);
  PairFrame P;
  pair_frame(st, F, G.L[layer].kind == kDisk, P);
  return pair_chi2(P, make_float4(hit3[0], hit3[1], hit3[2], 0.0f));
}

// FP64-covariance forms of the transport and the update (the fit's
// arithmetic), for comparing the building's FP32 covariance step by step
extern "C" double hs_predict64(const double* table, int nl, double bz, int layer, const double* p, const double* cov,
                               double* p_out, double* cov_out) {
  Geometry G = make_geo(table, nl, bz);
  StateT<double> st, out;
  st.x = p[0]; st.y = p[1]; st.z = p[2]; st.k = p[3]; st.phi = p[4]; st.th = p[5];
  for (int i = 0; i < 21; ++i) st.C[i] = cov[i];
  double cphi, sphi;
  sincos_d(st.phi, sphi, cphi);
  const double kappa = -kHcD * bz;
  const Layer& L = G.L[layer];
  const double s = path_to_layer(st, L, L.pos, cphi, sphi, kappa * st.k);
  if (!(s > 0.0)) return -1.0;
  transport(st, L, cphi, sphi, s, kappa, out);
  p_out[0] = out.x; p_out[1] = out.y; p_out[2] = out.z; p_out[3] = out.k; p_out[4] = out.phi; p_out[5] = out.th;
  for (int i = 0; i < 21; ++i) cov_out[i] = out.C[i];
  return s;
}

extern "C" double hs_update64(const double* table, int nl, int layer, const double* p, const double* cov,
                              const double* m, double* p_out, double* cov_out) {
  Geometry G = make_geo(table, nl, 0.0);
  StateT<double> st;
  st.x = p[0]; st.y = p[1]; st.z = p[2]; st.k = p[3]; st.phi = p[4]; st.th = p[5];
  for (int i = 0; i < 21; ++i) st.C[i] = cov[i];
  FrameT<double> F;
  make_frame(st, G.L[layer], F);
  const double c2 = kf_update(st, F, m[0], m[1], m[2]);
  p_out[0] = st.x; p_out[1] = st.y; p_out[2] = st.z; p_out[3] = st.k; p_out[4] = st.phi; p_out[5] = st.th;
  for (int i = 0; i < 21; ++i) cov_out[i] = st.C[i];
  return c2;
}

extern "C" int hs_seed_state64(const double* table, int nl, double bz, const float* x, const float* y,
                               const float* z, const int* layer, const int* sh, const float* prior, double* p_out,
                               double* cov_out, double* chi2) {
  Geometry G = make_geo(table, nl, bz);
  Prior pr{prior[0], prior[1], prior[2], prior[3]};
  double m[3][3];
  for (int i = 0; i < 3; ++i) {
    m[i][0] = x[sh[i]];
    m[i][1] = y[sh[i]];
    m[i][2] = z[sh[i]];
  }
  StateT<double> st;
  seed_estimate(G.bz, m[0], m[1], m[2], st);
  prior_cov(pr, st);
  const double kappa = -kHcD * G.bz;
  double c2sum = 0.0;
  for (int i = 0; i < 3; ++i) {
    const Layer& Ld = G.L[layer[sh[i]]];
    double c2 = 0.0;
    if (!filter_step(st, Ld, Ld.pos, kappa, i == 0, m[i], c2)) return 0;
    c2sum += c2;
  }
  p_out[0] = st.x; p_out[1] = st.y; p_out[2] = st.z; p_out[3] = st.k; p_out[4] = st.phi; p_out[5] = st.th;
  for (int i = 0; i < 21; ++i) cov_out[i] = st.C[i];
  *chi2 = c2sum;
  return 1;
}

// the binning kernel's FP32-first bin of a batch of points on `layer`
extern "C" void hs_hit_bin_fast_many(const double* table, int nl, int layer, const float* x, const float* y,
                                     const float* z, int n, int* out_fast, int* out_exact) {
  Geometry G = make_geo(table, nl, 0.0);
  for (int i = 0; i < n; ++i) {
    out_fast[i] = hit_bin_fast(G, layer, x[i], y[i], z[i]);
    out_exact[i] = hit_bin(G, layer, x[i], y[i], z[i]);
  }
}
