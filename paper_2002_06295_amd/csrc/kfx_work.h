// Per-thread work items of the track-building and fitting kernels.
//
// Each kernel of the plain path is a thin launcher around one of these
// functions (one call per thread); the fused persistent kernel reuses the
// same pieces per lane.  They are __host__ __device__ so that a test-only
// host build can check the kernel logic on the CPU; the library itself only
// runs them on the GPU.
//
// Paper: arXiv 2002.06295.  Sec. 1: building is a combinatorial search that
// starts from a seed in the innermost layers and proceeds outward with the
// propagate/update Kalman step; fitting applies the Kalman filter to the
// hits that building found.  Sec. 2: per layer, a seed keeps a bounded number
// of its children (the highest-ranked ones) and the bookkeeping of the
// explored candidates is compact.  Sec. 3: holes are counted the same way
// everywhere and take part in the ranking.
#pragma once

#include "kfx_math.h"

namespace kfx {

constexpr int kMaxK = 16;        // candidates per seed (compile-time cap)
constexpr int kMaxSteps = 40;    // surfaces crossed after the seed
constexpr int kSeedHits = 3;

// ---- hit binning ---------------------------------------------------------
// Per layer: n_eta equal bins of pseudorapidity over the layer's own range
// (barrel: asinh(z/R) over +-zmax; disk: asinh(Z/r) over [rmin, rmax]) and
// n_phi equal bins of phi over [-pi, pi).  Computed in FP64 from the FP32
// hit coordinates; an edge belongs to the upper bin, phi = pi wraps to 0,
// eta outside the range is clamped.  A hit with a coordinate that is not
// finite gets no bin (-1) and is not indexed.
KFX_HD int eta_bin(const Geometry& G, const Layer& Lr, double eta) {
  double f = floor((eta - Lr.eta_lo) / (Lr.eta_hi - Lr.eta_lo) * (double)G.n_eta);
  if (f < 0.0) f = 0.0;
  if (f > (double)(G.n_eta - 1)) f = (double)(G.n_eta - 1);
  return (int)f;
}

KFX_HD int phi_bin(const Geometry& G, double phi) {
  int b = (int)floor((phi + kPi) / (2.0 * kPi) * (double)G.n_phi);
  if (b >= G.n_phi) b -= G.n_phi;
  if (b < 0) b += G.n_phi;
  return b;
}

KFX_HD bool finite_hit(float x, float y, float z) {
  return __builtin_isfinite(x) && __builtin_isfinite(y) && __builtin_isfinite(z);
}

KFX_HD int hit_bin(const Geometry& G, int layer, float x, float y, float z) {
  if (!finite_hit(x, y, z)) return -1;
  const Layer& Lr = G.L[layer];
  const double xd = x, yd = y, zd = z;
  const double eta = Lr.kind == kBarrel ? asinh(zd / Lr.pos) : asinh(Lr.pos / sqrt(xd * xd + yd * yd));
  return eta_bin(G, Lr, eta) * G.n_phi + phi_bin(G, atan2(yd, xd));
}

// The same bin from FP32 estimates where they decide it: eta and phi from
// the short FP32 asinh and atan2 below (errors under 2e-6 and 1e-6), scaled
// to bin units; when the scaled value lies more than 2e-4 bin from every bin
// edge (the estimate's error in bin units is below 1e-5), its floor is the
// FP64 result's; otherwise the FP64 computation decides.  About one hit in
// a few thousand takes the FP64 path.
KFX_HD float asinh_win(float x);
KFX_HD float atan2_win(float y, float x);
KFX_HD bool near_edge(float f) {
  const float d = f - floorf(f);
  return d < 2e-4f || d > 1.0f - 2e-4f;
}
KFX_HD int hit_bin_fast(const Geometry& G, int layer, float x, float y, float z) {
  if (!finite_hit(x, y, z)) return -1;
  const Layer& Lr = G.L[layer];
  const float r = sqrtf(x * x + y * y);
  const float eta = Lr.kind == kBarrel ? asinh_win(z / (float)Lr.pos) : asinh_win((float)Lr.pos / r);
  const float fe = (eta - (float)Lr.eta_lo) * Lr.eta_scale;
  const float fp = (atan2_win(y, x) + 3.14159265358979f) * ((float)G.n_phi * 0.15915494309189535f);
  const bool clamped = fe < -2e-4f || fe > (float)G.n_eta + 2e-4f;
  // (a value within the margin of 0 or of the top edge counts as near an
  // edge too, which covers the clamping of eta and the wrap of phi)
  if (!__builtin_isfinite(fe) || !__builtin_isfinite(fp) || (!clamped && near_edge(fe)) || near_edge(fp) || r < 0.1f)
    return hit_bin(G, layer, x, y, z);
  int eb = (int)floorf(fe);
  eb = eb < 0 ? 0 : (eb > G.n_eta - 1 ? G.n_eta - 1 : eb);
  return eb * G.n_phi + (int)floorf(fp);
}

// ---- window: bins that can hold a hit with chi2 < cut ------------------
// The chi2 ellipsoid's bounding box |r_u| <= sqrt(cut S_uu) etc. mapped to
// phi and eta ranges, widened to cover FP32 rounding, so the window is a
// superset of the compatible hits.
struct Window {
  int eb0, eb1;  // eta bins, inclusive
  int pb0, npb;  // phi bins pb0 .. pb0 + npb - 1 (mod n_phi)
};

KFX_HD int eta_bin_f(const Geometry& G, const Layer& Lr, float eta) {
  float f = floorf((eta - (float)Lr.eta_lo) * Lr.eta_scale);
  f = fminf(fmaxf(f, 0.0f), (float)(G.n_eta - 1));
  return (int)f;
}

// Short FP32 forms of asinh and atan2 for the window bounds, whose margins
// (1e-5 absolute and more) cover their errors: asinh(x) = log(|x| +
// sqrt(x^2 + 1)) with the sign of x, within 1e-6 absolute for the
// arguments the geometry gives (|x| < 1e4); atan2 by octant reduction to
// atan on [0, 1], there an odd polynomial of degree 15 fitted to atan
// (Lawson-weighted least squares; 1.5e-7 in FP32), within 1e-6 overall.
KFX_HD float asinh_win(float x) {
  const float ax = fabsf(x);
  const float v = __builtin_log2f(ax + __builtin_sqrtf(fmaf(ax, ax, 1.0f))) * 0.6931471805599453f;
  return x < 0.0f ? -v : v;
}
KFX_HD float atan2_win(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float hi = fmaxf(ax, ay), lo = fminf(ax, ay);
  const float t = hi > 0.0f ? lo / hi : 0.0f;
  const float t2 = t * t;
  float p = -0.004054567310959101f;
  p = fmaf(p, t2, 0.021862957626581192f);
  p = fmaf(p, t2, -0.0559123270213604f);
  p = fmaf(p, t2, 0.0964219719171524f);
  p = fmaf(p, t2, -0.1390862911939621f);
  p = fmaf(p, t2, 0.19946566224098206f);
  p = fmaf(p, t2, -0.33329859375953674f);
  p = fmaf(p, t2, 0.9999993443489075f);
  float a = t * p;
  if (ay > ax) a = 1.5707963267948966f - a;
  if (x < 0.0f) a = 3.141592653589793f - a;
  return y < 0.0f ? -a : a;
}

// An upper bound of asin(w / r) for 0 <= w < r: tan(asin(x)) >= asin(x),
// i.e. w / sqrt(r^2 - w^2), wider by a relative (w/r)^2/3 when w/r is
// small; a superset window is all the scan needs.
KFX_HD float asin_upper(float w, float r) { return w / sqrtf((r - w) * (r + w)); }

KFX_HD Window window_bins(const Geometry& G, const Layer& Lr, const State& pr, const Frame& F,
                          float cut, float inflate = 1.0f) {
  const float infl = (1.0f + 1e-4f) * inflate;
  const float wu = sqrtf(cut * F.S[0]) * infl + 1e-5f;
  const float wv = sqrtf(cut * F.S[2]) * infl + 1e-5f;
  const float wn = sqrtf(cut * F.S[5]) * infl + 1e-5f;
  const float px = (float)pr.x, py = (float)pr.y;
  const float rp = sqrtf(px * px + py * py);
  const float php = atan2_win(py, px);
  Window w;
  if (!__builtin_isfinite(wu) || !__builtin_isfinite(wv) || !__builtin_isfinite(wn) || !__builtin_isfinite(rp) || !__builtin_isfinite(php) ||
      !__builtin_isfinite((float)pr.z)) {
    w.eb0 = 1;  // empty window
    w.eb1 = 0;
    w.pb0 = 0;
    w.npb = 0;
    return w;
  }
  float dphi, elo, ehi;
  if (Lr.kind == kBarrel) {
    const float rmin = rp - wn;
    dphi = (rmin <= 0.0f || wu >= rmin) ? 4.0f : asin_upper(wu, rmin) + 1e-5f;
    const float iR = 1.0f / (float)Lr.pos;
    elo = asinh_win(((float)pr.z - wv) * iR) - 1e-5f;
    ehi = asinh_win(((float)pr.z + wv) * iR) + 1e-5f;
  } else {
    const float rmin = rp - wv;
    const float rmax = sqrtf(wu * wu + (rp + wv) * (rp + wv));
    dphi = (rmin <= 0.0f || wu >= rmin) ? 4.0f : asin_upper(wu, rmin) + 1e-5f;
    const float Z = (float)Lr.pos;
    const float a = asinh_win(Z / rmax);
    const float b = rmin > 0.0f ? asinh_win(Z / rmin) : (Z > 0.0f ? 1e30f : -1e30f);
    elo = fminf(a, b) - 1e-5f;
    ehi = fmaxf(a, b) + 1e-5f;
  }
  w.eb0 = eta_bin_f(G, Lr, elo);
  w.eb1 = eta_bin_f(G, Lr, ehi);
  if (dphi >= 1.5f) {
    w.pb0 = 0;
    w.npb = G.n_phi;
  } else {
    const float ibw = (float)G.n_phi * (float)(0.5 / kPi);  // phi bins per radian
    const float pi = (float)kPi;
    int b0 = (int)floorf((php - dphi + pi) * ibw);
    int b1 = (int)floorf((php + dphi + pi) * ibw);
    int n = b1 - b0 + 1;
    if (n > G.n_phi) n = G.n_phi;
    b0 %= G.n_phi;
    if (b0 < 0) b0 += G.n_phi;
    w.pb0 = b0;
    w.npb = n;
  }
  return w;
}

// ---- candidate bookkeeping ---------------------------------------------
// meta word: bits 0-7 n_hits, 8-15 n_holes, 16-23 consecutive holes,
// 24-31 flags.
constexpr int kFlagLive = 1;   // slot holds a candidate
constexpr int kFlagDone = 2;   // candidate finished (no further surface)

KFX_HD int meta_pack(int nh, int nho, int consec, int flags) {
  return nh | (nho << 8) | (consec << 16) | (flags << 24);
}
KFX_HD int meta_nhits(int m) { return m & 0xff; }
KFX_HD int meta_nholes(int m) { return (m >> 8) & 0xff; }
KFX_HD int meta_consec(int m) { return (m >> 16) & 0xff; }
KFX_HD int meta_flags(int m) { return (m >> 24) & 0xff; }

// Ranking key of a child, smaller is better: more hits, then fewer holes,
// then smaller total chi2, then parent slot, then the child's rank among
// its parent's children (hits by (chi2, hit index), the hole after them).
KFX_HD uint64_t child_key(int nhits, int nholes, float chi2, int parent, int rank) {
  uint32_t cb;
  __builtin_memcpy(&cb, &chi2, 4);
  return ((uint64_t)(63 - nhits) << 58) | ((uint64_t)nholes << 52) | ((uint64_t)cb << 20) |
         ((uint64_t)parent << 10) | ((uint64_t)rank << 5);
}

// The ranking of a call: the key above, or a score (reading 19: Sec. 3
// re-tunes the score that decides which candidates are best, for short
// tracks; no formula is given) s = w_hit n_hits - w_hole n_holes - w_chi2
// chi2 in FP32, highest first, then parent slot, then rank.
struct RankW {
  float w_hit, w_hole, w_chi2;
  int on;
};

// Order-preserving integer image of a float (below).
KFX_HD uint32_t chi2_image(float c);

KFX_HD uint64_t rank_key(const RankW& w, int nhits, int nholes, float chi2, int parent, int rank) {
  if (!w.on) return child_key(nhits, nholes, chi2, parent, rank);
  const float sc = w.w_hit * (float)nhits - w.w_hole * (float)nholes - w.w_chi2 * chi2;
  return ((uint64_t)chi2_image(-sc) << 32) | ((uint64_t)parent << 10) | ((uint64_t)rank << 5);
}

// Child codes: hit index >= 0, kHole, kStop.
constexpr int kHole = -1;
constexpr int kStop = -2;

// Order-preserving integer image of a chi2 (a value rounded below zero, or
// -0, still sorts first; -0 and +0 map to the same image) and its inverse.
KFX_HD uint32_t chi2_image(float c) {
  uint32_t b;
  const float cz = c + 0.0f;  // -0 -> +0
  __builtin_memcpy(&b, &cz, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
KFX_HD float chi2_from_image(uint32_t k) {
  const uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  float c;
  __builtin_memcpy(&c, &b, 4);
  return c;
}
// (chi2, hit index) as one key, ascending in chi2 then in hit index
KFX_HD uint64_t pair_key(float c, int h) { return ((uint64_t)chi2_image(c) << 32) | (uint32_t)h; }
KFX_HD float pair_key_chi2(uint64_t k) { return chi2_from_image((uint32_t)(k >> 32)); }
KFX_HD int pair_key_hit(uint64_t k) { return (int)(uint32_t)k; }
constexpr uint64_t kNoKey = ~0ull;

// Best-K list of one candidate's compatible hits: the KM smallest
// (chi2, hit) keys in ascending order (empty entries kNoKey), held in
// registers; n = the number of valid entries, capped at the runtime K <= KM
// (entries from n on are not read).  Insertion is one compare-exchange
// pass over the unrolled list: no branches, and no element is indexed by a
// runtime value (which would put the list in scratch memory).
template <int KM>
struct BestK {
  uint64_t k[KM];
  int n;
};

template <int KM>
KFX_HD void bestk_init(BestK<KM>& b) {
#pragma unroll
  for (int i = 0; i < KM; ++i) b.k[i] = kNoKey;
  b.n = 0;
}

template <int KM>
KFX_HD void bestk_insert_key(BestK<KM>& b, int K, uint64_t key) {
#pragma unroll
  for (int i = 0; i < KM; ++i) {
    const uint64_t e = b.k[i];
    b.k[i] = key < e ? key : e;
    key = key < e ? e : key;
  }
  b.n = b.n < K ? b.n + 1 : K;
}

template <int KM>
KFX_HD void bestk_insert(BestK<KM>& b, int K, float c, int h) {
  bestk_insert_key(b, K, pair_key(c, h));
}

// key of the K-th entry of a full list (kNoKey otherwise): a pair enters
// the list only with a smaller key
template <int KM>
KFX_HD uint64_t bestk_threshold(const BestK<KM>& b, int K) {
  uint64_t t = kNoKey;
#pragma unroll
  for (int i = 0; i < KM; ++i)
    if (i == K - 1) t = b.k[i];
  return b.n == K ? t : kNoKey;
}

// ---- SoA state access ---------------------------------------------------
// par: [6][stride] float64 (x, y, z, k, phi, theta); cov: [21][stride]
// float32 (packed lower triangle).
struct StateSoA {
  double* par;
  float* cov;
  long stride;
};

KFX_HD void load_state(const StateSoA& a, long i, State& s) {
  s.x = a.par[i];
  s.y = a.par[a.stride + i];
  s.z = a.par[2 * a.stride + i];
  s.k = a.par[3 * a.stride + i];
  s.phi = a.par[4 * a.stride + i];
  s.th = a.par[5 * a.stride + i];
#pragma unroll
  for (int j = 0; j < 21; ++j) s.C[j] = a.cov[j * a.stride + i];
}

KFX_HD void store_state(const StateSoA& a, long i, const State& s) {
  a.par[i] = s.x;
  a.par[a.stride + i] = s.y;
  a.par[2 * a.stride + i] = s.z;
  a.par[3 * a.stride + i] = s.k;
  a.par[4 * a.stride + i] = s.phi;
  a.par[5 * a.stride + i] = s.th;
#pragma unroll
  for (int j = 0; j < 21; ++j) a.cov[j * a.stride + i] = s.C[j];
}

// ---- hits ----------------------------------------------------------------
struct HitsView {
  const float *x, *y, *z;
  const int* layer;
  const int* ev_off;   // [n_events + 1]
  int n_hits, n_events;
};

// Binned index: for event e, layer l, bin b the sorted hits (x, y, z, index
// as bits) occupy [off[key], off[key+1]), key = e ev_stride + l nb + b, with
// ev_stride = L nb (one counting sort over the batch) or L nb + 1 (one
// workgroup per event: the extra key of an event holds no bin).
struct BinIndex {
  const int* off;
  const float4* sorted;
  int n_layers, n_bins;
  long ev_stride;
};

KFX_HD long bin_key(const BinIndex& B, int ev, int layer, int bin) {
  return (long)ev * B.ev_stride + (long)layer * B.n_bins + bin;
}

// ---- window scan ---------------------------------------------------------
// The window's bins as contiguous ranges of the sorted hits: the phi bins of
// one eta row are adjacent in the index, so a row is one range (two when the
// phi range wraps at pi).  Range r of nrows * nseg: row r / nseg, segment
// r % nseg.
struct ScanWin {
  long row0;      // key of (event, layer, first eta row, phi bin 0)
  int nrows, nseg;
  int b0, b1;     // first segment: phi bins [b0, b1)
  int w1;         // second segment (wrap): phi bins [0, w1)
};

KFX_HD ScanWin scan_win(const Geometry& G, const BinIndex& B, int ev, int layer, const Window& w) {
  ScanWin s;
  const int wrap = w.pb0 + w.npb - G.n_phi;
  s.row0 = bin_key(B, ev, layer, 0) + (long)w.eb0 * G.n_phi;
  s.nrows = (w.eb1 >= w.eb0 && w.npb > 0) ? w.eb1 - w.eb0 + 1 : 0;
  s.nseg = wrap > 0 ? 2 : 1;
  s.b0 = w.pb0;
  s.b1 = wrap > 0 ? G.n_phi : w.pb0 + w.npb;
  s.w1 = wrap;
  if (s.nrows > 0 && 2 * w.npb > G.n_phi) {
    // more than half of phi: the whole rows instead (still a superset), and
    // consecutive whole rows are one contiguous range of the sorted hits
    s.b0 = 0;
    s.b1 = s.nrows * G.n_phi;
    s.nrows = 1;
    s.nseg = 1;
    s.w1 = 0;
  }
  return s;
}

KFX_HD int scan_nranges(const ScanWin& s) { return s.nrows * s.nseg; }

// sorted hits [a, e) of range r
KFX_HD void scan_range(const ScanWin& s, const BinIndex& B, int n_phi, int r, int& a, int& e) {
  const bool two = s.nseg == 2;
  const int row = two ? (r >> 1) : r;
  const bool second = two && (r & 1);
  const long k = s.row0 + (long)row * n_phi;
  a = B.off[k + (second ? 0 : s.b0)];
  e = B.off[k + (second ? s.w1 : s.b1)];
}

// What the chi2 of a candidate-hit pair needs: the predicted position, the
// azimuth (cos, sin) that defines the measurement frame, and S^-1.  The
// FP64 position is held as two FP32 parts, hi = its rounding to FP32 and lo
// = the rounding of the rest: m - x = (m - hi) - lo, where m - hi is exact
// for a hit near the prediction (Sterbenz) and lo is below 2^-24 |x|, so
// the residual comes out within an ulp of the FP64 difference rounded to
// FP32, in two FP32 subtractions instead of three FP64 operations and two
// conversions per coordinate of every hit scanned.
struct PairFrame {
  float xh, xl, yh, yl, zh, zl;
  float c, s;
  int disk;
  float Si[6];
};

KFX_HD void split_f64(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

KFX_HD void pair_frame(const State& pr, const Frame& F, bool disk, PairFrame& P) {
  split_f64(pr.x, P.xh, P.xl);
  split_f64(pr.y, P.yh, P.yl);
  split_f64(pr.z, P.zh, P.zl);
  P.c = F.h[0][1];
  P.s = -F.h[0][0];
  P.disk = disk ? 1 : 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) P.Si[i] = F.Si[i];
}

// chi2 of the pair: residual r = H (m - x), then r^T S^-1 r (the
// arithmetic of residual() and chi2_of() on the full frame, with the
// difference m - x from the two-part position).
KFX_HD float pair_chi2(const PairFrame& P, const float4& hv) {
  const float dx = (hv.x - P.xh) - P.xl, dy = (hv.y - P.yh) - P.yl;
  const float dz = (hv.z - P.zh) - P.zl;
  const bool disk = P.disk != 0;
  const float z0 = 0.0f, o1 = 1.0f;
  const float h[3][3] = {{-P.s, P.c, z0},
                         {disk ? P.c : z0, disk ? P.s : z0, disk ? z0 : o1},
                         {disk ? z0 : P.c, disk ? z0 : P.s, disk ? o1 : z0}};
  float r[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) r[a] = h[a][0] * dx + h[a][1] * dy + h[a][2] * dz;
  return r[0] * r[0] * P.Si[0] + r[1] * r[1] * P.Si[2] + r[2] * r[2] * P.Si[5] +
         2.0f * (r[0] * r[1] * P.Si[1] + r[0] * r[2] * P.Si[3] + r[1] * r[2] * P.Si[4]);
}

// Scan the window of one candidate and keep the best K compatible hits
// (chi2 < cut).  Returns the number of compatible hits found (all of them,
// not only K).
template <int KM>
KFX_HD int scan_window(const Geometry& G, const BinIndex& B, int ev, int layer, const State& pr,
                       const Frame& F, float cut, int K, BestK<KM>& best, float inflate = 1.0f) {
  const Layer& Lr = G.L[layer];
  const Window w = window_bins(G, Lr, pr, F, cut, inflate);
  const ScanWin sw = scan_win(G, B, ev, layer, w);
  PairFrame P;
  pair_frame(pr, F, Lr.kind == kDisk, P);
  bestk_init(best);
  int found = 0;
  const int nr = scan_nranges(sw);
  for (int r = 0; r < nr; ++r) {
    int a, e;
    scan_range(sw, B, G.n_phi, r, a, e);
    for (int q = a; q < e; ++q) {
      const float4 hv = B.sorted[q];
      const float c2 = pair_chi2(P, hv);
      if (c2 < cut) {
        int hid;
        __builtin_memcpy(&hid, &hv.w, 4);
        ++found;
        bestk_insert(best, K, c2, hid);
      }
    }
  }
  return found;
}

// Overlap recovery (a hit of an overlapping module on the same layer): on a
// state just updated with hit h1 on `layer`, the hits of the layer with an
// index above h1 and chi2 < cut (the search's window and pair chi2 on the
// updated state); returns the best by (chi2, index), or -1.
KFX_HD int recover_overlap(const Geometry& G, const BinIndex& B, int ev, int layer, const State& st, float cut,
                           int h1, float inflate, float& chi2_out) {
  const Layer& Lr = G.L[layer];
  Frame F;
  make_frame(st, Lr, F);
  const Window w = window_bins(G, Lr, st, F, cut, inflate);
  const ScanWin sw = scan_win(G, B, ev, layer, w);
  PairFrame P;
  pair_frame(st, F, Lr.kind == kDisk, P);
  uint64_t best = kNoKey;
  const int nr = scan_nranges(sw);
  for (int r = 0; r < nr; ++r) {
    int a, e;
    scan_range(sw, B, G.n_phi, r, a, e);
    for (int q = a; q < e; ++q) {
      const float4 hv = B.sorted[q];
      int hid;
      __builtin_memcpy(&hid, &hv.w, 4);
      if (hid <= h1) continue;
      const float c2 = pair_chi2(P, hv);
      if (c2 < cut) {
        const uint64_t k = pair_key(c2, hid);
        best = k < best ? k : best;
      }
    }
  }
  if (best == kNoKey) return -1;
  chi2_out = pair_key_chi2(best);
  return pair_key_hit(best);
}

// Kalman update in FP64 for either state type.
KFX_HD double update_at(StateT<double>& st, const Layer& Ld, const double m[3]) {
  FrameT<double> F;
  make_frame(st, Ld, F);
  return kf_update(st, F, m[0], m[1], m[2]);
}
KFX_HD float update_at(State& st, const Layer& Ld, const double m[3]) {
  return kf_update_fp64(st, Ld, m[0], m[1], m[2]);
}

// ---- one filter step: transport onto the hit's layer (not at the first
// hit, where the state starts on the hit), material noise, update.
template <class R>
KFX_HD bool filter_step(StateT<R>& st, const Layer& Ld, double r_surf, double kappa, bool first,
                        const double m[3], R& chi2) {
  if (first) {
    add_material(st, Ld);
  } else {
    double cphi, sphi;
    sincos_d(st.phi, sphi, cphi);
    const double s = path_to_layer(st, Ld, r_surf, cphi, sphi, kappa * st.k);
    if (!(s > 0.0)) return false;
    StateT<R> nx;
    transport(st, Ld, cphi, sphi, s, kappa, nx);
    st = nx;
  }
  chi2 = update_at(st, Ld, m);
  return true;
}

// ---- seed state: start estimate, then KF over the three seed hits ------
// The prior is ~1e4 times wider (in variance) than the hits, so the first
// updates cancel most of it: C+ = C - K H C keeps only ~1e-4 of C, which
// FP32 would resolve to ~1e-3.  These three updates run in FP64 (a handful
// per seed, at the unpacked FP32 rate on CDNA); the search then continues in
// FP32 from the rounded result.
KFX_HD bool seed_state(const Geometry& G, const HitsView& H, const int sh[3], const Prior& pr,
                       State& out, float& chi2) {
  double m[3][3];
  for (int i = 0; i < 3; ++i)
    if (sh[i] < 0 || sh[i] >= H.n_hits) return false;
  for (int i = 0; i < 3; ++i) {
    if (!finite_hit(H.x[sh[i]], H.y[sh[i]], H.z[sh[i]])) return false;  // three real points
    m[i][0] = H.x[sh[i]];
    m[i][1] = H.y[sh[i]];
    m[i][2] = H.z[sh[i]];
  }
  StateT<double> st;
  seed_estimate(G.bz, m[0], m[1], m[2], st);
  prior_cov(pr, st);
  const double kappa = -kHcD * G.bz;
  double c2sum = 0.0;
  for (int i = 0; i < 3; ++i) {
    const int l = H.layer[sh[i]];
    if (l < 0 || l >= G.n_layers) return false;
    const Layer& Ld = G.L[l];
    double c2 = 0.0;
    if (!filter_step(st, Ld, Ld.pos, kappa, i == 0, m[i], c2)) return false;
    c2sum += c2;
  }
  convert_state(st, out);
  chi2 = (float)c2sum;
  return true;
}

// ---- fit of one track over a fixed hit list ------------------------------
// Alignment of barrel layer l, a = (dr, drphi, dz): the hit recorded in the
// nominal frame moves to ((R+dr) (cos, sin)(phi_h + drphi/R), z + dz) and
// the track is propagated to the cylinder R + dr.  The field is B * fscale.
KFX_HD void aligned_hit(const Layer& Ld, float hx, float hy, float hz, const float* a, double m[3]) {
  if (Ld.kind == kBarrel) {
    const double dr = a ? (double)a[0] : 0.0, drphi = a ? (double)a[1] : 0.0, dz = a ? (double)a[2] : 0.0;
    const double x = hx, y = hy;
    const double r = sqrt(x * x + y * y);
    const double c = x / r, s = y / r;
    const double d = drphi / Ld.pos;
    double cd, sd;
    sincos_d(d, sd, cd);
    const double R = Ld.pos + dr;
    m[0] = R * (c * cd - s * sd);
    m[1] = R * (s * cd + c * sd);
    m[2] = (double)hz + dz;
  } else {
    m[0] = hx;
    m[1] = hy;
    m[2] = hz;
  }
}

struct FitOut {
  StateSoA state;     // per track
  float* chi2;
  int* ndof;
  int* status;        // 1 ok, 0 failed
  StateSoA ckpt;      // after hit i of track t: entry i * n_tracks + t (par == nullptr: none)
  int n_tracks;
};

KFX_HD void fit_track(const Geometry& G, const HitsView& H, const int* trk_off, const int* trk_hits,
                      int t, const Prior& pr, const float* align, float fscale, const FitOut& o) {
  const int b = trk_off[t], n = trk_off[t + 1] - trk_off[t];
  State st;
  double chi2 = 0.0;
  bool ok = n >= 3;
  // checkpoints beyond the caller's capacity: the track is not fitted
  const bool ckpt_fits = !o.ckpt.par || (long)(n - 1) * o.n_tracks + t < o.ckpt.stride;
  ok = ok && ckpt_fits;
  // a hit outside the arrays, on no layer or not finite fails the track;
  // each hit is checked where it is read (the filter below stops at the
  // first such hit, and a failed track's outputs are zeros whatever it had
  // filtered), so that its four values are fetched once per fit: scattered
  // over the tracks of a wavefront, every read costs a memory sector
  auto valid = [&](int h) {
    return h >= 0 && h < H.n_hits && H.layer[h] >= 0 && H.layer[h] < G.n_layers && finite_hit(H.x[h], H.y[h], H.z[h]);
  };
  double m0[3][3];
  for (int i = 0; ok && i < 3; ++i) {
    const int h = trk_hits[b + i];
    if (!valid(h)) {
      ok = false;
    } else {
      m0[i][0] = H.x[h];
      m0[i][1] = H.y[h];
      m0[i][2] = H.z[h];
    }
  }
  if (ok) {
    // The fit runs the whole filter with an FP64 covariance: a crossing at
    // angle a to the layer normal scales the covariance terms by 1/cos^2(a),
    // and over a few steep crossings the FP32 rounding of the covariance
    // (6e-8 relative per layer) grows to ~1e-3 in chi2; the gradient of the
    // fit needs the same precision.  The stored states are rounded to FP32.
    StateT<double> sd;
    seed_estimate(G.bz, m0[0], m0[1], m0[2], sd);
    prior_cov(pr, sd);
    const double kappa_d = -kHcD * G.bz * (double)fscale;
    for (int i = 0; i < n && ok; ++i) {
      const int h = trk_hits[b + i];
      if (i >= 3 && !valid(h)) {
        ok = false;
        break;
      }
      const int l = H.layer[h];
      const Layer& Ld = G.L[l];
      const float* a = align ? align + 3 * l : nullptr;
      double m[3];
      aligned_hit(Ld, H.x[h], H.y[h], H.z[h], a, m);
      const double r_surf = Ld.pos + ((a && Ld.kind == kBarrel) ? (double)a[0] : 0.0);
      double c2 = 0.0;
      ok = filter_step(sd, Ld, r_surf, kappa_d, i == 0, m, c2);
      chi2 += c2;
      if (ok && o.ckpt.par) {
        convert_state(sd, st);
        store_state(o.ckpt, (long)i * o.n_tracks + t, st);
      }
    }
    convert_state(sd, st);
  }
  if (!ok) {
    st.x = st.y = st.z = st.k = st.phi = st.th = 0.0;
    for (int j = 0; j < 21; ++j) st.C[j] = 0.0f;
    chi2 = 0.0;
  }
  store_state(o.state, t, st);
  o.chi2[t] = (float)chi2;
  o.ndof[t] = 2 * n - 5;
  o.status[t] = ok ? 1 : (ckpt_fits ? 0 : -1);
}

}  // namespace kfx
