// C ABI of libkfx.so (declared in include/kfx.h): argument checks, the
// context (geometry + workspace pool) and the calls into the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/kfx.h"
#include "kfx_internal.h"

using namespace kfx;

struct kfx_ctx {
  int device = 0;
  std::string err;
  Geometry host_geo{};
  Geometry* dev_geo = nullptr;
  bool have_geo = false;
  // workspace pool: named device buffers, grown on demand; `active` is the
  // pool in use (a graph being captured owns its own)
  std::map<std::string, std::pair<void*, size_t>> pool;
  std::map<std::string, std::pair<void*, size_t>>* active = &pool;
  int n_cu = 256;
  size_t max_lds = 65536;  // LDS a block may use
  // hit index of the last kfx_bin_hits / kfx_build_tracks call
  bool have_index = false;
  const void* index_hits_key[3] = {nullptr, nullptr, nullptr};
  int index_n_hits = -1, index_n_events = -1;
  BinWork bw{};
  bool bin_event_ok = false;  // one-workgroup-per-event binning available
  // optional timing of build calls: per call, events before binning, after
  // binning, after the seed start, after the search and after the output,
  // recorded on the caller's stream into a ring of `ring_n` calls
  bool timing = false;
  std::vector<hipEvent_t> ring;  // kEv per slot
  int ring_n = 0, ring_next = 0, ring_count = 0;
  hipEvent_t* slot_ev = nullptr;  // events of the call in progress
  // a second stream of the context: the fused build forks the seed start
  // onto it while the caller's stream bins the hits, then joins
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
};

// Scratch of kfx_fit_tracks_backward_noalloc: the per-block partial rows of
// the gradient live in this file-scope device array (one copy per GPU, kept
// until the process ends) instead of the context's workspace pool.  In host
// code the array's name is not a device address: kernels get the address
// that hipGetSymbolAddress returned on their device (g_scratch below).
constexpr size_t kNoAllocScratchDoubles = (size_t)1 << 20;  // 8 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];
constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxScratchDevices];  // device address per device, once resolved

namespace {

// Resolves the scratch array's address on `device` (current) once per
// device; called by kfx_create.
hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return hipSuccess;  // the entry point then refuses
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch[device] = static_cast<double*>(p);
  return e;
}

double* scratch_of(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    (void)hipGetDevice(&prev);
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (prev >= 0 && cur != prev) (void)hipSetDevice(prev);
  }
};

int fail(kfx_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int hip_check(kfx_ctx* c, hipError_t e, const char* what) {
  if (e == hipSuccess) return KFX_OK;
  return fail(c, KFX_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

// Named workspace of at least `bytes`, 256-byte aligned.  Growing waits for
// the stream so that queued work never sees a freed buffer.
void* ws(kfx_ctx* c, const char* name, size_t bytes, hipStream_t st, int& rc) {
  rc = KFX_OK;
  bytes = std::max<size_t>(bytes, 256);
  auto& pool = *c->active;
  auto it = pool.find(name);
  if (it != pool.end() && it->second.second >= bytes) return it->second.first;
  if (it != pool.end()) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(it->second.first);
    pool.erase(it);
  }
  void* p = nullptr;
  const size_t grown = bytes + bytes / 4;
  if (hipMalloc(&p, grown) != hipSuccess) {
    rc = fail(c, KFX_ENOMEM, std::string("workspace allocation failed: ") + name);
    return nullptr;
  }
  pool[name] = {p, grown};
  return p;
}

// the context's second stream and its fork / join events (created once)
int side_stream(kfx_ctx* c) {
  if (c->side) return KFX_OK;
  int rc = hip_check(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming), "fork event");
  if (!rc) rc = hip_check(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming), "join event");
  if (!rc) rc = hip_check(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking), "second stream");
  return rc;
}

bool is_finite(double v) { return std::isfinite(v); }

int check_hits(kfx_ctx* c, const kfx_hits* h) {
  if (!h) return fail(c, KFX_EINVAL, "hits is NULL");
  if (h->n_hits < 0 || h->n_events < 1) return fail(c, KFX_EINVAL, "n_hits < 0 or n_events < 1");
  if (h->n_hits > 0 && (!h->x || !h->y || !h->z || !h->layer))
    return fail(c, KFX_EINVAL, "hit arrays must not be NULL");
  if (!h->event_offsets) return fail(c, KFX_EINVAL, "event_offsets is NULL");
  return KFX_OK;
}

HitsView view(const kfx_hits* h) {
  HitsView v;
  v.x = h->x;
  v.y = h->y;
  v.z = h->z;
  v.layer = h->layer;
  v.ev_off = h->event_offsets;
  v.n_hits = h->n_hits;
  v.n_events = h->n_events;
  return v;
}

StateSoA soa(const kfx_states* s) {
  StateSoA a;
  a.par = s->par;
  a.cov = s->cov;
  a.stride = (long)s->stride;
  return a;
}

int check_states(kfx_ctx* c, const kfx_states* s, long n, const char* what) {
  if (!s || !s->par || !s->cov) return fail(c, KFX_EINVAL, std::string(what) + ": NULL state arrays");
  if (s->stride < n) return fail(c, KFX_EINVAL, std::string(what) + ": stride smaller than the entry count");
  return KFX_OK;
}

Prior prior_of(const kfx_prior* p) {
  Prior r;
  r.spos = p->spos;
  r.sk_rel = p->sk_rel;
  r.sphi = p->sphi;
  r.stheta = p->stheta;
  return r;
}

int check_prior(kfx_ctx* c, const kfx_prior* p) {
  if (!p) return fail(c, KFX_EINVAL, "prior is NULL");
  const float v[4] = {p->spos, p->sk_rel, p->sphi, p->stheta};
  for (float x : v)
    if (!std::isfinite(x) || x < 0.0f) return fail(c, KFX_EINVAL, "prior must be finite and >= 0");
  return KFX_OK;
}

// Events from which the automatic choice bins one event per workgroup (a
// quarter of the CUs busy at least; below, the counting sort over the whole
// batch spreads the hits over the machine).
constexpr int kBinEventMin = 64;

// Build the hit index into the context workspace.  binning: 0 automatic,
// 1 counting sort over the batch, 2 one workgroup per event (where the
// event's bins fit LDS); the stable order (bin_out, kfx_bin_hits) always
// takes the counting sort.
int build_index(kfx_ctx* c, const kfx_hits* h, int32_t* bin_out, bool stable, hipStream_t st, int binning = 1) {
  const Geometry& G = c->host_geo;
  const long nb = (long)G.n_eta * G.n_phi;
  const bool per_event = !stable && !bin_out && c->bin_event_ok && h->n_events > 0 &&
                         (binning == 2 || (binning == 0 && h->n_events >= kBinEventMin)) &&
                         bin_event_lds_bytes(G.n_layers * nb) <= c->max_lds;
  const long n_keys = (long)h->n_events * (G.n_layers * nb + (per_event ? 1 : 0));
  if (n_keys >= (1L << 31) - 2) return fail(c, KFX_EINVAL, "events x layers x bins exceeds 2^31");
  int rc;
  BinWork& w = c->bw;
  const long nh = std::max<long>(h->n_hits, 1);
  w.key = (int*)ws(c, "bin.key", nh * 4, st, rc); if (rc) return rc;
  w.counts = (int*)ws(c, "bin.counts", (n_keys + 1) * 4, st, rc); if (rc) return rc;
  w.rank = (int*)ws(c, "bin.rank", nh * 4, st, rc); if (rc) return rc;
  w.off = (int*)ws(c, "bin.off", (n_keys + 2) * 4, st, rc); if (rc) return rc;
  w.perm = (int*)ws(c, "bin.perm", nh * 4, st, rc); if (rc) return rc;
  w.sorted = (float4*)ws(c, "bin.sorted", nh * 16, st, rc); if (rc) return rc;
  w.scan_scratch = (int*)ws(c, "bin.scan", ((n_keys + 1) / 4096 + 4) * 4, st, rc); if (rc) return rc;
  if (per_event)
    launch_bin_events(c->dev_geo, view(h), G.n_layers, (int)nb, w, st);
  else
    launch_bin(c->dev_geo, view(h), G.n_layers, (int)nb, w, bin_out, stable, st);
  if ((rc = hip_check(c, hipGetLastError(), "binning kernels"))) return rc;
  c->have_index = true;
  c->index_hits_key[0] = h->x;
  c->index_hits_key[1] = h->layer;
  c->index_hits_key[2] = h->event_offsets;
  c->index_n_hits = h->n_hits;
  c->index_n_events = h->n_events;
  return KFX_OK;
}

BinIndex index_view(const kfx_ctx* c) {
  BinIndex B;
  B.off = c->bw.off;
  B.sorted = c->bw.sorted;
  B.n_layers = c->host_geo.n_layers;
  B.n_bins = c->host_geo.n_eta * c->host_geo.n_phi;
  B.ev_stride = c->bw.ev_stride;
  return B;
}

}  // namespace

extern "C" {

int kfx_create(int device, kfx_ctx** out) {
  if (!out) return KFX_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return KFX_EHIP;
  if (device < 0 || device >= n) return KFX_EINVAL;
  kfx_ctx* c = new kfx_ctx();
  c->device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
    c->n_cu = cus;
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
    c->max_lds = (size_t)lds;
  {
    DeviceGuard dg(device);
    // the per-event binning's LDS above the default limit of a launch (if
    // the runtime refuses, the counting sort over the batch is used)
    c->bin_event_ok = bin_event_init(c->max_lds) == hipSuccess;
    (void)hipGetLastError();
    if (resolve_scratch(device) != hipSuccess) {
      delete c;
      return KFX_EHIP;
    }
  }
  *out = c;
  return KFX_OK;
}

void kfx_destroy(kfx_ctx* c) {
  if (!c) return;
  {
    DeviceGuard g(c->device);
    for (auto& kv : c->pool) (void)hipFree(kv.second.first);
    if (c->dev_geo) (void)hipFree(c->dev_geo);
    for (auto& e : c->ring)
      if (e) (void)hipEventDestroy(e);
    if (c->side) {
      (void)hipStreamSynchronize(c->side);
      (void)hipStreamDestroy(c->side);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  }
  delete c;
}

const char* kfx_last_error(const kfx_ctx* c) { return c ? c->err.c_str() : "null context"; }

int kfx_load_layers(kfx_ctx* c, const double* table, int n_layers, double bz, int n_eta, int n_phi) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!table) return fail(c, KFX_EINVAL, "layer table is NULL");
  if (n_layers < 1 || n_layers > KFX_MAX_LAYERS) return fail(c, KFX_EINVAL, "n_layers out of range");
  if (n_eta < 1 || n_phi < 1 || n_eta > 4096 || n_phi > 4096) return fail(c, KFX_EINVAL, "bad bin counts");
  if (!is_finite(bz)) return fail(c, KFX_EINVAL, "non-finite field");
  Geometry G{};
  G.n_layers = n_layers;
  G.bz = bz;
  G.n_eta = n_eta;
  G.n_phi = n_phi;
  std::vector<int> bar, dp, dn;
  for (int i = 0; i < n_layers; ++i) {
    const double* r = table + 8 * i;
    for (int j = 0; j < 8; ++j)
      if (!is_finite(r[j])) return fail(c, KFX_EINVAL, "non-finite layer table entry");
    Layer& L = G.L[i];
    const int kind = (int)r[0];
    if ((kind != kBarrel && kind != kDisk) || (double)kind != r[0]) return fail(c, KFX_EINVAL, "layer kind must be 0 or 1");
    L.kind = kind;
    L.pos = r[1];
    L.lo = r[2];
    L.hi = r[3];
    if (!(L.lo < L.hi)) return fail(c, KFX_EINVAL, "layer lo >= hi");
    if (r[4] < 0 || r[5] <= 0 || r[6] <= 0 || r[7] <= 0) return fail(c, KFX_EINVAL, "x/X0 < 0 or sigma <= 0");
    L.x0 = (float)r[4];
    L.v_u = (float)(r[5] * r[5]);
    L.v_v = (float)(r[6] * r[6]);
    L.v_n = (float)(r[7] * r[7]);
    if (kind == kBarrel) {
      if (!(L.pos > 0)) return fail(c, KFX_EINVAL, "barrel radius <= 0");
      L.side = 0;
      L.eta_lo = std::asinh(L.lo / L.pos);
      L.eta_hi = std::asinh(L.hi / L.pos);
      bar.push_back(i);
    } else {
      if (L.pos == 0 || !(L.lo > 0)) return fail(c, KFX_EINVAL, "disk at z = 0 or r bound <= 0");
      L.side = L.pos > 0 ? 1 : -1;
      const double a = std::asinh(L.pos / L.hi), b = std::asinh(L.pos / L.lo);
      L.eta_lo = std::min(a, b);
      L.eta_hi = std::max(a, b);
      (L.pos > 0 ? dp : dn).push_back(i);
    }
  }
  for (int i = 0; i < n_layers; ++i) G.L[i].eta_scale = (float)(n_eta / (G.L[i].eta_hi - G.L[i].eta_lo));
  std::sort(bar.begin(), bar.end(), [&](int a, int b) { return G.L[a].pos < G.L[b].pos; });
  std::sort(dp.begin(), dp.end(), [&](int a, int b) { return G.L[a].pos < G.L[b].pos; });
  std::sort(dn.begin(), dn.end(), [&](int a, int b) { return G.L[a].pos > G.L[b].pos; });
  for (size_t i = 1; i < bar.size(); ++i)
    if (G.L[bar[i]].pos == G.L[bar[i - 1]].pos) return fail(c, KFX_EINVAL, "duplicate barrel radius");
  for (size_t i = 1; i < dp.size(); ++i)
    if (G.L[dp[i]].pos == G.L[dp[i - 1]].pos) return fail(c, KFX_EINVAL, "duplicate disk position");
  for (size_t i = 1; i < dn.size(); ++i)
    if (G.L[dn[i]].pos == G.L[dn[i - 1]].pos) return fail(c, KFX_EINVAL, "duplicate disk position");
  G.n_barrel = (int)bar.size();
  G.n_dpos = (int)dp.size();
  G.n_dneg = (int)dn.size();
  for (int i = 0; i < kMaxLayers; ++i) G.next_barrel[i] = G.brank[i] = -1;
  for (size_t i = 0; i < bar.size(); ++i) {
    G.barrel[i] = bar[i];
    G.brank[bar[i]] = (int)i;
    G.next_barrel[bar[i]] = (i + 1 < bar.size()) ? bar[i + 1] : -1;
  }
  for (size_t i = 0; i < dp.size(); ++i) G.dpos[i] = dp[i];
  for (size_t i = 0; i < dn.size(); ++i) G.dneg[i] = dn[i];
  nav_tables(G);
  DeviceGuard dg(c->device);
  if (!c->dev_geo) {
    if (hipMalloc(&c->dev_geo, sizeof(Geometry)) != hipSuccess) return fail(c, KFX_ENOMEM, "geometry allocation");
  }
  int rc = hip_check(c, hipMemcpy(c->dev_geo, &G, sizeof(Geometry), hipMemcpyHostToDevice), "geometry upload");
  if (rc) return rc;
  c->host_geo = G;
  c->have_geo = true;
  c->have_index = false;
  return KFX_OK;
}

int kfx_bin_hits(kfx_ctx* c, const kfx_hits* hits, int32_t* bin_out, int32_t* offsets_out, int32_t* perm_out,
                 void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!c->have_geo) return fail(c, KFX_ESTATE, "kfx_load_layers first");
  int rc = check_hits(c, hits);
  if (rc) return rc;
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  if ((rc = build_index(c, hits, bin_out, true, st))) return rc;
  const long n_keys = (long)hits->n_events * c->host_geo.n_layers * c->host_geo.n_eta * c->host_geo.n_phi;
  if (offsets_out &&
      (rc = hip_check(c, hipMemcpyAsync(offsets_out, c->bw.off, (n_keys + 1) * 4, hipMemcpyDeviceToDevice, st),
                      "offsets copy")))
    return rc;
  if (perm_out && hits->n_hits > 0 &&
      (rc = hip_check(c, hipMemcpyAsync(perm_out, c->bw.perm, (size_t)hits->n_hits * 4, hipMemcpyDeviceToDevice, st),
                      "perm copy")))
    return rc;
  return KFX_OK;
}

int kfx_index_keys_per_event(kfx_ctx* c, int64_t* keys) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!keys) return fail(c, KFX_EINVAL, "keys is NULL");
  if (!c->have_index) return fail(c, KFX_ESTATE, "no hit index on this context");
  *keys = c->bw.ev_stride;
  return KFX_OK;
}

int kfx_seed_states(kfx_ctx* c, const kfx_hits* hits, const int32_t* seeds, int32_t n, const kfx_prior* prior,
                    kfx_states* out, float* chi2, int32_t* status, void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!c->have_geo) return fail(c, KFX_ESTATE, "kfx_load_layers first");
  int rc = check_hits(c, hits);
  if (rc || (rc = check_prior(c, prior))) return rc;
  if (n < 0) return fail(c, KFX_EINVAL, "n < 0");
  if (n > 0 && (!seeds || !chi2 || !status)) return fail(c, KFX_EINVAL, "NULL seed arrays");
  if ((rc = check_states(c, out, n, "out"))) return rc;
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  launch_seed_states(c->dev_geo, view(hits), seeds, n, prior_of(prior), soa(out), chi2, status, st);
  return hip_check(c, hipGetLastError(), "seed kernel");
}

int kfx_step_compat(kfx_ctx* c, const kfx_hits* hits, const int32_t* cand_event, const int32_t* cand_layer,
                    const kfx_states* in, int32_t n, float chi2_cut, int32_t* next_layer, kfx_states* pred,
                    int32_t* pair_count, int32_t* pair_hit, float* pair_chi2, int32_t max_pairs, void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!c->have_geo) return fail(c, KFX_ESTATE, "kfx_load_layers first");
  int rc = check_hits(c, hits);
  if (rc) return rc;
  if (!c->have_index || c->index_hits_key[0] != hits->x || c->index_hits_key[1] != hits->layer ||
      c->index_hits_key[2] != hits->event_offsets || c->index_n_hits != hits->n_hits ||
      c->index_n_events != hits->n_events)
    return fail(c, KFX_ESTATE, "kfx_bin_hits on these hits first");
  if (n < 0 || max_pairs < 0) return fail(c, KFX_EINVAL, "n or max_pairs < 0");
  if (!(chi2_cut > 0.0f) || !std::isfinite(chi2_cut)) return fail(c, KFX_EINVAL, "chi2_cut must be finite and > 0");
  if (n > 0 && (!cand_event || !cand_layer || !next_layer || !pair_count || (max_pairs > 0 && (!pair_hit || !pair_chi2))))
    return fail(c, KFX_EINVAL, "NULL arrays");
  if ((rc = check_states(c, in, n, "in")) || (rc = check_states(c, pred, n, "pred"))) return rc;
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  launch_step_compat(c->dev_geo, view(hits), index_view(c), cand_event, cand_layer, soa(in), n, chi2_cut, next_layer,
                     soa(pred), pair_count, pair_hit, pair_chi2, max_pairs, st);
  return hip_check(c, hipGetLastError(), "step kernel");
}

namespace {
constexpr int kEv = 5;  // timing events per build call
// hit indices of the fused kernel's history words (27 bits for code + 2)
constexpr long kFusedMaxHits = (1L << 27) - 3;

// whether a fused launch shape's LDS (state slots, history, layer table)
// fits in a block
bool fused_shape_fits(const kfx_ctx* c, const kfx_build_params* p) {
  const int lanes = p->lanes_per_seed ? p->lanes_per_seed : fused_lanes_for(p->max_cands);
  const int threads = p->block_threads ? p->block_threads : 256;
  return fused_lds_bytes(lanes, threads, p->max_steps) + fused_static_lds_bytes() <= c->max_lds;
}

int build_impl(kfx_ctx* c, const kfx_hits* hits, const int32_t* seeds, const int32_t* seed_event, int32_t n_seeds,
               const kfx_build_params* p, kfx_tracks* out, hipStream_t st) {
  if (!c->have_geo) return fail(c, KFX_ESTATE, "kfx_load_layers first");
  int rc = check_hits(c, hits);
  if (rc) return rc;
  if (!p || !out) return fail(c, KFX_EINVAL, "params or out is NULL");
  if ((rc = check_prior(c, &p->prior))) return rc;
  if (n_seeds < 0) return fail(c, KFX_EINVAL, "n_seeds < 0");
  if (p->max_cands < 1 || p->max_cands > KFX_MAX_CANDS) return fail(c, KFX_EINVAL, "max_cands out of [1, 16]");
  if (p->max_steps < 1 || p->max_steps > KFX_MAX_STEPS) return fail(c, KFX_EINVAL, "max_steps out of [1, 40]");
  if (p->max_holes < 0 || p->max_holes > 200) return fail(c, KFX_EINVAL, "max_holes out of range");
  if (!(p->chi2_cut > 0.0f) || !std::isfinite(p->chi2_cut)) return fail(c, KFX_EINVAL, "chi2_cut must be finite and > 0");
  if (p->mode != KFX_MODE_PLAIN && p->mode != KFX_MODE_FUSED) return fail(c, KFX_EINVAL, "unknown mode");
  if (!(p->window_inflate == 0.0f || (p->window_inflate >= 1.0f && p->window_inflate <= 1e4f)))
    return fail(c, KFX_EINVAL, "window_inflate must be 0 or in [1, 1e4]");
  if (p->score && !(std::isfinite(p->score_hit) && std::isfinite(p->score_hole) && std::isfinite(p->score_chi2)))
    return fail(c, KFX_EINVAL, "score weights must be finite");
  if (p->binning < 0 || p->binning > 2) return fail(c, KFX_EINVAL, "binning must be 0, 1 or 2");
  if (p->block_threads != 0 && (p->block_threads < 64 || p->block_threads > 256 || p->block_threads % 64))
    return fail(c, KFX_EINVAL, "block_threads must be 0 or a multiple of 64 in [64, 256]");
  if (p->blocks < 0) return fail(c, KFX_EINVAL, "blocks < 0");
  if (p->scan_tile < 0) return fail(c, KFX_EINVAL, "scan_tile < 0");
  if (p->waves_per_simd < 0 || p->waves_per_simd > 2) return fail(c, KFX_EINVAL, "waves_per_simd must be 0, 1 or 2");
  if (p->lanes_per_seed != 0 && ((p->lanes_per_seed != 4 && p->lanes_per_seed != 6 && p->lanes_per_seed != 8 &&
                                  p->lanes_per_seed != 12 && p->lanes_per_seed != 16) ||
                                 p->lanes_per_seed < p->max_cands || (p->lanes_per_seed == 6 && p->max_cands < 5) ||
                                 (p->lanes_per_seed == 12 && p->max_cands < 9)))
    return fail(c, KFX_EINVAL,
                "lanes_per_seed must be 0, or 4, 6 (K of 5 or 6), 8, 12 (K of 9 to 12) or 16 and at least max_cands");
  {
    const int lanes = p->lanes_per_seed ? p->lanes_per_seed : fused_lanes_for(p->max_cands);
    if (p->seeds_per_wave < 0 || p->seeds_per_wave > 64 / lanes)
      return fail(c, KFX_EINVAL, "seeds_per_wave must be 0 or in [1, 64 / lanes_per_seed]");
    if (p->mode == KFX_MODE_FUSED) {
      if (!fused_shape_fits(c, p)) return fail(c, KFX_EINVAL, "launch shape needs more LDS than a block may use");
      if (hits->n_hits > kFusedMaxHits) return fail(c, KFX_EINVAL, "fused building takes at most 2^27 - 3 hits");
    }
  }
  const int K = p->max_cands;
  const long SK = (long)n_seeds * K;
  if (out->capacity < SK) {
    out->needed = SK;
    return fail(c, KFX_EOVERFLOW, "output capacity below n_seeds * max_cands");
  }
  if (out->max_hits < kSeedHits) return fail(c, KFX_EINVAL, "max_hits < 3");
  if (n_seeds > 0 && (!seeds || !seed_event || !out->n_cands || !out->hits || !out->n_hits || !out->n_holes ||
                      !out->chi2 || !out->stats))
    return fail(c, KFX_EINVAL, "NULL seed or output arrays");
  if ((rc = check_states(c, &out->state, SK, "out.state"))) return rc;
  hipEvent_t* tev = nullptr;
  if (c->timing) {
    tev = c->ring.data() + kEv * c->ring_next;
    if ((rc = hip_check(c, hipEventRecord(tev[0], st), "timing event"))) return rc;
  }
  auto close_timing = [&]() -> int {
    if (!tev) return KFX_OK;
    int r = hip_check(c, hipEventRecord(tev[4], st), "timing event");
    if (r) return r;
    c->ring_next = (c->ring_next + 1) % c->ring_n;
    c->ring_count = std::min(c->ring_count + 1, c->ring_n);
    return KFX_OK;
  };
  auto bin = [&]() -> int {
    // the building does not depend on the order within a bin: no sort
    int r = build_index(c, hits, nullptr, false, st, p->binning);
    if (!r && tev) r = hip_check(c, hipEventRecord(tev[1], st), "timing event");
    return r;
  };
  if (n_seeds == 0) {
    if ((rc = bin())) return rc;
    if (tev && ((rc = hip_check(c, hipEventRecord(tev[2], st), "timing event")) ||
                (rc = hip_check(c, hipEventRecord(tev[3], st), "timing event"))))
      return rc;
    return close_timing();
  }

  BuildArgs a{};
  a.G = c->dev_geo;
  a.H = view(hits);
  a.seeds = seeds;
  a.seed_event = seed_event;
  a.n_seeds = n_seeds;
  a.prior = prior_of(&p->prior);
  a.cut = p->chi2_cut;
  a.K = K;
  a.max_holes = p->max_holes;
  a.max_steps = p->max_steps;
  a.overlap = p->overlap ? 1 : 0;
  a.rank = RankW{p->score_hit, p->score_hole, p->score_chi2, p->score ? 1 : 0};
  a.inflate = p->window_inflate > 0.0f ? p->window_inflate : 1.0f;
  a.coop_min = p->scan_tile ? p->scan_tile : 64;
  {
    const int lanes = p->lanes_per_seed ? p->lanes_per_seed : fused_lanes_for(K);
    a.groups_per_wave = p->seeds_per_wave ? p->seeds_per_wave : 64 / lanes;
  }
  const long N = std::max<long>(SK, 1);
  auto alloc_states = [&](const char* name, StateSoA& s) -> int {
    char* base = (char*)ws(c, name, (size_t)N * (6 * 8 + 21 * 4), st, rc);
    if (rc) return rc;
    s.par = (double*)base;
    s.cov = (float*)(base + (size_t)N * 48);
    s.stride = N;
    return KFX_OK;
  };
  if ((rc = alloc_states("b.cand0", a.cand[0])) || (rc = alloc_states("b.cand1", a.cand[1])) ||
      (rc = alloc_states("b.pred", a.pred)))
    return rc;
  a.layer[0] = (int*)ws(c, "b.layer0", N * 4, st, rc); if (rc) return rc;
  a.layer[1] = (int*)ws(c, "b.layer1", N * 4, st, rc); if (rc) return rc;
  a.chi2[0] = (float*)ws(c, "b.chi20", N * 4, st, rc); if (rc) return rc;
  a.chi2[1] = (float*)ws(c, "b.chi21", N * 4, st, rc); if (rc) return rc;
  a.meta[0] = (int*)ws(c, "b.meta0", N * 4, st, rc); if (rc) return rc;
  a.meta[1] = (int*)ws(c, "b.meta1", N * 4, st, rc); if (rc) return rc;
  a.next_layer = (int*)ws(c, "b.next", N * 4, st, rc); if (rc) return rc;
  a.kid_c = (float*)ws(c, "b.kidc", N * K * 4, st, rc); if (rc) return rc;
  a.kid_h = (int*)ws(c, "b.kidh", N * K * 4, st, rc); if (rc) return rc;
  a.kid_n = (int*)ws(c, "b.kidn", N * 4, st, rc); if (rc) return rc;
  a.sel_parent = (int*)ws(c, "b.selp", N * 4, st, rc); if (rc) return rc;
  a.sel_code = (int*)ws(c, "b.selc", N * 4, st, rc); if (rc) return rc;
  a.sel_chi2 = (float*)ws(c, "b.selx", N * 4, st, rc); if (rc) return rc;
  // the per-step history in HBM: parent and code arrays of the plain path,
  // one packed word per entry for the fused kernel
  if (p->mode == KFX_MODE_PLAIN) {
    a.hist_parent = (signed char*)ws(c, "b.histp", (size_t)N * p->max_steps, st, rc); if (rc) return rc;
    a.hist_code = (int*)ws(c, "b.histc", (size_t)N * p->max_steps * 4, st, rc); if (rc) return rc;
  } else {
    a.hist_word = (unsigned int*)ws(c, "b.histw", (size_t)N * p->max_steps * 4, st, rc); if (rc) return rc;
  }
  if (a.overlap) {
    a.hist_ov = (int*)ws(c, "b.histo", (size_t)N * p->max_steps * 4, st, rc); if (rc) return rc;
  }
  a.n_steps = (int*)ws(c, "b.nsteps", (size_t)std::max(n_seeds, 1) * 4, st, rc); if (rc) return rc;
  a.stats = (unsigned long long*)out->stats;

  TracksOut o;
  o.n_cands = out->n_cands;
  o.hits = out->hits;
  o.n_hits = out->n_hits;
  o.n_holes = out->n_holes;
  o.chi2 = out->chi2;
  o.state = soa(&out->state);
  o.max_hits = out->max_hits;

  if (p->mode == KFX_MODE_PLAIN) {
    if ((rc = bin())) return rc;
    a.B = index_view(c);
    launch_build_plain(a, o, st, tev ? tev + 2 : nullptr);
  } else {
    int* counter = (int*)ws(c, "b.counter", 256, st, rc);
    if (rc) return rc;
    // the seed start reads only the hits: it runs on the second stream
    // while this one bins them
    if ((rc = side_stream(c)) || (rc = hip_check(c, hipEventRecord(c->ev_fork, st), "fork")) ||
        (rc = hip_check(c, hipStreamWaitEvent(c->side, c->ev_fork, 0), "fork")))
      return rc;
    launch_build_init(a, c->side);
    if ((rc = hip_check(c, hipEventRecord(c->ev_join, c->side), "join"))) return rc;
    if ((rc = bin())) return rc;
    a.B = index_view(c);
    if ((rc = hip_check(c, hipStreamWaitEvent(st, c->ev_join, 0), "join"))) return rc;
    const int threads = p->block_threads ? p->block_threads : 256;
    int blocks = p->blocks;
    if (blocks == 0) blocks = c->n_cu * 4;
    // no more groups than seeds need
    const int lanes = p->lanes_per_seed ? p->lanes_per_seed : fused_lanes_for(K);
    const int groups_per_block = (threads / 64) * a.groups_per_wave;
    const long max_blocks = (n_seeds + groups_per_block - 1) / groups_per_block;
    blocks = (int)std::max<long>(1, std::min<long>(blocks, max_blocks));
    launch_build_fused(a, o, counter, blocks, threads, lanes, p->waves_per_simd == 2 ? 2 : 1, st,
                       tev ? tev + 2 : nullptr);
  }
  if ((rc = hip_check(c, hipGetLastError(), "build kernels"))) return rc;
  return close_timing();
}
}  // namespace

int kfx_build_tracks(kfx_ctx* c, const kfx_hits* hits, const int32_t* seeds, const int32_t* seed_event,
                     int32_t n_seeds, const kfx_build_params* p, kfx_tracks* out, void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  DeviceGuard dg(c->device);
  return build_impl(c, hits, seeds, seed_event, n_seeds, p, out, (hipStream_t)stream);
}

int kfx_enable_timing(kfx_ctx* c, int n_calls) {
  if (!c || n_calls < 0 || n_calls > 4096) return KFX_EINVAL;
  c->err.clear();
  DeviceGuard dg(c->device);
  for (auto& e : c->ring)
    if (e) (void)hipEventDestroy(e);
  c->ring.assign(kEv * (size_t)n_calls, nullptr);
  for (auto& e : c->ring) {
    int rc = hip_check(c, hipEventCreate(&e), "event create");
    if (rc) return rc;
  }
  c->ring_n = n_calls;
  c->ring_next = 0;
  c->ring_count = 0;
  c->timing = n_calls > 0;
  return KFX_OK;
}

int kfx_build_times(kfx_ctx* c, float* ms, int n_calls) {
  if (!c || !ms || n_calls < 0) return KFX_EINVAL;
  c->err.clear();
  const int n = std::min(n_calls, c->ring_count);
  DeviceGuard dg(c->device);
  for (int i = 0; i < n; ++i) {
    // oldest of the last n first
    const int slot = ((c->ring_next - n + i) % c->ring_n + c->ring_n) % c->ring_n;
    hipEvent_t* e = c->ring.data() + kEv * slot;
    int rc = hip_check(c, hipEventSynchronize(e[4]), "event sync");
    if (rc) return rc;
    if ((rc = hip_check(c, hipEventElapsedTime(&ms[4 * i + 0], e[0], e[1]), "elapsed"))) return rc;
    if ((rc = hip_check(c, hipEventElapsedTime(&ms[4 * i + 1], e[2], e[3]), "elapsed"))) return rc;
    if ((rc = hip_check(c, hipEventElapsedTime(&ms[4 * i + 2], e[1], e[4]), "elapsed"))) return rc;
    if ((rc = hip_check(c, hipEventElapsedTime(&ms[4 * i + 3], e[0], e[4]), "elapsed"))) return rc;
  }
  return n;
}

// ---- HIP graph of one build -------------------------------------------------
struct kfx_graph {
  kfx_ctx* c = nullptr;
  std::map<std::string, std::pair<void*, size_t>> pool;  // the graph's own workspace
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {
void free_pool(std::map<std::string, std::pair<void*, size_t>>& pool) {
  for (auto& kv : pool) (void)hipFree(kv.second.first);
  pool.clear();
}
}  // namespace

int kfx_build_graph(kfx_ctx* c, const kfx_hits* hits, const int32_t* seeds, const int32_t* seed_event,
                    int32_t n_seeds, const kfx_build_params* p, kfx_tracks* out, kfx_graph** graph) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!graph) return fail(c, KFX_EINVAL, "graph is NULL");
  *graph = nullptr;
  DeviceGuard dg(c->device);
  hipStream_t cs = nullptr;
  int rc = hip_check(c, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "capture stream");
  if (rc) return rc;
  kfx_graph* g = new kfx_graph();
  g->c = c;
  auto* saved_active = c->active;
  const bool saved_timing = c->timing;
  c->active = &g->pool;
  c->timing = false;
  // an eager run sizes the graph's workspace, so that nothing is allocated
  // (and no stream waits) while capturing
  rc = build_impl(c, hits, seeds, seed_event, n_seeds, p, out, cs);
  if (!rc) rc = hip_check(c, hipStreamSynchronize(cs), "sizing run");
  if (!rc) rc = hip_check(c, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed), "begin capture");
  if (!rc) {
    const int brc = build_impl(c, hits, seeds, seed_event, n_seeds, p, out, cs);
    hipGraph_t gr = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &gr);
    if (brc) rc = brc;
    else rc = hip_check(c, e, "end capture");
    if (!rc) {
      g->graph = gr;
      rc = hip_check(c, hipGraphInstantiate(&g->exec, gr, nullptr, nullptr, 0), "graph instantiate");
    } else if (gr) {
      (void)hipGraphDestroy(gr);
    }
  }
  c->active = saved_active;
  c->timing = saved_timing;
  c->have_index = false;  // the index now lives in the graph's workspace
  (void)hipStreamSynchronize(cs);
  (void)hipStreamDestroy(cs);
  if (rc) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    free_pool(g->pool);
    delete g;
    return rc;
  }
  *graph = g;
  return KFX_OK;
}

int kfx_graph_launch(kfx_graph* g, void* stream) {
  if (!g || !g->exec) return KFX_EINVAL;
  DeviceGuard dg(g->c->device);
  return hip_check(g->c, hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
}

void kfx_graph_destroy(kfx_graph* g) {
  if (!g) return;
  {
    DeviceGuard dg(g->c->device);
    (void)hipDeviceSynchronize();
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    free_pool(g->pool);
  }
  delete g;
}

// ---- autotuner of the fused kernel's launch shape -------------------------
}  // extern "C"

namespace {
// Autotuner cache: key = device (architecture name, compute units) and
// workload signature; value = the launch shape and its time.  Optionally
// mirrored in the file named by KFX_AUTOTUNE_CACHE (lines "key<TAB>bt
// blocks lanes tile waves spw ms").
struct TuneEntry {
  int block_threads, blocks, lanes, tile, waves, spw;
  float ms;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
bool g_tune_loaded = false;

std::string tune_key(const kfx_ctx* c, const kfx_hits* h, int n_seeds, const kfx_build_params* p) {
  hipDeviceProp_t prop{};
  (void)hipGetDeviceProperties(&prop, c->device);
  char buf[512];
  snprintf(buf, sizeof(buf),
           "%s/%d|S%d|H%d|E%d|K%d|holes%d|steps%d|cut%.9g|infl%.9g|ov%d|score%d:%.9g:%.9g:%.9g|bin%d",
           prop.gcnArchName, prop.multiProcessorCount, n_seeds, h ? h->n_hits : -1, h ? h->n_events : -1,
           p->max_cands, p->max_holes, p->max_steps, (double)p->chi2_cut, (double)p->window_inflate,
           p->overlap ? 1 : 0, p->score ? 1 : 0, (double)p->score_hit, (double)p->score_hole,
           (double)p->score_chi2, p->binning);
  return buf;
}

void tune_load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char* path = std::getenv("KFX_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    const size_t tab = line.find('\t');
    if (tab == std::string::npos) continue;
    TuneEntry e{};
    if (sscanf(line.c_str() + tab + 1, "%d %d %d %d %d %d %f", &e.block_threads, &e.blocks, &e.lanes, &e.tile,
               &e.waves, &e.spw, &e.ms) == 7)
      g_tune[line.substr(0, tab)] = e;
  }
}

void tune_store(const std::string& key, const TuneEntry& e) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[key] = e;
  const char* path = std::getenv("KFX_AUTOTUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << '\t' << e.block_threads << ' ' << e.blocks << ' ' << e.lanes << ' ' << e.tile << ' ' << e.waves << ' '
    << e.spw << ' ' << e.ms << '\n';
}
}  // namespace

extern "C" {

void kfx_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
  g_tune_loaded = false;  // the file, if any, is read again on next use
}

int kfx_autotune_build(kfx_ctx* c, const kfx_hits* hits, const int32_t* seeds, const int32_t* seed_event,
                       int32_t n_seeds, kfx_build_params* p, kfx_tracks* out, int32_t reps, float* best_ms,
                       void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!p || !out) return fail(c, KFX_EINVAL, "params or out is NULL");
  if (reps < 1 || reps > 100) return fail(c, KFX_EINVAL, "reps out of [1, 100]");
  const std::string key = tune_key(c, hits, n_seeds, p);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    tune_load_locked();
    const auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      const TuneEntry& e = it->second;
      p->mode = KFX_MODE_FUSED;
      p->block_threads = e.block_threads;
      p->blocks = e.blocks;
      p->lanes_per_seed = e.lanes;
      p->scan_tile = e.tile;
      p->waves_per_simd = e.waves;
      p->seeds_per_wave = e.spw;
      if (best_ms) *best_ms = e.ms;
      return KFX_OK;
    }
  }
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  const bool saved_timing = c->timing;
  c->timing = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = hip_check(c, hipEventCreate(&e0), "event create");
  if (!rc) rc = hip_check(c, hipEventCreate(&e1), "event create");
  uint64_t saved_stats[3] = {0, 0, 0};
  if (!rc && out->stats)
    rc = hip_check(c, hipMemcpyAsync(saved_stats, out->stats, sizeof(saved_stats), hipMemcpyDeviceToHost, st),
                   "stats save");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(st), "stats save");
  kfx_build_params cur = *p;
  cur.mode = KFX_MODE_FUSED;
  const int lp0 = fused_lanes_pow2(p->max_cands);
  if (cur.block_threads == 0) cur.block_threads = 256;
  if (cur.blocks == 0) cur.blocks = c->n_cu * 4;
  if (cur.lanes_per_seed == 0) cur.lanes_per_seed = fused_lanes_for(p->max_cands);
  if (cur.scan_tile == 0) cur.scan_tile = 64;
  if (cur.waves_per_simd == 0) cur.waves_per_simd = 1;
  if (cur.seeds_per_wave == 0) cur.seeds_per_wave = 64 / cur.lanes_per_seed;
  auto timeit = [&](const kfx_build_params& q, float& ms) -> int {
    int r = build_impl(c, hits, seeds, seed_event, n_seeds, &q, out, st);  // warm-up
    if (r) return r;
    ms = 3.0e38f;
    for (int i = 0; i < reps; ++i) {
      if ((r = hip_check(c, hipEventRecord(e0, st), "event"))) return r;
      if ((r = build_impl(c, hits, seeds, seed_event, n_seeds, &q, out, st))) return r;
      if ((r = hip_check(c, hipEventRecord(e1, st), "event"))) return r;
      if ((r = hip_check(c, hipEventSynchronize(e1), "event"))) return r;
      float t = 0.0f;
      if ((r = hip_check(c, hipEventElapsedTime(&t, e0, e1), "elapsed"))) return r;
      ms = std::min(ms, t);
    }
    return KFX_OK;
  };
  float best = 3.0e38f;
  if (!rc) rc = timeit(cur, best);
  if (!rc && p->waves_per_simd == 0) {
    // start from the better of one and two wavefronts per SIMD: the other
    // parameters' best values depend on it, and a descent that starts on
    // the wrong side can settle there
    kfx_build_params q = cur;
    q.waves_per_simd = 3 - cur.waves_per_simd;
    float t = 0.0f;
    if (fused_shape_fits(c, &q) && !(rc = timeit(q, t)) && t < best) {
      best = t;
      cur = q;
    }
  }
  // coordinate descent: one parameter at a time, the others held; a second
  // sweep over the scan tile, the block size and the occupancy
  constexpr int kDims[] = {0, 1, 2, 3, 4, 5, 0, 1, 4};
  for (int dim : kDims) {
    if (rc) break;
    std::vector<kfx_build_params> cand;
    kfx_build_params q = cur;
    if (dim == 0) {
      for (int t : {16, 32, 64, 128, 256}) { q.scan_tile = t; cand.push_back(q); }
    } else if (dim == 1) {
      for (int t : {64, 128, 256}) { q.block_threads = t; cand.push_back(q); }
    } else if (dim == 2) {
      for (int b : {1, 2, 4, 8}) { q.blocks = c->n_cu * b; cand.push_back(q); }
    } else if (dim == 3) {
      // a full wavefront of seeds for each lane count (6-lane groups for K
      // of 5 or 6, 12-lane groups for K of 9 to 12)
      std::vector<int> ls;
      if (p->max_cands >= 5 && p->max_cands <= 6) ls.push_back(6);
      if (p->max_cands >= 9 && p->max_cands <= 12) ls.push_back(12);
      for (int l = lp0; l <= 16; l <<= 1) ls.push_back(l);
      for (int l : ls) {
        q.lanes_per_seed = l;
        q.seeds_per_wave = 64 / l;
        cand.push_back(q);
      }
    } else if (dim == 4) {
      for (int w : {1, 2}) { q.waves_per_simd = w; cand.push_back(q); }
    } else {
      for (int g = 2; g <= 64 / cur.lanes_per_seed; ++g) { q.seeds_per_wave = g; cand.push_back(q); }
    }
    for (const auto& v : cand) {
      if (v.scan_tile == cur.scan_tile && v.block_threads == cur.block_threads && v.blocks == cur.blocks &&
          v.lanes_per_seed == cur.lanes_per_seed && v.waves_per_simd == cur.waves_per_simd &&
          v.seeds_per_wave == cur.seeds_per_wave)
        continue;
      if (!fused_shape_fits(c, &v)) continue;
      float t = 0.0f;
      if ((rc = timeit(v, t))) break;
      if (t < best) {
        best = t;
        cur = v;
      }
    }
  }
  if (!rc && out->stats)
    rc = hip_check(c, hipMemcpyAsync(out->stats, saved_stats, sizeof(saved_stats), hipMemcpyHostToDevice, st),
                   "stats restore");
  if (!rc) rc = hip_check(c, hipStreamSynchronize(st), "stats restore");
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  c->timing = saved_timing;
  if (rc) return rc;
  p->mode = KFX_MODE_FUSED;
  p->block_threads = cur.block_threads;
  p->blocks = cur.blocks;
  p->lanes_per_seed = cur.lanes_per_seed;
  p->scan_tile = cur.scan_tile;
  p->waves_per_simd = cur.waves_per_simd;
  p->seeds_per_wave = cur.seeds_per_wave;
  if (best_ms) *best_ms = best;
  tune_store(key, TuneEntry{cur.block_threads, cur.blocks, cur.lanes_per_seed, cur.scan_tile, cur.waves_per_simd,
                            cur.seeds_per_wave, best});
  return KFX_OK;
}

int kfx_find_duplicates(kfx_ctx* c, const kfx_tracks* tracks, int32_t n_seeds, int32_t K, int32_t n_hits,
                        int32_t frac_num, int32_t frac_den, int32_t* dup_of, void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!tracks) return fail(c, KFX_EINVAL, "tracks is NULL");
  if (n_seeds < 0 || n_hits < 0) return fail(c, KFX_EINVAL, "n_seeds < 0 or n_hits < 0");
  if (K < 1 || K > KFX_MAX_CANDS) return fail(c, KFX_EINVAL, "K outside 1..KFX_MAX_CANDS");
  if (frac_num < 1 || frac_den < frac_num) return fail(c, KFX_EINVAL, "need 0 < frac_num <= frac_den");
  if (n_seeds == 0) return KFX_OK;
  const int H = tracks->max_hits;
  if (H < 1 || H > 64) return fail(c, KFX_EINVAL, "max_hits outside 1..64");
  if (tracks->capacity < (int64_t)n_seeds * K) return fail(c, KFX_EINVAL, "capacity < n_seeds * K");
  if ((int64_t)n_seeds * H > INT32_MAX) return fail(c, KFX_EINVAL, "n_seeds * max_hits exceeds 2^31 - 1");
  if (!tracks->n_cands || !tracks->hits || !tracks->n_hits || !tracks->n_holes || !tracks->chi2 || !dup_of)
    return fail(c, KFX_EINVAL, "NULL track arrays or dup_of");
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  const size_t SH = (size_t)n_seeds * H;
  int rc = KFX_OK;
  DupArgs a;
  a.n_cands = tracks->n_cands;
  a.hits = tracks->hits;
  a.n_hits_c = tracks->n_hits;
  a.n_holes_c = tracks->n_holes;
  a.chi2_c = tracks->chi2;
  a.S = n_seeds;
  a.K = K;
  a.H = H;
  a.n_hits = n_hits;
  a.num = frac_num;
  a.den = frac_den;
  a.dup_of = dup_of;
  a.list = (int*)ws(c, "dup.list", SH * 4, st, rc); if (rc) return rc;
  a.next = (int*)ws(c, "dup.next", SH * 4, st, rc); if (rc) return rc;
  a.key = (int4*)ws(c, "dup.key", (size_t)n_seeds * 16, st, rc); if (rc) return rc;
  a.head = (int*)ws(c, "dup.head", ((size_t)n_hits + 4) * 4, st, rc); if (rc) return rc;
  a.head2 = (int*)ws(c, "dup.head2", ((size_t)n_hits + 4) * 4, st, rc); if (rc) return rc;
  launch_find_duplicates(a, st);
  return hip_check(c, hipGetLastError(), "duplicate removal kernels");
}

int kfx_mask_hits(kfx_ctx* c, const kfx_tracks* tracks, int32_t n_seeds, int32_t K, const int32_t* dup_of,
                  int32_t min_hits, float max_chi2_ndof, const int32_t* layer_in, int32_t* layer_out,
                  int32_t n_hits, void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!tracks) return fail(c, KFX_EINVAL, "tracks is NULL");
  if (n_seeds < 0 || n_hits < 0) return fail(c, KFX_EINVAL, "n_seeds < 0 or n_hits < 0");
  if (K < 1 || K > KFX_MAX_CANDS) return fail(c, KFX_EINVAL, "K outside 1..KFX_MAX_CANDS");
  if (std::isnan(max_chi2_ndof)) return fail(c, KFX_EINVAL, "max_chi2_ndof is NaN");
  if (n_hits > 0 && (!layer_in || !layer_out)) return fail(c, KFX_EINVAL, "NULL layer arrays");
  if (n_seeds > 0) {
    if (tracks->max_hits < 1) return fail(c, KFX_EINVAL, "max_hits < 1");
    if (tracks->capacity < (int64_t)n_seeds * K) return fail(c, KFX_EINVAL, "capacity < n_seeds * K");
    if (!tracks->n_cands || !tracks->hits || !tracks->n_hits || !tracks->chi2)
      return fail(c, KFX_EINVAL, "NULL track arrays");
  }
  DeviceGuard dg(c->device);
  MaskArgs a;
  a.n_cands = tracks->n_cands;
  a.hits = tracks->hits;
  a.n_hits_c = tracks->n_hits;
  a.chi2_c = tracks->chi2;
  a.dup_of = dup_of;
  a.S = n_seeds;
  a.K = K;
  a.H = tracks->max_hits;
  a.n_hits = n_hits;
  a.min_hits = min_hits;
  a.max_chi2_ndof = max_chi2_ndof;
  a.layer_out = layer_out;
  launch_mask_hits(a, layer_in, (hipStream_t)stream);
  return hip_check(c, hipGetLastError(), "hit masking kernels");
}

int kfx_cluster_strips(kfx_ctx* c, const kfx_digis* d, const kfx_strip_calib* cal, const kfx_cluster_params* p,
                       kfx_clusters* out, void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!d || !cal || !p || !out) return fail(c, KFX_EINVAL, "NULL argument");
  if (d->n < 0 || d->n_events < 1 || !d->event_offsets) return fail(c, KFX_EINVAL, "bad digi sizes");
  if (d->n > 0 && (!d->module || !d->strip || !d->adc)) return fail(c, KFX_EINVAL, "NULL digi arrays");
  if (cal->n_modules < 1 || cal->strips_per_module < 1 ||
      (int64_t)cal->n_modules * cal->strips_per_module >= INT32_MAX)
    return fail(c, KFX_EINVAL, "bad calibration table size");
  if (!cal->noise || !cal->bad) return fail(c, KFX_EINVAL, "NULL calibration arrays");
  const double thr[3] = {p->seed_thr, p->chan_thr, p->clus_thr};
  for (double t : thr)
    if (!std::isfinite(t) || t < 0.0) return fail(c, KFX_EINVAL, "thresholds must be finite and >= 0");
  if (p->max_gap < 0 || p->max_gap > 64) return fail(c, KFX_EINVAL, "max_gap outside 0..64");
  if (out->capacity < 0 || !out->n_out) return fail(c, KFX_EINVAL, "bad output capacity or NULL n_out");
  if (out->capacity > 0 && (!out->event || !out->module || !out->first || !out->size || !out->charge ||
                            !out->barycenter))
    return fail(c, KFX_EINVAL, "NULL output arrays");
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  int rc = KFX_OK;
  StripArgs a;
  a.module = d->module;
  a.strip = d->strip;
  a.adc = d->adc;
  a.ev_off = d->event_offsets;
  a.n = d->n;
  a.n_events = d->n_events;
  a.noise = cal->noise;
  a.bad = cal->bad;
  a.n_modules = cal->n_modules;
  a.spm = cal->strips_per_module;
  a.seed_thr = p->seed_thr;
  a.chan_thr = p->chan_thr;
  a.clus_thr2 = p->clus_thr * p->clus_thr;
  a.max_gap = p->max_gap;
  a.min_charge = p->min_charge;
  // chunks of up to 8 modules whose calibration fits 32 KB of LDS; staged
  // when several events reuse it (a module wider than that, or a call of
  // fewer than four events, gathers from HBM what its digis need)
  a.chunk = std::max(1, std::min(8, (int)(32768 / strip_cal_lds(1, a.spm))));
  a.stage = (strip_cal_lds(a.chunk, a.spm) <= 32768 && d->n_events >= 4) ? 1 : 0;
  const long nchunks = strip_chunks(cal->n_modules, a.chunk);
  const size_t nec = (size_t)d->n_events * nchunks;
  a.bnd = (int*)ws(c, "strip.bnd", (size_t)d->n_events * (nchunks + 1) * 4, st, rc);
  if (rc) return rc;
  a.cnt = (int*)ws(c, "strip.cnt", (nec + 1) * 4, st, rc); if (rc) return rc;
  a.cnt_off = (int*)ws(c, "strip.cnt_off", (nec + 2) * 4, st, rc); if (rc) return rc;
  a.rec = (StripRec*)ws(c, "strip.rec", std::max<size_t>((size_t)d->n, 1) * sizeof(StripRec), st, rc);
  if (rc) return rc;
  int* scratch = (int*)ws(c, "strip.scan", ((nec + 1) / 4096 + 4) * 4, st, rc); if (rc) return rc;
  a.out_event = out->event;
  a.out_module = out->module;
  a.out_first = out->first;
  a.out_size = out->size;
  a.out_charge = out->charge;
  a.out_bary = out->barycenter;
  a.capacity = out->capacity;
  a.n_out = out->n_out;
  launch_cluster_strips(a, scratch, st);
  return hip_check(c, hipGetLastError(), "strip clustering kernels");
}

int kfx_fit_tracks(kfx_ctx* c, const kfx_hits* hits, const int32_t* trk_off, const int32_t* trk_hits,
                   int32_t n_tracks, const kfx_prior* prior, const float* align, float field_scale,
                   kfx_states* out, float* chi2, int32_t* ndof, int32_t* status, kfx_states* ckpt, void* stream) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!c->have_geo) return fail(c, KFX_ESTATE, "kfx_load_layers first");
  int rc = check_hits(c, hits);
  if (rc || (rc = check_prior(c, prior))) return rc;
  if (n_tracks < 0) return fail(c, KFX_EINVAL, "n_tracks < 0");
  if (!std::isfinite(field_scale)) return fail(c, KFX_EINVAL, "non-finite field scale");
  if (n_tracks > 0 && (!trk_off || !trk_hits || !chi2 || !ndof || !status))
    return fail(c, KFX_EINVAL, "NULL track arrays");
  if ((rc = check_states(c, out, n_tracks, "out"))) return rc;
  if (ckpt && (!ckpt->par || !ckpt->cov)) return fail(c, KFX_EINVAL, "ckpt: NULL state arrays");
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  FitOut o;
  o.state = soa(out);
  o.chi2 = chi2;
  o.ndof = ndof;
  o.status = status;
  if (ckpt) o.ckpt = soa(ckpt);
  else o.ckpt.par = nullptr, o.ckpt.cov = nullptr, o.ckpt.stride = 0;
  o.n_tracks = n_tracks;
  launch_fit(c->dev_geo, view(hits), trk_off, trk_hits, n_tracks, prior_of(prior), align, field_scale, o, st);
  return hip_check(c, hipGetLastError(), "fit kernel");
}

}  // extern "C"

namespace {
// The gradient of the fit: checks, then the adjoint kernels with their
// per-block partial rows in `partial` (nullptr: the workspace pool).
int backward_impl(kfx_ctx* c, const kfx_hits* hits, const int32_t* trk_off, const int32_t* trk_hits,
                  int32_t n_tracks, const kfx_prior* prior, const float* align, float field_scale,
                  const kfx_states* ckpt, const int32_t* status, const float* dchi2, int32_t dchi2_per_track,
                  double* dalign, double* dfield, void* stream, bool no_alloc) {
  if (!c) return KFX_EINVAL;
  c->err.clear();
  if (!c->have_geo) return fail(c, KFX_ESTATE, "kfx_load_layers first");
  int rc = check_hits(c, hits);
  if (rc || (rc = check_prior(c, prior))) return rc;
  if (n_tracks < 0) return fail(c, KFX_EINVAL, "n_tracks < 0");
  if (!std::isfinite(field_scale)) return fail(c, KFX_EINVAL, "non-finite field scale");
  if (!dalign || !dfield) return fail(c, KFX_EINVAL, "NULL gradient outputs");
  if (n_tracks > 0 && (!trk_off || !trk_hits || !status || !dchi2))
    return fail(c, KFX_EINVAL, "NULL track arrays");
  if (n_tracks > 0 && (!ckpt || !ckpt->par || !ckpt->cov)) return fail(c, KFX_EINVAL, "ckpt: NULL state arrays");
  const int nrow = 3 * c->host_geo.n_barrel + 1;
  const long nblocks = std::max(fit_backward_blocks(n_tracks), 1);
  double* partial = nullptr;
  if (no_alloc) {
    const size_t need = (size_t)nblocks * nrow;
    if (need > kNoAllocScratchDoubles)
      return fail(c, KFX_EOVERFLOW,
                  "kfx_fit_tracks_backward_noalloc: " + std::to_string(n_tracks) + " tracks need " +
                      std::to_string(need) + " float64 of scratch, the limit is " +
                      std::to_string(kNoAllocScratchDoubles) + " (" + std::to_string(nblocks) + " blocks of 64 tracks x " +
                      std::to_string(nrow) + " rows)");
    partial = scratch_of(c->device);
    if (!partial) return fail(c, KFX_ESTATE, "no scratch address for this device");
  }
  DeviceGuard dg(c->device);
  hipStream_t st = (hipStream_t)stream;
  if (!no_alloc) {
    partial = (double*)ws(c, "g.partial", (size_t)nblocks * nrow * sizeof(double), st, rc);
    if (rc) return rc;
  }
  StateSoA ck;
  if (n_tracks > 0) ck = soa(ckpt);
  else ck.par = nullptr, ck.cov = nullptr, ck.stride = 0;
  return hip_check(c,
                   launch_fit_backward(c->dev_geo, c->host_geo.n_barrel, c->host_geo.n_layers, view(hits), trk_off,
                                       trk_hits, n_tracks, prior_of(prior), align, field_scale, ck, status, dchi2,
                                       dchi2_per_track, partial, dalign, dfield, st),
                   "fit backward kernels");
}
}  // namespace

extern "C" {

int kfx_fit_tracks_backward(kfx_ctx* c, const kfx_hits* hits, const int32_t* trk_off, const int32_t* trk_hits,
                            int32_t n_tracks, const kfx_prior* prior, const float* align, float field_scale,
                            const kfx_states* ckpt, const int32_t* status, const float* dchi2,
                            int32_t dchi2_per_track, double* dalign, double* dfield, void* stream) {
  return backward_impl(c, hits, trk_off, trk_hits, n_tracks, prior, align, field_scale, ckpt, status, dchi2,
                       dchi2_per_track, dalign, dfield, stream, false);
}

int kfx_fit_tracks_backward_noalloc(kfx_ctx* c, const kfx_hits* hits, const int32_t* trk_off,
                                    const int32_t* trk_hits, int32_t n_tracks, const kfx_prior* prior,
                                    const float* align, float field_scale, const kfx_states* ckpt,
                                    const int32_t* status, const float* dchi2, int32_t dchi2_per_track,
                                    double* dalign, double* dfield, void* stream) {
  return backward_impl(c, hits, trk_off, trk_hits, n_tracks, prior, align, field_scale, ckpt, status, dchi2,
                       dchi2_per_track, dalign, dfield, stream, true);
}

}  // extern "C"
