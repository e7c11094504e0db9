// Track building work items: the beam search of Sec. 1-3 of the paper
// (arXiv 2002.06295) as four per-step pieces shared by the plain per-step
// kernels and the fused persistent kernel.
//
// Per step every live candidate of a seed is moved to its next surface,
// offers children (one per compatible hit, a hole child while its
// consecutive holes stay below the limit, or a stop child when it cannot
// continue), and the seed keeps the best K children by the ranking key of
// child_key().  Kept hit children get the Kalman update.
#pragma once

#include "kfx_work.h"

namespace kfx {

struct BuildArgs {
  const Geometry* G;
  HitsView H;
  BinIndex B;
  const int* seeds;       // [S][3]
  const int* seed_event;  // [S]
  int n_seeds;
  Prior prior;
  float cut;
  int K;
  int max_holes;
  int max_steps;
  int overlap;            // recover a second hit on the layer of a kept hit child
  RankW rank;             // ranking of the children (key or score)
  float inflate;          // window widening (>= 1; the window is a superset at 1)
  int coop_min;           // fused: window size scanned by the whole wave
  int groups_per_wave;    // fused: seed groups of a wavefront that take seeds
  // candidate slots (S K), two buffers used in turn
  StateSoA cand[2];
  int* layer[2];
  float* chi2[2];
  int* meta[2];
  // predicted state of each slot and its surface (-1 none, -2 empty slot)
  StateSoA pred;
  int* next_layer;
  // best K children (chi2, hit) of each slot and their count
  float* kid_c;
  int* kid_h;
  int* kid_n;
  // selection for each new slot: parent slot (-1 empty), child code, chi2
  int* sel_parent;
  int* sel_code;
  float* sel_chi2;
  // history of the plain path, per seed: [S][max_steps][K] parent slot and
  // child code (the fused kernel keeps its own in LDS)
  signed char* hist_parent;
  int* hist_code;
  // history of the fused kernel, per seed: [S][max_steps][K] words, the
  // child's code + 2 in bits 0-26 and its parent slot + 1 in bits 27-31
  unsigned int* hist_word;
  // with overlap recovery, both paths: the recovered hit of each history
  // entry, or -1 ([S][max_steps][K])
  int* hist_ov;
  int* n_steps;           // [S] steps recorded
  unsigned long long* stats;  // steps, pairs, updates
};

KFX_HD long hist_index(const BuildArgs& a, int seed, int t, int slot) {
  return ((long)seed * a.max_steps + t) * a.K + slot;
}

// Step 0: the seed state in slot 0 of each seed, other slots empty.
KFX_HD void init_seed_slots(const BuildArgs& a, int s) {
  const int* sh = a.seeds + 3 * s;
  State st;
  float c2 = 0.0f;
  const int ev = a.seed_event[s];
  const bool ok = ev >= 0 && ev < a.H.n_events && seed_state(*a.G, a.H, sh, a.prior, st, c2);
  for (int j = 0; j < a.K; ++j) {
    const long slot = (long)s * a.K + j;
    if (j == 0 && ok) {
      store_state(a.cand[0], slot, st);
      a.layer[0][slot] = a.H.layer[sh[2]];
      a.chi2[0][slot] = c2;
      a.meta[0][slot] = meta_pack(kSeedHits, 0, 0, kFlagLive);
    } else {
      a.meta[0][slot] = 0;
      a.layer[0][slot] = -1;
      a.chi2[0][slot] = 0.0f;
    }
  }
  if (a.n_steps) a.n_steps[s] = 0;  // the plain path's step count
}

// (a) navigate + transport (+ material) of one slot.  Returns 1 when a
// step was taken (a candidate moved to a surface).
KFX_HD int predict_slot(const BuildArgs& a, int cur, long slot) {
  const int m = a.meta[cur][slot];
  if (!(meta_flags(m) & kFlagLive)) {
    a.next_layer[slot] = -2;
    return 0;
  }
  if (meta_flags(m) & kFlagDone) {
    a.next_layer[slot] = -1;
    return 0;
  }
  const Geometry& G = *a.G;
  State st, pr;
  load_state(a.cand[cur], slot, st);
  double cphi, sphi;
  sincos_d(st.phi, sphi, cphi);
  const double kappa = -kHcD * G.bz;
  double s = 0.0;
  double sth, cth;
  sincos_d(st.th, sth, cth);
  const int nl = navigate(G, a.layer[cur][slot], st, cphi, sphi, sth, cth, kappa * st.k, s);
  if (nl < 0) {
    a.next_layer[slot] = -1;
    return 0;
  }
  transport(st, G.L[nl], cphi, sphi, sth, cth, s, kappa, pr);
  store_state(a.pred, slot, pr);
  a.next_layer[slot] = nl;
  return 1;
}

// (b) compatible hits of one predicted slot; keeps the best K.  Returns the
// number of compatible pairs.
KFX_HD int pairs_slot(const BuildArgs& a, long slot, int ev) {
  const int nl = a.next_layer[slot];
  if (nl < 0) {
    a.kid_n[slot] = 0;
    return 0;
  }
  State pr;
  load_state(a.pred, slot, pr);
  Frame F;
  make_frame(pr, a.G->L[nl], F);
  BestK<kMaxK> b;
  const int found = scan_window(*a.G, a.B, ev, nl, pr, F, a.cut, a.K, b, a.inflate);
#pragma unroll
  for (int r = 0; r < kMaxK; ++r)
    if (r < b.n) {
      a.kid_c[slot * a.K + r] = pair_key_chi2(b.k[r]);
      a.kid_h[slot * a.K + r] = pair_key_hit(b.k[r]);
    }
  a.kid_n[slot] = b.n;
  return found;
}

// Children of one parent slot, in rank order, as (key, code, chi2).
// Shared by the per-seed selection and the fused kernel's lane streams.
struct KidStream {
  int nh, nho, consec, parent;
  float chi2;
  int nkids;      // hit children available
  bool hole;      // hole child allowed
  bool stop;      // the single child is a stop child
  bool live;
};

KFX_HD KidStream kid_stream(const BuildArgs& a, int meta, float chi2, int next_layer, int nkids,
                            int parent) {
  KidStream k;
  k.live = (meta_flags(meta) & kFlagLive) != 0;
  k.nh = meta_nhits(meta);
  k.nho = meta_nholes(meta);
  k.consec = meta_consec(meta);
  k.parent = parent;
  k.chi2 = chi2;
  k.nkids = 0;
  k.hole = false;
  k.stop = false;
  if (!k.live) return k;
  if (next_layer < 0) {
    k.stop = true;
    return k;
  }
  k.nkids = nkids;
  k.hole = k.consec < a.max_holes;
  if (k.nkids == 0 && !k.hole) k.stop = true;
  return k;
}

// key of child number r of a stream (r < nkids: hit child r; r == nkids:
// hole; stop: r == 0) under the call's ranking w; ~0 when exhausted.
KFX_HD uint64_t kid_key(const RankW& w, const KidStream& k, int K, int r, const float* kc, float& chi2_out) {
  if (!k.live) return ~0ull;
  if (k.stop) {
    if (r > 0) return ~0ull;
    chi2_out = k.chi2;
    return rank_key(w, k.nh, k.nho, k.chi2, k.parent, 0);
  }
  if (r < k.nkids) {
    chi2_out = k.chi2 + kc[r];
    return rank_key(w, k.nh + 1, k.nho, chi2_out, k.parent, r);
  }
  if (r == k.nkids && k.hole) {
    chi2_out = k.chi2;
    return rank_key(w, k.nh, k.nho + 1, k.chi2, k.parent, K);
  }
  return ~0ull;
}

// (c) per seed: keep the best K children over all its parents.
KFX_HD void select_seed(const BuildArgs& a, int cur, int s) {
  const int K = a.K;
  KidStream ks[kMaxK];
  int pos[kMaxK];
  uint64_t head[kMaxK];
  float hc[kMaxK];
  for (int j = 0; j < K; ++j) {
    const long slot = (long)s * K + j;
    ks[j] = kid_stream(a, a.meta[cur][slot], a.chi2[cur][slot], a.next_layer[slot],
                       a.next_layer[slot] >= 0 ? a.kid_n[slot] : 0, j);
    pos[j] = 0;
    head[j] = kid_key(a.rank, ks[j], K, 0, a.kid_c + slot * K, hc[j]);
  }
  for (int i = 0; i < K; ++i) {
    int w = -1;
    uint64_t best = ~0ull;
    for (int j = 0; j < K; ++j)
      if (head[j] < best) {
        best = head[j];
        w = j;
      }
    const long out = (long)s * K + i;
    if (w < 0) {
      a.sel_parent[out] = -1;
      a.sel_code[out] = kStop;
      a.sel_chi2[out] = 0.0f;
      continue;
    }
    const long ps = (long)s * K + w;
    int code;
    if (ks[w].stop) code = kStop;
    else if (pos[w] < ks[w].nkids) code = a.kid_h[ps * K + pos[w]];
    else code = kHole;
    a.sel_parent[out] = w;
    a.sel_code[out] = code;
    a.sel_chi2[out] = hc[w];
    pos[w]++;
    head[w] = kid_key(a.rank, ks[w], K, pos[w], a.kid_c + ps * K, hc[w]);
  }
}

// (d) one new slot: copy its parent (predicted state for hit and hole
// children, current state for a stop child) and apply the update.
// Returns 1 when a Kalman update was applied.
KFX_HD int update_slot(const BuildArgs& a, int cur, int s, int j, int t) {
  const int nxt = 1 - cur;
  const long slot = (long)s * a.K + j;
  const int par = a.sel_parent[slot];
  const long hidx = hist_index(a, s, t, j);
  if (a.overlap) a.hist_ov[hidx] = -1;
  if (par < 0) {
    a.meta[nxt][slot] = 0;
    a.layer[nxt][slot] = -1;
    a.chi2[nxt][slot] = 0.0f;
    a.hist_parent[hidx] = -1;
    a.hist_code[hidx] = kStop;
    return 0;
  }
  const long ps = (long)s * a.K + par;
  const int code = a.sel_code[slot];
  const int pm = a.meta[cur][ps];
  State st;
  int upd = 0;
  float chi2 = a.sel_chi2[slot];
  if (code == kStop) {
    load_state(a.cand[cur], ps, st);
    a.layer[nxt][slot] = a.layer[cur][ps];
    a.meta[nxt][slot] = meta_pack(meta_nhits(pm), meta_nholes(pm), meta_consec(pm), kFlagLive | kFlagDone);
  } else {
    load_state(a.pred, ps, st);
    const int nl = a.next_layer[ps];
    a.layer[nxt][slot] = nl;
    if (code >= 0) {
      kf_update_fp64(st, a.G->L[nl], (double)a.H.x[code], (double)a.H.y[code], (double)a.H.z[code]);
      int nh = meta_nhits(pm) + 1;
      upd = 1;
      if (a.overlap) {
        float c2 = 0.0f;
        const int h2 = recover_overlap(*a.G, a.B, a.seed_event[s], nl, st, a.cut, code, a.inflate, c2);
        if (h2 >= 0) {
          kf_update_fp64(st, a.G->L[nl], (double)a.H.x[h2], (double)a.H.y[h2], (double)a.H.z[h2]);
          ++nh;
          ++upd;
          chi2 += c2;
          a.hist_ov[hidx] = h2;
        }
      }
      a.meta[nxt][slot] = meta_pack(nh, meta_nholes(pm), 0, kFlagLive);
    } else {
      a.meta[nxt][slot] = meta_pack(meta_nhits(pm), meta_nholes(pm) + 1, meta_consec(pm) + 1, kFlagLive);
    }
  }
  store_state(a.cand[nxt], slot, st);
  a.chi2[nxt][slot] = chi2;
  a.hist_parent[hidx] = (signed char)par;
  a.hist_code[hidx] = code;
  if (j == 0) a.n_steps[s] = t + 1;
  return upd;
}

// Output of building, per seed and slot (best first).
struct TracksOut {
  int* n_cands;     // [S]
  int* hits;        // [S][K][max_hits]: seed hits then one entry per step
                    // with a hit or a hole (-1); unused entries -3
  int* n_hits;      // [S][K]
  int* n_holes;     // [S][K]
  float* chi2;      // [S][K]
  StateSoA state;   // S K entries
  int max_hits;
};

// Hit list of one final slot, written to `out` (max_hits entries): the seed
// hits, then one entry per step with
// a hit or a hole (-1), `total` entries in all (stop entries add none),
// rebuilt from the per-step history by one backward walk over the parent
// pointers; the rest of the row -3 (all of it for a slot without a
// candidate).  T is the seed's step count; hist(t, slot, code, parent)
// reads the history entry of step t and slot.
template <class Hist>
KFX_HD void write_hit_row(const BuildArgs& a, int* out, int max_hits, int s, int j, int T, bool live, int total,
                          const Hist& hist) {
  // (hist(t, slot, code, parent, ov): ov is the hit recovered after `code`
  // on the same layer, or -1)
  if (!live) total = 0;
  {
    // unused entries: one by one up to a 16-byte boundary, then four at a
    // time (when the row is 16-byte aligned), then the rest
    int q = total < max_hits ? total : max_hits;
    if ((reinterpret_cast<uintptr_t>(out) & 15) == 0) {
      for (; q < max_hits && (q & 3); ++q) out[q] = -3;
      for (; q + 4 <= max_hits; q += 4) *reinterpret_cast<int4*>(out + q) = make_int4(-3, -3, -3, -3);
    }
    for (; q < max_hits; ++q) out[q] = -3;
  }
  if (!live) return;
  for (int q = 0; q < kSeedHits && q < max_hits; ++q) out[q] = a.seeds[3 * s + q];
  int w = total - 1, cj = j;
  for (int t = T - 1; t >= 0; --t) {
    int code, parent, ov;
    hist(t, cj, code, parent, ov);
    if (ov >= 0) {
      if (w < max_hits) out[w] = ov;
      --w;
    }
    if (code != kStop) {
      if (w < max_hits) out[w] = code >= 0 ? code : -1;
      --w;
    }
    cj = parent;
    if (cj < 0) break;  // (a slot without a candidate has no parent)
  }
}

template <class Hist>
KFX_HD void write_slot_hits(const BuildArgs& a, const TracksOut& o, int s, int j, int T, bool live, int total,
                            const Hist& hist) {
  write_hit_row(a, o.hits + ((long)s * a.K + j) * o.max_hits, o.max_hits, s, j, T, live, total, hist);
}

// Counts, chi2 sum and state of one final slot (m its meta word); zeros for
// a slot without a candidate.
KFX_HD void write_slot_summary(const TracksOut& o, long slot, int m, float chi2, const State& st) {
  if (!(meta_flags(m) & kFlagLive)) {
    o.n_hits[slot] = 0;
    o.n_holes[slot] = 0;
    o.chi2[slot] = 0.0f;
    State z;
    z.x = z.y = z.z = z.k = z.phi = z.th = 0.0;
    for (int q = 0; q < 21; ++q) z.C[q] = 0.0f;
    store_state(o.state, slot, z);
    return;
  }
  o.n_hits[slot] = meta_nhits(m);
  o.n_holes[slot] = meta_nholes(m);
  o.chi2[slot] = chi2;
  store_state(o.state, slot, st);
}

// The whole output of one final slot.
template <class Hist>
KFX_HD void write_slot_output(const BuildArgs& a, const TracksOut& o, int s, int j, int T, int m, float chi2,
                              const State& st, const Hist& hist) {
  const bool live = (meta_flags(m) & kFlagLive) != 0;
  write_slot_hits(a, o, s, j, T, live, meta_nhits(m) + meta_nholes(m), hist);
  write_slot_summary(o, (long)s * a.K + j, m, chi2, st);
}

// History entries of the plain path (HBM, per seed, step and slot).
struct HbmHist {
  const BuildArgs* a;
  int s;
  KFX_HD void operator()(int t, int j, int& code, int& parent, int& ov) const {
    const long h = hist_index(*a, s, t, j);
    code = a->hist_code[h];
    parent = a->hist_parent[h];
    ov = a->overlap ? a->hist_ov[h] : -1;
  }
};

// History entries of the fused kernel (HBM, one packed word per seed, step
// and slot).
struct HbmWordHist {
  const BuildArgs* a;
  int s;
  KFX_HD void operator()(int t, int j, int& code, int& parent, int& ov) const {
    const long h = hist_index(*a, s, t, j);
    const unsigned int e = a->hist_word[h];
    code = (int)(e & 0x7ffffffu) - 2;
    parent = (int)(e >> 27) - 1;
    ov = a->overlap ? a->hist_ov[h] : -1;
  }
};
KFX_HD unsigned int hist_word_pack(int code, int parent) {
  return (unsigned int)(code + 2) | ((unsigned int)(parent + 1) << 27);
}

// The same for a slot of the plain path's final candidate buffer.
KFX_HD void finalize_slot(const BuildArgs& a, int fin, const TracksOut& o, int s, int j) {
  const long slot = (long)s * a.K + j;
  State st;
  load_state(a.cand[fin], slot, st);
  write_slot_output(a, o, s, j, a.n_steps[s], a.meta[fin][slot], a.chi2[fin][slot], st, HbmHist{&a, s});
}

}  // namespace kfx
