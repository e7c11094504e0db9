// Internal interface between the C ABI (kfx_api.hip) and the kernels
// (kfx_kernels.hip): workspace layouts and launch wrappers.
#pragma once

#include <hip/hip_runtime.h>

#include "kfx_adjoint.h"
#include "kfx_build.h"

namespace kfx {

// Logical block of this workgroup when workgroups are dealt to the 8 XCDs
// in turn: XCD x takes logical blocks [x * per, (x + 1) * per), so that
// neighbouring logical blocks share an XCD and its L2; -1 = idle (launch
// 8 * per workgroups).
__device__ inline int xcd_block(int nblk) {
  const int per = (nblk + 7) >> 3;
  const int lb = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  return lb < nblk ? lb : -1;
}
inline int xcd_grid(int nblk) { return ((nblk + 7) >> 3) << 3; }

// Workspace of the hit binning (a counting sort keyed by event, layer and
// (eta, phi) bin).  counts must hold n_keys + 1 entries.
struct BinWork {
  int* key;       // [n_hits]
  int* counts;    // [n_keys + 1]
  int* rank;      // [n_hits]: place of a hit among its bin's hits
  int* off;       // [n_keys + 1]
  int* perm;      // [n_hits]
  float4* sorted; // [n_hits]
  int* scan_scratch;  // [n_keys / tile + 2]
  long ev_stride;     // keys per event of the index last built
};

// Duplicate removal over the best candidate (slot 0) of every seed.
struct DupArgs {
  const int* n_cands;    // [S]
  const int* hits;       // [S*K][H]
  const int* n_hits_c;   // [S*K]
  const int* n_holes_c;  // [S*K]
  const float* chi2_c;   // [S*K]
  int S, K, H, n_hits;   // seeds, slots per seed, list capacity, hit count
  int num, den;          // shared-hit fraction
  int* list;             // [S][H] ascending distinct hits of each track; the
                         // lists of a block's tracks back to back from the
                         // block's first row on
  int* next;             // [S][H] next entry holding the same hit, -1 at the end
  int* head;             // [n_hits] one holder's entry, -2 once the hit is
                         // known to be shared
  int* head2;            // [n_hits] of a shared hit: last entry pushed, -1 none
  int4* key;             // [S] n_hits, n_holes, chi2 bits, and the hit count
                         // of the list | its offset in the block's rows << 8
  int* dup_of;           // [S] output
};

// Hit masking between iterations over slot 0 of every seed.
struct MaskArgs {
  const int* n_cands;    // [S]
  const int* hits;       // [S*K][H]
  const int* n_hits_c;   // [S*K]
  const float* chi2_c;   // [S*K]
  const int* dup_of;     // [S] or NULL (every track counts as kept)
  int S, K, H, n_hits;
  int min_hits;
  float max_chi2_ndof;
  int* layer_out;        // [n_hits]
};

// Strip clustering over the digis of a batch of events.
// What the heads-and-walks pass keeps of a kept cluster, at its head
// digi: one 32-byte record, so that the write pass reads one line per
// cluster instead of a scattered word from each of several arrays.
struct __align__(32) StripRec {
  long sa;      // sum of strip * adc
  int last;     // last strip
  int charge;   // sum of adc
  int event;
  int module;
  int first;    // first strip
  int pad;
};

struct StripArgs {
  const int* module;        // [n] digis, sorted by (event, module, strip)
  const int* strip;         // [n]
  const unsigned short* adc;  // [n]
  const int* ev_off;        // [n_events + 1]
  int n, n_events;
  const float* noise;       // [n_modules * spm]
  const unsigned char* bad; // [n_modules * spm]
  int n_modules, spm;
  float seed_thr, chan_thr;
  double clus_thr2;         // clus_thr squared
  int max_gap, min_charge;
  int chunk;                // modules per chunk
  int stage;                // the chunk's calibration staged in LDS
  int* bnd;                 // [n_events * (chunks + 1)] first digi of each
                            // (event, module chunk)
  int* cnt;                 // [n_events * chunks] kept clusters of each
  int* cnt_off;             // [n_events * chunks + 1] their exclusive scan
  StripRec* rec;            // [n] kept clusters of (event, chunk) from the
                            // chunk's first digi on
  int* out_event;           // [capacity] kept clusters
  int* out_module;
  int* out_first;
  int* out_size;
  int* out_charge;
  float* out_bary;
  int capacity;
  int* n_out;               // [1] kept clusters (all, also beyond capacity)
};

void launch_fill(int* p, long n, int v, hipStream_t st);
void exclusive_scan(const int* in, long n, int* out, int* scratch, hipStream_t st);
void launch_bin(const Geometry* G, const HitsView& H, int n_layers, int n_bins, BinWork& w, int* bin_out,
                bool stable, hipStream_t st);
// One workgroup per event (sets w.ev_stride = n_layers * n_bins + 1):
// usable when bin_event_lds_bytes(n_layers * n_bins) fits a workgroup's LDS
// and bin_event_init has raised the kernel's dynamic LDS limit to it.
size_t bin_event_lds_bytes(long keys_per_event);
hipError_t bin_event_init(size_t max_lds);
void launch_bin_events(const Geometry* G, const HitsView& H, int n_layers, int n_bins, BinWork& w, hipStream_t st);
void launch_fit(const Geometry* G, const HitsView& H, const int* trk_off, const int* trk_hits, int n,
                const Prior& pr, const float* align, float fscale, const FitOut& o, hipStream_t st);
int fit_backward_blocks(int n);
hipError_t launch_fit_backward(const Geometry* G, int n_barrel, int n_layers, const HitsView& H, const int* trk_off,
                               const int* trk_hits, int n, const Prior& pr, const float* align, float fscale,
                               const StateSoA& ckpt, const int* status, const float* dchi2, int per_track,
                               double* partial, double* dalign, double* dfield, hipStream_t st);
void launch_seed_states(const Geometry* G, const HitsView& H, const int* seeds, int n, const Prior& pr,
                        const StateSoA& out, float* chi2, int* status, hipStream_t st);
void launch_step_compat(const Geometry* G, const HitsView& H, const BinIndex& B, const int* cand_event,
                        const int* cand_layer, const StateSoA& in, int n, float cut, int* next_layer,
                        const StateSoA& pred, int* pair_count, int* pair_hit, float* pair_chi2, int max_pairs,
                        hipStream_t st);
// ev: NULL, or two events recorded after the seed start and after the
// search (before the plain path's output kernel; the fused kernel writes
// its outputs itself, so its second event follows it)
void launch_build_plain(const BuildArgs& a, const TracksOut& o, hipStream_t st, const hipEvent_t* ev);
size_t fused_lds_bytes(int lanes, int threads, int max_steps);
size_t fused_static_lds_bytes();
void launch_build_init(const BuildArgs& a, hipStream_t st);
void launch_build_fused(const BuildArgs& a, const TracksOut& o, int* seed_counter, int blocks, int threads,
                        int lanes, int waves_per_simd, hipStream_t st, const hipEvent_t* ev);
int fused_lanes_for(int K);   // default lanes per seed group
int fused_lanes_pow2(int K);  // the smallest power of two >= max(K, 4)
void launch_find_duplicates(const DupArgs& a, hipStream_t st);
void launch_mask_hits(const MaskArgs& a, const int* layer_in, hipStream_t st);
int strip_chunks(int n_modules, int chunk);
size_t strip_cal_lds(int chunk, int spm);
void launch_cluster_strips(const StripArgs& a, int* scan_scratch, hipStream_t st);

}  // namespace kfx
