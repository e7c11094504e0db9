/*
 * kfx -- Kalman-filter track building and fitting on AMD Instinct MI355X
 * (gfx950).  C ABI of libkfx.so.
 *
 * What it computes (arXiv 2002.06295, "Reconstruction of Charged Particle
 * Tracks in Realistic Detector Geometry Using a Vectorized and Parallelized
 * Kalman Filter Algorithm"):
 *   Sec. 1   the Kalman filter propagates the track state (parameters and
 *            their uncertainties) from one layer to the next, material
 *            effects included, then updates it with the hit's position;
 *            track building is a combinatorial search for the hits of a
 *            track that starts from a seed in the innermost layers and
 *            proceeds outward; fitting applies the filter to the hits that
 *            building found.
 *   Sec. 2   lightweight geometry: barrel layers at their radius, forward
 *            layers at their z, hits known by their 3D position; per
 *            layer a seed keeps at most K candidates, its highest-ranked
 *            children.
 *   Sec. 3   missing hits are counted consistently and enter the score.
 *
 * Conventions.  Units cm, GeV, T, rad.  Field along +z.  Track state
 * p = (x, y, z, k = q/pT, phi, theta) with (x, y, z) on the current surface
 * and (phi, theta) the momentum direction there.  Covariances are the 21
 * floats of the lower triangle of the 6x6 matrix, row-major: element (i, j),
 * i >= j, at index i(i+1)/2 + j.
 *
 * Memory.  Every pointer marked "device" is HIP device memory owned by the
 * caller (the library never frees it); host pointers are read during the
 * call only.  The context owns its geometry and its workspaces (a pool that
 * grows on demand and is reused; growing synchronizes the given stream).
 * Calls are ordered on the given HIP stream (NULL = default stream) and do
 * not synchronize otherwise; results are valid once the stream has reached
 * them.
 *
 * Errors.  Every int-returning call returns KFX_OK (0) or a negative code;
 * kfx_last_error() gives a message.  Invalid arguments are rejected before
 * any work is queued.  A context is not thread-safe: one host thread at a
 * time.
 */
#ifndef KFX_H
#define KFX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KFX_OK 0
#define KFX_EINVAL (-1)     /* bad argument (sizes, NULL, non-finite, order) */
#define KFX_EOVERFLOW (-2)  /* output capacity too small; see kfx_tracks.needed */
#define KFX_EHIP (-3)       /* HIP runtime error */
#define KFX_ESTATE (-4)     /* call out of order (no geometry, no hit index) */
#define KFX_ENOMEM (-5)     /* workspace allocation failed */

#define KFX_MODE_PLAIN 0    /* one kernel per piece of each step */
#define KFX_MODE_FUSED 1    /* one persistent kernel for all steps */

#define KFX_MAX_LAYERS 64
#define KFX_MAX_CANDS 16
#define KFX_MAX_STEPS 40

typedef struct kfx_ctx kfx_ctx;

/* Track states, structure of arrays over `stride` entries (device).  The
 * six parameters are float64 (a float32 coordinate at 100 cm already has a
 * rounding error of ~2e-3 of the 20 um hit resolution); the covariance is
 * float32. */
typedef struct {
  double* par;     /* [6][stride] x, y, z, k, phi, theta (float64)        */
  float* cov;      /* [21][stride] packed covariance (float32)            */
  int64_t stride;  /* entries per row; >= number of states written        */
} kfx_states;

/* Hits of one or more events, structure of arrays (device).  Hits of
 * event e are [event_offsets[e], event_offsets[e+1]); hit indices are
 * global.  layer[i] outside [0, n_layers) marks a hit to ignore. */
typedef struct {
  const float* x;
  const float* y;
  const float* z;
  const int32_t* layer;
  const int32_t* event_offsets; /* [n_events + 1], device */
  int32_t n_hits;
  int32_t n_events;
} kfx_hits;

/* Prior covariance of the three-hit start estimate: diagonal with
 * sigma_pos^2 on x, y, z, (sk_rel |k|)^2, sigma_phi^2, sigma_theta^2. */
typedef struct {
  float spos, sk_rel, sphi, stheta;
} kfx_prior;

typedef struct {
  float chi2_cut;        /* keep candidate-hit pairs with 3x3 chi2 < cut      */
  int32_t max_cands;     /* K: candidates kept per seed, 1..KFX_MAX_CANDS     */
  int32_t max_holes;     /* a hole child is offered while consecutive holes
                            are below this                                    */
  int32_t max_steps;     /* surfaces searched after the seed, 1..KFX_MAX_STEPS */
  kfx_prior prior;
  int32_t mode;          /* KFX_MODE_PLAIN or KFX_MODE_FUSED                  */
  int32_t block_threads; /* fused: threads per block, 64..256, multiple of 64;
                            0 = library choice                                */
  int32_t blocks;        /* fused: persistent blocks; 0 = library choice      */
  int32_t lanes_per_seed;/* fused: lanes of the group that holds one seed's
                            candidates (one lane per slot): 4, 8 or 16, at
                            least K, or 6 for K of 5 or 6 (ten seeds a
                            wavefront), or 12 for K of 9 to 12 (five);
                            0 = 6 for K of 5 or 6, else the smallest power
                            of two that fits K                               */
  int32_t scan_tile;     /* fused: windows holding more hits than this are
                            scanned by the whole wavefront together; smaller
                            ones by their own lane; 0 = 64                    */
  int32_t waves_per_simd;/* fused: register budget of the kernel, 1 (all 512
                            registers of a lane) or 2 (256, two waves resident
                            per SIMD; K <= 6 fits it with at most a few
                            registers spilled, larger K spill more); 0 = 1  */
  int32_t seeds_per_wave;/* fused: seeds a wavefront works on at once, 1 ..
                            64 / lanes_per_seed (the rest of its lanes idle):
                            fewer seeds per wavefront spread a small event
                            over more SIMDs; 0 = 64 / lanes_per_seed         */
  float window_inflate;  /* factor widening every search window (>= 1; 0 =
                            1): the window is already a superset of the
                            compatible hits, so results do not change; a
                            wider one only reads more bins                   */
  int32_t overlap;       /* nonzero: overlap recovery -- after a kept hit
                            child is updated with hit h1, the best (chi2,
                            index) hit of the same layer with an index above
                            h1 and chi2 < chi2_cut against the updated state
                            is added as a second hit of that layer (one more
                            update, hit and chi2 term; right after h1 in the
                            hit list).  Sec. 3 of the paper names recovering
                            hits of overlapping modules as planned work. */
  int32_t score;         /* 0: children ranked by hits (more first), holes
                            (fewer first), chi2 sum (smaller first); nonzero:
                            by the score score_hit n_hits - score_hole
                            n_holes - score_chi2 chi2 (float32, higher
                            first).  Both then by parent slot and rank; Sec.
                            3 of the paper re-tunes the score for short
                            tracks without a formula.                        */
  float score_hit, score_hole, score_chi2;
  int32_t binning;       /* hit index of the build: 0 automatic (2 from 64
                            events on, else 1), 1 counting sort over the
                            whole batch with global atomics, 2 one workgroup
                            per event counting in LDS (falls back to 1 when
                            an event's bins do not fit LDS).  Same tracks
                            either way (the order within a bin differs).     */
} kfx_build_params;

/* Output of building, per seed s and slot j < K, best first (device). */
typedef struct {
  int32_t* n_cands;  /* [S] candidates kept                                   */
  int32_t* hits;     /* [S][K][max_hits]: the 3 seed hits, then one entry per
                        surface reached (hit index, or -1 for a hole; with
                        overlap recovery a recovered hit follows its
                        layer's hit); unused entries -3; a list longer than
                        max_hits is cut (n_hits and n_holes still count
                        all)                                                   */
  int32_t* n_hits;   /* [S][K]                                               */
  int32_t* n_holes;  /* [S][K]                                               */
  float* chi2;       /* [S][K] total chi2 (seed hits included)               */
  kfx_states state;  /* S*K entries: state on the last surface reached       */
  uint64_t* stats;   /* [3] device, added to: steps (candidate-surface pairs
                        propagated), compatible pairs, Kalman updates        */
  int32_t max_hits;  /* capacity of each hit list (>= 3)                     */
  int64_t capacity;  /* candidate entries allocated in the arrays (>= S*K)   */
  int64_t needed;    /* written on KFX_EOVERFLOW: entries required           */
} kfx_tracks;

/* Create a context on HIP device `device`.  *out receives the handle. */
int kfx_create(int device, kfx_ctx** out);

/* Release the context and its workspaces.  NULL is ignored.  The caller
 * must make sure no queued work still uses the context. */
void kfx_destroy(kfx_ctx* ctx);

/* Last error message of this context ("" if none; never NULL). */
const char* kfx_last_error(const kfx_ctx* ctx);

/* Load the geometry (Sec. 2: barrel cylinders at a radius, disks at a z).
 * table: host float64 [n_layers][8] rows (kind 0 barrel / 1 disk, pos = R
 * or Z, lo, hi = z bounds (barrel) or r bounds (disk), x/X0, sigma_u,
 * sigma_v, sigma_n), with u = r*phi direction, v = z (barrel) or r (disk),
 * n = surface normal.  bz: field [T].  n_eta x n_phi: hit bins per layer.
 * Copied; the caller may free the table.  KFX_EINVAL on more than
 * KFX_MAX_LAYERS layers, non-finite values, lo >= hi, a barrel radius or
 * disk bound <= 0, duplicate barrel radii or duplicate disk positions. */
int kfx_load_layers(kfx_ctx* ctx, const double* table, int n_layers, double bz, int n_eta,
                    int n_phi);

/* Hit index (Sec. 2 works with 3D hit positions; the (eta, phi) binning is
 * this library's index): bin of each hit, eta_bin * n_phi + phi_bin, in
 * FP64 from the FP32 coordinates, and a stable counting sort by
 * (event, layer, bin).  The index stays in the context for
 * kfx_step_compat on the same hits.  Optional device outputs (NULL to
 * skip): bin_out [n_hits] (-1 for ignored hits), offsets_out
 * [n_events * n_layers * n_eta * n_phi + 1], perm_out [n_hits] (hit
 * indices in index order; entries past offsets_out[last] unused). */
int kfx_bin_hits(kfx_ctx* ctx, const kfx_hits* hits, int32_t* bin_out, int32_t* offsets_out,
                 int32_t* perm_out, void* stream);

/* Start states of seeds (Sec. 1: seeds from the innermost layers): a
 * three-hit helix estimate at hit 1 with the prior covariance, then the
 * Kalman filter over the three hits.  seeds: device int32 [n][3] hit
 * indices.  out: state at hit 3; chi2 [n]; status [n] 1 = ok, 0 = failed
 * (a seed hit off the geometry or a surface not reached). */
int kfx_seed_states(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* seeds, int32_t n,
                    const kfx_prior* prior, kfx_states* out, float* chi2, int32_t* status,
                    void* stream);

/* One building step on given states (device inputs): navigate from
 * cand_layer to the next surface, propagate with material noise, and list
 * every hit of that surface in event cand_event with chi2 < chi2_cut,
 * ascending hit index.  Needs kfx_bin_hits on the same hits first
 * (KFX_ESTATE otherwise).  Outputs (device): next_layer [n] (-1: none),
 * pred (predicted states), pair_count [n] (all compatible hits, may exceed
 * max_pairs), pair_hit / pair_chi2 [n][max_pairs]. */
int kfx_step_compat(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* cand_event,
                    const int32_t* cand_layer, const kfx_states* in, int32_t n, float chi2_cut,
                    int32_t* next_layer, kfx_states* pred, int32_t* pair_count, int32_t* pair_hit,
                    float* pair_chi2, int32_t max_pairs, void* stream);

/* Track building (Sec. 1-3).  seeds: device int32 [n_seeds][3];
 * seed_event: device int32 [n_seeds].  Bins the hits, starts every seed,
 * then per step keeps the best K children of each seed.  KFX_EOVERFLOW
 * (with out->needed) when out->capacity < n_seeds * K.  KFX_MODE_FUSED
 * takes at most 2^27 - 3 hits (its per-step history words hold the hit
 * index in 27 bits) and a launch shape whose LDS fits in a block
 * (KFX_EINVAL otherwise). */
int kfx_build_tracks(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* seeds,
                     const int32_t* seed_event, int32_t n_seeds, const kfx_build_params* params,
                     kfx_tracks* out, void* stream);

/* Duplicate removal after building (abstract; Sec. 3: the duplicate
 * tracks that building produces are removed in a step of their own; the
 * paper gives no criterion, the reading below is this library's).
 * tracks: a building output (kfx_tracks of kfx_build_tracks, or the same
 * layout filled by the caller) of n_seeds seeds with K slots each; only
 * n_cands, hits, n_hits, n_holes and chi2 are read.  Each seed with
 * n_cands > 0 contributes one track, its slot 0.  The hits of a track are
 * the distinct entries h of its hit list with 0 <= h < n_hits (the hit
 * count of the batch); holes and padding are not hits.  Track b is a
 * duplicate of track a when they share at least one hit, frac_den * shared
 * >= frac_num * (hit count of the shorter of the two), and a ranks above b
 * in the building order: larger n_hits, then smaller n_holes, then smaller
 * chi2 (float32, must be finite), then smaller seed index.  The judgement
 * is pairwise.  Output dup_of: device int32 [n_seeds]: -2 for a seed
 * without a candidate, -1 for a kept track, else the seed of the
 * highest-ranked track of which it is a duplicate.  Needs 0 < frac_num <=
 * frac_den, max_hits <= 64, capacity >= n_seeds * K; the workspace grows
 * with n_seeds * max_hits and n_hits.  Deterministic. */
int kfx_find_duplicates(kfx_ctx* ctx, const kfx_tracks* tracks, int32_t n_seeds, int32_t K, int32_t n_hits,
                        int32_t frac_num, int32_t frac_den, int32_t* dup_of, void* stream);

/* Hit masking between iterations (Sec. 3: the hits used by tracks of good
 * quality are masked before the next iteration, which then searches fewer
 * hits).  Writes layer_out (device int32 [n_hits]) = layer_in, with -1 (a
 * hit every call ignores) at each valid hit index (0 <= h < n_hits) of the
 * hit list of every good track; layer_out may equal layer_in (in place).
 * A track is slot 0 of a seed with n_cands > 0 (layout as for
 * kfx_find_duplicates); it is good when dup_of is NULL or dup_of[s] == -1,
 * n_hits >= min_hits and chi2 <= max_chi2_ndof * (2 n_hits - 5), that
 * product formed in float32.  Deterministic (every write stores -1). */
int kfx_mask_hits(kfx_ctx* ctx, const kfx_tracks* tracks, int32_t n_seeds, int32_t K, const int32_t* dup_of,
                  int32_t min_hits, float max_chi2_ndof, const int32_t* layer_in, int32_t* layer_out,
                  int32_t n_hits, void* stream);

/* Silicon-strip digis of a batch of events (device).  Digis of event e are
 * [event_offsets[e], event_offsets[e+1]), sorted by (module, strip) with at
 * most one digi per strip (the results for unsorted digis are unspecified;
 * no access leaves the arrays); a digi whose (module, strip) lies outside
 * the calibration table is ignored. */
typedef struct {
  const int32_t* module;
  const int32_t* strip;
  const uint16_t* adc;
  const int32_t* event_offsets; /* [n_events + 1] */
  int32_t n;
  int32_t n_events;
} kfx_digis;

/* Calibration of the strip modules (device): noise in ADC counts and a bad
 * flag (nonzero = bad) per strip, index module * strips_per_module + strip. */
typedef struct {
  const float* noise;
  const uint8_t* bad;
  int32_t n_modules;
  int32_t strips_per_module;
} kfx_strip_calib;

typedef struct {
  float seed_thr;    /* seed strip: adc > seed_thr * noise (3), float32      */
  float chan_thr;    /* cluster strip: adc > chan_thr * noise (2), not bad,
                        float32 product                                      */
  double clus_thr;   /* kept: sum adc^2 > clus_thr^2 * sum noise^2 (5),
                        clus_thr^2 formed in float64                         */
  int32_t max_gap;   /* strips between two cluster strips, all bad (1)      */
  int32_t min_charge;/* kept: sum adc >= min_charge                         */
} kfx_cluster_params;

/* Kept clusters (device, caller-owned), in (event, module, first strip)
 * order. */
typedef struct {
  int32_t* event;
  int32_t* module;
  int32_t* first;      /* first strip                                      */
  int32_t* size;       /* last - first + 1 (bridged bad strips included)   */
  int32_t* charge;     /* sum of the ADCs                                  */
  float* barycenter;   /* sum(strip * adc) / sum(adc), float64 divide      */
  int32_t capacity;
  int32_t* n_out;      /* device int32 [1]: number of kept clusters; those
                          beyond capacity are counted but not written      */
} kfx_clusters;

/* Strip clustering (Sec. 4: the clustering of silicon-strip data ported to
 * GPUs for the HLT; thresholds and the gap rule as read in
 * kfx_cluster_params).  Two consecutive cluster strips of a module (in
 * digi order) join when at most max_gap strips lie between them and all
 * of those are bad; a cluster is a maximal chain and is kept when it holds
 * a seed strip, sum adc^2 > clus_thr^2 * sum noise^2 (noise^2 summed in
 * float64 in strip order) and sum adc >= min_charge.  All events of the
 * batch in one pass; deterministic.  KFX_EINVAL for bad sizes, NULL arrays,
 * non-finite or negative thresholds, max_gap outside 0..64, or
 * n_modules * strips_per_module >= 2^31. */
int kfx_cluster_strips(kfx_ctx* ctx, const kfx_digis* digis, const kfx_strip_calib* calib,
                       const kfx_cluster_params* params, kfx_clusters* out, void* stream);

/* Track fit (Sec. 1): the Kalman filter over fixed hit lists.  trk_off:
 * device int32 [n_tracks+1] into trk_hits (device int32 hit indices in
 * crossing order).  Starts at hit 1 from the three-hit estimate with the
 * prior, updates at hit 1, then propagates and updates through hit N.
 * align: device float32 [3 n_layers] (dr, drphi, dz) per layer or NULL;
 * for a barrel layer the hit moves to ((R+dr) cos(phi+drphi/R),
 * (R+dr) sin(phi+drphi/R), z+dz) and the track is propagated to radius
 * R+dr (disks are not aligned).  The field is bz * field_scale.
 * Outputs (device): state at hit N, chi2 [n] (float32, accumulated in
 * float64), ndof [n] = 2N - 5, status [n]: 1 ok, 0 failed (fewer than 3
 * hits, a hit off the geometry, a surface not reached), -1 checkpoint
 * capacity too small for this track.  ckpt: NULL, or states receiving the
 * filtered state after every hit, hit i of track t at entry
 * i * n_tracks + t (one row per hit number, so that the writes of one
 * step are coalesced); stride >= n_tracks * (longest track). */
int kfx_fit_tracks(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* trk_off,
                   const int32_t* trk_hits, int32_t n_tracks, const kfx_prior* prior,
                   const float* align, float field_scale, kfx_states* out, float* chi2,
                   int32_t* ndof, int32_t* status, kfx_states* ckpt, void* stream);

/* Adjoint of the fit (an addition to the paper, whose fit has no
 * alignment or field parameters): the gradient of L = sum_t w_t chi2_t over
 * the tracks with status 1 with respect to the alignment of every barrel
 * layer and the field scale, for the same inputs as a kfx_fit_tracks call
 * made with a checkpoint.  ckpt: the states that call wrote (read only);
 * status: its status array.  dchi2: device float32, w_t = dchi2[t] when
 * dchi2_per_track != 0, else w_t = dchi2[0] for every track.  The sweep
 * recomputes each step in float64 from the checkpointed state before it and
 * pulls the adjoint back through the update, the material noise, the
 * covariance transport, the helix and the path to the surface.  Outputs
 * (device, float64, overwritten): dalign [3 n_layers] (0 for disks), dfield
 * [1].  Per-track partial sums are reduced in a fixed order, so the result
 * is the same on every call. */
int kfx_fit_tracks_backward(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* trk_off,
                            const int32_t* trk_hits, int32_t n_tracks, const kfx_prior* prior,
                            const float* align, float field_scale, const kfx_states* ckpt,
                            const int32_t* status, const float* dchi2, int32_t dchi2_per_track,
                            double* dalign, double* dfield, void* stream);

/* The same gradient for callers that cannot allocate device memory (code
 * under HIP graph capture, tight training loops, harnesses that forbid
 * hipMalloc): identical arguments and results, but the per-block partial
 * rows go to a fixed device array inside the library (8 MiB per GPU, held
 * until the process ends) instead of the context's workspace pool, and the
 * call allocates nothing.  Limit: ceil(n_tracks / 64) * (3 * n_barrel + 1)
 * <= 2^20 float64 (about 1.29M tracks for 17 barrel layers); beyond it the
 * call returns KFX_EOVERFLOW before any work is queued.  Every call on one
 * GPU shares that array: calls that overlap on one GPU (several streams or
 * host threads at once) race; calls ordered on one stream do not.  Every
 * call overwrites the rows it uses before reading them. */
int kfx_fit_tracks_backward_noalloc(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* trk_off,
                                    const int32_t* trk_hits, int32_t n_tracks, const kfx_prior* prior,
                                    const float* align, float field_scale, const kfx_states* ckpt,
                                    const int32_t* status, const float* dchi2, int32_t dchi2_per_track,
                                    double* dalign, double* dfield, void* stream);

/* Keys per event of the hit index that the last kfx_bin_hits or
 * kfx_build_tracks call on this context built (host int64): n_layers *
 * n_eta * n_phi for the counting sort over the batch, one more for the
 * index made one workgroup per event (kfx_build_params.binning).
 * KFX_ESTATE when the context holds no index (none built yet, or the last
 * build was captured into a graph, which owns its index). */
int kfx_index_keys_per_event(kfx_ctx* ctx, int64_t* keys);

/* Timing of kfx_build_tracks with HIP events recorded on the caller's
 * stream, kept for the last n_calls calls (0 turns timing off; at most
 * 4096).  Off by default. */
int kfx_enable_timing(kfx_ctx* ctx, int n_calls);

/* Milliseconds of up to the last n_calls timed builds, oldest first, four
 * floats per call into ms (host): hit binning, the search (the fused
 * kernel, which also writes the outputs, or the per-step kernels of the
 * plain path), building (seed start, search, output; the fused build runs
 * its seed start on a second stream beside the binning), total.  Waits for
 * those events; returns the number of calls written (>= 0) or an error
 * code. */
int kfx_build_times(kfx_ctx* ctx, float* ms, int n_calls);

/* A HIP graph of one kfx_build_tracks call.  kfx_build_graph runs the call
 * once (sizing a workspace that the graph owns), then captures it on a
 * private stream and instantiates the graph; kfx_graph_launch replays it on
 * `stream` with the same device buffers (hits, seeds, seed_event, out),
 * whose contents the caller may change between launches (sizes and
 * parameters are fixed).  The graph holds no memset node: buffers are
 * cleared by kernels.  out->stats is added to on every launch.  Destroy
 * graphs before their context; kfx_graph_destroy waits for the device. */
typedef struct kfx_graph kfx_graph;
int kfx_build_graph(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* seeds, const int32_t* seed_event,
                    int32_t n_seeds, const kfx_build_params* params, kfx_tracks* out, kfx_graph** graph);
int kfx_graph_launch(kfx_graph* graph, void* stream);
void kfx_graph_destroy(kfx_graph* graph);

/* Autotuner of the fused kernel (the paper's Sec. 2 puts the parallel
 * tasks at the level of events, regions and seed bunches; how many seeds a
 * block holds and how windows are shared is a property of the workload).
 * Times kfx_build_tracks with HIP events on `stream` (one warm-up and `reps`
 * timed calls per shape, the minimum kept): first one and two wavefronts
 * per SIMD at the default shape (when waves_per_simd is 0), then from the
 * faster one parameter at a time: scan_tile in {16, 32, 64, 128, 256},
 * block_threads in {64, 128, 256}, blocks in {1, 2, 4, 8} per compute
 * unit, lanes_per_seed 6 (K of 5 or 6) or 12 (K of 9 to 12) and from
 * the smallest power of two >= K up to 16,
 * waves_per_simd in {1, 2}, seeds_per_wave from 2 up to 64 /
 * lanes_per_seed, then scan_tile, block_threads and waves_per_simd once
 * more.  Writes the fastest shape into
 * params (mode becomes KFX_MODE_FUSED) and its time into *best_ms
 * (nullable).  Every shape gives identical results; out holds the last
 * call's, out->stats is restored.  Synchronises the stream.
 *
 * Results are cached per device (its architecture name and compute-unit
 * count) and workload signature (seed, hit and event counts, K, holes,
 * steps, chi2 cut, window inflation, overlap recovery, score ranking,
 * binning): a call with a
 * cached key returns the cached shape and time without building (out is
 * then untouched).  When the environment variable KFX_AUTOTUNE_CACHE names
 * a file, the cache is read from it on first use and every new entry is
 * appended to it (one text line per entry), so later processes reuse it. */
int kfx_autotune_build(kfx_ctx* ctx, const kfx_hits* hits, const int32_t* seeds, const int32_t* seed_event,
                       int32_t n_seeds, kfx_build_params* params, kfx_tracks* out, int32_t reps,
                       float* best_ms, void* stream);

/* Empties the autotuner's in-process cache; the cache file, if one is
 * named, is read again on the next autotuner call. */
void kfx_autotune_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* KFX_H */
