// Strip clustering for gfx950 (MI355X): the three-threshold clustering of
// silicon-strip digis that the paper ports to GPUs for the HLT (Sec. 4):
// seed strips above seed_thr times their noise, clusters of the strips
// above chan_thr times their noise that are adjacent or separated only by a
// few bad strips, kept when the quadrature sum of the ADCs exceeds clus_thr
// times the quadrature sum of the noise and the charge reaches a minimum.
//
// Data-parallel over the digis of a whole batch of events (the paper's
// remedy for single-event GPU runs dominated by overheads): one thread per
// digi decides whether it starts a cluster and, if so, walks the cluster
// and decides whether it is kept; an exclusive scan of the kept flags gives
// every kept cluster its output slot, in (event, module, first strip)
// order; a second pass writes the kept clusters.  Digis are read once per
// pass (coalesced), neighbours through the caches.
#include <hip/hip_runtime.h>

#include "kfx_internal.h"

namespace kfx {

namespace {

__device__ inline int strip_event_of(const int* ev_off, int n_events, int i) {
  int lo = 0, hi = n_events;  // ev_off[lo] <= i < ev_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ev_off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

// candidate (not bad, adc > chan_thr * noise); *seed = adc > seed_thr * noise
__device__ inline bool strip_candidate(const StripArgs& a, int i, bool* seed, int* cal) {
  const int m = a.module[i], s = a.strip[i];
  if (m < 0 || m >= a.n_modules || s < 0 || s >= a.spm) return false;
  const int c = m * a.spm + s;
  if (a.bad[c]) return false;
  const float adc = (float)a.adc[i];
  const float nz = a.noise[c];
  if (!(adc > a.chan_thr * nz)) return false;
  *seed = adc > a.seed_thr * nz;
  *cal = c;
  return true;
}

// consecutive candidates j < i (digi order) of one cluster: same module, at
// most max_gap strips between them, all of them bad
__device__ inline bool strips_linked(const StripArgs& a, int j, int i) {
  const int m = a.module[j];
  if (a.module[i] != m) return false;
  const int sj = a.strip[j], si = a.strip[i];
  if (si <= sj || si - sj - 1 > a.max_gap) return false;
  for (int t = sj + 1; t < si; ++t)
    if (!a.bad[m * a.spm + t]) return false;
  return true;
}

// nearest candidate after digi k within max_gap + 1 digis of the event
__device__ inline int next_candidate(const StripArgs& a, int k, int ev_end, bool* seed, int* cal) {
  const int lim = min(ev_end, k + 2 + a.max_gap);
  for (int j = k + 1; j < lim; ++j)
    if (strip_candidate(a, j, seed, cal)) return j;
  return -1;
}

struct StripCluster {
  int first, last, charge;
  long sq, sa;
  double nsq;
  bool seed;
};

// does candidate i start a cluster?  (no linked candidate before it)
__device__ inline bool strip_head(const StripArgs& a, int i, int ev_start) {
  const int lo = max(ev_start, i - 1 - a.max_gap);
  for (int j = i - 1; j >= lo; --j) {
    bool sd;
    int c;
    if (strip_candidate(a, j, &sd, &c)) return !strips_linked(a, j, i);
  }
  return true;
}

// the cluster that starts at candidate i; true when it is kept
__device__ inline bool strip_walk(const StripArgs& a, int i, bool seed_i, int cal_i, int ev_end, StripCluster& cl) {
  int cur = i;
  bool sd = seed_i;
  int cal = cal_i;
  cl.first = a.strip[i];
  cl.charge = 0;
  cl.sq = 0;
  cl.sa = 0;
  cl.nsq = 0.0;
  cl.seed = false;
  for (;;) {
    const int q = a.adc[cur];
    const int s = a.strip[cur];
    cl.charge += q;
    cl.sq += (long)q * q;
    cl.sa += (long)s * q;
    const double nz = (double)a.noise[cal];
    cl.nsq += nz * nz;
    cl.seed |= sd;
    cl.last = s;
    bool sd2;
    int cal2;
    const int nx = next_candidate(a, cur, ev_end, &sd2, &cal2);
    if (nx < 0 || !strips_linked(a, cur, nx)) break;
    cur = nx, sd = sd2, cal = cal2;
  }
  return cl.seed && (double)cl.sq > a.clus_thr2 * cl.nsq && cl.charge >= a.min_charge;
}

}  // namespace

__global__ void __launch_bounds__(256) k_strip_flags(StripArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    int kept = 0;
    bool sd;
    int cal;
    if (strip_candidate(a, i, &sd, &cal)) {
      const int e = strip_event_of(a.ev_off, a.n_events, i);
      if (strip_head(a, i, a.ev_off[e])) {
        StripCluster cl;
        kept = strip_walk(a, i, sd, cal, a.ev_off[e + 1], cl) ? 1 : 0;
      }
    }
    a.flag[i] = kept;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.flag[a.n] = 0;
}

__global__ void __launch_bounds__(256) k_strip_write(StripArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    if (!a.flag[i]) continue;
    const int p = a.pos[i];
    if (p >= a.capacity) continue;
    bool sd;
    int cal;
    strip_candidate(a, i, &sd, &cal);
    const int e = strip_event_of(a.ev_off, a.n_events, i);
    StripCluster cl;
    strip_walk(a, i, sd, cal, a.ev_off[e + 1], cl);
    a.out_event[p] = e;
    a.out_module[p] = a.module[i];
    a.out_first[p] = cl.first;
    a.out_size[p] = cl.last - cl.first + 1;
    a.out_charge[p] = cl.charge;
    a.out_bary[p] = (float)((double)cl.sa / (double)cl.charge);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_out = a.pos[a.n];
}

void launch_cluster_strips(const StripArgs& a, int* scan_scratch, hipStream_t st) {
  const int nb = (int)std::min<long>(((long)a.n + 255) / 256, 16384);
  hipLaunchKernelGGL(k_strip_flags, dim3(std::max(nb, 1)), dim3(256), 0, st, a);
  exclusive_scan(a.flag, a.n, a.pos, scan_scratch, st);
  hipLaunchKernelGGL(k_strip_write, dim3(std::max(nb, 1)), dim3(256), 0, st, a);
}

}  // namespace kfx
