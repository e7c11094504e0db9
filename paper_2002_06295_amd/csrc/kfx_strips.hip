// Strip clustering for gfx950 (MI355X): the three-threshold clustering of
// silicon-strip digis that the paper ports to GPUs for the HLT (Sec. 4):
// seed strips above seed_thr times their noise, clusters of the strips
// above chan_thr times their noise that are adjacent or separated only by a
// few bad strips, kept when the quadrature sum of the ADCs exceeds clus_thr
// times the quadrature sum of the noise and the charge reaches a minimum.
//
// Data-parallel over the digis of a whole batch of events (the paper's
// remedy for single-event GPU runs dominated by overheads).  The first pass
// classifies every digi once (the calibration gathers, module-major across
// the events) into a code byte and its noise; in the second one thread per digi decides, from the codes of
// its neighbours, whether it starts a cluster, and if so walks the cluster
// and keeps its sums when the cluster passes; an exclusive scan of the
// kept flags gives every kept cluster its output slot, in (event, module,
// first strip) order; the last pass writes them.  Digis and codes are read
// coalesced, neighbours through the caches.
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

// consecutive cluster strips j < i (digi order) of one cluster: same module,
// at most max_gap strips between them, all of them bad
__device__ inline bool strips_linked(const StripArgs& a, int j, int i) {
  const int m = a.module[j];
  if (a.module[i] != m) return false;
  const int sj = a.strip[j], si = a.strip[i];
  if (si <= sj || si - sj - 1 > a.max_gap) return false;
  for (int t = sj + 1; t < si; ++t)
    if (!a.bad[m * a.spm + t]) return false;
  return true;
}

}  // namespace

// pass 1 runs module-major: block c owns modules [c * kStripChunk,
// (c + 1) * kStripChunk) and classifies their digis in every event, so that
// the chunk's calibration (noise and bad flags of its strips, ~60 KB) is
// fetched once and reused from the cache by all events, instead of every
// event gathering its own sectors of the table.  The events go in rounds
// of kStripEvents, whose gathers are all in flight together: the chunk's
// calibration is then read while it is in L2, once per round (in rounds of
// four, the tables of the ~120 chunks in flight on an XCD outgrew its L2
// between rounds and were fetched again for every round).
// bnd[e * (C + 1) + c] is the first digi of event e in chunk c (chunk 0
// starts at the event's first digi and chunk C is its end, so digis
// outside the table are classified too).
constexpr int kStripChunk = 16;
constexpr int kStripEvents = 16;

__global__ void __launch_bounds__(256) k_strip_bounds(StripArgs a, int C) {
  const long n_b = (long)a.n_events * (C + 1);
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n_b; t += (long)gridDim.x * blockDim.x) {
    const int e = (int)(t / (C + 1)), c = (int)(t - (long)e * (C + 1));
    const int lo = min(max(a.ev_off[e], 0), a.n), hi = min(max(a.ev_off[e + 1], lo), a.n);
    int b;
    if (c == 0) {
      b = lo;
    } else if (c == C) {
      b = hi;
    } else {
      // first digi of the event whose module is >= c * kStripChunk
      const int m = c * kStripChunk;
      int l = lo, h = hi;
      while (l < h) {
        const int mid = (l + h) >> 1;
        if (a.module[mid] < m) l = mid + 1; else h = mid;
      }
      b = l;
    }
    a.bnd[t] = b;
  }
}

// Code of a digi: bit 0 cluster strip (in the table, not bad, adc >
// chan_thr * noise), bit 1 seed (adc > seed_thr * noise); its noise (0 for
// a bad strip or one outside the table).
__global__ void __launch_bounds__(256) k_strip_codes(StripArgs a, int C) {
  const int c = blockIdx.x;
  for (int e0 = 0; e0 < a.n_events; e0 += kStripEvents) {
    int lo[kStripEvents], cnt[kStripEvents];
    int span = 0;
#pragma unroll
    for (int u = 0; u < kStripEvents; ++u) {
      const int e = e0 + u;
      lo[u] = 0;
      cnt[u] = 0;
      if (e < a.n_events) {
        lo[u] = a.bnd[(long)e * (C + 1) + c];
        cnt[u] = max(a.bnd[(long)e * (C + 1) + c + 1] - lo[u], 0);
      }
      span = max(span, cnt[u]);
    }
    for (int k = threadIdx.x; k < span; k += blockDim.x) {
      int cal[kStripEvents], qq[kStripEvents];
#pragma unroll
      for (int u = 0; u < kStripEvents; ++u) {
        const bool in = k < cnt[u];
        const int i = lo[u] + k;
        const int m = in ? a.module[i] : -1;
        const int st = in ? a.strip[i] : 0;
        qq[u] = in ? (int)a.adc[i] : 0;
        cal[u] = (m >= 0 && m < a.n_modules && st >= 0 && st < a.spm) ? m * a.spm + st : -1;
      }
      float nzv[kStripEvents];
      bool bd[kStripEvents];
#pragma unroll
      for (int u = 0; u < kStripEvents; ++u) {
        nzv[u] = cal[u] >= 0 ? a.noise[cal[u]] : 0.0f;
        bd[u] = cal[u] >= 0 ? a.bad[cal[u]] != 0 : true;
      }
#pragma unroll
      for (int u = 0; u < kStripEvents; ++u) {
        if (k >= cnt[u]) continue;
        unsigned char cd = 0;
        float nzo = 0.0f;
        if (cal[u] >= 0 && !bd[u]) {
          nzo = nzv[u];
          const float adc = (float)qq[u];
          if (adc > a.chan_thr * nzv[u]) cd = (unsigned char)(1 | ((adc > a.seed_thr * nzv[u]) ? 2 : 0));
        }
        a.code[lo[u] + k] = cd;
        a.nz[lo[u] + k] = nzo;
      }
    }
  }
}

// pass 2: a cluster strip with no linked cluster strip before it starts a
// cluster; it walks the cluster (the nearest cluster strip after the
// current one, within max_gap + 1 digis of the event, while linked) and
// flags it when kept, storing its last strip, charge and sum strip * adc
__global__ void __launch_bounds__(256) k_strip_flags(StripArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    int kept = 0;
    // a digi outside every event's range (before the first event, after
    // the last, or skipped by offsets that go backwards) was not
    // classified: its code byte is not read
    const int e = strip_event_of(a.ev_off, a.n_events, i);
    // clamped to the digis, so that malformed offsets cannot lead a walk
    // out of the arrays
    const int ev_start = max(a.ev_off[e], 0), ev_end = min(a.ev_off[e + 1], a.n);
    const bool in_event = i >= ev_start && i < ev_end;
    const unsigned char ci = in_event ? a.code[i] : 0;
    if (ci & 1) {
      bool head = true;
      for (int j = i - 1, lo = max(ev_start, i - 1 - a.max_gap); j >= lo; --j)
        if (a.code[j] & 1) {
          head = !strips_linked(a, j, i);
          break;
        }
      if (head) {
        int cur = i, charge = 0, last = 0;
        long sq = 0, sa = 0;
        double nsq = 0.0;
        bool seed = false;
        for (;;) {
          const int q = a.adc[cur];
          const int st = a.strip[cur];
          charge += q;
          sq += (long)q * q;
          sa += (long)st * q;
          const double nzd = (double)a.nz[cur];
          nsq += nzd * nzd;
          seed |= (a.code[cur] & 2) != 0;
          last = st;
          int nx = -1;
          for (int j = cur + 1, lim = min(ev_end, cur + 2 + a.max_gap); j < lim; ++j)
            if (a.code[j] & 1) {
              nx = j;
              break;
            }
          if (nx < 0 || !strips_linked(a, cur, nx)) break;
          cur = nx;
        }
        if (seed && (double)sq > a.clus_thr2 * nsq && charge >= a.min_charge) {
          kept = 1;
          StripRec r;
          r.sa = sa;
          r.last = last;
          r.charge = charge;
          r.event = e;
          r.module = a.module[i];
          r.first = a.strip[i];
          r.pad = 0;
          a.rec[i] = r;
        }
      }
    }
    a.flag[i] = kept;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.flag[a.n] = 0;
}

// pass 3 (after the scan of the flags): the kept clusters in order; digi i
// is kept when the scan steps after it (pos[i + 1] > pos[i]: two coalesced
// reads instead of the flags and a scattered read of the kept ones' slots)
__global__ void __launch_bounds__(256) k_strip_write(StripArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    const int p = a.pos[i];
    if (a.pos[i + 1] == p) continue;
    if (p >= a.capacity) continue;
    const StripRec r = a.rec[i];
    a.out_event[p] = r.event;
    a.out_module[p] = r.module;
    a.out_first[p] = r.first;
    a.out_size[p] = r.last - r.first + 1;
    a.out_charge[p] = r.charge;
    a.out_bary[p] = (float)((double)r.sa / (double)r.charge);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_out = a.pos[a.n];
}

int strip_chunks(int n_modules) { return (n_modules + kStripChunk - 1) / kStripChunk; }

void launch_cluster_strips(const StripArgs& a, int* scan_scratch, hipStream_t st) {
  const int nb = std::max(1, (int)std::min<long>(((long)a.n + 255) / 256, 16384));
  const int C = strip_chunks(a.n_modules);
  const long n_b = (long)a.n_events * (C + 1);
  hipLaunchKernelGGL(k_strip_bounds, dim3((unsigned)std::min<long>((n_b + 255) / 256, 16384)), dim3(256), 0, st, a, C);
  hipLaunchKernelGGL(k_strip_codes, dim3((unsigned)C), dim3(256), 0, st, a, C);
  hipLaunchKernelGGL(k_strip_flags, dim3(nb), dim3(256), 0, st, a);
  exclusive_scan(a.flag, a.n, a.pos, scan_scratch, st);
  hipLaunchKernelGGL(k_strip_write, dim3(nb), dim3(256), 0, st, a);
}

}  // namespace kfx
