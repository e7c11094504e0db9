// Strip clustering for gfx950 (MI355X): the three-threshold clustering of
// silicon-strip digis that the paper ports to GPUs for the HLT (Sec. 4):
// seed strips above seed_thr times their noise, clusters of the strips
// above chan_thr times their noise that are adjacent or separated only by a
// few bad strips, kept when the quadrature sum of the ADCs exceeds clus_thr
// times the quadrature sum of the noise and the charge reaches a minimum.
//
// Data-parallel over the digis of a whole batch of events (the paper's
// remedy for single-event GPU runs dominated by overheads).  The first pass
// classifies every digi once (the calibration gathers) into a code byte and
// its noise; in the second one thread per digi decides, from the codes of
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

// code of a digi: bit 0 cluster strip (not bad, adc > chan_thr * noise),
// bit 1 seed (adc > seed_thr * noise); 0 for a digi outside the table
__device__ inline unsigned char strip_code(const StripArgs& a, int i, float* nz_out) {
  const int m = a.module[i], s = a.strip[i];
  *nz_out = 0.0f;
  if (m < 0 || m >= a.n_modules || s < 0 || s >= a.spm) return 0;
  const int c = m * a.spm + s;
  if (a.bad[c]) return 0;
  const float adc = (float)a.adc[i];
  const float nz = a.noise[c];
  *nz_out = nz;
  if (!(adc > a.chan_thr * nz)) return 0;
  return (unsigned char)(1 | ((adc > a.seed_thr * nz) ? 2 : 0));
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

// pass 1: the code and noise of every digi (coalesced writes)
__global__ void __launch_bounds__(256) k_strip_codes(StripArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    float nz;
    a.code[i] = strip_code(a, i, &nz);
    a.nz[i] = nz;
  }
}

// pass 2: a cluster strip with no linked cluster strip before it starts a
// cluster; it walks the cluster (the nearest cluster strip after the
// current one, within max_gap + 1 digis of the event, while linked) and
// flags it when kept, storing its last strip, charge and sum strip * adc
__global__ void __launch_bounds__(256) k_strip_flags(StripArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    int kept = 0;
    const unsigned char ci = a.code[i];
    if (ci & 1) {
      const int e = strip_event_of(a.ev_off, a.n_events, i);
      // clamped to the digis, so that malformed offsets cannot lead a walk
      // out of the arrays
      const int ev_start = max(a.ev_off[e], 0), ev_end = min(a.ev_off[e + 1], a.n);
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
          a.st_last[i] = last;
          a.st_charge[i] = charge;
          a.st_sa[i] = sa;
          a.st_event[i] = e;
        }
      }
    }
    a.flag[i] = kept;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.flag[a.n] = 0;
}

// pass 3 (after the scan of the flags): the kept clusters in order
__global__ void __launch_bounds__(256) k_strip_write(StripArgs a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += gridDim.x * blockDim.x) {
    if (!a.flag[i]) continue;
    const int p = a.pos[i];
    if (p >= a.capacity) continue;
    const int first = a.strip[i];
    const int charge = a.st_charge[i];
    a.out_event[p] = a.st_event[i];
    a.out_module[p] = a.module[i];
    a.out_first[p] = first;
    a.out_size[p] = a.st_last[i] - first + 1;
    a.out_charge[p] = charge;
    a.out_bary[p] = (float)((double)a.st_sa[i] / (double)charge);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_out = a.pos[a.n];
}

void launch_cluster_strips(const StripArgs& a, int* scan_scratch, hipStream_t st) {
  const int nb = std::max(1, (int)std::min<long>(((long)a.n + 255) / 256, 16384));
  hipLaunchKernelGGL(k_strip_codes, dim3(nb), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_strip_flags, dim3(nb), dim3(256), 0, st, a);
  exclusive_scan(a.flag, a.n, a.pos, scan_scratch, st);
  hipLaunchKernelGGL(k_strip_write, dim3(nb), dim3(256), 0, st, a);
}

}  // namespace kfx
