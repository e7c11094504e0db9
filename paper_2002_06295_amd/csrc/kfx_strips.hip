// Strip clustering for gfx950 (MI355X): the three-threshold clustering of
// silicon-strip digis that the paper ports to GPUs for the HLT (Sec. 4):
// seed strips above seed_thr times their noise, clusters of the strips
// above chan_thr times their noise that are adjacent or separated only by a
// few bad strips, kept when the quadrature sum of the ADCs exceeds clus_thr
// times the quadrature sum of the noise and the charge reaches a minimum.
//
// Data-parallel over the digis of a whole batch of events (the paper's
// remedy for single-event GPU runs dominated by overheads), in one pass
// over the digis: a block per chunk of modules holds the chunk's
// calibration in LDS and takes the chunk's digis event by event; one
// thread per digi decides whether it starts a cluster, and if so walks the
// cluster and keeps its sums when the cluster passes; the kept clusters of
// each (event, chunk) are compacted in the block.  An exclusive scan of the
// per-(event, chunk) counts gives every kept cluster its output slot, in
// (event, module, first strip) order, and a last pass moves them there.
#include <hip/hip_runtime.h>

#include "kfx_internal.h"

namespace kfx {

namespace {

constexpr int kStripThreads = 512;  // 8 wavefronts

// LDS of the strip clustering block: the chunk's calibration (4-byte noise
// and 1-byte bad flag per strip), then one window per wavefront (module,
// strip and noise 4 bytes each, ADC 2, code 1 per digi); 16-byte aligned
__host__ __device__ inline size_t strip_cal_lds_al(int chunk, int spm) {
  return ((size_t)chunk * spm * 5 + 15) & ~(size_t)15;
}
__host__ __device__ inline size_t strip_win_lds(int wn) { return ((size_t)wn * 15 + 15) & ~(size_t)15; }

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline bool in_table(const StripArgs& a, int m, int s) {
  return m >= 0 && m < a.n_modules && s >= 0 && s < a.spm;
}

// The calibration a block works with: its chunk's modules [m0, m0 + nm)
// staged in LDS (nm = 0 when the table is not staged), any other module
// read from HBM.
struct Calib {
  const float* nz;
  const unsigned char* bd;
  int m0, nm;
  __device__ float noise(const StripArgs& a, int m, int s) const {
    return (m >= m0 && m < m0 + nm) ? nz[(m - m0) * a.spm + s] : a.noise[(long)m * a.spm + s];
  }
  __device__ bool bad(const StripArgs& a, int m, int s) const {
    return ((m >= m0 && m < m0 + nm) ? bd[(m - m0) * a.spm + s] : a.bad[(long)m * a.spm + s]) != 0;
  }
};

// Code of a digi (module m, strip st, ADC q): bit 0 cluster strip (in the
// table, not bad, adc > chan_thr * noise), bit 1 seed (adc > seed_thr *
// noise); nzo its noise.
__device__ inline unsigned int code_from(const StripArgs& a, const Calib& K, int m, int st, int q, float& nzo) {
  nzo = 0.0f;
  if (!in_table(a, m, st) || K.bad(a, m, st)) return 0u;
  const float nzv = K.noise(a, m, st);
  nzo = nzv;
  const float adc = (float)q;
  if (!(adc > a.chan_thr * nzv)) return 0u;
  return 1u | ((adc > a.seed_thr * nzv) ? 2u : 0u);
}

// consecutive cluster strips j < i (digi order) of one cluster, given
// their modules and strips: same module, at most max_gap strips between
// them, all of them bad
__device__ inline bool strips_linked(const StripArgs& a, const Calib& K, int mj, int sj, int mi, int si) {
  if (mi != mj) return false;
  if (si <= sj || si - sj - 1 > a.max_gap) return false;
  for (int t = sj + 1; t < si; ++t)
    if (!K.bad(a, mj, t)) return false;
  return true;
}

// A wavefront's window of digis [w0, w1) in LDS: module, strip, ADC, code
// and noise of each; a digi outside it is read from HBM.  The window's
// digis of modules outside the block's chunk (the digis around the chunk's
// edges) are not classified when the window is filled, and a digi read
// from HBM is not classified when read (code kUnclassified): the cluster
// searches below look at such a digi's code only when a digi of the
// searched module lies beyond it, which in sorted input never happens, and
// then classify it (resolve).  `sorted`: the window's digis are in
// ascending module order.
constexpr unsigned int kUnclassified = 4;

struct Win {
  int w0, w1;
  bool sorted;
  int* m;
  int* s;
  float* nz;
  unsigned short* q;
  unsigned char* c;
};

struct Digi {
  int m, s, q;
  unsigned int code;
  float nz;
};

__device__ inline Digi digi_at(const StripArgs& a, const Win& w, int j) {
  Digi d;
  if (j >= w.w0 && j < w.w1) {
    const int k = j - w.w0;
    d.m = w.m[k];
    d.s = w.s[k];
    d.q = w.q[k];
    d.code = w.c[k];
    d.nz = w.nz[k];
  } else {
    d.m = a.module[j];
    d.s = a.strip[j];
    d.q = a.adc[j];
    d.code = kUnclassified;
    d.nz = 0.0f;
  }
  return d;
}

__device__ inline void resolve(const StripArgs& a, const Calib& K, Digi& d) {
  if (d.code == kUnclassified) d.code = code_from(a, K, d.m, d.s, d.q, d.nz);
}

// The chunk's calibration (ncal strips from module m0 on) into LDS: 16-byte
// loads, four per thread in flight, where both tables' ranges are 16-byte
// aligned and whole (the common case: strips_per_module a multiple of 16),
// else one strip at a time.
__device__ inline void stage_calibration(const StripArgs& a, int m0, int ncal, float* nz_l, unsigned char* bd_l,
                                         int tid) {
  const float* nz = a.noise + (long)m0 * a.spm;
  const unsigned char* bd = a.bad + (long)m0 * a.spm;
  const bool al = ((reinterpret_cast<uintptr_t>(nz) | reinterpret_cast<uintptr_t>(bd)) & 15) == 0 &&
                  ((size_t)a.chunk * a.spm * 4 & 15) == 0 && (ncal & 15) == 0;  // bd_l's offset too
  if (al) {
    const float4* nz4 = reinterpret_cast<const float4*>(nz);
    const uint4* bd16 = reinterpret_cast<const uint4*>(bd);
    float4* nzl4 = reinterpret_cast<float4*>(nz_l);
    uint4* bdl16 = reinterpret_cast<uint4*>(bd_l);
    const int n4 = ncal >> 2, n16 = ncal >> 4;
    // iteration i: noise words tid + T (4 i + u), u < 4, and bad-flag word
    // tid + T i (a quarter as many; T threads); indices clamped to the last word
    // (which is then copied by several threads, with the same value) so
    // that no load waits behind a branch
    for (int k = tid; k < n4; k += 4 * kStripThreads) {
      const int kb = min(tid + ((k - tid) >> 2), n16 - 1);
      int ix[4];
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ix[u] = min(k + u * kStripThreads, n4 - 1);
        v[u] = nz4[ix[u]];
      }
      const uint4 w = bd16[kb];
#pragma unroll
      for (int u = 0; u < 4; ++u) nzl4[ix[u]] = v[u];
      bdl16[kb] = w;
    }
  } else {
    for (int k = tid; k < ncal; k += kStripThreads) {
      nz_l[k] = nz[k];
      bd_l[k] = bd[k];
    }
  }
}

// a digi of module m among the digis [j0, j1)
__device__ inline bool module_in(const StripArgs& a, const Win& w, int m, int j0, int j1) {
  for (int t = j0; t < j1; ++t)
    if (((t >= w.w0 && t < w.w1) ? w.m[t - w.w0] : a.module[t]) == m) return true;
  return false;
}

}  // namespace

// The digis of event e in chunk c (a chunk: `chunk` consecutive modules)
// are [bnd[e * (C + 1) + c], bnd[e * (C + 1) + c + 1]): chunk 0 starts at the
// event's first digi and chunk C - 1 ends at its last, so digis outside
// the table are covered too.  Offsets are clamped to the digis.
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
      // first digi of the event whose module is >= c * chunk
      const int m = c * a.chunk;
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

// One pass over the digis, module-major: block c stages the calibration of
// its chunk (noise and bad flags of `chunk` modules, 30 KB for 8 modules of
// 768 strips) in LDS once, then each of its wavefronts takes the chunk's
// digis of one event after another (wavefront w: events w, w + 8, ...), 64
// at a time: the 64 digis and max_gap + 1 on each side are read and
// classified once into an LDS window, where the neighbour tests and walks
// find them (a walk that leaves the window reads HBM).  A
// cluster strip whose nearest cluster strip before it (within max_gap + 1
// digis of the event: a linked one cannot be farther) is not linked to it
// starts a cluster; its thread walks the cluster forward the same way,
// summing charge, sum adc^2, sum strip * adc and sum noise^2 in strip order.
// The kept clusters of (event, chunk) are compacted by a ballot and stored
// from the chunk's first digi on (never more clusters than digis), in digi
// order, with their count; k_strip_emit then moves them to their place in
// the output.  The calibration is read once and the digis once
// (neighbours through the caches; the window's digis of the neighbouring
// chunks are not classified, as the Win note says); no per-digi codes or
// flags go through HBM.
__global__ void __launch_bounds__(kStripThreads) k_strip_cluster(StripArgs a, int C) {
  extern __shared__ __align__(16) unsigned char cal_lds[];
  // neighbouring chunks on one XCD: the digis at their common edge are
  // read through one L2
  const int c = xcd_block(C), tid = threadIdx.x, lane = tid & 63;
  if (c < 0) return;  // whole block
  Calib K;
  K.m0 = c * a.chunk;
  K.nm = a.stage ? max(0, min(a.chunk, a.n_modules - K.m0)) : 0;
  const int chunk_lo = K.m0, chunk_hi = K.m0 + a.chunk;
  float* nz_l = reinterpret_cast<float*>(cal_lds);
  unsigned char* bd_l = cal_lds + (size_t)a.chunk * a.spm * 4;
  K.nz = nz_l;
  K.bd = bd_l;
  stage_calibration(a, K.m0, K.nm * a.spm, nz_l, bd_l, tid);
  // this wavefront's window: 64 digis and max_gap + 1 on each side
  const int halo = a.max_gap + 1, wn = 64 + 2 * halo;
  unsigned char* wbase = cal_lds + strip_cal_lds_al(a.stage ? a.chunk : 0, a.spm) + (size_t)(tid >> 6) * strip_win_lds(wn);
  Win W;
  W.m = reinterpret_cast<int*>(wbase);
  W.s = W.m + wn;
  W.nz = reinterpret_cast<float*>(W.s + wn);
  W.q = reinterpret_cast<unsigned short*>(W.nz + wn);
  W.c = reinterpret_cast<unsigned char*>(W.q + wn);
  __syncthreads();
  for (int e = tid >> 6; e < a.n_events; e += kStripThreads / 64) {
    const int ev_start = min(max(a.ev_off[e], 0), a.n), ev_end = min(max(a.ev_off[e + 1], ev_start), a.n);
    const int lo = a.bnd[(long)e * (C + 1) + c];
    const int hi = max(a.bnd[(long)e * (C + 1) + c + 1], lo);
    int running = 0;
    for (int base = lo; base < hi; base += 64) {
      // the window's digis, classified once, in LDS
      W.w0 = max(ev_start, base - halo);
      W.w1 = min(ev_end, base + 64 + halo);
      auto put = [&](int k, int m, int st, int q) {
        float nzj = 0.0f;
        W.c[k] = (m >= chunk_lo && m < chunk_hi) ? (unsigned char)code_from(a, K, m, st, q, nzj)
                                                 : (unsigned char)kUnclassified;
        W.m[k] = m;
        W.s[k] = st;
        W.q[k] = (unsigned short)q;
        W.nz[k] = nzj;
      };
      // two digis a lane at a time, their loads together (the second index
      // clamped to the window's last digi, written then twice, alike)
      for (int j = W.w0 + lane; j < W.w1; j += 128) {
        const int j2 = min(j + 64, W.w1 - 1);
        const int m = a.module[j], st = a.strip[j], q = a.adc[j];
        const int m2 = a.module[j2], st2 = a.strip[j2], q2 = a.adc[j2];
        put(j - W.w0, m, st, q);
        put(j2 - W.w0, m2, st2, q2);
      }
      wave_sync();
      {
        bool up = true;
        for (int k = lane; k + 1 < W.w1 - W.w0; k += 64) up &= W.m[k] <= W.m[k + 1];
        W.sorted = __ballot(!up) == 0;
      }
      const int i = base + lane;
      int kept = 0;
      StripRec r;
      Digi di = Digi{0, 0, 0, 0u, 0.0f};
      if (i < hi) {
        di = digi_at(a, W, i);
        resolve(a, K, di);
      }
      if (di.code & 1u) {
        bool head = true;
        for (int j = i - 1, jl = max(ev_start, i - 1 - a.max_gap); j >= jl; --j) {
          Digi dj = digi_at(a, W, j);
          // past a digi of another module, only a digi of di.m farther back
          // could still be linked to di; without one, di heads a cluster
          // whatever the codes in between (in a sorted window, [jl, j) lies
          // in it and holds none)
          if (dj.m != di.m && (W.sorted || !module_in(a, W, di.m, jl, j))) break;
          resolve(a, K, dj);
          if (dj.code & 1u) {
            head = !strips_linked(a, K, dj.m, dj.s, di.m, di.s);
            break;
          }
        }
        if (head) {
          int cur = i, charge = 0, last = 0;
          Digi dc = di;
          long sq = 0, sa = 0;
          double nsq = 0.0;
          bool seed = false;
          for (;;) {
            charge += dc.q;
            sq += (long)dc.q * dc.q;
            sa += (long)dc.s * dc.q;
            const double nzd = (double)dc.nz;
            nsq += nzd * nzd;
            seed |= (dc.code & 2u) != 0;
            last = dc.s;
            int nx = -1;
            Digi dn = dc;
            for (int j = cur + 1, lim = min(ev_end, cur + 2 + a.max_gap); j < lim; ++j) {
              Digi dj = digi_at(a, W, j);
              // the same: without a digi of dc.m from j on, the cluster ends
              if (dj.m != dc.m && ((W.sorted && lim <= W.w1) || !module_in(a, W, dc.m, j + 1, lim))) break;
              resolve(a, K, dj);
              if (dj.code & 1u) {
                nx = j;
                dn = dj;
                break;
              }
            }
            if (nx < 0 || !strips_linked(a, K, dc.m, dc.s, dn.m, dn.s)) break;
            cur = nx;
            dc = dn;
          }
          if (seed && (double)sq > a.clus_thr2 * nsq && charge >= a.min_charge) {
            kept = 1;
            r.sa = sa;
            r.last = last;
            r.charge = charge;
            r.event = e;
            r.module = di.m;
            r.first = di.s;
            r.pad = 0;
          }
        }
      }
      const unsigned long long km = __ballot(kept);
      if (kept) a.rec[lo + running + __popcll(km & ((1ull << lane) - 1ull))] = r;
      running += __popcll(km);
      wave_sync();  // the window is refilled for the next 64 digis
    }
    if (lane == 0) a.cnt[(long)e * C + c] = running;
  }
}

// The kept clusters to their output slots (offsets: the exclusive scan of
// the per-(event, chunk) counts, event-major): one wavefront per (event,
// chunk), coalesced reads of its records and coalesced writes.
__global__ void __launch_bounds__(256) k_strip_emit(StripArgs a, int C) {
  const long nw = (long)a.n_events * C;
  const int lane = threadIdx.x & 63;
  const long step = ((long)gridDim.x * blockDim.x) >> 6;
  for (long w = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6; w < nw; w += step) {
    const int e = (int)(w / C), c = (int)(w - (long)e * C);
    const int lo = a.bnd[(long)e * (C + 1) + c];
    const int k0 = a.cnt_off[w], cnt = a.cnt[w];
    for (int k = lane; k < cnt; k += 64) {
      const int p = k0 + k;
      if (p >= a.capacity) break;
      const StripRec r = a.rec[lo + k];
      a.out_event[p] = r.event;
      a.out_module[p] = r.module;
      a.out_first[p] = r.first;
      a.out_size[p] = r.last - r.first + 1;
      a.out_charge[p] = r.charge;
      a.out_bary[p] = (float)((double)r.sa / (double)r.charge);
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.n_out = a.cnt_off[nw];
}

int strip_chunks(int n_modules, int chunk) { return (n_modules + chunk - 1) / chunk; }

size_t strip_cal_lds(int chunk, int spm) { return (size_t)chunk * spm * 5; }

size_t strip_cluster_lds(int chunk, int spm, int stage, int max_gap) {
  return strip_cal_lds_al(stage ? chunk : 0, spm) + (kStripThreads / 64) * strip_win_lds(64 + 2 * (max_gap + 1));
}

void launch_cluster_strips(const StripArgs& a, int* scan_scratch, hipStream_t st) {
  const int C = strip_chunks(a.n_modules, a.chunk);
  const long n_b = (long)a.n_events * (C + 1);
  hipLaunchKernelGGL(k_strip_bounds, dim3((unsigned)std::min<long>((n_b + 255) / 256, 16384)), dim3(256), 0, st, a, C);
  hipLaunchKernelGGL(k_strip_cluster, dim3((unsigned)xcd_grid(C)), dim3(kStripThreads),
                     strip_cluster_lds(a.chunk, a.spm, a.stage, a.max_gap), st, a, C);
  const long nw = (long)a.n_events * C;
  exclusive_scan(a.cnt, nw, a.cnt_off, scan_scratch, st);
  const long nb = std::max<long>(1, std::min<long>((nw * 64 + 255) / 256, 16384));
  hipLaunchKernelGGL(k_strip_emit, dim3((unsigned)nb), dim3(256), 0, st, a, C);
}

}  // namespace kfx
