// HIP kernels for gfx950 (MI355X): hit binning, seed states, the plain
// per-step building path, the fused persistent building kernel, the Kalman
// fit and its adjoint.  Launch wrappers at the bottom are called by the C
// ABI (kfx_api.hip).
//
// Paper: arXiv 2002.06295, Sec. 1-3 (Kalman-filter track building and
// fitting over a lightweight barrel/disk geometry, at most K candidates
// per seed kept at each layer).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>

#include "kfx_build.h"
#include "kfx_internal.h"

namespace kfx {

// ---------------------------------------------------------------- utility

__global__ void __launch_bounds__(256) k_fill_i32(int* p, long n, int v) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = v;
}
// the same with 16-byte stores (p 16-byte aligned), the last n % 4 by the
// first threads
__global__ void __launch_bounds__(256) k_fill_i32x4(int* p, long n, int v) {
  const long n4 = n >> 2;
  int4* q = reinterpret_cast<int4*>(p);
  const int4 v4 = make_int4(v, v, v, v);
  const long stride = (long)gridDim.x * blockDim.x;
  const long i0 = blockIdx.x * (long)blockDim.x + threadIdx.x;
  for (long i = i0; i < n4; i += stride) q[i] = v4;
  if (i0 < (n & 3)) p[(n4 << 2) + i0] = v;
}

// Exclusive scan of int32 in three passes: block sums, scan of the sums,
// block-local scan plus offset.  Each block covers kScanTile elements.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

template <int NT = kScanThreads>
__device__ inline int block_exclusive_scan(int v, int* lds, int& total) {
  // wave-level inclusive scan (64 lanes), then across the NT / 64 waves
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds[wid] = x;
  __syncthreads();
  int base = 0, tot = 0;
  for (int w = 0; w < NT / 64; ++w) {
    if (w < wid) base += lds[w];
    tot += lds[w];
  }
  __syncthreads();
  total = tot;
  return base + x - v;
}

__global__ void __launch_bounds__(256) k_scan_reduce(const int* in, long n, int* block_sums) {
  __shared__ int lds[kScanThreads / 64];
  const long base = (long)blockIdx.x * kScanTile;
  int s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const long idx = base + (long)i * kScanThreads + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  int tot;
  block_exclusive_scan(s, lds, tot);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(256) k_scan_sums(int* sums, int nb) {
  // single block: sequential over chunks of kScanThreads
  __shared__ int lds[kScanThreads / 64];
  int carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int i = b0 + threadIdx.x;
    const int v = i < nb ? sums[i] : 0;
    int tot;
    const int ex = block_exclusive_scan(v, lds, tot);
    if (i < nb) sums[i] = carry + ex;
    carry += tot;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_scan_apply(const int* in, long n, const int* block_offsets, int* out) {
  __shared__ int lds[kScanThreads / 64];
  // thread t owns the contiguous run [t*items, (t+1)*items) of the tile
  const long base = (long)blockIdx.x * kScanTile + (long)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_exclusive_scan(s, lds, tot) + block_offsets[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

// The apply pass for few blocks: each block adds up the totals of the
// blocks before it itself (no separate pass over the totals).
constexpr int kScanFewBlocks = 64;
__global__ void __launch_bounds__(256) k_scan_apply_few(const int* in, long n, const int* block_sums, int* out) {
  __shared__ int lds[kScanThreads / 64];
  __shared__ int base_sh;
  if (threadIdx.x < 64) {
    int v = threadIdx.x < blockIdx.x ? block_sums[threadIdx.x] : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) base_sh = v;
  }
  __syncthreads();
  const long base = (long)blockIdx.x * kScanTile + (long)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0;
    s += v[i];
  }
  int tot;
  int ex = block_exclusive_scan(s, lds, tot) + base_sh;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = ex;
    ex += v[i];
  }
}

// exclusive scan of n values; out has n + 1 entries (out[n] = total)
void exclusive_scan(const int* in, long n, int* out, int* scratch, hipStream_t st) {
  const long nb = (n + 1 + kScanTile - 1) / kScanTile;
  if (nb <= kScanFewBlocks) {
    hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, st, in, n, scratch);
    hipLaunchKernelGGL(k_scan_apply_few, dim3(nb), dim3(kScanThreads), 0, st, in, n + 1, scratch, out);
    return;
  }
  // treat in[n] as 0 by scanning n + 1 values where the last is read as 0:
  // simplest is to scan n values and compute the total from the sums.
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanThreads), 0, st, in, n, scratch);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, st, scratch, (int)nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanThreads), 0, st, in, n + 1, scratch, out);
}

// ------------------------------------------------------------- binning (a1)
__device__ inline int event_of(const int* ev_off, int n_events, int hit) {
  int lo = 0, hi = n_events;  // ev_off[lo] <= hit < ev_off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (ev_off[mid] <= hit) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_bin_keys(const Geometry* __restrict__ G, HitsView H, long ev_stride,
                                                  int* key_out, int* bin_out, int* counts, int* rank) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H.n_hits) return;
  const int l = H.layer[i];
  const int nb = G->n_eta * G->n_phi;
  int bin = -1;
  long key = -1;
  if (l >= 0 && l < G->n_layers) bin = hit_bin_fast(*G, l, H.x[i], H.y[i], H.z[i]);
  if (bin >= 0) {
    const int e = event_of(H.ev_off, H.n_events, i);
    key = (long)e * ev_stride + (long)l * nb + bin;
    // the hit's place among its bin's hits (arrival order; the per-bin sort
    // restores ascending hit index)
    rank[i] = atomicAdd(counts + key, 1);
  }
  key_out[i] = (int)key;
  if (bin_out) bin_out[i] = bin;
}

__global__ void __launch_bounds__(256) k_bin_scatter(HitsView H, const int* key, const int* off, const int* rank, int* perm,
                                                     float4* sorted) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H.n_hits) return;
  const int k = key[i];
  if (k < 0) return;
  const int p = off[k] + rank[i];
  if (perm) perm[p] = i;
  if (sorted) {
    // unsorted bins: the hit goes to its place at once
    float w;
    __builtin_memcpy(&w, &i, 4);
    sorted[p] = make_float4(H.x[i], H.y[i], H.z[i], w);
  }
}

// bins hold a handful of hits: insertion sort by hit index gives the same
// order as a stable sort, whatever order the atomics produced
__global__ void __launch_bounds__(256) k_bin_sort(const int* off, long n_keys, int* perm) {
  const long k = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (k >= n_keys) return;
  const int a = off[k], b = off[k + 1];
  for (int i = a + 1; i < b; ++i) {
    const int v = perm[i];
    int j = i - 1;
    while (j >= a && perm[j] > v) {
      perm[j + 1] = perm[j];
      --j;
    }
    perm[j + 1] = v;
  }
}

// only the first off[n_keys] entries of perm are filled (hits with a layer
// id outside the geometry are not indexed)
__global__ void __launch_bounds__(256) k_bin_gather(HitsView H, const int* perm, const int* n_valid, float4* sorted) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= *n_valid) return;
  const int h = perm[p];
  float w;
  __builtin_memcpy(&w, &h, 4);
  sorted[p] = make_float4(H.x[h], H.y[h], H.z[h], w);
}

// ---- binning of a batch of events: one workgroup per event ---------------
// With many events, each workgroup takes one event: its hits are counted
// per (layer, bin) in LDS, the counts are scanned there, and every hit gets
// its place in the event's own part [ev_off[e], ev_off[e+1]) of the sorted
// array (offsets clamped to the hit count).  No global atomics and no scan
// over the whole key space are needed.  The index then has n_layers *
// n_bins + 1 keys per event: the last holds no bin, and its range is the
// tail of the event's part that its hits without a bin leave unused.  The
// counters are 8 bits, four to a word; a bin that reaches 255 hits (far
// more than a bin of these geometries holds) makes the workgroup count the
// event again with global atomics, which have no such limit.  The scan
// also keeps the offset of every group of 8 keys in LDS, so that a hit's
// place is found there (the group's offset plus the counts of the keys
// before it in the group) rather than by a read of the offsets in HBM.  The
// hits are then moved by k_bin_place, with the blocks over the hits dealt to the
// XCDs in contiguous ranges: the 16-byte writes of an XCD then land in the
// few events it is placing at the time, whose part of the sorted array its
// L2 holds until the lines are whole (moved by the workgroup of each event,
// the writes of the 32 events in flight on an XCD outgrew its L2 and left
// as partial lines: three quarters of the binning time).
constexpr int kBinEvThreads = 1024;
constexpr int kBinEvBatch = 4;  // hits per thread in flight in the passes over the hits
constexpr unsigned int kNoBin = 0xffffffffu;

// packed: on return, the hit's place in the sorted array (-1: none; hits
// outside every event's range keep what the caller filled in)
__global__ void __launch_bounds__(kBinEvThreads) k_bin_event(const Geometry* __restrict__ G, HitsView H,
                                                            long ev_stride, unsigned int* packed, int* rank,
                                                            int* gcounts, int* off) {
  extern __shared__ unsigned int bin_cnt[];
  __shared__ int wsum[kBinEvThreads / 64];
  __shared__ int ovf;
  const int e = blockIdx.x;
  const int tid = threadIdx.x;
  const int n = H.n_hits;
  const int lo = min(max(H.ev_off[e], 0), n);
  const int hi = min(max(H.ev_off[e + 1], lo), n);
  const int L = G->n_layers, nb = G->n_eta * G->n_phi;
  const int nk = L * nb;
  const int ng = (nk + 7) >> 3;  // groups of 8 keys
  const int nw = 2 * ng;         // counter words (4 keys each)
  unsigned int* goff = bin_cnt + nw;  // [ng] global offset of each group
  const long kbase = (long)e * ev_stride;
  for (int i = tid; i < nw; i += kBinEvThreads) bin_cnt[i] = 0u;
  if (tid == 0) ovf = 0;
  __syncthreads();
  // count: key = layer * n_bins + bin and the hit's place among its bin's
  // hits, packed as key | place << 24 (kNoBin: no bin)
  constexpr int kStep = kBinEvThreads * kBinEvBatch;
  for (int i0 = lo + tid; i0 < hi; i0 += kStep) {
    int l[kBinEvBatch];
    float x[kBinEvBatch], y[kBinEvBatch], z[kBinEvBatch];
#pragma unroll
    for (int u = 0; u < kBinEvBatch; ++u) {
      const int i = i0 + u * kBinEvThreads;
      l[u] = i < hi ? H.layer[i] : -1;
      x[u] = i < hi ? H.x[i] : 0.0f;
      y[u] = i < hi ? H.y[i] : 0.0f;
      z[u] = i < hi ? H.z[i] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kBinEvBatch; ++u) {
      const int i = i0 + u * kBinEvThreads;
      if (i >= hi) break;
      unsigned int p = kNoBin;
      if (l[u] >= 0 && l[u] < L) {
        const int b = hit_bin_fast(*G, l[u], x[u], y[u], z[u]);
        if (b >= 0) {
          const int key = l[u] * nb + b;
          const int sh = (key & 3) << 3;
          const unsigned int r = (atomicAdd(&bin_cnt[key >> 2], 1u << sh) >> sh) & 255u;
          if (r == 255u) ovf = 1;
          p = (unsigned int)key | (r << 24);
        }
      }
      packed[i] = p;
    }
  }
  __syncthreads();
  const bool glob = ovf != 0;  // the same for the whole workgroup
  if (glob) {
    for (int k = tid; k < nk; k += kBinEvThreads) gcounts[kbase + k] = 0;
    __syncthreads();
    for (int i = lo + tid; i < hi; i += kBinEvThreads) {
      const unsigned int p = packed[i];
      if (p != kNoBin) rank[i] = atomicAdd(&gcounts[kbase + (p & 0xffffffu)], 1);
    }
    __syncthreads();
  }
  // exclusive scan of the counts in tiles of 4 keys per thread; the
  // offsets are global positions (the event's part starts at lo)
  int running = lo;
  for (int w0 = 0; w0 < nw; w0 += kBinEvThreads) {
    const int wi = w0 + tid;
    int c[4] = {0, 0, 0, 0};
    if (wi < nw) {
      if (!glob) {
        const unsigned int v = bin_cnt[wi];
        c[0] = (int)(v & 255u);
        c[1] = (int)((v >> 8) & 255u);
        c[2] = (int)((v >> 16) & 255u);
        c[3] = (int)(v >> 24);
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j)
          c[j] = 4 * wi + j < nk ? __hip_atomic_load(&gcounts[kbase + 4 * wi + j], __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT)
                                 : 0;
      }
    }
    int tot;
    int pre = running + block_exclusive_scan<kBinEvThreads>(c[0] + c[1] + c[2] + c[3], wsum, tot);
    if (wi < nw && !(wi & 1)) goff[wi >> 1] = (unsigned int)pre;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (4 * wi + j < nk) off[kbase + 4 * wi + j] = pre;
      pre += c[j];
    }
    running += tot;
  }
  if (tid == 0) {
    off[kbase + nk] = running;                              // the unused tail
    if (e == (int)gridDim.x - 1) off[kbase + ev_stride] = hi;  // one past the last key
  }
  __syncthreads();
  // places: each thread handles the hits it counted
  for (int i0 = lo + tid; i0 < hi; i0 += kStep) {
    unsigned int p[kBinEvBatch];
    int r[kBinEvBatch];
#pragma unroll
    for (int u = 0; u < kBinEvBatch; ++u) {
      const int i = i0 + u * kBinEvThreads;
      p[u] = i < hi ? packed[i] : kNoBin;
      r[u] = (glob && p[u] != kNoBin) ? rank[i] : (int)(p[u] >> 24);
    }
#pragma unroll
    for (int u = 0; u < kBinEvBatch; ++u) {
      const int i = i0 + u * kBinEvThreads;
      if (i >= hi) break;
      unsigned int q = kNoBin;
      if (p[u] != kNoBin) {
        const int key = (int)(p[u] & 0xffffffu);
        if (glob) {
          q = (unsigned int)(off[kbase + key] + r[u]);
        } else {
          // the counts of the keys before this one in its group of 8
          const int g = key >> 3, j = key & 7;
          const unsigned int w0 = bin_cnt[2 * g], w1 = bin_cnt[2 * g + 1];
          const unsigned int m0 = j >= 4 ? 0xffffffffu : (j == 0 ? 0u : 0xffffffffu >> (32 - 8 * j));
          const unsigned int m1 = j <= 4 ? 0u : 0xffffffffu >> (64 - 8 * j);
          const unsigned int before = __builtin_amdgcn_sad_u8(w0 & m0, 0u, 0u) + __builtin_amdgcn_sad_u8(w1 & m1, 0u, 0u);
          q = goff[g] + before + (unsigned int)r[u];
        }
      }
      packed[i] = q;
    }
  }
}

// The hits to their places (pos[i] < 0: none), blocks in XCD order.
__global__ void __launch_bounds__(256) k_bin_place(HitsView H, const int* pos, int nblk, float4* sorted) {
  const int lb = xcd_block(nblk);
  if (lb < 0) return;
  const int i = lb * 256 + (int)threadIdx.x;
  if (i >= H.n_hits) return;
  const int p = pos[i];
  if (p < 0) return;
  float w;
  __builtin_memcpy(&w, &i, 4);
  sorted[p] = make_float4(H.x[i], H.y[i], H.z[i], w);
}

// ---------------------------------------------------------------- fit (a10)
// Two wavefronts per SIMD (at most 256 registers a lane; the FP64 filter
// step needs about that many): 200k tracks are ~3 wavefronts per SIMD, and
// two resident at a time hide part of each other's latency.
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_fit(const Geometry* __restrict__ G, HitsView H, const int* trk_off,
                                             const int* trk_hits, int n_tracks, Prior pr,
                                             const float* align, float fscale, FitOut o) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tracks) return;
  fit_track(*G, H, trk_off, trk_hits, t, pr, align, fscale, o);
}

// ------------------------------------------------------------ fit adjoint
// One track per lane.  Each lane adds its track's gradient into its own
// column of an LDS table (rows: dr, drphi, dz per barrel layer by radius,
// then the field scale), so no two lanes write one word.  The wave then sums
// every row over its 64 lanes with a fixed butterfly and writes one partial
// row per block, and k_grad_reduce sums the partials in block order: the
// result does not depend on scheduling.
struct LdsAcc {
  double* col;  // this lane's column: row q at col[q * 64]
  const int* brank;
  int nb;
  __device__ void add(int l, int c, double v) {
    const int r = brank[l];
    if (r >= 0) col[(3 * r + c) * 64] += v;
  }
  __device__ void field(double v) { col[(3 * nb) * 64] += v; }
};

__global__ void __launch_bounds__(64) k_fit_backward(const Geometry* __restrict__ G, HitsView H, const int* trk_off,
                                                     const int* trk_hits, int n_tracks, Prior pr,
                                                     const float* align, float fscale, StateSoA ckpt,
                                                     const int* status, const float* dchi2, int per_track,
                                                     double* partial) {
  extern __shared__ double acc_lds[];
  const int lane = threadIdx.x;
  const int nb = G->n_barrel;
  const int nrow = 3 * nb + 1;
  for (int q = 0; q < nrow; ++q) acc_lds[q * 64 + lane] = 0.0;
  const int t = blockIdx.x * 64 + lane;
  if (t < n_tracks && status[t] == 1) {
    const double w = per_track ? (double)dchi2[t] : (double)dchi2[0];
    if (w != 0.0) {
      LdsAcc acc{acc_lds + lane, G->brank, nb};
      fit_track_backward(*G, H, trk_off, trk_hits, t, pr, align, fscale, ckpt, n_tracks, w, acc);
    }
  }
  __syncthreads();
  for (int q = 0; q < nrow; ++q) {
    double v = acc_lds[q * 64 + lane];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) partial[(long)blockIdx.x * nrow + q] = v;
  }
}

// dalign[3 l + c] = sum over blocks of the partial rows (0 for disks),
// dfield = the last row.  One workgroup per output: thread t adds the
// partials of blocks t, t + 256, ... in that order, then a fixed tree over
// the 256 sums; the order depends only on the number of blocks, so the
// result does not depend on scheduling.  (Summed by one thread, the
// thousands of dependent adds of a large fit took longer than the adjoint.)
constexpr int kReduceThreads = 256;
__global__ void __launch_bounds__(kReduceThreads) k_grad_reduce(const Geometry* __restrict__ G, const double* partial,
                                                                int nblocks, double* dalign, double* dfield) {
  __shared__ double part[kReduceThreads];
  const int i = blockIdx.x;
  const int nl = G->n_layers, nrow = 3 * G->n_barrel + 1;
  if (i > 3 * nl) return;
  int row = nrow - 1;
  if (i < 3 * nl) {
    const int r = G->brank[i / 3];
    if (r < 0) {
      if (threadIdx.x == 0) dalign[i] = 0.0;
      return;
    }
    row = 3 * r + i % 3;
  }
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kReduceThreads) s += partial[(long)b * nrow + row];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = kReduceThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (i < 3 * nl) dalign[i] = part[0];
    else *dfield = part[0];
  }
}

// ------------------------------------------------------ seeds and step (a2-a6)
__global__ void __launch_bounds__(128) k_seed_states(const Geometry* __restrict__ G, HitsView H, const int* seeds, int n, Prior pr,
                              StateSoA out, float* chi2, int* status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  State st;
  float c2 = 0.0f;
  const bool ok = seed_state(*G, H, seeds + 3 * s, pr, st, c2);
  if (!ok) {
    st.x = st.y = st.z = st.k = st.phi = st.th = 0.0;
    for (int j = 0; j < 21; ++j) st.C[j] = 0.0f;
    c2 = 0.0f;
  }
  store_state(out, s, st);
  chi2[s] = c2;
  status[s] = ok ? 1 : 0;
}

// One building step on given states: navigate, transport, then list every
// compatible hit through the binned index (ascending hit index).
__global__ void __launch_bounds__(128) k_step_compat(const Geometry* __restrict__ G, HitsView H, BinIndex B, const int* cand_event,
                              const int* cand_layer, StateSoA in, int n, float cut, int* next_layer,
                              StateSoA pred, int* pair_count, int* pair_hit, float* pair_chi2,
                              int max_pairs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  State st, pr;
  load_state(in, i, st);
  double cphi, sphi, sth, cth;
  sincos_d(st.phi, sphi, cphi);
  sincos_d(st.th, sth, cth);
  const double kappa = -kHcD * G->bz;
  double s = 0.0;
  const int cl = cand_layer[i], ce = cand_event[i];
  const int nl = (cl >= 0 && cl < G->n_layers && ce >= 0 && ce < H.n_events)
                     ? navigate(*G, cl, st, cphi, sphi, sth, cth, kappa * st.k, s) : -1;
  next_layer[i] = nl;
  if (nl < 0) {
    pair_count[i] = 0;
    return;
  }
  transport(st, G->L[nl], cphi, sphi, sth, cth, s, kappa, pr);
  store_state(pred, i, pr);
  Frame F;
  make_frame(pr, G->L[nl], F);
  const Window w = window_bins(*G, G->L[nl], pr, F, cut);
  const ScanWin sw = scan_win(*G, B, ce, nl, w);
  PairFrame P;
  pair_frame(pr, F, G->L[nl].kind == kDisk, P);
  int cnt = 0;
  int* oh = pair_hit + (long)i * max_pairs;
  float* oc = pair_chi2 + (long)i * max_pairs;
  const int nr = scan_nranges(sw);
  for (int r = 0; r < nr; ++r) {
    int qa, qe;
    scan_range(sw, B, G->n_phi, r, qa, qe);
    for (int q = qa; q < qe; ++q) {
      const float4 hv = B.sorted[q];
      const float c2 = kfx::pair_chi2(P, hv);
      if (c2 < cut) {
        int hid;
        __builtin_memcpy(&hid, &hv.w, 4);
        // keep the max_pairs smallest hit indices, ascending
        int k = cnt < max_pairs ? cnt : max_pairs;
        if (k == max_pairs && (k == 0 || oh[k - 1] < hid)) k = -1;
        if (k >= 0) {
          if (k == max_pairs) --k;  // the largest kept one drops out
          while (k > 0 && oh[k - 1] > hid) {
            oh[k] = oh[k - 1];
            oc[k] = oc[k - 1];
            --k;
          }
          oh[k] = hid;
          oc[k] = c2;
        }
        ++cnt;
      }
    }
  }
  pair_count[i] = cnt;
}

// -------------------------------------------------- plain building path (a3-a9)
__device__ inline void add_stat(unsigned long long* p, unsigned long long v) {
  // one atomic per wave
  const unsigned long long lo = v;
  unsigned long long s = lo;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0 && s) atomicAdd(p, s);
}

// Two wavefronts per SIMD (at most 256 registers; the FP64 seed fit needs
// a little more, and spills a few): one seed per thread, so a batch's
// seeds are many rounds of the machine, and two resident wavefronts hide
// part of each other's latency.
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(2, 2))) k_build_init(BuildArgs a) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n_seeds) return;
  init_seed_slots(a, s);
}

__global__ void __launch_bounds__(128) k_build_predict(BuildArgs a, int cur) {
  const long slot = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int took = 0;
  if (slot < (long)a.n_seeds * a.K) took = predict_slot(a, cur, slot);
  add_stat(a.stats + 0, (unsigned long long)took);
}

__global__ void __launch_bounds__(128) k_build_pairs(BuildArgs a) {
  const long slot = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int found = 0;
  if (slot < (long)a.n_seeds * a.K) found = pairs_slot(a, slot, a.seed_event[slot / a.K]);
  add_stat(a.stats + 1, (unsigned long long)found);
}

__global__ void __launch_bounds__(128) k_build_select(BuildArgs a, int cur) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= a.n_seeds) return;
  select_seed(a, cur, s);
}

__global__ void __launch_bounds__(128) k_build_update(BuildArgs a, int cur, int t) {
  const long slot = blockIdx.x * (long)blockDim.x + threadIdx.x;
  int upd = 0;
  if (slot < (long)a.n_seeds * a.K) upd = update_slot(a, cur, (int)(slot / a.K), (int)(slot % a.K), t);
  add_stat(a.stats + 2, (unsigned long long)upd);
}

__global__ void __launch_bounds__(128) k_build_finalize(BuildArgs a, int fin, TracksOut o) {
  const long slot = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (slot >= (long)a.n_seeds * a.K) return;
  const int s = (int)(slot / a.K), j = (int)(slot % a.K);
  finalize_slot(a, fin, o, s, j);
  if (j == 0) {
    int n = 0;
    for (int q = 0; q < a.K; ++q) n += (meta_flags(a.meta[fin][(long)s * a.K + q]) & kFlagLive) ? 1 : 0;
    o.n_cands[s] = n;
  }
}

// Hit lists of the fused build (the fused kernel wrote the counts, chi2
// sums and states itself).  A block takes `rs` consecutive seeds (128 / the
// power of two >= K, so that the walks fill the block): it first copies the
// steps each seed took of its history (n_steps x K words, contiguous in
// HBM) into LDS with coalesced 16-byte loads, then one thread per (seed,
// slot) walks its slot's parent pointers in LDS.  A walk is a chain of
// dependent reads; in LDS each costs tens of cycles instead of an HBM round
// trip.  A thread fetches its row's counts before the copy, so that their
// latency overlaps it.  When the block's rows fit in LDS too (stage_rows),
// they are built there and then written to HBM as one contiguous range (the
// rows of consecutive seeds are adjacent), in 16-byte stores across the
// block; otherwise each thread writes its row.  Small blocks (about 30 KB
// of LDS for K = 6) let five share a CU, each in its own phase.
constexpr int kRowThreads = 128;
constexpr size_t kRowLds = 65536;

struct LdsWordHist {
  const unsigned int* h;  // the seed's history, [t][K]
  const int* ov;          // its recovered hits, [t][K] (nullptr: no recovery)
  int K;
  __device__ void operator()(int t, int j, int& code, int& parent, int& o) const {
    const unsigned int e = h[t * K + j];
    code = (int)(e & 0x7ffffffu) - 2;
    parent = (int)(e >> 27) - 1;
    o = ov ? ov[t * K + j] : -1;
  }
};

// the first n words of src to dst by `tps` threads (sub = 0 .. tps - 1), 16
// bytes at a time where both are aligned; rounding n up to whole 16-byte
// chunks stays within `cap` words
__device__ inline void copy_prefix(unsigned int* dst, const unsigned int* src, int n, int cap, int sub, int tps) {
  if (((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15) == 0 && (cap & 3) == 0) {
    const int n4 = (n + 3) >> 2;
    for (int i = sub; i < n4; i += tps) reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
  } else {
    for (int i = sub; i < n; i += tps) dst[i] = src[i];
  }
}

__global__ void __launch_bounds__(kRowThreads) k_build_fused_rows(BuildArgs a, TracksOut o, int rs, int stage_rows) {
  // [rs][max_steps][K] history words, with recovery as many recovered hits,
  // then (stage_rows) the [rs K][max_hits] rows
  extern __shared__ __align__(16) unsigned int hist_lds[];
  const int K = a.K;
  const long s0 = (long)blockIdx.x * rs;
  const int ns = (int)min((long)rs, (long)a.n_seeds - s0);
  const int per = a.max_steps * K;  // words per seed
  int* ov_lds = a.overlap ? reinterpret_cast<int*>(hist_lds + (size_t)rs * per) : nullptr;
  // this thread's row: seed q / K, slot q % K (rs K <= the block's threads)
  const int q = threadIdx.x;
  const bool has_row = q < ns * K;
  int T = 0, total = 0;
  bool live = false;
  if (has_row) {
    const long s = s0 + q / K, slot = s * K + q % K;
    T = min(a.n_steps[s], a.max_steps);
    const int nc = o.n_cands[s], nh = o.n_hits[slot], nho = o.n_holes[slot];
    live = q % K < nc;
    total = live ? nh + nho : 0;
  }
  {
    // the steps each seed took: kRowThreads / rs threads per seed
    const int tps = kRowThreads / rs, sl = threadIdx.x / tps, sub = threadIdx.x % tps;
    if (sl < ns) {
      const int used = min(a.n_steps[s0 + sl], a.max_steps) * K;
      copy_prefix(hist_lds + sl * per, a.hist_word + (s0 + sl) * per, used, per, sub, tps);
      if (ov_lds)
        copy_prefix(reinterpret_cast<unsigned int*>(ov_lds) + sl * per,
                    reinterpret_cast<const unsigned int*>(a.hist_ov) + (s0 + sl) * per, used, per, sub, tps);
    }
  }
  __syncthreads();
  const int H = o.max_hits;
  // rows after the histories, at a 16-byte boundary (as the launch sized it)
  const size_t hwords = (size_t)rs * per * (a.overlap ? 2 : 1);
  int* rows = reinterpret_cast<int*>(reinterpret_cast<char*>(hist_lds) + ((hwords * 4 + 15) & ~(size_t)15));
  if (has_row) {
    const int sl = q / K, j = q % K;
    const long s = s0 + sl, slot = s * K + j;
    int* out = stage_rows ? rows + (size_t)q * H : o.hits + slot * H;
    write_hit_row(a, out, H, (int)s, j, T, live, total,
                  LdsWordHist{hist_lds + sl * per, ov_lds ? ov_lds + sl * per : nullptr, K});
  }
  if (!stage_rows) return;
  __syncthreads();
  // the block's rows are one contiguous range of o.hits
  int* dst = o.hits + s0 * K * H;
  const long n = (long)ns * K * H;
  if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
    const long n4 = n >> 2;
    for (long i = threadIdx.x; i < n4; i += kRowThreads)
      reinterpret_cast<int4*>(dst)[i] = reinterpret_cast<const int4*>(rows)[i];
    for (long i = (n4 << 2) + threadIdx.x; i < n; i += kRowThreads) dst[i] = rows[i];
  } else {
    for (long i = threadIdx.x; i < n; i += kRowThreads) dst[i] = rows[i];
  }
}

// ---------------------------------------------- fused persistent kernel (a12)
// One wavefront runs 64 / G seed groups of G lanes (G = lanes per seed:
// 4, 8 or 16 and >= K, or 6 for K of 5 or 6 and 12 for K of 9 to 12, which
// leave 4 of the 64 lanes idle); each lane holds one candidate slot in registers
// for the whole search.  A group takes a new seed from a device counter as
// soon as its seed finishes, so uneven events and candidates of uneven
// length share the machine.  The per-step pieces are those of the plain
// path: navigate + transport, window scan, selection (here K rounds of a
// segmented wavefront minimum over the lanes' child streams) and update;
// states move between lanes through LDS.
struct FusedShared {
  // per lane: the state its children start from -- the prediction on the
  // next surface, or the current state when its child is a stop child --
  // with its layer, and the candidate's meta and chi2
  double par[6];
  float cov[21];
  int layer;
  int meta;
  float chi2;
  // the child picked for this slot by the selection (written by the winner)
  int sel_code;
  float sel_chi2;
};

template <class FS>
__device__ inline void lds_put(FS& d, const State& s, int layer) {
  double* p = d.par;
  p[0] = s.x; p[1] = s.y; p[2] = s.z; p[3] = s.k; p[4] = s.phi; p[5] = s.th;
#pragma unroll
  for (int q = 0; q < 21; ++q) d.cov[q] = s.C[q];
  d.layer = layer;
}

template <class FS>
__device__ inline void lds_get(const FS& d, State& s) {
  const double* p = d.par;
  s.x = p[0]; s.y = p[1]; s.z = p[2]; s.k = p[3]; s.phi = p[4]; s.th = p[5];
#pragma unroll
  for (int q = 0; q < 21; ++q) s.C[q] = d.cov[q];
}

__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Minimum of a 64-bit key over aligned groups of G lanes (G = 4, 8, 16)
// with DPP lane moves: a mirror within the row of 16, a mirror within the
// half row of 8, then the two quad exchanges.  Each step pairs every lane
// with one whose partial set is disjoint from its own, so after the steps
// every lane of a group holds the group's minimum.
template <int CTRL>
__device__ inline uint64_t dpp_min_step(uint64_t v) {
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xf, 0xf, false);
  const uint64_t o = ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
  return o < v ? o : v;
}

// Groups of 6 or 12 lanes (lanes G j .. G j + G - 1; the last 4 lanes of
// the wavefront idle) do not align with the DPP rows: lane shuffles
// instead.  A lane that holds the minimum over c consecutive lanes of its
// group (counted round the group) takes the minimum with the lane
// min(c, G - c) places further round, which holds the next ones; from
// c = 1 this covers the group in 3 steps for G = 6 (1, 2, 2) and 4 for
// G = 12 (1, 2, 4, 4).
__device__ inline uint64_t shfl_min_step(uint64_t v, int src) {
  const int lo = __shfl((int)(uint32_t)v, src, 64);
  const int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
  const uint64_t o = ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo;
  return o < v ? o : v;
}
template <int G>
__device__ inline uint64_t group_min_rot(uint64_t v, int glane, int gl) {
#pragma unroll
  for (int c = 1; c < G; c += (c < G - c ? c : G - c)) {
    const int off = c < G - c ? c : G - c;
    const int j = gl + off;
    v = shfl_min_step(v, glane + (j >= G ? j - G : j));
  }
  return v;
}

template <int G>
__device__ inline uint64_t group_min(uint64_t v) {
  static_assert(G == 4 || G == 8 || G == 16, "group of 4, 8 or 16 lanes");
  if (G >= 16) v = dpp_min_step<0x140>(v);  // row_mirror
  if (G >= 8) v = dpp_min_step<0x141>(v);   // row_half_mirror
  v = dpp_min_step<0x4E>(v);                // quad_perm [2, 3, 0, 1]
  v = dpp_min_step<0xB1>(v);                // quad_perm [1, 0, 3, 2]
  return v;
}

// Navigation of the fused kernel, kept out of line: inlined into the
// persistent loop, its FP64 crossing code raised the loop's register peak by
// about a hundred VGPRs (the scheduler interleaves it with the live state of
// the other phases); as a call it needs no more than its own working set.
// Scalars in, scalars out: nothing goes through scratch memory.
struct NavResult {
  double s;
  int layer;
};
__device__ __attribute__((noinline)) NavResult navigate_call(const Geometry& G, int cur, double x, double y, double z,
                                                             double k, double phi, double th, double cphi, double sphi,
                                                             double sth, double cth, double omega) {
  State st;
  st.x = x;
  st.y = y;
  st.z = z;
  st.k = k;
  st.phi = phi;
  st.th = th;
  NavResult r;
  r.layer = navigate(G, cur, st, cphi, sphi, sth, cth, omega, r.s);
  return r;
}

// ---- window scan of a wavefront -----------------------------------------
// The windows of one step differ wildly in size: a candidate that crosses a
// layer almost tangentially can cover the whole layer, and a lane-private
// scan would leave the wave waiting on its largest window.  Each lane first
// counts the hits of its window.  Windows of at most `coop_min` hits are
// scanned by their own lane.  Each larger one is then scanned by the whole
// wave in turn: its owner's frame, window and admission threshold are
// broadcast with readlane, the 64 lanes read 64 consecutive hits of a range
// at a time (one coalesced load), and a lane keeps a pair only if its chi2 is
// below the cut and it would enter the owner's best-K list (ordered by chi2,
// then hit index) as it stood at the start of the chunk.  The kept pairs are
// handed to the owner through readlane, in ballot order, and the owner counts
// every pair under the cut from a ballot.  The best-K set and the count do
// not depend on the order of insertion, so the result is the lane-private
// scan's.
__device__ inline double rl_d(double v, int l) {
  uint64_t b;
  __builtin_memcpy(&b, &v, 8);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
  const uint64_t r = ((uint64_t)hi << 32) | lo;
  double d;
  __builtin_memcpy(&d, &r, 8);
  return d;
}
__device__ inline float rl_f(float v, int l) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l)); }
__device__ inline int rl_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ inline long rl_l(long v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
  return (long)(((uint64_t)hi << 32) | lo);
}

template <int KM>
__device__ int wave_scan(const BinIndex& B, int n_phi, int lane, bool has, const ScanWin& sw, const PairFrame& pf,
                         float cut, int K, int coop_min, BestK<KM>& best) {
  bestk_init(best);
  int found = 0;
  const int nr = has ? scan_nranges(sw) : 0;
  // bounds of the first kR ranges, loaded together and kept for the scan
  // (a window rarely has more); the others are loaded where needed
  constexpr int kR = 4;
  int ra[kR], re[kR];
#pragma unroll
  for (int r = 0; r < kR; ++r) {
    ra[r] = 0;
    re[r] = 0;
    if (r < nr) scan_range(sw, B, n_phi, r, ra[r], re[r]);
  }
  int total_mine = 0;
#pragma unroll
  for (int r = 0; r < kR; ++r) total_mine += re[r] - ra[r];
  for (int r = kR; r < nr; ++r) {
    int qa, qe;
    scan_range(sw, B, n_phi, r, qa, qe);
    total_mine += qe - qa;
  }
  const bool big = total_mine > coop_min;
  // lane-private scan of the small windows, four loads in flight
  if (has && !big) {
    for (int r = 0; r < nr; ++r) {
      int qa = ra[0], qe = re[0];
#pragma unroll
      for (int i = 1; i < kR; ++i)
        if (r == i) {
          qa = ra[i];
          qe = re[i];
        }
      if (r >= kR) scan_range(sw, B, n_phi, r, qa, qe);
      for (int q = qa; q < qe; q += 4) {
        float4 hv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) hv[u] = q + u < qe ? B.sorted[q + u] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float c2 = pair_chi2(pf, hv[u]);
          if (q + u < qe && c2 < cut) {
            int hid;
            __builtin_memcpy(&hid, &hv[u].w, 4);
            ++found;
            bestk_insert(best, K, c2, hid);
          }
        }
      }
    }
  }
  // the large windows, one owner at a time, by the whole wave
  unsigned long long owners = __ballot(big);
  while (owners) {
    const int o = __ffsll((long long)owners) - 1;
    owners &= owners - 1ull;
    PairFrame P;
    P.xh = rl_f(pf.xh, o);
    P.xl = rl_f(pf.xl, o);
    P.yh = rl_f(pf.yh, o);
    P.yl = rl_f(pf.yl, o);
    P.zh = rl_f(pf.zh, o);
    P.zl = rl_f(pf.zl, o);
    P.c = rl_f(pf.c, o);
    P.s = rl_f(pf.s, o);
    P.disk = rl_i(pf.disk, o);
#pragma unroll
    for (int i = 0; i < 6; ++i) P.Si[i] = rl_f(pf.Si[i], o);
    ScanWin W;
    W.row0 = rl_l(sw.row0, o);
    W.nrows = rl_i(sw.nrows, o);
    W.nseg = rl_i(sw.nseg, o);
    W.b0 = rl_i(sw.b0, o);
    W.b1 = rl_i(sw.b1, o);
    W.w1 = rl_i(sw.w1, o);
    // the owner's admission threshold: a pair must have a smaller key
    uint64_t thr = rl_l((long)bestk_threshold(best, K), o);
    const int nro = W.nrows * W.nseg;
    for (int r = 0; r < nro; ++r) {
      int qa, qe;
      scan_range(W, B, n_phi, r, qa, qe);
      // four loads of 64 consecutive hits per pass; the next pass's loads
      // are issued before this pass is processed
      float4 nx[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int q = qa + 64 * u + lane;
        nx[u] = q < qe ? B.sorted[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
      for (int base = qa; base < qe; base += 256) {
        float4 hv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          hv[u] = nx[u];
          const int q = base + 256 + 64 * u + lane;
          nx[u] = q < qe ? B.sorted[q] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        // keys of the pairs under the cut that would enter the owner's list
        uint64_t kk[4];
        int n_under = 0, n_keep = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const float c2 = pair_chi2(P, hv[u]);
          int hid;
          __builtin_memcpy(&hid, &hv[u].w, 4);
          const uint64_t pk = pair_key(c2, hid);
          const bool under = base + 64 * u + lane < qe && c2 < cut;
          const bool keep = under && pk < thr;
          kk[u] = keep ? pk : kNoKey;
          n_under += __popcll(__ballot(under));
          n_keep += __popcll(__ballot(keep));
        }
        if (lane == o) found += n_under;
        if (n_keep == 0) continue;
        if (n_keep <= 3) {
          // few: hand them over one by one
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            unsigned long long mk = __ballot(kk[u] != kNoKey);
            while (mk) {
              const int b = __ffsll((long long)mk) - 1;
              mk &= mk - 1ull;
              const uint64_t k1 = (uint64_t)rl_l((long)kk[u], b);
              if (lane == o) bestk_insert_key(best, K, k1);
            }
          }
        } else {
          // many (hits sorted by phi approach the window centre with
          // falling chi2): each lane sorts its four keys, then rounds of a
          // wave minimum over the lanes' smallest remaining keys hand the
          // pass's keys to the owner smallest first, at most K of them,
          // stopping at the first that no longer enters the list
#define KFX_CX(a, b)                                  \
  {                                                   \
    const uint64_t lo_ = kk[a] < kk[b] ? kk[a] : kk[b]; \
    kk[b] = kk[a] < kk[b] ? kk[b] : kk[a];            \
    kk[a] = lo_;                                      \
  }
          KFX_CX(0, 1) KFX_CX(2, 3) KFX_CX(0, 2) KFX_CX(1, 3) KFX_CX(1, 2)
#undef KFX_CX
          for (int i = 0; i < K; ++i) {
            const uint64_t m = group_min<16>(kk[0]);
            const uint64_t r0 = (uint64_t)rl_l((long)m, 0), r1 = (uint64_t)rl_l((long)m, 16);
            const uint64_t r2 = (uint64_t)rl_l((long)m, 32), r3 = (uint64_t)rl_l((long)m, 48);
            const uint64_t a01 = r0 < r1 ? r0 : r1, a23 = r2 < r3 ? r2 : r3;
            const uint64_t mn = a01 < a23 ? a01 : a23;
            if (!(mn < thr)) break;  // none left (kNoKey), or no longer enters
            if (lane == o) bestk_insert_key(best, K, mn);
            thr = rl_l((long)bestk_threshold(best, K), o);
            if (kk[0] == mn) {  // keys are unique (hit index): one lane advances
              kk[0] = kk[1];
              kk[1] = kk[2];
              kk[2] = kk[3];
              kk[3] = kNoKey;
            }
          }
        }
        thr = rl_l((long)bestk_threshold(best, K), o);
      }
    }
  }
  return found;
}

// KM: capacity of a candidate's best-K list (>= K; the lane count unless a
// shorter list is instantiated for smaller K)
template <int G_LANES, int OCC, int KM = G_LANES>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OCC, OCC)))
k_build_fused(BuildArgs a, TracksOut o, int* seed_counter) {
  extern __shared__ unsigned char smem_raw[];
  using FS = FusedShared;
  FS* sh = reinterpret_cast<FS*>(smem_raw);
  // the layer table is read at every step with lane-dependent indices: keep
  // a copy in LDS
  __shared__ Geometry g_lds;
  {
    const int* src = reinterpret_cast<const int*>(a.G);
    int* dst = reinterpret_cast<int*>(&g_lds);
    for (int i = threadIdx.x; i < (int)(sizeof(Geometry) / 4); i += blockDim.x) dst[i] = src[i];
    __syncthreads();
  }
  const Geometry& G = g_lds;
  const int lane = threadIdx.x & 63;
  const int gl = lane % G_LANES;                // slot within the seed
  const int glane = lane - gl;                  // the group's first lane in the wave
  const int gbase = (int)(threadIdx.x & ~63u) + glane;
  const int K = a.K;
  const double kappa = -kHcD * G.bz;
  const unsigned long long gmask = ((G_LANES == 64) ? ~0ull : ((1ull << G_LANES) - 1ull)) << glane;

  // per-lane counters (a lane sees at most a few thousand steps per launch)
  unsigned int n_steps = 0, n_pairs = 0, n_upd = 0;
  // groups beyond the wave's quota never take a seed
  int seed = (lane / G_LANES) < a.groups_per_wave ? -1 : -2;
  // a group's next seed is fetched when it takes its current one, so that
  // the counter's latency overlaps the search (first lane of the group)
  int pend = (seed == -1 && gl == 0) ? atomicAdd(seed_counter, 1) : -1;
  int t = 0;
  // register state of this lane's slot
  State st;
  int layer = -1, meta = 0;
  float chi2 = 0.0f;
  FS& me = sh[threadIdx.x];

  while (true) {
    // a group without a seed takes the next one (all lanes take part in
    // the broadcast; only groups that need a seed use it)
    const bool need = seed == -1;
    const int ns = __shfl(pend, gbase & 63, 64);
    if (need) {
      if (ns < a.n_seeds) {
        if (gl == 0) pend = atomicAdd(seed_counter, 1);
        seed = ns;
        t = 0;
        meta = 0;
        layer = -1;
        chi2 = 0.0f;
        if (gl == 0) {
          // start state written by the seed kernel into slot 0
          const long s0 = (long)seed * K;
          meta = a.meta[0][s0];
          if (meta_flags(meta) & kFlagLive) {
            load_state(a.cand[0], s0, st);
            layer = a.layer[0][s0];
            chi2 = a.chi2[0][s0];
          }
        }
      } else {
        seed = -2;  // nothing left for this group
      }
    }
    const bool active = seed >= 0;
    if (__ballot(active) == 0) break;

    // ---- (a) navigate + transport.  The children's start state goes to
    // LDS at once: the prediction, or the current state when there is no
    // next surface (a stop child).  A lane at the hole limit may still end
    // as a stop child after the scan (no compatible hit): it parks its
    // current state in its own slot of the candidate buffer (unused by this
    // kernel after the seed start), so that no current state stays live in
    // registers through the scan.
    int nl = -2;
    const bool live = active && (meta_flags(meta) & kFlagLive) && gl < K;
    BestK<KM> best;
    {
      ScanWin sw;
      PairFrame pf;
      {
        State pr;
        if (live) {
          if (meta_flags(meta) & kFlagDone) {
            nl = -1;
          } else {
            double cphi, sphi;
            sincos_d(st.phi, sphi, cphi);
            double s = 0.0;
            double sth, cth;
            sincos_d(st.th, sth, cth);
            const NavResult r = navigate_call(G, layer, st.x, st.y, st.z, st.k, st.phi, st.th, cphi, sphi, sth, cth,
                                              kappa * st.k);
            nl = r.layer;
            s = r.s;
            if (nl >= 0) {
              transport(st, G.L[nl], cphi, sphi, sth, cth, s, kappa, pr);
              ++n_steps;
            }
          }
        }
        me.meta = meta;
        me.chi2 = chi2;
        if (nl < 0) {
          lds_put(me, st, layer);
        } else {
          lds_put(me, pr, nl);
          if (meta_consec(meta) >= a.max_holes) store_state(a.cand[0], (long)seed * K + gl, st);
          // ---- (b) the window of the prediction
          Frame F;
          const Layer& Ln = G.L[nl];
          make_frame(pr, Ln, F);
          sw = scan_win(G, a.B, a.seed_event[seed], nl, window_bins(G, Ln, pr, F, a.cut, a.inflate));
          pair_frame(pr, F, Ln.kind == kDisk, pf);
        }
      }
      // ---- window scan, best K hit children in registers
      n_pairs += (unsigned int)wave_scan(a.B, G.n_phi, lane, nl >= 0, sw, pf, a.cut, K, a.coop_min, best);
    }
    const KidStream ks = kid_stream(a, live ? meta : 0, chi2, nl, best.n, gl);
    if (nl >= 0 && ks.stop) {
      State cur;
      load_state(a.cand[0], (long)seed * K + gl, cur);
      lds_put(me, cur, layer);
    }
    // ---- (c) selection: K rounds of a segmented minimum over the lanes'
    // stream heads; round i fills new slot i (lane gbase + i).  A lane's
    // stream is its stop child, or its hit children by (chi2, hit) followed
    // by the hole; the head is formed from the front of the best-K list,
    // which shifts by one when the lane wins.
    int idx = 0;
    int my_parent = -1, my_code = kStop;
    float my_chi2 = 0.0f;
    for (int i = 0; i < K; ++i) {
      uint64_t head = ~0ull;
      int hcode = kStop;
      float hchi2 = 0.0f;
      if (ks.live) {
        if (ks.stop) {
          if (idx == 0) {
            head = rank_key(a.rank, ks.nh, ks.nho, ks.chi2, ks.parent, 0);
            hchi2 = ks.chi2;
          }
        } else if (idx < best.n) {
          hchi2 = ks.chi2 + pair_key_chi2(best.k[0]);
          head = rank_key(a.rank, ks.nh + 1, ks.nho, hchi2, ks.parent, idx);
          hcode = pair_key_hit(best.k[0]);
        } else if (idx == best.n && ks.hole) {
          head = rank_key(a.rank, ks.nh, ks.nho + 1, ks.chi2, ks.parent, K);
          hcode = kHole;
          hchi2 = ks.chi2;
        }
      }
      // no group of the wave has a child left: the remaining slots stay empty
      if (__ballot(head != ~0ull) == 0) break;
      uint64_t mn;
      if constexpr (G_LANES == 6 || G_LANES == 12) mn = group_min_rot<G_LANES>(head, glane, gl);
      else mn = group_min<G_LANES>(head);
      const unsigned long long win = __ballot(head == mn && mn != ~0ull) & gmask;
      // winner lane in the wave (unique: keys differ by parent slot); it
      // hands its child to the lane of new slot i through LDS
      const int wl = win ? __ffsll((long long)win) - 1 : 0;
      if (win && gl == i) my_parent = wl - glane;
      if (win && lane == wl) {
        sh[gbase + i].sel_code = hcode;
        sh[gbase + i].sel_chi2 = hchi2;
        ++idx;
#pragma unroll
        for (int q = 0; q + 1 < KM; ++q) best.k[q] = best.k[q + 1];
        best.k[KM - 1] = kNoKey;
      }
    }
    wave_sync();
    if (my_parent >= 0) {
      my_code = me.sel_code;
      my_chi2 = me.sel_chi2;
    }
    // ---- (d) children: copy the parent's state from LDS, update hit children
    // (the lane's state is reassigned on every path, so that the old one is
    // dead from the prediction on and holds no registers through the scan)
    int new_meta = 0, new_layer = -1, h2 = -1;
    const FS& par = sh[gbase + (my_parent >= 0 ? my_parent : 0)];
    lds_get(par, st);
    if (active && gl < K) {
      if (my_parent >= 0) {
        State& ns = st;
        const int pm = par.meta;
        new_layer = par.layer;
        if (my_code == kStop) {
          new_meta = meta_pack(meta_nhits(pm), meta_nholes(pm), meta_consec(pm), kFlagLive | kFlagDone);
        } else if (my_code >= 0) {
          kf_update_fp64(ns, G.L[new_layer], (double)a.H.x[my_code], (double)a.H.y[my_code],
                         (double)a.H.z[my_code]);
          int nh = meta_nhits(pm) + 1;
          ++n_upd;
          if (a.overlap) {
            float c2 = 0.0f;
            h2 = recover_overlap(G, a.B, a.seed_event[seed], new_layer, ns, a.cut, my_code, a.inflate, c2);
            if (h2 >= 0) {
              kf_update_fp64(ns, G.L[new_layer], (double)a.H.x[h2], (double)a.H.y[h2], (double)a.H.z[h2]);
              ++nh;
              ++n_upd;
              my_chi2 += c2;
            }
          }
          new_meta = meta_pack(nh, meta_nholes(pm), 0, kFlagLive);
        } else {
          new_meta = meta_pack(meta_nhits(pm), meta_nholes(pm) + 1, meta_consec(pm) + 1, kFlagLive);
        }
      }
      a.hist_word[hist_index(a, seed, t, gl)] = hist_word_pack(my_parent >= 0 ? my_code : kStop, my_parent);
      if (a.overlap) a.hist_ov[hist_index(a, seed, t, gl)] = h2;
    }
    wave_sync();
    if (active) {
      meta = (gl < K) ? new_meta : 0;
      layer = new_layer;
      chi2 = my_chi2;
      ++t;
    }
    // ---- a group whose candidates are all done (or a full history) ends
    const bool running = active && (meta_flags(meta) & kFlagLive) && !(meta_flags(meta) & kFlagDone);
    const unsigned long long run_mask = __ballot(running) & gmask;
    if (active && (run_mask == 0 || t >= a.max_steps)) {
      // the seed's counts, chi2 sums and states; its hit lists are rebuilt
      // from the history by k_build_fused_rows after this kernel
      const unsigned long long live_mask = __ballot(gl < K && (meta_flags(meta) & kFlagLive)) & gmask;
      if (gl == 0) {
        o.n_cands[seed] = __popcll(live_mask);
        a.n_steps[seed] = t;
      }
      if (gl < K) write_slot_summary(o, (long)seed * K + gl, meta, chi2, st);
      seed = -1;
    }
  }
  add_stat(a.stats + 0, n_steps);
  add_stat(a.stats + 1, n_pairs);
  add_stat(a.stats + 2, n_upd);
}

// ------------------------------------------------------ duplicate removal
// After building, the best candidate of every seed is one track; a track is
// a duplicate of a higher-ranked track when their hit sets overlap by at
// least frac_num / frac_den of the shorter one (abstract and Sec. 3: the
// duplicates the building produces are removed in a step of their own).
//
// One wavefront per track, lane k on entry k of its list (at most 64).  The
// first pass sorts the list across the lanes (bitonic network on shuffles),
// drops repeats and non-hits (ballot compaction), stores the ascending list
// and writes each entry (entry = track * H + position) to head[hit]; the
// next two passes find the shared hits and push only their entries onto a
// per-hit linked list with an atomic exchange (head2[hit] -> entry ->
// next[entry] -> ...).  The last pass walks, lane per shared hit, the list
// of the hit's other holders, merges the track's list with those of the
// holders that rank above it, and reduces the lanes' best partners.  The
// per-hit arrays span the whole batch, so blocks are ordered so that each
// XCD (and its L2) works through one contiguous range of seeds, i.e. of
// events and their hits.

constexpr int kDupRows = 4;  // tracks (wavefronts) per block

// ascending sort of one value per lane over the 64 lanes
__device__ inline int wave_sort_asc(int v, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int o = __shfl_xor(v, j, 64);
      const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
      v = keep_min ? min(v, o) : max(v, o);
    }
  }
  return v;
}

// The lists of a block's tracks lie back to back in the block's segment of
// the list array (kDupRows * H entries from the block's first track on), so
// that the later passes, which read a list's entries only, fetch about one
// line for the four short lists together; key.w holds a track's list length
// (bits 0-7) and its offset in the segment (bits 8 on).
__device__ inline int dup_len(int w) { return w & 0xff; }
__device__ inline const int* dup_list(const DupArgs& a, int b, int w) {
  return a.list + (long)(b / kDupRows) * kDupRows * a.H + (w >> 8);
}

__global__ void __launch_bounds__(256) k_dup_lists(DupArgs a, int nblk) {
  __shared__ int nrow[kDupRows];
  const int lb = xcd_block(nblk);
  if (lb < 0) return;  // whole block
  const int lane = threadIdx.x & 63, wv = (int)(threadIdx.x >> 6);
  const int b = lb * kDupRows + wv;
  const bool valid = b < a.S;  // whole wavefront
  const int H = a.H;
  const int nc = valid ? a.n_cands[b] : 0;
  int v = INT_MAX;
  if (nc > 0 && lane < H) {
    const int h = a.hits[(long)b * a.K * H + lane];
    if (h >= 0 && h < a.n_hits) v = h;
  }
  v = wave_sort_asc(v, lane);
  const int prev = __shfl_up(v, 1, 64);
  const bool keep = v != INT_MAX && (lane == 0 || v != prev);
  const unsigned long long m = __ballot(keep);
  const int n = __popcll(m);
  const int pos = __popcll(m & ((1ull << lane) - 1ull));
  if (lane == 0) nrow[wv] = n;
  __syncthreads();
  if (!valid) return;
  int off = 0;
  for (int w = 0; w < wv; ++w) off += nrow[w];
  if (keep) {
    a.list[(long)lb * kDupRows * H + off + pos] = v;
    a.head[v] = b * H + pos;  // one of the hit's holders wins
  }
  if (lane == 0) {
    const long e = (long)b * a.K;
    a.key[b] = nc > 0 ? make_int4(a.n_hits_c[e], a.n_holes_c[e], __float_as_int(a.chi2_c[e]), n | (off << 8))
                      : make_int4(0, 0, 0, 0);
    a.dup_of[b] = nc > 0 ? -1 : -2;
  }
}

// An entry that does not find itself in head[hit] shares its hit with
// another track: it marks the hit (head = -2; every holder but one sees a
// foreign entry, so a shared hit always ends marked) and clears the hit's
// list head.  Only the entries of marked hits are pushed (with an atomic
// exchange) onto a linked list per hit; a hit held by one track, the
// common case, costs a plain store and two reads.
__global__ void __launch_bounds__(256) k_dup_mark(DupArgs a, int nblk) {
  const int lb = xcd_block(nblk);
  if (lb < 0) return;
  const int lane = threadIdx.x & 63;
  const int b = lb * kDupRows + (int)(threadIdx.x >> 6);
  if (b >= a.S) return;
  const int H = a.H;
  const int w = a.key[b].w, nb = dup_len(w);
  if (lane < nb) {
    const int h = dup_list(a, b, w)[lane];
    if (a.head[h] != b * H + lane) {
      a.head[h] = -2;
      a.head2[h] = -1;
    }
  }
}

__global__ void __launch_bounds__(256) k_dup_push(DupArgs a, int nblk) {
  const int lb = xcd_block(nblk);
  if (lb < 0) return;
  const int lane = threadIdx.x & 63;
  const int b = lb * kDupRows + (int)(threadIdx.x >> 6);
  if (b >= a.S) return;
  const int H = a.H;
  const int w = a.key[b].w, nb = dup_len(w);
  if (lane < nb) {
    const int h = dup_list(a, b, w)[lane];
    if (a.head[h] == -2) {
      const int e = b * H + lane;
      a.next[e] = atomicExch(a.head2 + h, e);
    }
  }
}

// rank of the building order: more hits, fewer holes, smaller chi2, lower
// seed index (x = n_hits, y = n_holes, z = chi2 bits)
__device__ inline bool ranks_above(const int4& x, int xs, const int4& y, int ys) {
  if (x.x != y.x) return x.x > y.x;
  if (x.y != y.y) return x.y < y.y;
  const float cx = __int_as_float(x.z), cy = __int_as_float(y.z);
  if (cx != cy) return cx < cy;
  return xs < ys;
}

// The wave judges one candidate partner J at a time: J's list is loaded
// one entry per lane and every lane tests its own hit against it, so the
// shared count is a ballot.  Lane k walks the holders of its track's hit k
// and offers the next holder that ranks above the track and above the best
// partner so far; a lane whose offer was judged, or can no longer win,
// moves on.  Every holder that could become the best is judged with its
// exact shared count, so the result is the highest-ranked qualifying
// partner whatever the order of the chains.
__global__ void __launch_bounds__(256) k_dup_find(DupArgs a, int nblk) {
  const int lb = xcd_block(nblk);
  if (lb < 0) return;
  const int lane = threadIdx.x & 63;
  const int b = lb * kDupRows + (int)(threadIdx.x >> 6);
  if (b >= a.S) return;  // whole wavefront
  const int4 kb = a.key[b];
  const int nb = dup_len(kb.w);
  if (nb == 0) return;  // dup_of already -1 (no hits) or -2 (no track)
  const int H = a.H;
  const int h = lane < nb ? dup_list(a, b, kb.w)[lane] : -1;
  int e = (lane < nb && a.head[h] == -2) ? a.head2[h] : -1;  // -1: no other holder
  int best = -1;  // uniform across the wave
  int4 kbest = make_int4(0, 0, 0, 0);
  int j = -1;  // this lane's offer
  int4 kj = make_int4(0, 0, 0, 0);
  // next holder on this lane's chain that could still become the best
  auto advance = [&]() {
    j = -1;
    while (e >= 0) {
      const int jj = e / H;
      e = a.next[e];
      if (jj == b) continue;
      const int4 kjj = a.key[jj];
      if (!ranks_above(kjj, jj, kb, b)) continue;
      if (best >= 0 && !ranks_above(kjj, jj, kbest, best)) continue;
      j = jj;
      kj = kjj;
      break;
    }
  };
  advance();
  for (;;) {
    const unsigned long long m = __ballot(j >= 0);
    if (m == 0) break;
    const int l = __ffsll((long long)m) - 1;
    const int J = rl_i(j, l);
    const int4 kJ = make_int4(rl_i(kj.x, l), rl_i(kj.y, l), rl_i(kj.z, l), rl_i(kj.w, l));
    const int nJ = dup_len(kJ.w);
    const int v = lane < nJ ? dup_list(a, J, kJ.w)[lane] : -2;
    bool hit = false;
    for (int y = 0; y < nJ; ++y) hit |= (lane < nb) && (h == rl_i(v, y));
    const int shared = __popcll(__ballot(hit));
    const int shorter = nb < nJ ? nb : nJ;
    if ((long)a.den * shared >= (long)a.num * shorter && (best < 0 || ranks_above(kJ, J, kbest, best))) {
      best = J;
      kbest = kJ;
    }
    if (j == J || (j >= 0 && best >= 0 && !ranks_above(kj, j, kbest, best))) advance();
  }
  if (lane == 0 && best >= 0) a.dup_of[b] = best;
}

// ------------------------------------------------ hit masking (iterations)
// Between iterations the hits of good tracks are taken out of the next
// iteration's input (Sec. 3): a copy of the layer array with -1 (no layer:
// ignored by every call) at the valid hits of every good track.  Good: a
// kept track (dup_of -1, or any track without dup_of) with n_hits >=
// min_hits and chi2 <= max_chi2_ndof * (2 n_hits - 5) in float32.

__global__ void __launch_bounds__(256) k_copy_i32(const int* __restrict__ in, int* __restrict__ out, long n) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) out[i] = in[i];
}

// one thread per list entry of slot 0
__global__ void __launch_bounds__(256) k_mask_hits(MaskArgs a) {
  const long n = (long)a.S * a.H;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int s = (int)(i / a.H), k = (int)(i - (long)s * a.H);
    if (a.n_cands[s] <= 0) continue;
    if (a.dup_of && a.dup_of[s] != -1) continue;
    const long e = (long)s * a.K;
    const int nh = a.n_hits_c[e];
    if (nh < a.min_hits) continue;
    const float cut = a.max_chi2_ndof * (float)(2 * nh - 5);
    if (!(a.chi2_c[e] <= cut)) continue;
    const int h = a.hits[e * a.H + k];
    if (h >= 0 && h < a.n_hits) a.layer_out[h] = -1;
  }
}

// ---------------------------------------------------------------- launchers
static inline unsigned nblk(long n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_fill(int* p, long n, int v, hipStream_t st) {
  if (n <= 0) return;
  if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && n >= 1024) {
    const long blocks = std::min<long>(nblk(n >> 2, 256), 8192);
    hipLaunchKernelGGL(k_fill_i32x4, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
    return;
  }
  const long blocks = std::min<long>(nblk(n, 256), 65536);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, st, p, n, v);
}

// stable: hits of one bin in ascending hit index (else in the order the
// atomics gave them, which the building does not depend on: its best-K
// sets and counts ignore the scan order, ties go by hit index)
void launch_bin(const Geometry* G, const HitsView& H, int n_layers, int n_bins, BinWork& w,
                int* bin_out, bool stable, hipStream_t st) {
  w.ev_stride = (long)n_layers * n_bins;
  const long n_keys = (long)H.n_events * w.ev_stride;
  launch_fill(w.counts, n_keys + 1, 0, st);
  if (H.n_hits > 0)
    hipLaunchKernelGGL(k_bin_keys, dim3(nblk(H.n_hits, 256)), dim3(256), 0, st, G, H, w.ev_stride, w.key, bin_out,
                       w.counts, w.rank);
  exclusive_scan(w.counts, n_keys, w.off, w.scan_scratch, st);
  if (H.n_hits > 0)
    hipLaunchKernelGGL(k_bin_scatter, dim3(nblk(H.n_hits, 256)), dim3(256), 0, st, H, w.key, w.off, w.rank,
                       stable ? w.perm : nullptr, stable ? nullptr : w.sorted);
  if (stable) {
    // hits of a bin in ascending index, then the hits re-laid in that order
    hipLaunchKernelGGL(k_bin_sort, dim3(nblk(n_keys, 256)), dim3(256), 0, st, w.off, n_keys, w.perm);
    if (H.n_hits > 0)
      hipLaunchKernelGGL(k_bin_gather, dim3(nblk(H.n_hits, 256)), dim3(256), 0, st, H, w.perm, w.off + n_keys,
                         w.sorted);
  }
}

size_t bin_event_dyn_lds(long keys_per_event) {
  const long ng = (keys_per_event + 7) / 8;
  return (size_t)ng * 12;  // two counter words and one offset per group of 8 keys
}
size_t bin_event_lds_bytes(long keys_per_event) {
  return bin_event_dyn_lds(keys_per_event) + sizeof(int) * (kBinEvThreads / 64 + 1);
}

hipError_t bin_event_init(size_t max_lds) {
  const size_t dyn = max_lds - sizeof(int) * (kBinEvThreads / 64 + 1);
  return hipFuncSetAttribute((const void*)k_bin_event, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn);
}

void launch_bin_events(const Geometry* G, const HitsView& H, int n_layers, int n_bins, BinWork& w, hipStream_t st) {
  const long nk = (long)n_layers * n_bins;
  w.ev_stride = nk + 1;
  if (H.n_events <= 0) return;
  // a hit outside every event's range has no place
  if (H.n_hits > 0) launch_fill(w.key, H.n_hits, -1, st);
  hipLaunchKernelGGL(k_bin_event, dim3(H.n_events), dim3(kBinEvThreads), bin_event_dyn_lds(nk), st, G, H,
                     w.ev_stride, reinterpret_cast<unsigned int*>(w.key), w.rank, w.counts, w.off);
  if (H.n_hits > 0) {
    const int nb = (int)nblk(H.n_hits, 256);
    hipLaunchKernelGGL(k_bin_place, dim3((nb + 7) / 8 * 8), dim3(256), 0, st, H, w.key, nb, w.sorted);
  }
}

void launch_fit(const Geometry* G, const HitsView& H, const int* trk_off, const int* trk_hits, int n,
                const Prior& pr, const float* align, float fscale, const FitOut& o, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fit, dim3(nblk(n, 128)), dim3(128), 0, st, G, H, trk_off, trk_hits, n, pr, align, fscale, o);
}

int fit_backward_blocks(int n) { return (n + 63) / 64; }

hipError_t launch_fit_backward(const Geometry* G, int n_barrel, int n_layers, const HitsView& H, const int* trk_off,
                               const int* trk_hits, int n, const Prior& pr, const float* align, float fscale,
                               const StateSoA& ckpt, const int* status, const float* dchi2, int per_track,
                               double* partial, double* dalign, double* dfield, hipStream_t st) {
  const int nrow = 3 * n_barrel + 1;
  const int nblocks = fit_backward_blocks(n);
  const size_t shmem = (size_t)nrow * 64 * sizeof(double);
  if (n > 0) {
    if (shmem > 65536) {
      const hipError_t e = hipFuncSetAttribute((const void*)k_fit_backward,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_fit_backward, dim3(nblocks), dim3(64), shmem, st, G, H, trk_off, trk_hits, n, pr, align,
                       fscale, ckpt, status, dchi2, per_track, partial);
  }
  const int nout = 3 * n_layers + 1;
  hipLaunchKernelGGL(k_grad_reduce, dim3(nout), dim3(kReduceThreads), 0, st, G, partial, n > 0 ? nblocks : 0, dalign,
                     dfield);
  return hipGetLastError();
}

void launch_seed_states(const Geometry* G, const HitsView& H, const int* seeds, int n, const Prior& pr,
                        const StateSoA& out, float* chi2, int* status, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_seed_states, dim3(nblk(n, 128)), dim3(128), 0, st, G, H, seeds, n, pr, out, chi2, status);
}

void launch_step_compat(const Geometry* G, const HitsView& H, const BinIndex& B, const int* cand_event,
                        const int* cand_layer, const StateSoA& in, int n, float cut, int* next_layer,
                        const StateSoA& pred, int* pair_count, int* pair_hit, float* pair_chi2,
                        int max_pairs, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_step_compat, dim3(nblk(n, 128)), dim3(128), 0, st, G, H, B, cand_event, cand_layer, in, n,
                     cut, next_layer, pred, pair_count, pair_hit, pair_chi2, max_pairs);
}

void launch_build_plain(const BuildArgs& a, const TracksOut& o, hipStream_t st, const hipEvent_t* ev) {
  const long nslots = (long)a.n_seeds * a.K;
  if (a.n_seeds <= 0) return;
  hipLaunchKernelGGL(k_build_init, dim3(nblk(a.n_seeds, 128)), dim3(128), 0, st, a);
  if (ev) (void)hipEventRecord(ev[0], st);
  int cur = 0;
  for (int t = 0; t < a.max_steps; ++t) {
    hipLaunchKernelGGL(k_build_predict, dim3(nblk(nslots, 128)), dim3(128), 0, st, a, cur);
    hipLaunchKernelGGL(k_build_pairs, dim3(nblk(nslots, 128)), dim3(128), 0, st, a);
    hipLaunchKernelGGL(k_build_select, dim3(nblk(a.n_seeds, 128)), dim3(128), 0, st, a, cur);
    hipLaunchKernelGGL(k_build_update, dim3(nblk(nslots, 128)), dim3(128), 0, st, a, cur, t);
    cur = 1 - cur;
  }
  if (ev) (void)hipEventRecord(ev[1], st);
  hipLaunchKernelGGL(k_build_finalize, dim3(nblk(nslots, 128)), dim3(128), 0, st, a, cur, o);
}

int fused_lanes_pow2(int K) {
  int g = 4;
  while (g < K) g <<= 1;
  return g;
}
// default lanes per seed group: 6 for K of 5 or 6 (ten seeds a wavefront;
// 13 % faster on the batched workload than 8), else the power of two
int fused_lanes_for(int K) { return (K == 5 || K == 6) ? 6 : fused_lanes_pow2(K); }

// Start states of the fused build (FP64 seed phase) in their own kernel, so
// that its FP64 temporaries do not set the register budget of the
// persistent kernel; it needs only the hits, not their bin index.
void launch_build_init(const BuildArgs& a, hipStream_t st) {
  if (a.n_seeds <= 0) return;
  hipLaunchKernelGGL(k_build_init, dim3(nblk(a.n_seeds, 128)), dim3(128), 0, st, a);
}

void launch_build_fused(const BuildArgs& a, const TracksOut& o, int* seed_counter, int blocks, int threads,
                        int lanes, int waves_per_simd, hipStream_t st, const hipEvent_t* ev) {
  if (a.n_seeds <= 0) return;
  launch_fill(seed_counter, 1, 0, st);
  if (ev) (void)hipEventRecord(ev[0], st);
  const size_t shmem = fused_lds_bytes(lanes, threads, a.max_steps);
#define KFX_FUSED(GL, OC) \
  hipLaunchKernelGGL((k_build_fused<GL, OC>), dim3(blocks), dim3(threads), shmem, st, a, o, seed_counter)
#define KFX_FUSED_KM(GL, OC, KM) \
  hipLaunchKernelGGL((k_build_fused<GL, OC, KM>), dim3(blocks), dim3(threads), shmem, st, a, o, seed_counter)
  const bool two = waves_per_simd == 2;
  switch (lanes) {
    case 4:
      if (two) KFX_FUSED(4, 2); else KFX_FUSED(4, 1);
      break;
    case 6:
      if (two) KFX_FUSED_KM(6, 2, 6); else KFX_FUSED_KM(6, 1, 6);
      break;
    case 12:
      if (two) KFX_FUSED_KM(12, 2, 12); else KFX_FUSED_KM(12, 1, 12);
      break;
    case 8:
      // K of 5 or 6 keeps a 6-entry best-K list
      if (a.K <= 6 && a.K >= 5) {
        if (two) KFX_FUSED_KM(8, 2, 6); else KFX_FUSED_KM(8, 1, 6);
      } else {
        if (two) KFX_FUSED(8, 2); else KFX_FUSED(8, 1);
      }
      break;
    default:
      // K of 9 to 12 keeps a 12-entry best-K list (fewer registers)
      if (a.K <= 12) {
        if (two) KFX_FUSED_KM(16, 2, 12); else KFX_FUSED_KM(16, 1, 12);
      } else {
        if (two) KFX_FUSED(16, 2); else KFX_FUSED(16, 1);
      }
      break;
  }
#undef KFX_FUSED
#undef KFX_FUSED_KM
  if (ev) (void)hipEventRecord(ev[1], st);
  const int rs = kRowThreads / fused_lanes_pow2(a.K);
  const size_t hist_lds = (size_t)rs * a.max_steps * a.K * 4 * (a.overlap ? 2 : 1);
  // the hit rows are staged too when they fit; the history part is
  // rounded to 16 bytes so that the rows start aligned
  const size_t hist_al = (hist_lds + 15) & ~(size_t)15;
  const size_t rows_lds = (size_t)rs * a.K * o.max_hits * 4;
  const int stage = hist_al + rows_lds <= kRowLds ? 1 : 0;
  hipLaunchKernelGGL(k_build_fused_rows, dim3((unsigned)((a.n_seeds + rs - 1) / rs)), dim3(kRowThreads),
                     stage ? hist_al + rows_lds : hist_lds, st, a, o, rs, stage);
}

// Dynamic LDS of a fused launch: the lanes' state slots (the history goes
// to HBM); the layer table comes on top of it.
size_t fused_lds_bytes(int lanes, int threads, int max_steps) {
  (void)lanes;
  (void)max_steps;
  return sizeof(FusedShared) * threads;
}
size_t fused_static_lds_bytes() { return sizeof(Geometry); }

void launch_find_duplicates(const DupArgs& a, hipStream_t st) {
  if (a.S <= 0) return;
  const int nblk = (a.S + kDupRows - 1) / kDupRows;
  const dim3 grid((unsigned)(8 * ((nblk + 7) / 8)));
  hipLaunchKernelGGL(k_dup_lists, grid, dim3(64 * kDupRows), 0, st, a, nblk);
  hipLaunchKernelGGL(k_dup_mark, grid, dim3(64 * kDupRows), 0, st, a, nblk);
  hipLaunchKernelGGL(k_dup_push, grid, dim3(64 * kDupRows), 0, st, a, nblk);
  hipLaunchKernelGGL(k_dup_find, grid, dim3(64 * kDupRows), 0, st, a, nblk);
}

void launch_mask_hits(const MaskArgs& a, const int* layer_in, hipStream_t st) {
  if (a.n_hits > 0 && layer_in != a.layer_out) {
    const long nb = std::min<long>(((long)a.n_hits + 255) / 256, 4096);
    hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)nb), dim3(256), 0, st, layer_in, a.layer_out, (long)a.n_hits);
  }
  const long n = (long)a.S * a.H;
  if (n <= 0 || a.n_hits <= 0) return;
  const long nb = std::min<long>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_mask_hits, dim3((unsigned)nb), dim3(256), 0, st, a);
}

}  // namespace kfx
