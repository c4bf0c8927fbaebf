// Fits whose rows stay in host memory: the GPU analog of the paper's
// semi-external-memory k-means (Section "Semi-External Memory", its I/O
// minimization and its partitioned row cache).
//
// The points are processed in passes over batches of consecutive rows.  A
// batch's rows live in a device staging buffer at the batch-local index of
// their point, so every kernel of the in-memory iteration (filter, tile,
// recheck, exact update) runs on a batch unchanged: it sees the batch as a
// problem of its own whose labels and bounds are views into the global
// arrays.  A pass either copies the whole batch (one DMA, for full passes)
// or fetches only the rows it will read: the rows of the points that fail
// MTI Clause 1, the paper's rule that a point pruned by Clause 1 requests no
// row data.  A fetched row comes from the device row cache when it holds the
// point (HBM to HBM) and from host memory otherwise (read by the kernel over
// the host link).
//
// The row cache follows the paper's lazily refreshed cache of active rows: at
// the refresh iterations (the first at the cache interval I, each later one
// twice as many iterations after the previous) the rows of that iteration's
// active points (those that fail Clause 1) replace the cache's contents, the
// lowest point indices first up to the capacity.  The new contents go to the
// second of two regions while the current one still serves the iteration;
// the point-to-slot map switches when the iteration ends.  Admission order
// is fixed by a scan of per-segment counts, so the cache holds the same rows
// on every run.
#include "common.h"

namespace knor {

constexpr int kFetchThreads = 1024;      // one block per segment of kSeg points
static_assert(kSeg == 4 * kFetchThreads, "four points per thread");

// Candidates (points that fail Clause 1, or every point with all) of one
// segment of a batch, in point order, into cand[]; returns their count.
// Thread t owns points 4t .. 4t + 3 of the segment.
__device__ __forceinline__ int segment_candidates(
    int64_t n, int64_t p0, const int32_t* __restrict__ labels, const float* __restrict__ u,
    const float* __restrict__ drift, const float* __restrict__ s_half, int all, int* cand,
    int* wcnt) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t pb = p0 + 4 * threadIdx.x;
  bool c[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    c[e] = false;
    if (pb + e < n) {
      if (all) {
        c[e] = true;
      } else {
        const int a = labels[pb + e];
        float ub;
        c[e] = !clause1_keeps(u[pb + e], drift[a], s_half[a], &ub);
      }
    }
  }
  const int cl = (int)c[0] + (int)c[1] + (int)c[2] + (int)c[3];
  int x = cl;                                   // inclusive scan over the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wcnt[wave] = x;
  __syncthreads();
  int before = 0, total = 0;
  for (int w = 0; w < kFetchThreads / 64; ++w) {
    const int v = wcnt[w];
    before += w < wave ? v : 0;
    total += v;
  }
  int pos = before + x - cl;
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (c[e]) cand[pos++] = 4 * (int)threadIdx.x + e;
  __syncthreads();
  return total;
}

// Blocks walk the batch's segments (segment blockIdx.x, then every
// gridDim.x-th): a small grid keeps most compute units free for the compute
// stream, which works on the previous batch meanwhile, while enough reads
// stay in flight for the host link.  Count mode (seg_count != null): each
// segment's candidate count only.  Otherwise every candidate's row goes to
// stage[p] (p batch-local): from cache[pslot[p]] when pslot[p] >= 0, else
// from the host rows Xh.  With adm_rows (a refresh iteration), candidate c
// of a segment also goes to slot adm_base[seg] + c of the new cache region
// when that slot is below adm_cap, and the slot records the point's global
// index.  io (this iteration): [1] rows read from host memory, [2] rows
// read from the cache, [3] rows admitted.
constexpr int kFetchInFlight = 8;       // 16-byte reads per thread before their stores
template <typename T>
__global__ __launch_bounds__(kFetchThreads) void stream_fetch_kernel(
    const T* __restrict__ Xh, int64_t n, int d, const int32_t* __restrict__ labels,
    const float* __restrict__ u, const float* __restrict__ drift,
    const float* __restrict__ s_half, int all, const int* __restrict__ pslot,
    const T* __restrict__ cache, T* __restrict__ stage, T* __restrict__ adm_rows,
    int* __restrict__ adm_pts, const int64_t* __restrict__ adm_base, int64_t adm_cap,
    int64_t gid0, int* __restrict__ seg_count, unsigned long long* __restrict__ io,
    const int* __restrict__ conv, int iter, int vec) {
  __shared__ int cand[kSeg];
  __shared__ int src[kSeg];
  __shared__ int wcnt[kFetchThreads / 64];
  __shared__ int nhit;
  if (*conv < iter) return;                     // uniform
  const int nseg = (int)((n + kSeg - 1) / kSeg);
  unsigned long long miss_tot = 0, hit_tot = 0, adm_tot = 0;   // thread 0's sums
  for (int seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
    const int64_t p0 = (int64_t)seg * kSeg;
    __syncthreads();                            // the previous segment's LDS is free
    if (threadIdx.x == 0) nhit = 0;
    const int na = segment_candidates(n, p0, labels, u, drift, s_half, all, cand, wcnt);
    if (seg_count) {
      if (threadIdx.x == 0) seg_count[seg] = na;
      continue;
    }
    int hits = 0;
    for (int c = threadIdx.x; c < na; c += kFetchThreads) {
      const int sl = pslot ? pslot[p0 + cand[c]] : -1;
      src[c] = sl;
      hits += sl >= 0 ? 1 : 0;
    }
    if (hits) atomicAdd(&nhit, hits);           // LDS
    int64_t base = 0, nadm = 0;
    if (adm_rows) {
      base = adm_base[seg];
      nadm = adm_cap - base;
      nadm = nadm < 0 ? 0 : (nadm > na ? na : nadm);
    }
    __syncthreads();
    if (vec) {
      // 16-byte pieces, kFetchInFlight in flight per thread before their stores
      const int nv = d * (int)sizeof(T) / 16;
      const int tot = na * nv;
      for (int e0 = threadIdx.x; e0 < tot; e0 += kFetchInFlight * kFetchThreads) {
        uint4 w[kFetchInFlight];
        int cc[kFetchInFlight], vv[kFetchInFlight];
#pragma unroll
        for (int r = 0; r < kFetchInFlight; ++r) {
          const int e = e0 + r * kFetchThreads;
          cc[r] = e < tot ? e / nv : -1;
          vv[r] = cc[r] >= 0 ? e - cc[r] * nv : 0;
          if (cc[r] >= 0) {
            const int sl = src[cc[r]];
            const uint4* from =
                sl >= 0 ? reinterpret_cast<const uint4*>(cache + (size_t)sl * d)
                        : reinterpret_cast<const uint4*>(Xh + (size_t)(p0 + cand[cc[r]]) * d);
            w[r] = from[vv[r]];
          }
        }
#pragma unroll
        for (int r = 0; r < kFetchInFlight; ++r) {
          if (cc[r] < 0) continue;
          const int64_t p = p0 + cand[cc[r]];
          reinterpret_cast<uint4*>(stage + (size_t)p * d)[vv[r]] = w[r];
          if (cc[r] < nadm)
            reinterpret_cast<uint4*>(adm_rows + (size_t)(base + cc[r]) * d)[vv[r]] = w[r];
        }
      }
    } else {
      const int tot = na * d;
      for (int e = threadIdx.x; e < tot; e += kFetchThreads) {
        const int c = e / d, i = e - c * d;
        const int64_t p = p0 + cand[c];
        const int sl = src[c];
        const T v = sl >= 0 ? cache[(size_t)sl * d + i] : Xh[(size_t)p * d + i];
        stage[(size_t)p * d + i] = v;
        if (c < nadm) adm_rows[(size_t)(base + c) * d + i] = v;
      }
    }
    for (int c = threadIdx.x; c < nadm; c += kFetchThreads)
      adm_pts[base + c] = (int)(gid0 + p0 + cand[c]);
    __syncthreads();
    if (threadIdx.x == 0) {
      miss_tot += (unsigned long long)(na - nhit);
      hit_tot += (unsigned long long)nhit;
      adm_tot += (unsigned long long)nadm;
    }
  }
  if (threadIdx.x == 0 && !seg_count) {
    if (miss_tot) atomicAdd(io + 1, miss_tot);
    if (hit_tot) atomicAdd(io + 2, hit_tot);
    if (adm_tot) atomicAdd(io + 3, adm_tot);
  }
}

// Exclusive prefix of the per-segment counts: base[s] for s < nseg and the
// total in base[nseg].  One block walks the counts 1024 at a time.
__global__ __launch_bounds__(1024) void stream_scan_kernel(const int* __restrict__ cnt,
                                                           int nseg, int64_t* __restrict__ base,
                                                           const int* __restrict__ conv,
                                                           int iter) {
  __shared__ int64_t wsum[16];
  __shared__ int64_t carry;
  if (*conv < iter) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int s0 = 0; s0 < nseg; s0 += 1024) {
    const int s = s0 + (int)threadIdx.x;
    const int64_t v = s < nseg ? cnt[s] : 0;
    int64_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wave] = x;
    __syncthreads();
    int64_t before = carry, tot = 0;
    for (int w = 0; w < 16; ++w) {
      before += w < wave ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (s < nseg) base[s] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) base[nseg] = carry;
}

// pslot[pts[i]] = -1 for the cnt points of the region being retired.
__global__ void stream_unmap_kernel(int* __restrict__ pslot, const int* __restrict__ pts,
                                    const int64_t* __restrict__ cnt,
                                    const int* __restrict__ conv, int iter) {
  if (*conv < iter) return;
  const int64_t m = *cnt;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    pslot[pts[i]] = -1;
}

// pslot[pts[i]] = i for the min(total, cap) admitted points; the region's
// count goes to cnt_out.
__global__ void stream_map_kernel(int* __restrict__ pslot, const int* __restrict__ pts,
                                  const int64_t* __restrict__ total, int64_t cap,
                                  int64_t* __restrict__ cnt_out,
                                  const int* __restrict__ conv, int iter) {
  if (*conv < iter) return;
  const int64_t m = *total < cap ? *total : cap;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    pslot[pts[i]] = (int)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) *cnt_out = m;
}

// Blocks of the fetch kernel: one per segment up to this many (it walks the
// rest); the count pass, which reads no rows, takes one block per segment.
constexpr int kFetchGrid = 128;

hipError_t launch_stream_fetch(const StreamFetch& f, hipStream_t s) {
  const int nseg = nseg_of_n(f.n);
  if (nseg == 0) return hipSuccess;
  const int grid = f.seg_count ? nseg : (nseg < kFetchGrid ? nseg : kFetchGrid);
  const size_t esz = f.dt == KNOR_F32 ? 4 : 2;
  const size_t rb = (size_t)f.d * esz;
  const bool al = ((uintptr_t)f.Xh & 15) == 0 && ((uintptr_t)f.stage & 15) == 0 &&
                  ((uintptr_t)f.cache & 15) == 0 && ((uintptr_t)f.adm_rows & 15) == 0;
  const int vec = (rb % 16 == 0 && al) ? 1 : 0;
  if (f.dt == KNOR_F32)
    hipLaunchKernelGGL(stream_fetch_kernel<float>, dim3(grid), dim3(kFetchThreads), 0, s,
                       (const float*)f.Xh, f.n, f.d, f.labels, f.u, f.drift, f.s_half, f.all,
                       f.pslot, (const float*)f.cache, (float*)f.stage, (float*)f.adm_rows,
                       f.adm_pts, f.adm_base, f.adm_cap, f.gid0, f.seg_count, f.io, f.conv,
                       f.iter, vec);
  else if (f.dt == KNOR_BF16)
    hipLaunchKernelGGL(stream_fetch_kernel<uint16_t>, dim3(grid), dim3(kFetchThreads), 0, s,
                       (const uint16_t*)f.Xh, f.n, f.d, f.labels, f.u, f.drift, f.s_half,
                       f.all, f.pslot, (const uint16_t*)f.cache, (uint16_t*)f.stage,
                       (uint16_t*)f.adm_rows, f.adm_pts, f.adm_base, f.adm_cap, f.gid0,
                       f.seg_count, f.io, f.conv, f.iter, vec);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_stream_scan(const int* cnt, int nseg, int64_t* base, const int* conv,
                              int iter, hipStream_t s) {
  hipLaunchKernelGGL(stream_scan_kernel, dim3(1), dim3(1024), 0, s, cnt, nseg, base, conv,
                     iter);
  return hipGetLastError();
}

hipError_t launch_stream_remap(int* pslot, const int* old_pts, const int64_t* old_cnt,
                               const int* new_pts, const int64_t* total, int64_t cap,
                               int64_t* new_cnt, const int* conv, int iter, hipStream_t s) {
  int64_t blocks = (cap + 255) / 256;
  const unsigned g = (unsigned)(blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks));
  hipLaunchKernelGGL(stream_unmap_kernel, dim3(g), dim3(256), 0, s, pslot, old_pts, old_cnt,
                     conv, iter);
  hipLaunchKernelGGL(stream_map_kernel, dim3(g), dim3(256), 0, s, pslot, new_pts, total, cap,
                     new_cnt, conv, iter);
  return hipGetLastError();
}

}  // namespace knor
