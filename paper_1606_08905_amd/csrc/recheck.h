// The FP64 recheck of points the matrix-core tiles could not decide: every
// distance is the canonical FP64 form of the definition (index order, one
// rounding per operation), and the lexicographic (D, j) minimum gives the
// lowest-index argmin (Mhembere et al., HPDC'17, Algorithm 1).  Two paths:
// recheck_small (latency: few points per workgroup) and recheck_blocked
// (throughput: many points).  Used by the recheck kernel and, for small
// slices, by the tile kernels themselves after their last unit.
#pragma once

#include <math.h>

#include "common.h"

namespace knor {

// Sixteen dimensions [i0, i0 + 16) of a point row, as FP64.  `full` means
// the chunk lies inside the row and the row start is 16-byte aligned, so the
// chunk is read with 16-byte loads; otherwise dimensions past the end are
// clamped to the last one (valid addresses; the caller drops them).
template <typename T>
__device__ __forceinline__ void load_x_chunk(const T* __restrict__ x, int i0,
                                             int d, bool full, double (&xv)[16]) {
  if (full) {
    if constexpr (sizeof(T) == 4) {
#pragma unroll
      for (int q4 = 0; q4 < 4; ++q4) {
        const float4 v = reinterpret_cast<const float4*>(x + i0)[q4];
        xv[4 * q4] = v.x; xv[4 * q4 + 1] = v.y;
        xv[4 * q4 + 2] = v.z; xv[4 * q4 + 3] = v.w;
      }
      return;
    } else if constexpr (sizeof(T) == 2) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint4 v = reinterpret_cast<const uint4*>(x + i0)[h];
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          xv[8 * h + 2 * e] = (double)__uint_as_float(w[e] << 16);
          xv[8 * h + 2 * e + 1] = (double)__uint_as_float(w[e] & 0xffff0000u);
        }
      }
      return;
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int dim = (i0 + q < d) ? (i0 + q) : (d - 1);
    xv[q] = to_f64<T>(x[dim]);
  }
}

// Throughput path of the FP64 recheck, for workgroups with many near-tie
// points: tiles of 64 points x 64 centroids, staged dimension-major in LDS
// (16 dimensions per stage); thread (tp, tc) keeps the 4 x 4 canonical
// accumulators of points 4tp.. and centroids 4tc.. -- each is the index-order
// FP64 sum of the definition, one rounding per operation -- then the
// lexicographic (D, j) minimum over the 16 lanes that share a point.
constexpr int kRbP = 64, kRbC = 64, kRbD = 16;
constexpr int kRecheckBlockedMin = 48;

template <typename T, typename PointOf>
__device__ unsigned long long recheck_blocked(
    const T* __restrict__ X, int d, const double* __restrict__ C64, int k, int nf,
    PointOf point_of, int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ dirty) {
  __shared__ __attribute__((aligned(16))) double sx[kRbD][kRbP];
  __shared__ __attribute__((aligned(16))) double sc[kRbD][kRbC];
  __shared__ int sp[kRbP];
  const int tp = threadIdx.x >> 4, tc = threadIdx.x & 15;
  unsigned long long changes = 0;
  for (int f0 = 0; f0 < nf; f0 += kRbP) {
    __syncthreads();
    if (threadIdx.x < kRbP) sp[threadIdx.x] = f0 + threadIdx.x < nf ? point_of(f0 + threadIdx.x) : -1;
    __syncthreads();
    double best[4];
    int bj[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) { best[r] = INFINITY; bj[r] = 0x7fffffff; }
    for (int c0 = 0; c0 < k; c0 += kRbC) {
      double acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
      for (int i0 = 0; i0 < d; i0 += kRbD) {
        const int lim = d - i0 < kRbD ? d - i0 : kRbD;
        __syncthreads();
        for (int e = threadIdx.x; e < kRbD * kRbP; e += 256) {
          const int pp = e / kRbD, ii = e - pp * kRbD;
          const int p = sp[pp];
          sx[ii][pp] = (p >= 0 && ii < lim) ? to_f64<T>(X[(size_t)p * d + i0 + ii]) : 0.0;
          const int j = c0 + pp;
          sc[ii][pp] = (j < k && ii < lim) ? C64[(size_t)j * d + i0 + ii] : 0.0;
        }
        __syncthreads();
        for (int ii = 0; ii < lim; ++ii) {
          double xv[4], cv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) xv[r] = sx[ii][4 * tp + r];
#pragma unroll
          for (int q = 0; q < 4; ++q) cv[q] = sc[ii][4 * tc + q];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const double t = __dsub_rn(xv[r], cv[q]);
              acc[r][q] = __dadd_rn(acc[r][q], __dmul_rn(t, t));
            }
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int j = c0 + 4 * tc + q;
        if (j < k)
#pragma unroll
          for (int r = 0; r < 4; ++r)
            if (acc[r][q] < best[r] || (acc[r][q] == best[r] && j < bj[r])) {
              best[r] = acc[r][q];
              bj[r] = j;
            }
      }
    }
    // minimum over the 16 lanes (tc) of each point group
#pragma unroll
    for (int off = 1; off < 16; off <<= 1)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double ob = __shfl_xor(best[r], off);
        const int oj = __shfl_xor(bj[r], off);
        if (ob < best[r] || (ob == best[r] && oj < bj[r])) { best[r] = ob; bj[r] = oj; }
      }
    if (tc < 4) {
      const int r = tc;
      const int p = sp[4 * tp + r];
      double bv = best[0];
      int jv = bj[0];
#pragma unroll
      for (int q = 1; q < 4; ++q)
        if (q == r) { bv = best[q]; jv = bj[q]; }
      if (p >= 0) {
        const int32_t old = labels[p];
        if (old != jv) {                     // unchanged labels are not rewritten
          labels[p] = jv;
          ++changes;
          mark_dirty(dirty, old, jv);
        }
        if (ub) ub[p] = f32_up(sqrt(bv) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
      }
    }
  }
  return changes;
}

// Latency path of the FP64 recheck: the workgroup's 256 threads are split
// into groups of tpf threads, each group takes one near-tie point and its
// threads split the centroids.  tpf starts at tpf_max = min(256, pow2 >= k)
// and is halved until all nf points fit in one pass, so that a workgroup
// costs a fixed number of dependent memory round trips.  Each distance is
// the canonical FP64 form.  With LDSC the FP64 centroids are staged into sC
// (row stride d + 1 doubles); otherwise they are read from the transposed
// global copy CT, which makes the threads' reads contiguous.  The
// lexicographic (D, j) minimum is the lowest-index argmin.  TWO: two
// centroids per step (more loads in flight, more registers).  Every thread
// of the workgroup calls this with the same nf.
template <typename T, bool LDSC, bool TWO = true, typename PointOf>
__device__ unsigned long long recheck_small(
    const T* __restrict__ X, int d, int vec, const double* __restrict__ C64,
    const double* __restrict__ CT, double* sC, int k, int tpf_max, int nf,
    PointOf point_of, int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ dirty) {
  __shared__ double red_d[4];
  __shared__ int red_j[4];
  int tpf = tpf_max;
  while (tpf > 1 && (256 / tpf) < nf) tpf >>= 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = 256 / tpf;                   // points per pass
  const int gsel = threadIdx.x / tpf, t = threadIdx.x % tpf;
  // the first pass's point index is fetched before the centroid staging
  int p_next = gsel < nf ? point_of(gsel) : 0;
  const int ldc = d + 1;
  if constexpr (LDSC) {
    for (int e = threadIdx.x; e < k * d; e += 256) {
      const int jj = e / d, ii = e - jj * d;
      sC[jj * ldc + ii] = C64[e];
    }
    __syncthreads();
  }
  unsigned long long changes = 0;
  for (int f0 = 0; f0 < nf; f0 += G) {
    const int f = f0 + gsel;
    const bool live_f = f < nf;
    const int p = p_next;
    if (f0 + G < nf) p_next = f + G < nf ? point_of(f + G) : 0;
    const T* x = X + (size_t)p * d;
    const int32_t old = (live_f && t == 0) ? labels[p] : 0;
    double best = INFINITY;
    int a = 0x7fffffff;
    constexpr int kC = 16;                   // dimensions loaded together
    // two centroids per step (j and j + tpf), so that both rows' loads are
    // in flight together; a thread visits its centroids in increasing
    // index, so a strict "<" keeps the lowest index
    for (int j = t; live_f && j < k; j += (TWO ? 2 : 1) * tpf) {
      const bool has2 = TWO && j + tpf < k;
      const int j2 = has2 ? j + tpf : j;
      double acc = 0.0, acc2 = 0.0;
      for (int i0 = 0; i0 < d; i0 += kC) {
        double cv[kC], cv2[kC], xv[kC];
        load_x_chunk<T>(x, i0, d, vec && i0 + kC <= d, xv);
#pragma unroll
        for (int q = 0; q < kC; ++q) {
          const int dim = (i0 + q < d) ? (i0 + q) : (d - 1);
          if constexpr (LDSC) {
            cv[q] = sC[j * ldc + dim];
            if constexpr (TWO) cv2[q] = sC[j2 * ldc + dim];
          } else {
            cv[q] = CT[(size_t)dim * k + j];
            if constexpr (TWO) cv2[q] = CT[(size_t)dim * k + j2];
          }
        }
#pragma unroll
        for (int q = 0; q < kC; ++q)
          if (i0 + q < d) {
            const double dd = __dsub_rn(xv[q], cv[q]);
            acc = __dadd_rn(acc, __dmul_rn(dd, dd));
            if constexpr (TWO) {
              const double dd2 = __dsub_rn(xv[q], cv2[q]);
              acc2 = __dadd_rn(acc2, __dmul_rn(dd2, dd2));
            }
          }
      }
      if (acc < best) { best = acc; a = j; }
      if (has2 && acc2 < best) { best = acc2; a = j2; }
    }
    // minimum within the wave part of the group
    const int span = tpf < 64 ? tpf : 64;
    for (int off = span >> 1; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oa = __shfl_xor(a, off);
      if (ob < best || (ob == best && oa < a)) { best = ob; a = oa; }
    }
    // groups wider than a wave combine their waves through LDS
    if (tpf > 64) {
      __syncthreads();
      if (lane == 0) { red_d[wave] = best; red_j[wave] = a; }
      __syncthreads();
      const int w0 = (gsel * tpf) >> 6, nw = tpf >> 6;
      best = red_d[w0];
      a = red_j[w0];
      for (int w = 1; w < nw; ++w) {
        const double ob = red_d[w0 + w];
        const int oa = red_j[w0 + w];
        if (ob < best || (ob == best && oa < a)) { best = ob; a = oa; }
      }
    }
    if (live_f && t == 0) {
      if (old != a) {                        // unchanged labels are not rewritten
        labels[p] = a;
        ++changes;
        mark_dirty(dirty, old, a);
      }
      if (ub) ub[p] = f32_up(sqrt(best) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
    }
  }
  return changes;
}

}  // namespace knor
