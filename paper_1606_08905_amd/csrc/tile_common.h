// Pieces shared by the matrix-core distance tiles (tile_f32.hip,
// tile_bf16.hip): per-wave top-2 state, the merge of the four lane groups of
// a 16x16 MFMA output, the decision of each point against the rounding
// bound of its tile type, and the unit and recheck-slice bookkeeping.
//
// A tile type T provides: PB (blocks of 16 points per wave), KS (MFMA
// K-steps per row), Frag (one lane's B operand of one K-step) and
// bound(xn2, R2) -> E, an upper bound on |y~_j - y_j| for every centroid j,
// where y_j = |c_j|^2 - 2 x.c_j exactly and y~_j is the tile's value,
// xn2 >= |x|^2 and R2 >= max_j |c_j|^2.
#pragma once

#include <math.h>

#include "recheck.h"

namespace knor {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTileThreads = 256;

// min / max without NaN canonicalisation (inputs are finite or +inf)
__device__ __forceinline__ float fmax_nc(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, INFINITY);
}

// Per-wave state for PB blocks of 16 points.
template <class T>
struct WaveState {
  typename T::Frag bx[T::PB][T::KS];
  int64_t pid[T::PB];
  bool valid[T::PB];
  double xs[T::PB];
  float b1[T::PB], b2[T::PB];
  int i1[T::PB];
  int32_t old[T::PB];     // previous label (loaded with the point)
};

// Largest fp32(|c|^2) over the real centroids of a staged chunk.
__device__ __forceinline__ float chunk_cmax(const float* sN, int cc, int c0,
                                            int k, int lane) {
  float mx = 0.0f;
  for (int e = lane; e < cc; e += 64)
    if (c0 + e < k) mx = fmax_nc(mx, sN[e]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax_nc(mx, __shfl_xor(mx, off));
  return mx;
}

// Combine the four lane groups (each saw a different quarter of centroids).
template <class T>
__device__ __forceinline__ void merge_groups(WaveState<T>& w) {
  constexpr int PB = T::PB;
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const float ob1 = __shfl_xor(w.b1[pb], off);
      const float ob2 = __shfl_xor(w.b2[pb], off);
      const int oi1 = __shfl_xor(w.i1[pb], off);
      w.xs[pb] += __shfl_xor(w.xs[pb], off);
      // second best of the union: min(max(b1, ob1), min(b2, ob2))
      const float hi = w.b1[pb] < ob1 ? ob1 : w.b1[pb];
      const float lo2 = w.b2[pb] < ob2 ? w.b2[pb] : ob2;
      const float nb2 = hi < lo2 ? hi : lo2;
      const bool take = ob1 < w.b1[pb] || (ob1 == w.b1[pb] && oi1 < w.i1[pb]);
      w.i1[pb] = take ? oi1 : w.i1[pb];
      w.b1[pb] = take ? ob1 : w.b1[pb];
      w.b2[pb] = nb2;
    }
  }
}

// Decide each point (lane group g finalises point block pb with pb % 4 == g).
// With E the tile's error bound, the point is decided iff
//   y_2nd - y_best > 2E + 2.01 (d+2) 2^-53 (|x|^2 + y_best + E):
// every other centroid's exact squared distance then exceeds the chosen
// one's by more than the FP64 evaluation error of the definition, so the
// FP64 argmin (with its lowest-index rule) picks the same centroid.
// Writes labels / bounds of decided points; returns per-block flags.
template <class T>
__device__ __forceinline__ void finalize_points(
    WaveState<T>& w, float cmax, int d, int grp, int recheck_all,
    int32_t* __restrict__ labels, float* __restrict__ ub, int* __restrict__ dirty,
    bool (&flag)[T::PB], bool& changed) {
  constexpr int PB = T::PB;
  static_assert(PB <= 4, "one finalised point per lane");
  // R2 >= max |c|^2: cmax is the largest fp32(|c|^2), within 2^-24 of it
  const double R2 = (double)cmax * (1.0 + 2.384185791015625e-07);  // 1+2^-22
  const double e64 = (double)(d + 2) * 1.1102230246251565e-16;     // (d+2)2^-53
  changed = false;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    flag[pb] = false;
    if (!(w.valid[pb] && (pb & 3) == grp)) continue;
    // xs sums exact squares in FP64: at most (d+4) roundings of 2^-53
    const double xn2 = w.xs[pb] * (1.0 + (double)(d + 4) * 2.220446049250313e-16);
    const double E = T::bound(xn2, R2, d);
    const double y1 = (double)w.b1[pb], y2 = (double)w.b2[pb];
    double dbest = xn2 + y1 + E;
    if (!(dbest > 0.0)) dbest = 0.0;
    const double thr = 2.0 * E + 2.01 * e64 * dbest;
    const double gap = y2 - y1;
    flag[pb] = recheck_all || !(gap > thr);
    if (!flag[pb]) {
      const int64_t p = w.pid[pb];
      const int32_t old = w.old[pb];
      labels[p] = w.i1[pb];
      if (old != w.i1[pb]) {
        changed = true;
        mark_dirty(dirty, old, w.i1[pb]);
      }
      if (ub) ub[p] = f32_up(sqrt(dbest) * (1.0 + 8.881784197001252e-16));
    }
  }
}

// Unit -> (range of points) of a dense or segmented pass.  Segmented units
// are ordered tile-major (all segments' first tiles, then second tiles, ...)
// so that occupied units spread over the grid.  sSeg: the segment counts
// staged in LDS, or null.
__device__ __forceinline__ bool unit_range(int64_t unit, int up, int64_t n,
                                           const int* __restrict__ seg_cnt,
                                           const int* sSeg, int nseg, int64_t& q0,
                                           int64_t& m, int64_t& base) {
  if (seg_cnt) {
    const int64_t t = unit / nseg;
    const int s = (int)(unit - t * nseg);
    m = sSeg ? sSeg[s] : seg_cnt[s];
    q0 = t * up;
    base = (int64_t)s * kSeg;
    return q0 < m;
  }
  m = n;
  q0 = unit * up;
  base = 0;
  return true;
}

// Segmented pass: stage the segment counts in LDS (when there are at most
// kSegCache segments) and each wave's largest count of occupied units of
// any segment into sWmax[wave].  After the caller's next barrier,
// seg_units_bound() gives the number of units worth visiting: units are
// tile-major, so every unit past (max tiles) x nseg is empty.
constexpr int kSegCache = 1024;

__device__ __forceinline__ void seg_stage(const int* __restrict__ seg_cnt, int nseg,
                                          int up, int* sSeg, int* sWmax) {
  int mx = 0;
  for (int e = threadIdx.x; e < nseg; e += blockDim.x) {
    const int c = seg_cnt[e];
    if (nseg <= kSegCache) sSeg[e] = c;
    const int t = (c + up - 1) / up;
    mx = t > mx ? t : mx;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const int o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if ((threadIdx.x & 63) == 0) sWmax[threadIdx.x >> 6] = mx;
}

__device__ __forceinline__ int64_t seg_units_bound(const int* sWmax, int nseg,
                                                   int64_t nunits) {
  int mx = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) mx = sWmax[w] > mx ? sWmax[w] : mx;
  const int64_t b = (int64_t)mx * nseg;
  return b < nunits ? b : nunits;
}

// After its last unit (and a barrier), a tile workgroup with at most
// fuse_max near-tie points rechecks them itself and reports an empty slice;
// larger slices are left to the recheck kernel.  Returns the slice length
// left for that kernel.
constexpr int kFuseRecheckMax = 64;

// threads per point of the latency path: min(256, pow2 >= k)
inline int fuse_tpf(int k) {
  int t = 1;
  while (t < k && t < 256) t *= 2;
  return t;
}

template <typename X_T>
__device__ __forceinline__ int recheck_own_slice(
    const X_T* __restrict__ X, int d, int vecx, const double* __restrict__ CT,
    int k, int tpf_max, int fuse_max, const int* slice, int nf,
    int32_t* __restrict__ labels, float* __restrict__ ub, int* __restrict__ dirty,
    unsigned long long* __restrict__ row) {
  if (nf == 0 || nf > fuse_max || !CT) return nf;
  const unsigned long long ch = recheck_small<X_T, false, false>(
      X, d, vecx, nullptr, CT, nullptr, k, tpf_max, nf,
      [&](int f) { return slice[f]; }, labels, ub, dirty);
  const int q[1] = {SLOT_CHANGED};
  const unsigned long long v[1] = {ch};
  block_add_slots<1>(row, q, v);
  return 0;
}

// Append this wave's flagged points to the workgroup's slice.
template <class T>
__device__ __forceinline__ int append_flags(const WaveState<T>& w,
                                            const bool (&flag)[T::PB],
                                            int* sFlag, int* __restrict__ slice,
                                            int lane) {
  int total = 0;
#pragma unroll
  for (int pb = 0; pb < T::PB; ++pb) total += __popcll(__ballot(flag[pb]));
  if (total == 0) return 0;
  int base = 0;
  if (lane == 0) base = atomicAdd(sFlag, total);           // LDS
  base = __shfl(base, 0);
#pragma unroll
  for (int pb = 0; pb < T::PB; ++pb) {
    const uint64_t fm = __ballot(flag[pb]);
    if (flag[pb]) slice[base + __popcll(fm & lanemask_lt())] = (int)w.pid[pb];
    base += __popcll(fm);
  }
  return total;
}

}  // namespace knor
