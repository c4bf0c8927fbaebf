// Pieces shared by the matrix-core distance tiles (tile_f32.hip,
// tile_bf16.hip): per-wave top-3 state, the merge of the four lane groups of
// a 16x16 MFMA output, the decision of each point against the rounding
// bound of its tile type, and the unit and recheck-slice bookkeeping.
//
// A tile type T provides: PB (blocks of 16 points per wave), KS (MFMA
// K-steps per row), Frag (one lane's B operand of one K-step) and
// bound(xn2, R2) -> E, an upper bound on |y~_j - y_j| for every centroid j,
// where y_j = |c_j|^2 - 2 x.c_j exactly and y~_j is the tile's value,
// xn2 >= |x|^2 and R2 >= max_j |c_j|^2.  For the two-candidate FP64 pass it
// also gives the dimension each lane group holds: NS steps of NE elements,
// dim(s, g, e) and xval(bx, s, e) (the exact point value), such that the
// order (s, g, e) is increasing dimension order; PAIR enables that pass.
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

// Per-wave state for PB blocks of 16 points: per point the three smallest
// tile values b1 <= b2 <= b3 seen so far, the index of b1 and of b2.
template <class T>
struct WaveState {
  typename T::Frag bx[T::PB][T::KS];
  int64_t pid[T::PB];
  bool valid[T::PB];
  double xs[T::PB];
  float b1[T::PB], b2[T::PB], b3[T::PB];
  int i1[T::PB], i2[T::PB];
  int32_t old[T::PB];     // previous label (loaded with the point)
};

__device__ __forceinline__ void top3_reset(float& b1, float& b2, float& b3,
                                           int& i1, int& i2) {
  b1 = INFINITY; b2 = INFINITY; b3 = INFINITY;
  i1 = 0; i2 = 0;
}

// Insert tile value y of centroid j (a lane visits its centroids in
// increasing index, so a strict "<" keeps the lowest index on ties).
// b3 and b2 are medians of three (for b1 <= b2 <= b3 the median of
// (b2, b3, y) is the third smallest of {b1, b2, b3, y}).
__device__ __forceinline__ void top3_insert(float& b1, float& b2, float& b3,
                                            int& i1, int& i2, float y, int j) {
  const bool lt1 = y < b1, lt2 = y < b2;
  b3 = __builtin_amdgcn_fmed3f(b2, b3, y);
  b2 = __builtin_amdgcn_fmed3f(b1, b2, y);
  const int t = lt2 ? j : i2;
  i2 = lt1 ? i1 : t;
  i1 = lt1 ? j : i1;
  b1 = lt1 ? y : b1;
}

// The two smallest values and the index of the smallest (for tiles that
// never resolve two-candidate points: the third value is not kept).
__device__ __forceinline__ void top2_insert(float& b1, float& b2, int& i1, float y, int j) {
  const bool lt1 = y < b1;
  b2 = __builtin_amdgcn_fmed3f(b1, b2, y);
  i1 = lt1 ? j : i1;
  b1 = lt1 ? y : b1;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// The same without the second index (three values, best index).
__device__ __forceinline__ void top3_insert_lite(float& b1, float& b2, float& b3,
                                                 int& i1, float y, int j) {
  const bool lt1 = y < b1;
  b3 = __builtin_amdgcn_fmed3f(b2, b3, y);
  b2 = __builtin_amdgcn_fmed3f(b1, b2, y);
  i1 = lt1 ? j : i1;
  b1 = lt1 ? y : b1;
}

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

// Largest fp32(|c|^2) over all k centroids, read from memory by one wave
// (8 loads per lane in flight): the same value as chunk_cmax over every
// chunk of a pass that compares each point with all centroids.
__device__ __forceinline__ float all_cmax(const float* __restrict__ cn, int k, int lane) {
  float mx = 0.0f;
  for (int e0 = 0; e0 < k; e0 += 64 * 8) {
    float v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 64 * q + lane;
      v[q] = cn[e < k ? e : 0];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (e0 + 64 * q + lane < k) mx = fmax_nc(mx, v[q]);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmax_nc(mx, __shfl_xor(mx, off));
  return mx;
}

// Combine the four lane groups (each saw a different quarter of centroids).
// For two sorted triples a and o the union's second smallest is
// min(max(a1, o1), a2, o2) and its third smallest is
// min(a3, o3, max(a2, o1), max(a1, o2)).
template <class T, bool I2 = true>
__device__ __forceinline__ void merge_groups(WaveState<T>& w) {
  constexpr int PB = T::PB;
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const float a1 = w.b1[pb], a2 = w.b2[pb], a3 = w.b3[pb];
      const int ia1 = w.i1[pb], ia2 = I2 ? w.i2[pb] : 0;
      const float o1 = __shfl_xor(a1, off);
      const float o2 = __shfl_xor(a2, off);
      const float o3 = __shfl_xor(a3, off);
      const int io1 = __shfl_xor(ia1, off);
      const int io2 = I2 ? __shfl_xor(ia2, off) : 0;
      w.xs[pb] += __shfl_xor(w.xs[pb], off);
      const bool take = o1 < a1 || (o1 == a1 && io1 < ia1);
      // second: after a1 comes min(a2, o1); after o1 comes min(a1, o2)
      const float s_a = o1 < a2 ? o1 : a2;
      const int is_a = o1 < a2 ? io1 : ia2;
      const float s_o = a1 <= o2 ? a1 : o2;
      const int is_o = a1 <= o2 ? ia1 : io2;
      const float m21 = a2 < o1 ? o1 : a2, m12 = a1 < o2 ? o2 : a1;
      float t3 = a3 < o3 ? a3 : o3;
      t3 = t3 < m21 ? t3 : m21;
      t3 = t3 < m12 ? t3 : m12;
      w.b1[pb] = take ? o1 : a1;
      w.i1[pb] = take ? io1 : ia1;
      w.b2[pb] = take ? s_o : s_a;
      if (I2) w.i2[pb] = take ? is_o : is_a;
      w.b3[pb] = t3;
    }
  }
}

// Canonical FP64 squared distance D(x, c_j) of the point in column
// `lane & 15` (every lane returns the value of its column).  The sum runs
// in increasing dimension order as one chain: the lane group holding the
// next dimensions continues the running sum, which moves to it with a lane
// rotation by 16 after each group's part.  Each lane first loads its own
// dimensions of c_j (one memory round trip).
template <class T>
__device__ __forceinline__ double chain_dist(const typename T::Frag (&bx)[T::KS],
                                             bool need, int j,
                                             const double* __restrict__ C64, int d,
                                             int grp, int lane) {
  constexpr int NS = T::NS, NE = T::NE;
  double c[NS][NE];
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int dim = T::dim(s, grp, e);
      c[s][e] = (need && dim < d) ? C64[(size_t)j * d + dim] : 0.0;
    }
  double a = 0.0;
  const int from = (lane + 48) & 63;          // the lane 16 below, cyclically
#pragma unroll
  for (int s = 0; s < NS; ++s)
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (grp == g && need) {
#pragma unroll
        for (int e = 0; e < NE; ++e) {
          if (T::dim(s, g, e) < d) {
            const double t = __dsub_rn(T::xval(bx, s, e), c[s][e]);
            a = __dadd_rn(a, __dmul_rn(t, t));
          }
        }
      }
      a = __shfl(a, from);
    }
  // after the last group's part the sum sits in lane group 0
  return __shfl(a, lane & 15);
}

// Points resolved from two canonical distances after the workgroup's last
// unit: (point, best index, second index, previous label), in LDS.  A point
// that finds the list full goes to the full FP64 recheck instead.
constexpr int kPairCap = 128;

// The tile's decision for one point from its three smallest values (xs:
// the FP64 sum of its squares, cmax: the largest fp32(|c|^2)).  With E the
// tile's error bound, the point is decided iff
//   y_2nd - y_best > 2E + 2.01 (d+2) 2^-53 (|x|^2 + y_best + E):
// every other centroid's exact squared distance then exceeds the chosen
// one's by more than the FP64 evaluation error of the definition, so the
// FP64 argmin (with its lowest-index rule) picks the same centroid.
// If instead only the third smallest value clears that margin, every
// centroid other than the two best is excluded the same way, and the FP64
// argmin over all centroids is the FP64 argmin of those two ("pair").
// dbest bounds the squared distance to the best centroid from above.
struct Decision {
  bool decided, pair;
  double dbest;
};

template <class T>
__device__ __forceinline__ Decision decide_point(double xs, float b1, float b2,
                                                 float b3, float cmax, int d,
                                                 bool recheck_all, bool pairs) {
  // R2 >= max |c|^2: cmax is the largest fp32(|c|^2), within 2^-24 of it
  const double R2 = (double)cmax * (1.0 + 2.384185791015625e-07);  // 1+2^-22
  const double e64 = (double)(d + 2) * 1.1102230246251565e-16;     // (d+2)2^-53
  // xs sums exact squares in FP64: at most (d+4) roundings of 2^-53
  const double xn2 = xs * (1.0 + (double)(d + 4) * 2.220446049250313e-16);
  const double E = T::bound(xn2, R2, d);
  const double y1 = (double)b1;
  Decision r;
  r.dbest = xn2 + y1 + E;
  if (!(r.dbest > 0.0)) r.dbest = 0.0;
  const double thr = 2.0 * E + 2.01 * e64 * r.dbest;
  r.decided = !recheck_all && (double)b2 - y1 > thr;
  r.pair = pairs && !recheck_all && !r.decided && (double)b3 - y1 > thr;
  return r;
}

// Write a decided point's bound, and its label when it changed (old is the
// label the point had before this pass).
__device__ __forceinline__ bool commit_label(int64_t p, int32_t old, int32_t a,
                                             float bnd, int32_t* __restrict__ labels,
                                             float* __restrict__ ub,
                                             int* __restrict__ dirty) {
  if (ub) ub[p] = bnd;
  if (old == a) return false;
  labels[p] = a;
  mark_dirty(dirty, old, a);
  return true;
}

// Decide each point: lane group g finalises point block g (g < PB; the
// merged values are equal in every group), so the bound arithmetic runs
// once per lane instead of once per block.  Decided points get their label
// and bound; pair points are queued for the tail (with the second index
// when I2); the rest are flagged for the full FP64 recheck.
template <class T, bool I2 = true>
__device__ __forceinline__ void finalize_points(
    WaveState<T>& w, float cmax, int d, int grp, int recheck_all, bool pairs,
    int4* sPair, int* sPairN, int32_t* __restrict__ labels,
    float* __restrict__ ub, int* __restrict__ dirty, bool& flag, int& pid,
    bool& changed) {
  constexpr int PB = T::PB;
  static_assert(PB <= 4, "one finalised point per lane");
  // this lane's block
  bool valid = w.valid[0];
  double xs = w.xs[0];
  float b1 = w.b1[0], b2 = w.b2[0], b3 = w.b3[0];
  int i1 = w.i1[0], i2 = I2 ? w.i2[0] : -1;
  int64_t p = w.pid[0];
  int32_t old = w.old[0];
#pragma unroll
  for (int pb = 1; pb < PB; ++pb) {
    const bool m = grp == pb;                  // selects, not an indexed copy
    valid = m ? w.valid[pb] : valid;
    xs = m ? w.xs[pb] : xs;
    b1 = m ? w.b1[pb] : b1;
    b2 = m ? w.b2[pb] : b2;
    b3 = m ? w.b3[pb] : b3;
    i1 = m ? w.i1[pb] : i1;
    if (I2) i2 = m ? w.i2[pb] : i2;
    p = m ? w.pid[pb] : p;
    old = m ? w.old[pb] : old;
  }
  const bool own = grp < PB && valid;
  pid = (int)p;
  changed = false;
  flag = false;
  Decision dc{false, false, 0.0};
  if (own) dc = decide_point<T>(xs, b1, b2, b3, cmax, d, recheck_all, pairs);
  bool pair = dc.pair;
  if (pairs) {
    const uint64_t m = __ballot(pair);
    if (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      int base = 0;
      if (lane_id() == leader) base = atomicAdd(sPairN, __popcll(m));   // LDS
      base = __shfl(base, leader);
      if (pair) {
        const int slot = base + __popcll(m & lanemask_lt());
        if (slot < kPairCap)
          sPair[slot] = make_int4(pid, i1, i2, old);
        else
          pair = false;                        // list full: full recheck
      }
    }
  }
  if (!own) return;
  flag = !dc.decided && !pair;
  if (!dc.decided) return;
  changed = commit_label(p, old, i1, f32_up(sqrt(dc.dbest) * (1.0 + 8.881784197001252e-16)),
                         labels, ub, dirty);
}

// Upper bound on the distance from a canonical FP64 squared distance.
__device__ __forceinline__ float pair_bound(double D, int d) {
  return f32_up(sqrt(D) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
}

// The queued two-candidate points (after a barrier; every thread calls this
// with the same count np <= kPairCap): each wave takes 16 at a time in the
// tile's lane layout, loads their rows and both centroids' FP64 values, and
// the owner lane keeps the lower canonical distance (lower index on a tie).
// Returns this thread's count of changed labels.
template <class T, typename X_T>
__device__ __forceinline__ unsigned long long resolve_pairs(
    const X_T* __restrict__ X, int d, int vec, const double* __restrict__ C64,
    const int4* sPair, int np, int32_t* __restrict__ labels,
    float* __restrict__ ub, int* __restrict__ dirty) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  unsigned long long chg = 0;
  for (int e0 = wave * 16; e0 < np; e0 += kTileThreads / 4) {
    const int e = e0 + col;
    const bool need = e < np;
    const int4 q = need ? sPair[e] : make_int4(0, 0, 0, 0);
    typename T::Frag bx[T::KS];
    T::load_row(bx, X, (int64_t)q.x, d, grp, vec, need);
    const double D1 = chain_dist<T>(bx, need, q.y, C64, d, grp, lane);
    const double D2 = chain_dist<T>(bx, need, q.z, C64, d, grp, lane);
    if (need && grp == 0) {
      const bool second = D2 < D1 || (D2 == D1 && q.z < q.y);
      chg += commit_label(q.x, q.w, second ? q.z : q.y,
                          pair_bound(second ? D2 : D1, d), labels, ub, dirty);
    }
  }
  return chg;
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
  stage_batched<8, int>(
      nseg, [&](int e) { return seg_cnt[e]; },
      [&](int e, int c) {
        if (nseg <= kSegCache) sSeg[e] = c;
        const int t = (c + up - 1) / up;
        mx = t > mx ? t : mx;
      });
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
__device__ __forceinline__ int append_flags(bool flag, int pid, int* sFlag,
                                            int* __restrict__ slice, int lane) {
  const uint64_t fm = __ballot(flag);
  if (fm == 0) return 0;
  const int total = __popcll(fm);
  int base = 0;
  if (lane == 0) base = atomicAdd(sFlag, total);           // LDS
  base = __shfl(base, 0);
  if (flag) slice[base + __popcll(fm & lanemask_lt())] = pid;
  return total;
}

}  // namespace knor
