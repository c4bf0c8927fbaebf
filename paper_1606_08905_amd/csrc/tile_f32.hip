// FP32 matrix-core distance tile with the argmin fused into its epilogue
// (the nearest-centroid loop of Mhembere et al., HPDC'17, Algorithm 1).
//
// For a point x and centroid c the tile computes y = |c|^2 - 2 x.c on
// v_mfma_f32_16x16x4f32: the accumulator starts at fp32(|c|^2) and the A
// operand holds -2 * fp32(c) (an exact scaling).  The epilogue keeps, per
// point, the smallest y, its centroid index and the second smallest y.
//
// Lane layout of v_mfma_f32_16x16x4f32 used here: lane l = 16*g + c supplies
// A[c][g] and B[g][c] and receives D[4g + r][c], r = 0..3.  Rows of A are
// centroids, columns of B are points, so every lane owns one point column
// and reduces over the 4 centroid rows it receives.  The contraction index
// is permuted so that lane group g owns the KS = DP/4 consecutive dimensions
// [g*KS, (g+1)*KS) of both operands.
//
// Rounding bound (u = 2^-24, R^2 >= max_j |c_j|^2, |x| the point norm): the
// FP32 result y_j differs from the exact |c_j|^2 - 2 x.c_j by at most
//   E = u * ((2d + 5) R^2 + (4d + 10) |x| R) * (1 + 2^-10),
// which covers the rounding of c to FP32, of |c|^2 to FP32, of every product
// and of every accumulation step (each counted with 2u, so that any faithful
// rounding inside the matrix core is covered).  The point is decided by the
// tile iff  y_2nd - y_best > 2E + 2.01 (d+2) 2^-53 (|x|^2 + y_best + E):
// then every other centroid's exact squared distance exceeds the best one's
// by more than the FP64 evaluation error of the definition, so the FP64
// argmin (and its lowest-index rule) must select the same centroid.  Every
// other point goes to its unit's slice of the FP64 recheck list.
//
// Two schedules:
//  resident  all centroids fit in LDS: staged once per workgroup, then each
//            wave works through its own 16*PB-point units with no barrier;
//  chunked   centroids stream through LDS in chunks shared by the four
//            waves of a workgroup, which finalise 64*PB-point units.
#include <math.h>

#include "common.h"

namespace knor {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kTileThreads = 256;
constexpr size_t kResidentLds = 65536;

template <int DP>
struct F32Tile {
  static constexpr int KS = DP / 4;                    // dims per lane group
  static constexpr int PB = DP >= 256 ? 1 : (DP >= 128 ? 2 : 4);
  static constexpr int LDA = DP + 4;                   // LDS row stride
  static constexpr int CK = (4096 / DP) < 16 ? 16 : (4096 / DP);
  static constexpr int WUP = 16 * PB;                  // points per wave unit
  static constexpr int BUP = 4 * WUP;                  // points per block unit
};

static int pb_of(int dp) { return dp >= 256 ? 1 : (dp >= 128 ? 2 : 4); }

bool tile_f32_resident(int dp, int kpad) {
  return (size_t)kpad * (dp + 4) * 4 + (size_t)kpad * 4 <= kResidentLds;
}

int tile_f32_unit_points(int dp, int kpad) {
  return (tile_f32_resident(dp, kpad) ? 16 : 64) * pb_of(dp);
}

// min / max without NaN canonicalisation (inputs are finite or +inf)
__device__ __forceinline__ float fmin_nc(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, -INFINITY);
}
__device__ __forceinline__ float fmax_nc(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, INFINITY);
}

template <int KS>
__device__ __forceinline__ void load_slice(float (&dst)[KS], const float* src) {
  if constexpr (KS % 4 == 0) {
#pragma unroll
    for (int s = 0; s < KS; s += 4) {
      float4 v = *reinterpret_cast<const float4*>(src + s);
      dst[s] = v.x; dst[s + 1] = v.y; dst[s + 2] = v.z; dst[s + 3] = v.w;
    }
  } else {
    static_assert(KS % 2 == 0, "slice width");
#pragma unroll
    for (int s = 0; s < KS; s += 2) {
      float2 v = *reinterpret_cast<const float2*>(src + s);
      dst[s] = v.x; dst[s + 1] = v.y;
    }
  }
}

// Per-wave state for PB blocks of 16 points.
template <int DP>
struct WaveState {
  static constexpr int KS = F32Tile<DP>::KS, PB = F32Tile<DP>::PB;
  float bx[PB][KS];
  int64_t pid[PB];
  bool valid[PB];
  double xs[PB];
  float b1[PB], b2[PB];
  int i1[PB];
};

// Load the wave's points q0 + pb*16 + col (pb < PB) of a range of length m;
// with a list, point = list[base + q].
template <int DP>
__device__ __forceinline__ void load_points(WaveState<DP>& w,
                                            const float* __restrict__ X, int d,
                                            int vec, const int* __restrict__ list,
                                            int64_t base, int64_t q0, int64_t m,
                                            int col, int grp) {
  constexpr int KS = F32Tile<DP>::KS, PB = F32Tile<DP>::PB;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t q = q0 + pb * 16 + col;
    w.valid[pb] = q < m;
    const int64_t p = w.valid[pb] ? (list ? (int64_t)list[base + q] : q) : 0;
    w.pid[pb] = p;
    const float* xr = X + (size_t)p * d + grp * KS;
    if (w.valid[pb] && vec) {
      load_slice<KS>(w.bx[pb], xr);
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int dim = grp * KS + s;
        w.bx[pb][s] = (w.valid[pb] && dim < d) ? xr[s] : 0.0f;
      }
    }
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const double v = (double)w.bx[pb][s];
      acc = acc + v * v;
    }
    w.xs[pb] = acc;
    w.b1[pb] = INFINITY;
    w.b2[pb] = INFINITY;
    w.i1[pb] = 0;
  }
}

// One block of 16 centroids (rows of A from LDS, norms as the accumulator
// seed) against the wave's PB point blocks.  The PB accumulation chains are
// interleaved so consecutive matrix instructions are independent.
template <int DP>
__device__ __forceinline__ void tile_block(WaveState<DP>& w, const float* arow,
                                           const float* nrow, int jb) {
  constexpr int KS = F32Tile<DP>::KS, PB = F32Tile<DP>::PB;
  float a[KS];
  load_slice<KS>(a, arow);
  f4 init;
  init[0] = nrow[0]; init[1] = nrow[1]; init[2] = nrow[2]; init[3] = nrow[3];
  f4 acc[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) acc[pb] = init;
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
      acc[pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], w.bx[pb][s], acc[pb], 0, 0, 0);
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float y = acc[pb][r];
      w.b2[pb] = __builtin_amdgcn_fmed3f(w.b1[pb], w.b2[pb], y);
      const bool lt = y < w.b1[pb];
      w.i1[pb] = lt ? (jb + r) : w.i1[pb];
      w.b1[pb] = fmin_nc(w.b1[pb], y);
    }
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

// Combine the four lane groups (each saw a different quarter of centroids).
template <int DP>
__device__ __forceinline__ void merge_groups(WaveState<DP>& w) {
  constexpr int PB = F32Tile<DP>::PB;
#pragma unroll
  for (int off = 16; off <= 32; off <<= 1) {
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const float ob1 = __shfl_xor(w.b1[pb], off);
      const float ob2 = __shfl_xor(w.b2[pb], off);
      const int oi1 = __shfl_xor(w.i1[pb], off);
      w.xs[pb] += __shfl_xor(w.xs[pb], off);
      const float nb2 = fmin_nc(fmax_nc(w.b1[pb], ob1), fmin_nc(w.b2[pb], ob2));
      const bool take = ob1 < w.b1[pb] || (ob1 == w.b1[pb] && oi1 < w.i1[pb]);
      w.i1[pb] = take ? oi1 : w.i1[pb];
      w.b1[pb] = fmin_nc(w.b1[pb], ob1);
      w.b2[pb] = nb2;
    }
  }
}

// Decide each point (lane group g finalises point block pb with pb % 4 == g).
// Writes labels / bounds of decided points; returns per-block flags.
template <int DP>
__device__ __forceinline__ void finalize_points(
    WaveState<DP>& w, float cmax, int d, int grp, int recheck_all,
    int32_t* __restrict__ labels, float* __restrict__ ub, int* __restrict__ dirty,
    bool (&flag)[F32Tile<DP>::PB], bool& changed) {
  constexpr int PB = F32Tile<DP>::PB;
  static_assert(PB <= 4, "one finalised point per lane");
  const double R2 = (double)cmax * (1.0 + 2.384185791015625e-07);  // 1+2^-22
  const double u24 = 5.9604644775390625e-08;                        // 2^-24
  const double e64 = (double)(d + 2) * 1.1102230246251565e-16;     // (d+2)2^-53
  changed = false;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    flag[pb] = false;
    if (!(w.valid[pb] && (pb & 3) == grp)) continue;
    const double xn2 = w.xs[pb] * (1.0 + (double)(d + 4) * 2.220446049250313e-16);
    const double E = u24 * ((2.0 * d + 5.0) * R2 + (4.0 * d + 10.0) * sqrt(xn2 * R2)) *
                     (1.0 + 9.765625e-04);
    const double y1 = (double)w.b1[pb], y2 = (double)w.b2[pb];
    double dbest = xn2 + y1 + E;
    if (!(dbest > 0.0)) dbest = 0.0;
    const double thr = 2.0 * E + 2.01 * e64 * dbest;
    const double gap = y2 - y1;
    flag[pb] = recheck_all || !(gap > thr);
    if (!flag[pb]) {
      const int64_t p = w.pid[pb];
      const int32_t old = labels[p];
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
// so that occupied units spread over the grid.
__device__ __forceinline__ bool unit_range(int64_t unit, int up, int64_t n,
                                           const int* __restrict__ seg_cnt,
                                           int nseg, int64_t& q0, int64_t& m,
                                           int64_t& base) {
  if (seg_cnt) {
    const int64_t t = unit / nseg;
    const int s = (int)(unit - t * nseg);
    m = seg_cnt[s];
    q0 = t * up;
    base = (int64_t)s * kSeg;
    return q0 < m;
  }
  m = n;
  q0 = unit * up;
  base = 0;
  return true;
}

template <int DP>
__global__ __launch_bounds__(kTileThreads) void tile_f32_resident_kernel(
    const float* __restrict__ X, int64_t n, int d,
    const float* __restrict__ Cm2, const float* __restrict__ cn, int k,
    int kpad, const int* __restrict__ list, const int* __restrict__ seg_cnt,
    int nseg, int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ flags, int* __restrict__ ucnt,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int* __restrict__ dirty, int recheck_all, int vec) {
  using T = F32Tile<DP>;
  constexpr int LDA = T::LDA, PB = T::PB, WUP = T::WUP;
  extern __shared__ __attribute__((aligned(16))) float smem[];
  float* sC = smem;
  float* sN = smem + (size_t)kpad * LDA;
  if (*conv < iter) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;

  for (int e = threadIdx.x; e < kpad * (DP / 4); e += kTileThreads) {
    const int r = e / (DP / 4), q4 = e - r * (DP / 4);
    *reinterpret_cast<float4*>(&sC[r * LDA + q4 * 4]) =
        *reinterpret_cast<const float4*>(Cm2 + (size_t)r * DP + q4 * 4);
  }
  for (int e = threadIdx.x; e < kpad; e += kTileThreads) sN[e] = cn[e];
  __syncthreads();
  const float cmax = chunk_cmax(sN, kpad, 0, k, lane);

  const int64_t nwu = seg_cnt ? (int64_t)nseg * (kSeg / WUP) : (n + WUP - 1) / WUP;
  WaveState<DP> w;
  unsigned long long tot_flag = 0, tot_chg = 0;
  for (int64_t wu = (int64_t)blockIdx.x * 4 + wave; wu < nwu;
       wu += (int64_t)gridDim.x * 4) {
    int64_t q0, m, base;
    if (!unit_range(wu, WUP, n, seg_cnt, nseg, q0, m, base)) {
      if (lane == 0) ucnt[wu] = 0;
      continue;
    }
    load_points<DP>(w, X, d, vec, list, base, q0, m, col, grp);
    for (int cb = 0; cb < kpad; cb += 16)
      tile_block<DP>(w, &sC[(cb + col) * LDA + grp * T::KS], &sN[cb + 4 * grp],
                     cb + 4 * grp);
    merge_groups<DP>(w);
    bool flag[PB], changed;
    finalize_points<DP>(w, cmax, d, grp, recheck_all, labels, ub, dirty, flag,
                        changed);
    int nf = 0;
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const uint64_t fm = __ballot(flag[pb]);
      if (flag[pb]) flags[wu * WUP + nf + __popcll(fm & lanemask_lt())] = (int)w.pid[pb];
      nf += __popcll(fm);
    }
    const int nc = __popcll(__ballot(changed));
    if (lane == 0) {
      ucnt[wu] = nf;
      tot_flag += nf;
      tot_chg += nc;
    }
  }
  const int q[2] = {SLOT_FLAGGED, SLOT_CHANGED};
  const unsigned long long v[2] = {tot_flag, tot_chg};
  block_add_slots<2>(row, q, v);
}

template <int DP>
__global__ __launch_bounds__(kTileThreads) void tile_f32_chunked_kernel(
    const float* __restrict__ X, int64_t n, int d,
    const float* __restrict__ Cm2, const float* __restrict__ cn, int k,
    int kpad, const int* __restrict__ list, const int* __restrict__ seg_cnt,
    int nseg, int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ flags, int* __restrict__ ucnt,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int* __restrict__ dirty, int recheck_all, int vec) {
  using T = F32Tile<DP>;
  constexpr int LDA = T::LDA, PB = T::PB, CK = T::CK, WUP = T::WUP, BUP = T::BUP;
  __shared__ __attribute__((aligned(16))) float sC[CK * LDA];
  __shared__ float sN[CK];
  __shared__ int sFlag, sChg;
  if (*conv < iter) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t units = seg_cnt ? (int64_t)nseg * (kSeg / BUP) : (n + BUP - 1) / BUP;

  WaveState<DP> w;
  unsigned long long tot_flag = 0, tot_chg = 0;
  for (int64_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    int64_t q0, m, base;
    if (!unit_range(unit, BUP, n, seg_cnt, nseg, q0, m, base)) {
      if (threadIdx.x == 0) ucnt[unit] = 0;
      continue;                                // uniform over the workgroup
    }
    load_points<DP>(w, X, d, vec, list, base, q0 + wave * WUP, m, col, grp);
    float cmax = 0.0f;
    for (int c0 = 0; c0 < kpad; c0 += CK) {
      const int cc = (kpad - c0) < CK ? (kpad - c0) : CK;
      __syncthreads();
      if (c0 == 0 && threadIdx.x == 0) { sFlag = 0; sChg = 0; }
      for (int e = threadIdx.x; e < cc * (DP / 4); e += kTileThreads) {
        const int r = e / (DP / 4), q4 = e - r * (DP / 4);
        *reinterpret_cast<float4*>(&sC[r * LDA + q4 * 4]) =
            *reinterpret_cast<const float4*>(Cm2 + (size_t)(c0 + r) * DP + q4 * 4);
      }
      for (int e = threadIdx.x; e < cc; e += kTileThreads) sN[e] = cn[c0 + e];
      __syncthreads();
      cmax = fmax_nc(cmax, chunk_cmax(sN, cc, c0, k, lane));
      for (int cb = 0; cb < cc; cb += 16)
        tile_block<DP>(w, &sC[(cb + col) * LDA + grp * T::KS], &sN[cb + 4 * grp],
                       c0 + cb + 4 * grp);
    }
    merge_groups<DP>(w);
    bool flag[PB], changed;
    finalize_points<DP>(w, cmax, d, grp, recheck_all, labels, ub, dirty, flag,
                        changed);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const uint64_t fm = __ballot(flag[pb]);
      if (fm) {
        int fb = 0;
        if (lane == __ffsll((unsigned long long)fm) - 1) fb = atomicAdd(&sFlag, __popcll(fm));
        fb = __shfl(fb, __ffsll((unsigned long long)fm) - 1);
        if (flag[pb]) flags[unit * BUP + fb + __popcll(fm & lanemask_lt())] = (int)w.pid[pb];
      }
    }
    const uint64_t cm = __ballot(changed);
    if (cm && lane == __ffsll((unsigned long long)cm) - 1) atomicAdd(&sChg, __popcll(cm));
    __syncthreads();
    if (threadIdx.x == 0) {
      ucnt[unit] = sFlag;
      tot_flag += sFlag;
      tot_chg += sChg;
    }
  }
  const int q[2] = {SLOT_FLAGGED, SLOT_CHANGED};
  const unsigned long long v[2] = {tot_flag, tot_chg};
  block_add_slots<2>(row, q, v);
}

template <int DP>
static hipError_t launch_dp(const CentroidOps& o, const AssignJob& j,
                            hipStream_t s) {
  using T = F32Tile<DP>;
  const int vec = (int)(j.d == DP && ((uintptr_t)j.X & 15) == 0);
  const bool seg = j.seg_cnt != nullptr;
  if (tile_f32_resident(DP, o.kpad)) {
    const int64_t nwu = seg ? (int64_t)j.nseg * (kSeg / T::WUP) : (j.n + T::WUP - 1) / T::WUP;
    int64_t blocks = (nwu + 3) / 4;
    const int grid = (int)(blocks < 1024 ? (blocks < 1 ? 1 : blocks) : 1024);
    const size_t lds = (size_t)o.kpad * T::LDA * 4 + (size_t)o.kpad * 4;
    hipLaunchKernelGGL(tile_f32_resident_kernel<DP>, dim3(grid), dim3(kTileThreads),
                       lds, s, (const float*)j.X, j.n, j.d, o.Cm2, o.cn, o.k,
                       o.kpad, j.list, j.seg_cnt, j.nseg, j.labels, j.u, j.flags,
                       j.ucnt, j.row, j.conv, j.iter, j.dirty, j.recheck_all, vec);
  } else {
    const int64_t units = seg ? (int64_t)j.nseg * (kSeg / T::BUP) : (j.n + T::BUP - 1) / T::BUP;
    const int grid = (int)(units < 2048 ? (units < 1 ? 1 : units) : 2048);
    hipLaunchKernelGGL(tile_f32_chunked_kernel<DP>, dim3(grid), dim3(kTileThreads),
                       0, s, (const float*)j.X, j.n, j.d, o.Cm2, o.cn, o.k,
                       o.kpad, j.list, j.seg_cnt, j.nseg, j.labels, j.u, j.flags,
                       j.ucnt, j.row, j.conv, j.iter, j.dirty, j.recheck_all, vec);
  }
  return hipGetLastError();
}

hipError_t launch_tile_f32(const CentroidOps& o, const AssignJob& j,
                           hipStream_t s) {
  switch (o.dp) {
    case 8: return launch_dp<8>(o, j, s);
    case 16: return launch_dp<16>(o, j, s);
    case 32: return launch_dp<32>(o, j, s);
    case 64: return launch_dp<64>(o, j, s);
    case 128: return launch_dp<128>(o, j, s);
    case 256: return launch_dp<256>(o, j, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace knor
