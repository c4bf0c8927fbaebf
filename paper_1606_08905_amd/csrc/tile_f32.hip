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
// argmin (and its lowest-index rule) must select the same centroid.  A point
// for which only the third smallest clears that margin is resolved after
// the workgroup's last unit from the canonical FP64 distances to its two
// best centroids.  Every other point goes to its workgroup's slice of the
// FP64 recheck list.
//
// Two schedules:
//  resident  all centroids fit in LDS: staged once per workgroup, then each
//            wave works through its own 16*PB-point units with no barrier;
//  chunked   centroids stream through LDS in chunks shared by the four
//            waves of a workgroup, which finalise 64*PB-point units.
#include <math.h>

#include "tile_f32.h"

namespace knor {

constexpr size_t kResidentLds = 65536;
#ifndef KNOR_RESIDENT_GRID
#define KNOR_RESIDENT_GRID 1024
#endif
constexpr int kResidentGrid = KNOR_RESIDENT_GRID;
constexpr int kChunkedGrid = kTileMaxGrid;
static_assert(kResidentGrid <= kTileMaxGrid, "grid bound");

// Point blocks of 16 per wave: fewer for wide rows (register budget).
constexpr int res_pb(int dp) { return dp >= 128 ? 1 : 2; }
constexpr int chk_pb(int dp) { return dp >= 256 ? 1 : (dp >= 128 ? 2 : 4); }

bool tile_f32_resident(int dp, int kpad) {
  return (size_t)kpad * (dp + 4) * 4 + (size_t)kpad * 4 <= kResidentLds;
}

// Point blocks per wave that fit the register budget of a row width.
bool tile_f32_pb_ok(int dp, int pb) {
  if (pb != 1 && pb != 2 && pb != 4) return false;
  if (dp >= 256) return pb == 1;
  if (dp >= 128) return pb <= 2;
  return true;
}

void tile_f32_default(int dp, int kpad, int* pb, int* resident) {
  *resident = tile_f32_resident(dp, kpad) ? 1 : 0;
  *pb = *resident ? res_pb(dp) : chk_pb(dp);
}

TileGeom tile_f32_geometry(int dp, int kpad, int pb, int resident, int64_t n,
                           bool seg, int nseg) {
  (void)dp;
  (void)kpad;
  TileGeom g{};
  g.resident = resident != 0;
  if (g.resident) {
    const int wup = 16 * pb;
    const int64_t nwu = seg ? (int64_t)nseg * (kSeg / wup) : (n + wup - 1) / wup;
    int64_t blocks = (nwu + 3) / 4;
    g.grid = (int)(blocks < kResidentGrid ? (blocks < 1 ? 1 : blocks) : kResidentGrid);
    const int64_t per_wave = (nwu + 4LL * g.grid - 1) / (4LL * g.grid);
    g.cap = per_wave * 4 * wup;
  } else {
    const int bup = 64 * pb;
    const int64_t units = seg ? (int64_t)nseg * (kSeg / bup) : (n + bup - 1) / bup;
    g.grid = (int)(units < kChunkedGrid ? (units < 1 ? 1 : units) : kChunkedGrid);
    g.cap = (units + g.grid - 1) / g.grid * bup;
  }
  return g;
}

TileGeom tile_geometry(const CentroidOps& o, knor_dtype dt, int64_t n,
                       bool seg, int nseg) {
  if (dt == KNOR_BF16) return tile_bf16_geometry(o.dpb, o.kpad, n, seg, nseg);
  return tile_f32_geometry(o.dp, o.kpad, o.tpb, o.tres, n, seg, nseg);
}

int64_t tile_flag_capacity(const CentroidOps& o, knor_dtype dt, int64_t n,
                           int nseg) {
  const TileGeom a = tile_geometry(o, dt, n, false, nseg);
  const TileGeom b = tile_geometry(o, dt, n, true, nseg);
  const int64_t ca = (int64_t)a.grid * a.cap, cb = (int64_t)b.grid * b.cap;
  return ca > cb ? ca : cb;
}

// Load the wave's points q0 + pb*16 + col (pb < PB) of a range of length m;
// with a list, point = list[base + q].  The lane group that will finalise a
// point block also fetches the points' previous labels here, so that the
// read overlaps the matrix work.
template <class T>
__device__ __forceinline__ void load_points(WaveState<T>& w,
                                            const float* __restrict__ X, int d,
                                            int vec, const int* __restrict__ list,
                                            const int32_t* __restrict__ labels,
                                            int64_t base, int64_t q0, int64_t m,
                                            int col, int grp) {
  constexpr int KS = T::KS, PB = T::PB;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t q = q0 + pb * 16 + col;
    w.valid[pb] = q < m;
    const int64_t p = w.valid[pb] ? (list ? (int64_t)list[base + q] : q) : 0;
    w.pid[pb] = p;
    w.old[pb] = (w.valid[pb] && (pb & 3) == grp) ? labels[p] : 0;
    T::load_row(w.bx[pb], X, p, d, grp, vec, w.valid[pb]);
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const double v = (double)w.bx[pb][s];
      acc = acc + v * v;
    }
    w.xs[pb] = acc;
    top3_reset(w.b1[pb], w.b2[pb], w.b3[pb], w.i1[pb], w.i2[pb]);
  }
}

// Two-candidate points of the resident schedule, whose main loop keeps no
// second index: each wave takes 16 queued points, sweeps them again over
// the staged centroids with the full state, and decides them again from
// those values; pairs are resolved from their two canonical FP64 distances,
// and a point that no longer qualifies is decided or appended to the
// recheck slice.  Returns this thread's count of changed labels.
template <int DP>
__device__ __forceinline__ unsigned long long resweep_pairs(
    const float* __restrict__ X, int d, int vec, const double* __restrict__ C64,
    const float* sC, const float* sN, int kpad, float cmax, const int4* sPair,
    int np, int* sFlag, int* __restrict__ slice, int32_t* __restrict__ labels,
    float* __restrict__ ub, int* __restrict__ dirty) {
  using T1 = F32Tile<DP, 1>;
  constexpr int KS = T1::KS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  unsigned long long chg = 0;
  for (int e0 = wave * 16; e0 < np; e0 += kTileThreads / 4) {
    const int e = e0 + col;
    const bool need = e < np;
    const int4 q = need ? sPair[e] : make_int4(0, 0, 0, 0);
    WaveState<T1> w;
    T1::load_row(w.bx[0], X, (int64_t)q.x, d, grp, vec, need);
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const double v = (double)w.bx[0][s];
      acc = acc + v * v;
    }
    w.xs[0] = acc;
    top3_reset(w.b1[0], w.b2[0], w.b3[0], w.i1[0], w.i2[0]);
    tile_sweep<T1, true>(w, sC, sN, kpad, 0, col, grp);
    merge_groups<T1, true>(w);
    const bool own = need && grp == 0;
    Decision dc{false, false, 0.0};
    if (own) dc = decide_point<T1>(w.xs[0], w.b1[0], w.b2[0], w.b3[0], cmax, d, false, true);
    // the chain runs over the four lanes of a column
    const bool pr = __shfl(dc.pair ? 1 : 0, col) != 0;
    double D1 = 0.0, D2 = 0.0;
    if (__ballot(pr)) {
      D1 = chain_dist<T1>(w.bx[0], pr, w.i1[0], C64, d, grp, lane);
      D2 = chain_dist<T1>(w.bx[0], pr, w.i2[0], C64, d, grp, lane);
    }
    bool flag = false;
    if (own) {
      if (dc.decided) {
        chg += commit_label(q.x, q.w, w.i1[0],
                            f32_up(sqrt(dc.dbest) * (1.0 + 8.881784197001252e-16)),
                            labels, ub, dirty);
      } else if (dc.pair) {
        const bool second = D2 < D1 || (D2 == D1 && w.i2[0] < w.i1[0]);
        chg += commit_label(q.x, q.w, second ? w.i2[0] : w.i1[0],
                            pair_bound(second ? D2 : D1, d), labels, ub, dirty);
      } else {
        flag = true;
      }
    }
    append_flags(flag, q.x, sFlag, slice, lane);
  }
  return chg;
}

template <int DP, int PB_>
__global__ __launch_bounds__(kTileThreads) void tile_f32_resident_kernel(
    const float* __restrict__ X, int64_t n, int d,
    const float* __restrict__ Cm2, const float* __restrict__ cn, int k,
    int kpad, const int* __restrict__ list, const int* __restrict__ seg_cnt,
    int nseg, int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ flags, int64_t cap, int* __restrict__ ucnt,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int* __restrict__ dirty, int recheck_all, int vec,
    const double* __restrict__ CT, const double* __restrict__ C64, int tpf_max,
    int fuse_max, int vecx) {
  using T = F32Tile<DP, PB_>;
  constexpr int LDA = T::LDA, PB = T::PB, WUP = T::WUP;
  extern __shared__ __attribute__((aligned(16))) float smem[];
  __shared__ int sFlag, sPairN;
  __shared__ int4 sPair[kPairCap];
  float* sC = smem;
  float* sN = smem + (size_t)kpad * LDA;
  const int cv = *conv;                        // tested after the staging loads
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const bool pairs = T::PAIR && C64 != nullptr;

  __shared__ int sSeg[kSegCache], sWmax[kTileThreads / 64];
  if (threadIdx.x == 0) { sFlag = 0; sPairN = 0; }
  if (seg_cnt) seg_stage(seg_cnt, nseg, WUP, sSeg, sWmax);
  stage_cents<T, 8>(sC, sN, Cm2, cn, 0, kpad);
  if (cv < iter) return;
  __syncthreads();
  const float cmax = chunk_cmax(sN, kpad, 0, k, lane);

  int* slice = flags + (int64_t)blockIdx.x * cap;
  int64_t nwu = seg_cnt ? (int64_t)nseg * (kSeg / WUP) : (n + WUP - 1) / WUP;
  if (seg_cnt) nwu = seg_units_bound(sWmax, nseg, nwu);
  const int* segc = (seg_cnt && nseg <= kSegCache) ? sSeg : nullptr;
  WaveState<T> w;
  unsigned long long tot_flag = 0, tot_chg = 0;
  for (int64_t wu = (int64_t)blockIdx.x * 4 + wave; wu < nwu;
       wu += (int64_t)gridDim.x * 4) {
    int64_t q0, m, base;
    if (!unit_range(wu, WUP, n, seg_cnt, segc, nseg, q0, m, base)) continue;
    load_points<T>(w, X, d, vec, list, labels, base, q0, m, col, grp);
    tile_sweep<T, false, true>(w, sC, sN, kpad, 0, col, grp);
    merge_groups<T, false>(w);
    bool flag, changed;
    int fp;
    finalize_points<T, false>(w, cmax, d, grp, recheck_all, pairs, sPair, &sPairN,
                              labels, ub, dirty, flag, fp, changed);
    const int nf = append_flags(flag, fp, &sFlag, slice, lane);
    const int nc = __popcll(__ballot(changed));
    if (lane == 0) {
      tot_flag += nf;
      tot_chg += nc;
    }
  }
  __syncthreads();
  const int np = sPairN < kPairCap ? sPairN : kPairCap;
  if constexpr (T::PAIR)
    if (np)
      tot_chg += resweep_pairs<DP>(X, d, vec, C64, sC, sN, kpad, cmax, sPair, np,
                                   &sFlag, slice, labels, ub, dirty);
  const int q[2] = {SLOT_FLAGGED, SLOT_CHANGED};
  const unsigned long long v[2] = {tot_flag + (threadIdx.x == 0 ? np : 0), tot_chg};
  block_add_slots<2>(row, q, v);               // includes a barrier
  const int left = recheck_own_slice<float>(X, d, vecx, CT, k, tpf_max, fuse_max, slice,
                                         sFlag, labels, ub, dirty, row);
  if (threadIdx.x == 0) ucnt[blockIdx.x] = left;
}

template <int DP, int PB_>
__global__ __launch_bounds__(kTileThreads) void tile_f32_chunked_kernel(
    const float* __restrict__ X, int64_t n, int d,
    const float* __restrict__ Cm2, const float* __restrict__ cn, int k,
    int kpad, const int* __restrict__ list, const int* __restrict__ seg_cnt,
    int nseg, int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ flags, int64_t cap, int* __restrict__ ucnt,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int* __restrict__ dirty, int recheck_all, int vec,
    const double* __restrict__ CT, const double* __restrict__ C64, int tpf_max,
    int fuse_max, int vecx) {
  using T = F32Tile<DP, PB_>;
  constexpr int LDA = T::LDA, PB = T::PB, CK = T::CK, WUP = T::WUP, BUP = T::BUP;
  __shared__ __attribute__((aligned(16))) float sC[CK * LDA];
  __shared__ __attribute__((aligned(16))) float sN[CK];
  __shared__ int sFlag, sChg, sPairN;
  __shared__ int4 sPair[kPairCap];
  const int cv = *conv;                        // tested after the first loads
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const bool pairs = T::PAIR && C64 != nullptr;
  __shared__ int sSeg[kSegCache], sWmax[kTileThreads / 64];
  int64_t units = seg_cnt ? (int64_t)nseg * (kSeg / BUP) : (n + BUP - 1) / BUP;
  if (threadIdx.x == 0) { sFlag = 0; sChg = 0; sPairN = 0; }
  if (seg_cnt) seg_stage(seg_cnt, nseg, BUP, sSeg, sWmax);
  if (cv < iter) return;
  __syncthreads();
  if (seg_cnt) units = seg_units_bound(sWmax, nseg, units);
  const int* segc = (seg_cnt && nseg <= kSegCache) ? sSeg : nullptr;

  int* slice = flags + (int64_t)blockIdx.x * cap;
  // every point meets every centroid: the rounding bound's largest norm is
  // the same for all units, taken once per wave
  const float cmax = all_cmax(cn, k, lane);
  WaveState<T> w;
  for (int64_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    int64_t q0, m, base;
    if (!unit_range(unit, BUP, n, seg_cnt, segc, nseg, q0, m, base))
      continue;                                // uniform over the workgroup
    load_points<T>(w, X, d, vec, list, labels, base, q0 + wave * WUP, m, col, grp);
    for (int c0 = 0; c0 < kpad; c0 += CK) {
      const int cc = (kpad - c0) < CK ? (kpad - c0) : CK;
      __syncthreads();
      stage_cents<T, 2>(sC, sN, Cm2, cn, c0, cc);     // point state is live here
      __syncthreads();
      tile_sweep<T, false>(w, sC, sN, cc, c0, col, grp);
    }
    // one index per point: a two-candidate point goes to the FP64 recheck
    // with the undecided ones (centroids are not resident for a re-sweep)
    merge_groups<T, false>(w);
    bool flag, changed;
    int fp;
    finalize_points<T, false>(w, cmax, d, grp, recheck_all, false, sPair, &sPairN,
                              labels, ub, dirty, flag, fp, changed);
    append_flags(flag, fp, &sFlag, slice, lane);
    const uint64_t cm = __ballot(changed);
    if (cm && lane == 0) atomicAdd(&sChg, __popcll(cm));
  }
  __syncthreads();
  const int np = sPairN < kPairCap ? sPairN : kPairCap;
  unsigned long long pch = 0;
  if constexpr (T::PAIR)
    if (np) pch = resolve_pairs<T, float>(X, d, vec, C64, sPair, np, labels, ub, dirty);
  const int q[2] = {SLOT_FLAGGED, SLOT_CHANGED};
  const unsigned long long v[2] = {threadIdx.x == 0 ? (unsigned long long)(sFlag + np) : 0ull,
                                   (threadIdx.x == 0 ? (unsigned long long)sChg : 0ull) + pch};
  block_add_slots<2>(row, q, v);               // includes a barrier
  const int left = recheck_own_slice<float>(X, d, vecx, CT, k, tpf_max, fuse_max, slice,
                                         sFlag, labels, ub, dirty, row);
  if (threadIdx.x == 0) ucnt[blockIdx.x] = left;
}

template <int DP, int PB>
static hipError_t launch_dp_pb(const CentroidOps& o, const AssignJob& j,
                               hipStream_t s) {
  const int vec = (int)(j.d == DP && ((uintptr_t)j.X & 15) == 0);
  const int vecx = (int)(j.d % 4 == 0 && ((uintptr_t)j.X & 15) == 0);
  const bool seg = j.seg_cnt != nullptr;
  const TileGeom g = tile_f32_geometry(DP, o.kpad, PB, o.tres, j.n, seg, j.nseg);
  if (g.resident) {
    using T = F32Tile<DP, PB>;
    const size_t lds = (size_t)o.kpad * T::LDA * 4 + (size_t)o.kpad * 4;
    if (lds > 49152) {   // with the static arrays, past the default 64 KB
      hipError_t e = hipFuncSetAttribute(
          reinterpret_cast<const void*>(&tile_f32_resident_kernel<DP, PB>),
          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((tile_f32_resident_kernel<DP, PB>), dim3(g.grid),
                       dim3(kTileThreads), lds, s, (const float*)j.X, j.n, j.d,
                       o.Cm2, o.cn, o.k, o.kpad, j.list, j.seg_cnt, j.nseg,
                       j.labels, j.u, j.flags, g.cap, j.ucnt, j.row, j.conv,
                       j.iter, j.dirty, j.recheck_all, vec, o.CT, o.C64, fuse_tpf(o.k),
                       j.recheck_all ? 0 : kFuseRecheckMax, vecx);
  } else {
    hipLaunchKernelGGL((tile_f32_chunked_kernel<DP, PB>), dim3(g.grid),
                       dim3(kTileThreads), 0, s, (const float*)j.X, j.n, j.d,
                       o.Cm2, o.cn, o.k, o.kpad, j.list, j.seg_cnt, j.nseg,
                       j.labels, j.u, j.flags, g.cap, j.ucnt, j.row, j.conv,
                       j.iter, j.dirty, j.recheck_all, vec, o.CT, o.C64, fuse_tpf(o.k),
                       j.recheck_all ? 0 : kFuseRecheckMax, vecx);
  }
  return hipGetLastError();
}

template <int DP>
static hipError_t launch_dp(const CentroidOps& o, const AssignJob& j,
                            hipStream_t s) {
  if (o.tres && !tile_f32_resident(DP, o.kpad)) return hipErrorInvalidValue;
  switch (o.tpb) {
    case 1: return launch_dp_pb<DP, 1>(o, j, s);
    case 2:
      if constexpr (DP < 256) return launch_dp_pb<DP, 2>(o, j, s);
      break;
    case 4:
      if constexpr (DP < 128) return launch_dp_pb<DP, 4>(o, j, s);
      break;
  }
  return hipErrorInvalidValue;
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

// ---------------------------------------------------------------------------
// the tile's values and bound, for checking the bound (knor_tile_values)
// ---------------------------------------------------------------------------

// Y[p][j] = the tile's FP32 value of |c_j|^2 - 2 x_p.c_j (the same operands
// and accumulation as every pass above), E[p] = the bound its decision uses
// with R^2 taken over all k centroids.  One wave per 16 points.
template <int DP>
__global__ __launch_bounds__(256) void tile_values_f32_kernel(
    const float* __restrict__ X, int64_t n, int d, const float* __restrict__ Cm2,
    const float* __restrict__ cn, int k, int kpad, float* __restrict__ Y,
    double* __restrict__ E, int vec) {
  using T = F32Tile<DP, 1>;
  constexpr int KS = T::KS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t p = ((int64_t)blockIdx.x * 4 + wave) * 16 + col;
  if (((int64_t)blockIdx.x * 4 + wave) * 16 >= n) return;
  float cmax = 0.0f;
  for (int j = lane; j < k; j += 64) cmax = fmax_nc(cmax, cn[j]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cmax = fmax_nc(cmax, __shfl_xor(cmax, o));
  float bx[1][KS];
  T::load_row(bx[0], X, p < n ? p : 0, d, grp, vec, p < n);
  double xs = 0.0;
#pragma unroll
  for (int s = 0; s < KS; ++s) {
    const double v = (double)bx[0][s];
    xs = xs + v * v;
  }
  xs += __shfl_xor(xs, 16);
  xs += __shfl_xor(xs, 32);
  for (int jb = 0; jb < kpad; jb += 16) {
    ABlock<T> o;
    load_ablock<T>(o, Cm2 + (size_t)(jb + col) * DP + grp * KS, cn + jb + 4 * grp);
    f4 acc[1];
    tile_block_acc<T>(acc, bx, o);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = jb + 4 * grp + r;
      if (p < n && j < k) Y[(size_t)p * k + j] = acc[0][r];
    }
  }
  if (grp == 0 && p < n) {
    const double R2 = (double)cmax * (1.0 + 2.384185791015625e-07);
    E[p] = T::bound(xs * (1.0 + (double)(d + 4) * 2.220446049250313e-16), R2, d);
  }
}

hipError_t launch_tile_values_f32(const CentroidOps& o, const float* X, int64_t n, int d,
                                  float* Y, double* E, hipStream_t s) {
  const dim3 grid((unsigned)((n + 63) / 64));
  auto go = [&](auto kern, int DP) {
    const int vec = (int)(d == DP && ((uintptr_t)X & 15) == 0);
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, X, n, d, o.Cm2, o.cn, o.k, o.kpad, Y, E,
                       vec);
    return hipGetLastError();
  };
  switch (o.dp) {
    case 8: return go(tile_values_f32_kernel<8>, 8);
    case 16: return go(tile_values_f32_kernel<16>, 16);
    case 32: return go(tile_values_f32_kernel<32>, 32);
    case 64: return go(tile_values_f32_kernel<64>, 64);
    case 128: return go(tile_values_f32_kernel<128>, 128);
    case 256: return go(tile_values_f32_kernel<256>, 256);
  }
  return hipErrorInvalidValue;
}

}  // namespace knor
