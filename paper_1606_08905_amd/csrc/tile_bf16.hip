// BF16 matrix-core distance tile with the argmin fused into its epilogue
// (the nearest-centroid loop of Mhembere et al., HPDC'17, Algorithm 1) for
// points stored as BF16.
//
// The points are exact BF16 operands.  The centroid operand is -2c split
// into two BF16 terms, A_hi = bf16(-2c) and A_lo = bf16(-2c - A_hi) (the
// difference is exact in FP64), so that |-2c - A_hi - A_lo| <= 2^-15 |c| per
// element (+2^-134 below the normal range).  Both terms go through
// v_mfma_f32_16x16x32_bf16 into one FP32 accumulator seeded with
// fp32(|c|^2): y~_j approximates y_j = |c_j|^2 - 2 x.c_j.
//
// Rounding bound (u = 2^-24, R^2 >= max_j |c_j|^2, dp the padded dimension):
//   E = [u R^2 + 2u (2 dp + 1)(R^2 + 2.02 |x| R) + 2^-15 |x| R
//        + 2^-100 (1 + R)(1 + |x|)] (1 + 2^-10)
// covering the rounding of |c|^2 to FP32, the accumulation of the 2 dp + 1
// terms (every product of two BF16 values is exact in FP32; each step is
// counted at 2u of the running sum of magnitudes, so any faithful rounding
// inside the matrix core is covered; sum of magnitudes <= R^2 + 2.02|x|R),
// the two-term representation of -2c, and subnormals flushed by the matrix
// core.  The decision rule and the FP64 recheck of undecided points are the
// FP32 tile's (tile_common.h); the two-candidate pass is not used here.
//
// Lane layout: lane l = 16 g + c supplies eight consecutive elements
// [8g, 8g + 8) of the 32-element K-step for row c of A (a centroid) and
// column c of B (a point), and receives D[4g + r][c], r = 0..3 -- A and B
// use the same K-index mapping, so the contraction pairs equal dimensions.
//
// Two schedules (as for FP32): resident (hi and lo copies of all centroids
// in LDS, staged once per workgroup; each wave works through 16*PB-point
// units without barriers) and chunked (centroid chunks shared by the four
// waves of a workgroup).  Four point blocks per wave at dp <= 64 give each
// LDS fragment four uses, which keeps LDS reads under the matrix rate.
#include <math.h>

#include "tile_common.h"

namespace knor {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr size_t kBfResidentLds = 81920;   // at most two workgroups per CU
constexpr int kBfChunkedGrid = kTileMaxGrid;

constexpr int bf_pb(int dp) { return dp <= 64 ? 4 : (dp <= 128 ? 2 : 1); }
constexpr int bf_ck(int dp) {
  return dp <= 32 ? 256 : (dp <= 64 ? 128 : (dp <= 128 ? 64 : 32));
}

template <int DP>
struct Bf16Tile {
  using Frag = bf8;
  static constexpr int KS = DP / 32;                   // K-steps per row
  static constexpr int PB = bf_pb(DP);
  static constexpr int LDA = DP + 8;                   // LDS row stride (bf16)
  static constexpr int CK = bf_ck(DP);                 // chunk of centroids
  static constexpr int WUP = 16 * PB;                  // points per wave unit
  static constexpr int BUP = 4 * WUP;                  // points per block unit
  // lane group g holds dimensions [32 s + 8 g, 32 s + 8 g + 8) of K-step s.
  // The two-candidate pass stays off: with four point blocks per wave the
  // third value and second index add registers that cost one wave per SIMD
  // at dp = 64, which costs more than the full recheck it saves.
  static constexpr bool PAIR = false;
  static constexpr int NS = KS, NE = 8;
  __device__ static constexpr int dim(int s, int g, int e) { return 32 * s + 8 * g + e; }
  __device__ static double xval(const Frag (&bx)[KS], int s, int e) {
    const uint4 v = __builtin_bit_cast(uint4, bx[s]);
    const uint32_t wd = (e >> 1) == 0 ? v.x : ((e >> 1) == 1 ? v.y : ((e >> 1) == 2 ? v.z : v.w));
    return (double)__uint_as_float((e & 1) ? (wd & 0xffff0000u) : (wd << 16));
  }
  // this lane group's dimensions of row p as B fragments (zero past d or
  // when !valid)
  __device__ static void load_row(Frag (&bx)[KS], const uint16_t* __restrict__ X,
                                  int64_t p, int d, int grp, int vec, bool valid) {
    const uint16_t* xr = X + (size_t)p * d;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int d0 = s * 32 + grp * 8;
      uint32_t wd[4];
      if (valid && vec && d0 + 8 <= d) {
        const uint4 v = *reinterpret_cast<const uint4*>(xr + d0);
        wd[0] = v.x; wd[1] = v.y; wd[2] = v.z; wd[3] = v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t lo = (valid && d0 + 2 * e < d) ? xr[d0 + 2 * e] : 0u;
          const uint32_t hi = (valid && d0 + 2 * e + 1 < d) ? xr[d0 + 2 * e + 1] : 0u;
          wd[e] = lo | (hi << 16);
        }
      }
      const uint4 v4 = {wd[0], wd[1], wd[2], wd[3]};
      bx[s] = __builtin_bit_cast(bf8, v4);
    }
  }
  // load_row for loads that stay in flight across other work: with vec, the
  // loads are unconditional (row 0 stands in for an invalid point and the
  // value is replaced by zero afterwards), so no branch joins with a load
  // outstanding
  template <bool VEC>
  __device__ static void load_row_ahead(Frag (&bx)[KS], const uint16_t* __restrict__ X,
                                        int64_t p, int d, int grp, bool valid) {
    if constexpr (!VEC) {
      load_row(bx, X, p, d, grp, 0, valid);
      return;
    }
    const uint16_t* xr = X + (size_t)(valid ? p : 0) * d;
    uint4 v[KS];
#pragma unroll
    for (int s = 0; s < KS; ++s) v[s] = *reinterpret_cast<const uint4*>(xr + s * 32 + grp * 8);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const uint4 z = {0u, 0u, 0u, 0u};
      bx[s] = __builtin_bit_cast(bf8, valid ? v[s] : z);
    }
  }
  __device__ static double bound(double xn2, double R2, int) {
    const double u24 = 5.9604644775390625e-08;
    const double xn = sqrt(xn2), R = sqrt(R2);
    const double xr = xn * R;
    return (u24 * R2 + 2.0 * u24 * (2.0 * DP + 1.0) * (R2 + 2.02 * xr) +
            3.0517578125e-05 * xr +                       // 2^-15
            7.888609052210118e-31 * (1.0 + R) * (1.0 + xn)) *   // 2^-100
           (1.0 + 9.765625e-04);
  }
};

static size_t bf_resident_bytes(int dp, int kpad) {
  return (size_t)kpad * (dp + 8) * 2 * 2 + (size_t)kpad * 4;
}

static size_t device_lds_limit() {
  int dev = 0, v = 65536;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
          hipSuccess)
    v = 65536;
  return (size_t)v;
}

bool tile_bf16_resident(int dp, int kpad) {
  const size_t need = bf_resident_bytes(dp, kpad);
  const size_t lim = device_lds_limit();
  return need <= kBfResidentLds && need <= lim;
}

TileGeom tile_bf16_geometry(int dp, int kpad, int64_t n, bool seg, int nseg) {
  TileGeom g{};
  g.resident = tile_bf16_resident(dp, kpad);
  const int pb = bf_pb(dp);
  if (g.resident) {
    const int wup = 16 * pb;
    const int64_t nwu = seg ? (int64_t)nseg * (kSeg / wup) : (n + wup - 1) / wup;
    const size_t per_cu = 163840 / bf_resident_bytes(dp, kpad);
    const int cap_grid = 256 * (int)(per_cu < 1 ? 1 : (per_cu > 4 ? 4 : per_cu));
    const int64_t blocks = (nwu + 3) / 4;
    g.grid = (int)(blocks < cap_grid ? (blocks < 1 ? 1 : blocks) : cap_grid);
    const int64_t per_wave = (nwu + 4LL * g.grid - 1) / (4LL * g.grid);
    g.cap = per_wave * 4 * wup;
  } else {
    const int bup = 64 * pb;
    const int64_t units = seg ? (int64_t)nseg * (kSeg / bup) : (n + bup - 1) / bup;
    g.grid = (int)(units < kBfChunkedGrid ? (units < 1 ? 1 : units) : kBfChunkedGrid);
    g.cap = (units + g.grid - 1) / g.grid * bup;
  }
  return g;
}

// The wave's points q0 + pb*16 + col of a range of length m (through the
// list when given), as B fragments; dimensions past d are zero.  Also the
// FP64 partial |x|^2 over this lane group's dimensions and, for the lane
// group that finalises the block, the previous label.
template <class T>
__device__ __forceinline__ void load_points_bf(
    WaveState<T>& w, const uint16_t* __restrict__ X, int d, int vec,
    const int* __restrict__ list, const int32_t* __restrict__ labels,
    int64_t base, int64_t q0, int64_t m, int col, int grp) {
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
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double v = T::xval(w.bx[pb], s, e);
        acc = acc + v * v;
      }
    w.xs[pb] = acc;
    top3_reset(w.b1[pb], w.b2[pb], w.b3[pb], w.i1[pb], w.i2[pb]);
  }
}

// load_points_bf in two halves for a pipelined unit loop: the loads of a
// unit's rows and labels (indices given), and, once they are needed, the
// squared norms and the reset of the running minima.
template <class T, bool VEC>
__device__ __forceinline__ void issue_points_bf(WaveState<T>& w, const uint16_t* __restrict__ X,
                                                int d, const int32_t* __restrict__ labels,
                                                bool listed, const int64_t (&q)[T::PB],
                                                const int (&raw)[T::PB],
                                                const bool (&valid)[T::PB], int grp) {
#pragma unroll
  for (int pb = 0; pb < T::PB; ++pb) {
    const int64_t pid = valid[pb] ? (listed ? (int64_t)raw[pb] : q[pb]) : 0;
    w.valid[pb] = valid[pb];
    w.pid[pb] = pid;
    w.old[pb] = labels[pid];                  // unconditional (point 0 stands in); see finish
    T::template load_row_ahead<VEC>(w.bx[pb], X, pid, d, grp, valid[pb]);
  }
}

template <class T>
__device__ __forceinline__ void finish_points_bf(WaveState<T>& w, int grp) {
#pragma unroll
  for (int pb = 0; pb < T::PB; ++pb) {
    w.old[pb] = (w.valid[pb] && (pb & 3) == grp) ? w.old[pb] : 0;
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < T::KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double v = T::xval(w.bx[pb], s, e);
        acc = acc + v * v;
      }
    w.xs[pb] = acc;
    top3_reset(w.b1[pb], w.b2[pb], w.b3[pb], w.i1[pb], w.i2[pb]);
  }
}

template <class T>
struct ABlockBf {
  bf8 hi[T::KS], lo[T::KS];
  f4 init;
};

template <class T>
__device__ __forceinline__ void load_ablock_bf(ABlockBf<T>& o, const uint16_t* hrow,
                                               const uint16_t* lrow,
                                               const float* nrow) {
#pragma unroll
  for (int s = 0; s < T::KS; ++s) {
    o.hi[s] = *reinterpret_cast<const bf8*>(hrow + s * 32);
    o.lo[s] = *reinterpret_cast<const bf8*>(lrow + s * 32);
  }
  o.init = *reinterpret_cast<const f4*>(nrow);
}

// One block of 16 centroids against the wave's PB point blocks: the small
// (lo) terms first, then the hi terms, with the PB chains interleaved.
template <class T>
__device__ __forceinline__ void tile_block_bf_acc(f4 (&acc)[T::PB],
                                                  const bf8 (&bx)[T::PB][T::KS],
                                                  const ABlockBf<T>& o) {
  constexpr int KS = T::KS, PB = T::PB;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) acc[pb] = o.init;
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
      acc[pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.lo[s], bx[pb][s], acc[pb], 0, 0, 0);
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
      acc[pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(o.hi[s], bx[pb][s], acc[pb], 0, 0, 0);
}

// Epilogue per value: the two smallest values and the index of the smallest
// (the two-candidate pass is off, so neither a third value nor a second
// index is kept; b3 stays +inf).
template <class T>
__device__ __forceinline__ void tile_block_bf(WaveState<T>& w,
                                              const ABlockBf<T>& o, int jb) {
  constexpr int PB = T::PB;
  f4 acc[PB];
  tile_block_bf_acc<T>(acc, w.bx, o);
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      top2_insert(w.b1[pb], w.b2[pb], w.i1[pb], acc[pb][r], jb + r);
}

template <class T>
__device__ __forceinline__ void tile_sweep_bf(WaveState<T>& w, const uint16_t* sH,
                                              const uint16_t* sL, const float* sN,
                                              int cc, int c0, int col, int grp) {
  constexpr int LDA = T::LDA;
  // two operand buffers used in turn (no register copy between blocks)
  ABlockBf<T> a0, a1;
  auto load = [&](ABlockBf<T>& o, int cb) {
    load_ablock_bf<T>(o, &sH[(cb + col) * LDA + grp * 8], &sL[(cb + col) * LDA + grp * 8],
                      &sN[cb + 4 * grp]);
  };
  load(a0, 0);
  for (int cb = 0; cb < cc; cb += 32) {
    if (cb + 16 < cc) load(a1, cb + 16);
    tile_block_bf<T>(w, a0, c0 + cb + 4 * grp);
    if (cb + 16 >= cc) break;
    if (cb + 32 < cc) load(a0, cb + 32);
    tile_block_bf<T>(w, a1, c0 + cb + 16 + 4 * grp);
  }
}

// rows [c0, c0 + cc) of the global hi/lo copies (row stride DP) into LDS
// (row stride LDA), 16 bytes per piece with four pieces of each copy per
// thread in flight, and their norms
template <int DP, int LDA>
__device__ __forceinline__ void stage_bf(uint16_t* sH, uint16_t* sL, float* sN,
                                         const uint16_t* __restrict__ Chi,
                                         const uint16_t* __restrict__ Clo,
                                         const float* __restrict__ cn, int c0,
                                         int cc) {
  constexpr int Q = DP / 8;
  struct HL { uint4 h, l; };
  stage_batched<4, HL>(
      cc * Q,
      [&](int e) {
        const int r = e / Q, q8 = e - r * Q;
        const size_t src = (size_t)(c0 + r) * DP + q8 * 8;
        return HL{*reinterpret_cast<const uint4*>(Chi + src),
                  *reinterpret_cast<const uint4*>(Clo + src)};
      },
      [&](int e, HL v) {
        const int r = e / Q, q8 = e - r * Q;
        *reinterpret_cast<uint4*>(&sH[r * LDA + q8 * 8]) = v.h;
        *reinterpret_cast<uint4*>(&sL[r * LDA + q8 * 8]) = v.l;
      });
  stage_batched<8, float>(
      cc, [&](int e) { return cn[c0 + e]; }, [&](int e, float v) { sN[e] = v; });
}

template <int DP, bool VEC>
__global__ __launch_bounds__(kTileThreads) void tile_bf16_resident_kernel(
    const uint16_t* __restrict__ X, int64_t n, int d,
    const uint16_t* __restrict__ Chi, const uint16_t* __restrict__ Clo,
    const float* __restrict__ cn, int k, int kpad,
    const int* __restrict__ list, const int* __restrict__ seg_cnt, int nseg,
    int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ flags, int64_t cap, int* __restrict__ ucnt,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int* __restrict__ dirty, int recheck_all, int vec,
    const double* __restrict__ CT, const double* __restrict__ C64, int tpf_max,
    int fuse_max, int vecx) {
  using T = Bf16Tile<DP>;
  constexpr int LDA = T::LDA, PB = T::PB, WUP = T::WUP;
  extern __shared__ __attribute__((aligned(16))) uint16_t smem_bf[];
  __shared__ int sFlag, sPairN;
  __shared__ int4 sPair[kPairCap];
  uint16_t* sH = smem_bf;
  uint16_t* sL = smem_bf + (size_t)kpad * LDA;
  float* sN = reinterpret_cast<float*>(smem_bf + (size_t)2 * kpad * LDA);
  const int cv = *conv;                        // tested after the staging loads
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const bool pairs = T::PAIR && C64 != nullptr;

  __shared__ int sSeg[kSegCache], sWmax[kTileThreads / 64];
  if (threadIdx.x == 0) { sFlag = 0; sPairN = 0; }
  if (seg_cnt) seg_stage(seg_cnt, nseg, WUP, sSeg, sWmax);
  stage_bf<DP, LDA>(sH, sL, sN, Chi, Clo, cn, 0, kpad);
  if (cv < iter) return;
  __syncthreads();
  const float cmax = chunk_cmax(sN, kpad, 0, k, lane);

  int* slice = flags + (int64_t)blockIdx.x * cap;
  int64_t nwu = seg_cnt ? (int64_t)nseg * (kSeg / WUP) : (n + WUP - 1) / WUP;
  if (seg_cnt) nwu = seg_units_bound(sWmax, nseg, nwu);
  const int* segc = (seg_cnt && nseg <= kSegCache) ? sSeg : nullptr;
  unsigned long long tot_flag = 0, tot_chg = 0;
  WaveState<T> w;
  // Rows up to 128 wide run the wave's units as a two-stage pipeline: while
  // a unit is swept, the next unit's rows and labels are loaded (their list
  // entries were read one unit earlier) and the list entries of the unit
  // after that.  Every such load is unconditional and its value untouched
  // until the next unit starts, so no wait inside the sweep drains them.
  constexpr bool PIPE = DP <= 128;
  const int64_t stride = (int64_t)gridDim.x * 4;
  int64_t q0, m, base;
  auto advance = [&](int64_t& u) {            // the wave's next non-empty unit from u
    for (; u < nwu; u += stride)
      if (unit_range(u, WUP, n, seg_cnt, segc, nseg, q0, m, base)) return true;
    return false;
  };
  int64_t nq[PB];
  int nraw[PB];
  bool nval[PB];
  auto unit_pids = [&](bool ok) {
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      nq[pb] = q0 + pb * 16 + col;
      nval[pb] = ok && nq[pb] < m;
      nraw[pb] = list ? list[nval[pb] ? base + nq[pb] : 0] : 0;
    }
  };
  int64_t wu = (int64_t)blockIdx.x * 4 + wave;
  bool hcur = advance(wu), hnext = false;
  int64_t wn_u = wu + stride;
  if constexpr (PIPE) {
    unit_pids(hcur);
    issue_points_bf<T, VEC>(w, X, d, labels, list != nullptr, nq, nraw, nval, grp);
    hnext = hcur && advance(wn_u);
    unit_pids(hnext);
  }
  while (hcur) {                              // wave-uniform
    bool hafter = false;
    WaveState<T> wn;
    if constexpr (PIPE) {
      finish_points_bf<T>(w, grp);            // waits for this unit's rows
      // the unit after next is found before the next unit's loads are
      // issued (the search reads segment counts; its waits would drain them)
      wn_u += stride;
      hafter = hnext && advance(wn_u);
      issue_points_bf<T, VEC>(wn, X, d, labels, list != nullptr, nq, nraw, nval, grp);
      unit_pids(hafter);
    } else {
      load_points_bf<T>(w, X, d, vec, list, labels, base, q0, m, col, grp);
    }
    tile_sweep_bf<T>(w, sH, sL, sN, kpad, 0, col, grp);
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
    if constexpr (PIPE) {
      w = wn;
      hcur = hnext;
      hnext = hafter;
    } else {
      wu += stride;
      hcur = advance(wu);
    }
  }
  __syncthreads();
  const int np = sPairN < kPairCap ? sPairN : kPairCap;
  if constexpr (T::PAIR)
    if (np) tot_chg += resolve_pairs<T, uint16_t>(X, d, vec, C64, sPair, np, labels, ub, dirty);
  const int q[2] = {SLOT_FLAGGED, SLOT_CHANGED};
  const unsigned long long v[2] = {tot_flag + (threadIdx.x == 0 ? np : 0), tot_chg};
  block_add_slots<2>(row, q, v);               // includes a barrier
  const int left = recheck_own_slice<uint16_t>(X, d, vecx, CT, k, tpf_max, fuse_max, slice,
                                         sFlag, labels, ub, dirty, row);
  if (threadIdx.x == 0) ucnt[blockIdx.x] = left;
}

template <int DP>
__global__ __launch_bounds__(kTileThreads) void tile_bf16_chunked_kernel(
    const uint16_t* __restrict__ X, int64_t n, int d,
    const uint16_t* __restrict__ Chi, const uint16_t* __restrict__ Clo,
    const float* __restrict__ cn, int k, int kpad,
    const int* __restrict__ list, const int* __restrict__ seg_cnt, int nseg,
    int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ flags, int64_t cap, int* __restrict__ ucnt,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int* __restrict__ dirty, int recheck_all, int vec,
    const double* __restrict__ CT, const double* __restrict__ C64, int tpf_max,
    int fuse_max, int vecx) {
  using T = Bf16Tile<DP>;
  constexpr int LDA = T::LDA, PB = T::PB, CK = T::CK, WUP = T::WUP, BUP = T::BUP;
  __shared__ __attribute__((aligned(16))) uint16_t sH[CK * LDA];
  __shared__ __attribute__((aligned(16))) uint16_t sL[CK * LDA];
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
  WaveState<T> w;
  for (int64_t unit = blockIdx.x; unit < units; unit += gridDim.x) {
    int64_t q0, m, base;
    if (!unit_range(unit, BUP, n, seg_cnt, segc, nseg, q0, m, base))
      continue;                                // uniform over the workgroup
    load_points_bf<T>(w, X, d, vec, list, labels, base, q0 + wave * WUP, m, col, grp);
    float cmax = 0.0f;
    for (int c0 = 0; c0 < kpad; c0 += CK) {
      const int cc = (kpad - c0) < CK ? (kpad - c0) : CK;
      __syncthreads();
      stage_bf<DP, LDA>(sH, sL, sN, Chi, Clo, cn, c0, cc);
      __syncthreads();
      cmax = fmax_nc(cmax, chunk_cmax(sN, cc, c0, k, lane));
      tile_sweep_bf<T>(w, sH, sL, sN, cc, c0, col, grp);
    }
    merge_groups<T, false>(w);
    bool flag, changed;
    int fp;
    finalize_points<T, false>(w, cmax, d, grp, recheck_all, pairs, sPair, &sPairN,
                       labels, ub, dirty, flag, fp, changed);
    append_flags(flag, fp, &sFlag, slice, lane);
    const uint64_t cm = __ballot(changed);
    if (cm && lane == 0) atomicAdd(&sChg, __popcll(cm));
  }
  __syncthreads();
  const int np = sPairN < kPairCap ? sPairN : kPairCap;
  unsigned long long pch = 0;
  if constexpr (T::PAIR)
    if (np) pch = resolve_pairs<T, uint16_t>(X, d, vec, C64, sPair, np, labels, ub, dirty);
  const int q[2] = {SLOT_FLAGGED, SLOT_CHANGED};
  const unsigned long long v[2] = {threadIdx.x == 0 ? (unsigned long long)(sFlag + np) : 0ull,
                                   (threadIdx.x == 0 ? (unsigned long long)sChg : 0ull) + pch};
  block_add_slots<2>(row, q, v);               // includes a barrier
  const int left = recheck_own_slice<uint16_t>(X, d, vecx, CT, k, tpf_max, fuse_max, slice,
                                         sFlag, labels, ub, dirty, row);
  if (threadIdx.x == 0) ucnt[blockIdx.x] = left;
}

template <int DP>
static hipError_t launch_bf_dp(const CentroidOps& o, const AssignJob& j,
                               hipStream_t s) {
  const int vec = (int)(j.d % 8 == 0 && ((uintptr_t)j.X & 15) == 0);
  const int vecx = vec;
  const bool seg = j.seg_cnt != nullptr;
  const TileGeom g = tile_bf16_geometry(DP, o.kpad, j.n, seg, j.nseg);
  if (g.resident) {
    const size_t lds = bf_resident_bytes(DP, o.kpad);
    // rows of exactly DP columns, 16-byte aligned, get the branch-free loads
    auto kern = vec ? &tile_bf16_resident_kernel<DP, true> : &tile_bf16_resident_kernel<DP, false>;
    if (lds > 49152) {   // with the static arrays, past the default 64 KB
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(kern, dim3(g.grid), dim3(kTileThreads),
                       lds, s, (const uint16_t*)j.X, j.n, j.d, o.Chi, o.Clo, o.cn,
                       o.k, o.kpad, j.list, j.seg_cnt, j.nseg, j.labels, j.u,
                       j.flags, g.cap, j.ucnt, j.row, j.conv, j.iter, j.dirty,
                       j.recheck_all, vec, o.CT, o.C64, fuse_tpf(o.k),
                       j.recheck_all ? 0 : kFuseRecheckMax, vecx);
  } else {
    hipLaunchKernelGGL(tile_bf16_chunked_kernel<DP>, dim3(g.grid), dim3(kTileThreads),
                       0, s, (const uint16_t*)j.X, j.n, j.d, o.Chi, o.Clo, o.cn,
                       o.k, o.kpad, j.list, j.seg_cnt, j.nseg, j.labels, j.u,
                       j.flags, g.cap, j.ucnt, j.row, j.conv, j.iter, j.dirty,
                       j.recheck_all, vec, o.CT, o.C64, fuse_tpf(o.k),
                       j.recheck_all ? 0 : kFuseRecheckMax, vecx);
  }
  return hipGetLastError();
}

hipError_t launch_tile_bf16(const CentroidOps& o, const AssignJob& j,
                            hipStream_t s) {
  switch (o.dpb) {
    case 32: return launch_bf_dp<32>(o, j, s);
    case 64: return launch_bf_dp<64>(o, j, s);
    case 128: return launch_bf_dp<128>(o, j, s);
    case 256: return launch_bf_dp<256>(o, j, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// the tile's values and bound, for checking the bound (knor_tile_values)
// ---------------------------------------------------------------------------

// Y[p][j] = the tile's FP32 value of |c_j|^2 - 2 x_p.c_j (the same operands
// and accumulation as every pass above), E[p] = the bound its decision uses
// with R^2 taken over all k centroids.  One wave per 16 * PB points.
template <int DP>
__global__ __launch_bounds__(256) void tile_values_bf16_kernel(
    const uint16_t* __restrict__ X, int64_t n, int d, const uint16_t* __restrict__ Chi,
    const uint16_t* __restrict__ Clo, const float* __restrict__ cn, int k, int kpad,
    float* __restrict__ Y, double* __restrict__ E, int vec) {
  using T = Bf16Tile<DP>;
  constexpr int PB = T::PB, KS = T::KS;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t p0 = ((int64_t)blockIdx.x * 4 + wave) * 16 * PB;
  if (p0 >= n) return;
  float cmax = 0.0f;
  for (int j = lane; j < k; j += 64) cmax = fmax_nc(cmax, cn[j]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) cmax = fmax_nc(cmax, __shfl_xor(cmax, o));
  bf8 bx[PB][KS];
  double xs[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t p = p0 + pb * 16 + col;
    T::load_row(bx[pb], X, p < n ? p : 0, d, grp, vec, p < n);
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const double v = T::xval(bx[pb], s, e);
        acc = acc + v * v;
      }
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    xs[pb] = acc;
  }
  for (int jb = 0; jb < kpad; jb += 16) {
    ABlockBf<T> o;
    load_ablock_bf<T>(o, Chi + (size_t)(jb + col) * DP + grp * 8,
                      Clo + (size_t)(jb + col) * DP + grp * 8, cn + jb + 4 * grp);
    f4 acc[PB];
    tile_block_bf_acc<T>(acc, bx, o);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int64_t p = p0 + pb * 16 + col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j = jb + 4 * grp + r;
        if (p < n && j < k) Y[(size_t)p * k + j] = acc[pb][r];
      }
    }
  }
  if (grp == 0) {
    const double R2 = (double)cmax * (1.0 + 2.384185791015625e-07);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int64_t p = p0 + pb * 16 + col;
      if (p < n) E[p] = T::bound(xs[pb] * (1.0 + (double)(d + 4) * 2.220446049250313e-16), R2, d);
    }
  }
}

hipError_t launch_tile_values_bf16(const CentroidOps& o, const uint16_t* X, int64_t n,
                                   int d, float* Y, double* E, hipStream_t s) {
  const int vec = (int)(((uintptr_t)X & 15) == 0 && d % 8 == 0);
  auto go = [&](auto kern, int pb) {
    const int64_t per = 64LL * pb;
    hipLaunchKernelGGL(kern, dim3((unsigned)((n + per - 1) / per)), dim3(256), 0, s, X, n, d,
                       o.Chi, o.Clo, o.cn, o.k, o.kpad, Y, E, vec);
    return hipGetLastError();
  };
  switch (o.dpb) {
    case 32: return go(tile_values_bf16_kernel<32>, bf_pb(32));
    case 64: return go(tile_values_bf16_kernel<64>, bf_pb(64));
    case 128: return go(tile_values_bf16_kernel<128>, bf_pb(128));
    case 256: return go(tile_values_bf16_kernel<256>, bf_pb(256));
  }
  return hipErrorInvalidValue;
}

}  // namespace knor
