// The FP32 matrix-core tile type shared by the distance tiles over FP32
// points (tile_f32.hip: dense and survivor-list passes; tile_cand.hip: the
// Clause-2 candidate-list pass): operand layout of v_mfma_f32_16x16x4f32,
// row loads, the rounding bound of one tile value, and the per-block
// sweep with the top-3 epilogue.
#pragma once

#include "tile_common.h"

namespace knor {

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

template <int DP, int PB_>
struct F32Tile {
  using Frag = float;
  static constexpr int KS = DP / 4;                    // dims per lane group
  static constexpr int PB = PB_;
  static constexpr int LDA = DP + 4;                   // LDS row stride
  static constexpr int CK = (4096 / DP) < 16 ? 16 : (4096 / DP);
  static constexpr int WUP = 16 * PB;                  // points per wave unit
  static constexpr int BUP = 4 * WUP;                  // points per block unit
  // lane group g holds dimensions [g KS, (g + 1) KS): one step of KS
  static constexpr bool PAIR = KS <= 16;
  static constexpr int NS = 1, NE = KS;
  __device__ static constexpr int dim(int, int g, int e) { return g * KS + e; }
  __device__ static double xval(const Frag (&bx)[KS], int, int e) {
    return (double)bx[e];
  }
  // this lane group's dimensions of row p (zero past d or when !valid)
  __device__ static void load_row(Frag (&bx)[KS], const float* __restrict__ X,
                                  int64_t p, int d, int grp, int vec, bool valid) {
    const float* xr = X + (size_t)p * d + grp * KS;
    if (valid && vec) {
      load_slice<KS>(bx, xr);
    } else {
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        const int dim = grp * KS + s;
        bx[s] = (valid && dim < d) ? xr[s] : 0.0f;
      }
    }
  }
  // u = 2^-24.  Rounding c to FP32 (2u|x||c| after the -2 scaling), |c|^2
  // to FP32 (u R^2), each of the d products and d+1 accumulation steps at
  // 2u of the running magnitude; plus 2^-100 (1 + R) for subnormals flushed
  // by the matrix core.
  __device__ static double bound(double xn2, double R2, int d) {
    const double u24 = 5.9604644775390625e-08;
    const double xr = sqrt(xn2 * R2);
    return (u24 * ((2.0 * d + 5.0) * R2 + (4.0 * d + 10.0) * xr) +
            7.888609052210118e-31 * (1.0 + sqrt(R2))) * (1.0 + 9.765625e-04);
  }
};

// Operands of one block of 16 centroids: A slice (rows from LDS) and the
// accumulator seed (their norms).
template <class T>
struct ABlock {
  float a[T::KS];
  f4 init;
};

template <class T>
__device__ __forceinline__ void load_ablock(ABlock<T>& o, const float* arow,
                                            const float* nrow) {
  load_slice<T::KS>(o.a, arow);
  o.init = *reinterpret_cast<const f4*>(nrow);
}

// One block of 16 centroids against the wave's PB point blocks.  The PB
// accumulation chains are interleaved so consecutive matrix instructions are
// independent.  Epilogue per value: the three smallest values by two
// medians of three, and the index of the smallest (I2: of the two smallest)
// by selects.
// The tile values of one block of 16 centroids for PB point blocks: the
// accumulator seeded with fp32(|c|^2), then one MFMA per K-step in order.
// Every pass of the tile (and the bound check's value dump) uses this, so a
// pair's value depends on nothing but its two operands.
template <class T>
__device__ __forceinline__ void tile_block_acc(f4 (&acc)[T::PB],
                                               const typename T::Frag (&bx)[T::PB][T::KS],
                                               const ABlock<T>& o) {
  constexpr int KS = T::KS, PB = T::PB;
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) acc[pb] = o.init;
#pragma unroll
  for (int s = 0; s < KS; ++s)
#pragma unroll
    for (int pb = 0; pb < PB; ++pb)
      acc[pb] = __builtin_amdgcn_mfma_f32_16x16x4f32(o.a[s], bx[pb][s], acc[pb], 0, 0, 0);
}

template <class T, bool I2>
__device__ __forceinline__ void tile_block(WaveState<T>& w, const ABlock<T>& o,
                                           int jb) {
  constexpr int PB = T::PB;
  f4 acc[PB];
  tile_block_acc<T>(acc, w.bx, o);
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (I2)
        top3_insert(w.b1[pb], w.b2[pb], w.b3[pb], w.i1[pb], w.i2[pb], acc[pb][r], jb + r);
      else
        top3_insert_lite(w.b1[pb], w.b2[pb], w.b3[pb], w.i1[pb], acc[pb][r], jb + r);
    }
}

// All centroid blocks [c0, c0 + cc) staged at sC/sN, with the next block's
// operands loaded from LDS before the current block's matrix work.
template <class T, bool I2, bool PP = false>
__device__ __forceinline__ void tile_sweep(WaveState<T>& w, const float* sC,
                                           const float* sN, int cc, int c0,
                                           int col, int grp) {
  constexpr int LDA = T::LDA, KS = T::KS;
  auto load = [&](ABlock<T>& o, int cb) {
    load_ablock<T>(o, &sC[(cb + col) * LDA + grp * KS], &sN[cb + 4 * grp]);
  };
  if constexpr (PP) {
    // two operand buffers used in turn (no register copy between blocks;
    // a few more registers live)
    ABlock<T> a0, a1;
    load(a0, 0);
    for (int cb = 0; cb < cc; cb += 32) {
      if (cb + 16 < cc) load(a1, cb + 16);
      tile_block<T, I2>(w, a0, c0 + cb + 4 * grp);
      if (cb + 16 >= cc) break;
      if (cb + 32 < cc) load(a0, cb + 32);
      tile_block<T, I2>(w, a1, c0 + cb + 16 + 4 * grp);
    }
  } else {
    ABlock<T> cur, nxt;
    load(cur, 0);
    for (int cb = 0; cb < cc; cb += 16) {
      if (cb + 16 < cc) load(nxt, cb + 16);
      tile_block<T, I2>(w, cur, c0 + cb + 4 * grp);
      cur = nxt;
    }
  }
}

// Rows [c0, c0 + cc) of -2c (row stride DP) into LDS (row stride LDA) and
// their norms, B 16-byte loads per thread in flight.
template <class T, int B>
__device__ __forceinline__ void stage_cents(float* sC, float* sN,
                                            const float* __restrict__ Cm2,
                                            const float* __restrict__ cn, int c0,
                                            int cc) {
  constexpr int Q = T::KS;                     // 16-byte pieces per row (DP / 4)
  stage_batched<B, float4>(
      cc * Q,
      [&](int e) {
        const int r = e / Q, q4 = e - r * Q;
        return *reinterpret_cast<const float4*>(Cm2 + (size_t)(c0 + r) * (4 * Q) + q4 * 4);
      },
      [&](int e, float4 v) {
        const int r = e / Q, q4 = e - r * Q;
        *reinterpret_cast<float4*>(&sC[r * T::LDA + q4 * 4]) = v;
      });
  stage_batched<B, float>(
      cc, [&](int e) { return cn[c0 + e]; }, [&](int e, float v) { sN[e] = v; });
}


}  // namespace knor
