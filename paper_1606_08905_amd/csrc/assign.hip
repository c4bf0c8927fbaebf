// Assignment step: nearest centroid of every point (Mhembere et al., HPDC'17,
// Algorithm 1, the nearest-centroid loop with a strict "<").
//
// Two forms:
//  * assign_mfma_f32: the distance tile y_j = |c_j|^2 - 2 x.c_j on the FP32
//    matrix cores (v_mfma_f32_16x16x4f32), centroids staged through LDS,
//    points held in registers, argmin fused into the epilogue as a running
//    (best, second-best, best-index) per point.  A point is final only if
//    the gap between its two smallest y exceeds a proven bound on the FP32
//    rounding error (plus the FP64 evaluation error of the definition);
//    otherwise it is appended to the recheck list.
//  * exact assignment in FP64 (the definition itself), used for FP64 data and
//    for the recheck list.
#include <float.h>
#include <math.h>

#include "common.h"

namespace knor {

typedef float f4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// centroid operands
// ---------------------------------------------------------------------------

// One wave per centroid row: Cm2 = -2 * RNE_fp32(c) (exact scaling), zero
// padded to dp columns; cn = RNE_fp32(sum_i c_i^2) with the sum in FP64.
// Rows k..kpad-1 are padding: Cm2 = 0, cn = +inf (they can never be chosen).
__global__ __launch_bounds__(256) void prep_centroids_kernel(
    const double* __restrict__ C64, int k, int kpad, int d, int dp,
    float* __restrict__ Cm2, float* __restrict__ cn,
    uint16_t* __restrict__ Cbf) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (j >= kpad) return;
  double ss = 0.0;
  for (int i = lane; i < dp; i += 64) {
    float v = 0.0f;
    if (j < k && i < d) {
      double c = C64[(size_t)j * d + i];
      v = (float)c;
      ss = __dadd_rn(ss, __dmul_rn(c, c));
      if (Cbf) {
        // BF16 = RNE of the FP64 value
        uint64_t b = (uint64_t)__double_as_longlong(c);
        double a = fabs(c);
        uint16_t out = 0;
        if (a != 0.0) {
          int e = ilogb(a);
          if (e < -126) e = -126;
          double q = ldexp(a, 7 - e);
          double r = rint(q);
          float y = (float)ldexp(r, e - 7);
          out = (uint16_t)(__float_as_uint(y) >> 16);
        }
        Cbf[(size_t)j * dp + i] = out | (uint16_t)((b >> 48) & 0x8000u);
      }
    } else if (Cbf) {
      Cbf[(size_t)j * dp + i] = 0;
    }
    Cm2[(size_t)j * dp + i] = -2.0f * v;
  }
  for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
  if (lane == 0) cn[j] = (j < k) ? (float)ss : INFINITY;
}

hipError_t launch_prep_centroids(const CentroidOps& o, hipStream_t s) {
  int blocks = (o.kpad + 3) / 4;
  hipLaunchKernelGGL(prep_centroids_kernel, dim3(blocks), dim3(256), 0, s,
                     o.C64, o.k, o.kpad, o.d, o.dp, o.Cm2, o.cn, o.Cbf);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 MFMA distance tile + fused argmin
// ---------------------------------------------------------------------------
//
// Lane layout of v_mfma_f32_16x16x4f32 used here: lane l = 16*g + c supplies
// A[c][g] and B[g][c] and receives D[4g + r][c], r = 0..3.  Rows of A are
// centroids, columns of B are points, so every lane owns one point column
// and reduces over the 4 centroid rows it receives.  The contraction index
// is permuted so that lane group g owns the KS = DP/4 consecutive dimensions
// [g*KS, (g+1)*KS): both operands use the same permutation, and each lane
// loads its slice of a row with 16-byte vector loads.
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
// argmin (and its lowest-index rule) must select the same centroid.

constexpr int kTileThreads = 256;

// Load KS consecutive floats (16-byte aligned when KS >= 4, 8-byte when 2).
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

template <int DP>
struct TileCfg {
  static constexpr int KS = DP / 4;                      // k-steps per MFMA
  static constexpr int CK = (4096 / DP) < 16 ? 16 : (4096 / DP);
  static constexpr int LDA = DP + 4;                     // LDS row stride
  static constexpr int PB = DP >= 256 ? 1 : (DP >= 128 ? 2 : 4);
  static constexpr int TP = 4 * 16 * PB;                 // points per tile
};

template <int DP>
__global__ __launch_bounds__(kTileThreads) void assign_mfma_f32(
    const float* __restrict__ X, int64_t n, int d,
    const float* __restrict__ Cm2, const float* __restrict__ cn, int k,
    int kpad, const int* __restrict__ list,
    const unsigned long long* __restrict__ list_len,
    int32_t* __restrict__ labels, float* __restrict__ ub,
    int* __restrict__ flags, unsigned long long* __restrict__ ctr,
    const int* __restrict__ done, int recheck_all, int vec) {
  using C = TileCfg<DP>;
  constexpr int KS = C::KS, CK = C::CK, LDA = C::LDA, PB = C::PB, TP = C::TP;
  __shared__ __attribute__((aligned(16))) float sC[CK * LDA];
  __shared__ float sN[CK];

  if (*done) return;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int col = lane & 15;
  const int grp = lane >> 4;
  const int64_t m = list ? (int64_t)(*list_len) : n;
  const int64_t ntiles = (m + TP - 1) / TP;

  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    float bx[PB][KS];
    int64_t pid[PB];
    bool valid[PB];
    double xs[PB];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      int64_t q = tile * TP + (int64_t)(wave * 16 * PB + pb * 16 + col);
      valid[pb] = q < m;
      int64_t p = valid[pb] ? (list ? (int64_t)list[q] : q) : 0;
      pid[pb] = p;
      const float* row = X + (size_t)p * d + grp * KS;
      if (valid[pb] && vec) {
        load_slice<KS>(bx[pb], row);
      } else {
#pragma unroll
        for (int s = 0; s < KS; ++s) {
          int dim = grp * KS + s;
          bx[pb][s] = (valid[pb] && dim < d) ? row[s] : 0.0f;
        }
      }
      double acc = 0.0;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        double v = (double)bx[pb][s];
        acc = acc + v * v;
      }
      xs[pb] = acc;
    }

    float b1[PB], b2[PB];
    int i1[PB];
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      b1[pb] = INFINITY;
      b2[pb] = INFINITY;
      i1[pb] = 0;
    }
    float cmax = 0.0f;

    for (int c0 = 0; c0 < kpad; c0 += CK) {
      const int cc = (kpad - c0) < CK ? (kpad - c0) : CK;
      __syncthreads();
      for (int e = threadIdx.x; e < cc * (DP / 4); e += kTileThreads) {
        int r = e / (DP / 4), q4 = e - r * (DP / 4);
        float4 v = *reinterpret_cast<const float4*>(Cm2 + (size_t)(c0 + r) * DP + q4 * 4);
        *reinterpret_cast<float4*>(&sC[r * LDA + q4 * 4]) = v;
      }
      for (int e = threadIdx.x; e < cc; e += kTileThreads) sN[e] = cn[c0 + e];
      __syncthreads();

      for (int cb = 0; cb < cc; cb += 16) {
        float a[KS];
        load_slice<KS>(a, &sC[(cb + col) * LDA + grp * KS]);
        f4 init;
        init[0] = sN[cb + 4 * grp + 0];
        init[1] = sN[cb + 4 * grp + 1];
        init[2] = sN[cb + 4 * grp + 2];
        init[3] = sN[cb + 4 * grp + 3];
        const int jb = c0 + cb + 4 * grp;
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (jb + r < k) cmax = fmaxf(cmax, init[r]);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          f4 acc = init;
#pragma unroll
          for (int s = 0; s < KS; ++s)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], bx[pb][s], acc, 0, 0, 0);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            float y = acc[r];
            b2[pb] = __builtin_amdgcn_fmed3f(b1[pb], b2[pb], y);
            bool lt = y < b1[pb];
            i1[pb] = lt ? (jb + r) : i1[pb];
            b1[pb] = fminf(b1[pb], y);
          }
        }
      }
    }

    // merge the four lane groups (each saw a different quarter of centroids)
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) {
      cmax = fmaxf(cmax, __shfl_xor(cmax, off));
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) {
        float ob1 = __shfl_xor(b1[pb], off);
        float ob2 = __shfl_xor(b2[pb], off);
        int oi1 = __shfl_xor(i1[pb], off);
        xs[pb] += __shfl_xor(xs[pb], off);
        float nb2 = fminf(fmaxf(b1[pb], ob1), fminf(b2[pb], ob2));
        bool take = ob1 < b1[pb] || (ob1 == b1[pb] && oi1 < i1[pb]);
        i1[pb] = take ? oi1 : i1[pb];
        b1[pb] = fminf(b1[pb], ob1);
        b2[pb] = nb2;
      }
    }

    const double R2 = (double)cmax * (1.0 + 2.384185791015625e-07);  // 1+2^-22
    const double u24 = 5.9604644775390625e-08;                        // 2^-24
    const double e64 = (double)(d + 2) * 1.1102230246251565e-16;     // (d+2)2^-53
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const bool mine = valid[pb] && ((pb & 3) == grp);
      bool flag = false, changed = false;
      if (mine) {
        double xn2 = xs[pb] * (1.0 + (double)(d + 4) * 2.220446049250313e-16);
        double E = u24 * ((2.0 * d + 5.0) * R2 + (4.0 * d + 10.0) * sqrt(xn2 * R2)) *
                   (1.0 + 9.765625e-04);
        double y1 = (double)b1[pb], y2 = (double)b2[pb];
        double dbest = xn2 + y1 + E;
        if (!(dbest > 0.0)) dbest = 0.0;
        double thr = 2.0 * E + 2.01 * e64 * dbest;
        double gap = y2 - y1;
        flag = recheck_all || !(gap > thr);
        if (!flag) {
          int64_t p = pid[pb];
          int32_t old = labels[p];
          labels[p] = i1[pb];
          changed = old != i1[pb];
          if (ub) ub[p] = f32_up(sqrt(dbest) * (1.0 + 8.881784197001252e-16));
        }
      }
      wave_count(mine, &ctr[CNT_SCANNED]);
      wave_count(changed, &ctr[CNT_CHANGED]);
      wave_append(flag, (int)pid[pb], &ctr[CNT_RECHECKED], flags);
    }
  }
}

template <int DP>
static hipError_t launch_mfma_dp(const CentroidOps& o, const AssignJob& j,
                                 hipStream_t s) {
  using C = TileCfg<DP>;
  int64_t tiles = (j.n + C::TP - 1) / C::TP;
  int grid = (int)(tiles < 2048 ? (tiles < 1 ? 1 : tiles) : 2048);
  hipLaunchKernelGGL(assign_mfma_f32<DP>, dim3(grid), dim3(kTileThreads), 0,
                     s, (const float*)j.X, j.n, j.d, o.Cm2, o.cn, o.k, o.kpad,
                     j.list, j.list_len, j.labels, j.u, j.flags, j.ctr, j.done,
                     j.recheck_all,
                     (int)(j.d == DP && ((uintptr_t)j.X & 15) == 0));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exact FP64 assignment (the definition)
// ---------------------------------------------------------------------------

// One lane per point: used for FP64 data.  Centroid rows are read with
// wave-uniform addresses (scalar loads).
template <typename T>
__global__ __launch_bounds__(256) void exact_assign_lane(
    const T* __restrict__ X, int64_t n, int d, const double* __restrict__ C64,
    int k, const int* __restrict__ list,
    const unsigned long long* __restrict__ list_len,
    int32_t* __restrict__ labels, float* __restrict__ ub,
    unsigned long long* __restrict__ ctr, const int* __restrict__ done,
    double* __restrict__ dist2) {
  if (*done) return;
  const int64_t m = list ? (int64_t)(*list_len) : n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x; q0 < m; q0 += stride) {
    int64_t q = q0 + threadIdx.x;
    bool valid = q < m;
    bool changed = false;
    if (valid) {
      int64_t p = list ? (int64_t)list[q] : q;
      const T* x = X + (size_t)p * d;
      double best = INFINITY;
      int a = 0;
      for (int j = 0; j < k; ++j) {
        double D = dist2_canon<T>(x, C64 + (size_t)j * d, d);
        if (D < best) { best = D; a = j; }
      }
      int32_t old = labels[p];
      labels[p] = a;
      changed = old != a;
      if (ub) ub[p] = f32_up(sqrt(best) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
      if (dist2) dist2[p] = best;
    }
    wave_count(valid, &ctr[CNT_SCANNED]);
    wave_count(changed, &ctr[CNT_CHANGED]);
  }
}

// One wave per listed point, lanes over centroids: the FP64 recheck.  The
// lexicographic (D, j) minimum over lanes is the lowest-index argmin.
template <typename T>
__global__ __launch_bounds__(256) void exact_recheck_wave(
    const T* __restrict__ X, int d, const double* __restrict__ C64, int k,
    const int* __restrict__ list, const unsigned long long* __restrict__ list_len,
    int32_t* __restrict__ labels, float* __restrict__ ub,
    unsigned long long* __restrict__ ctr, const int* __restrict__ done) {
  if (*done) return;
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)(*list_len);
  const int64_t wstride = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t q = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
       q < m; q += wstride) {
    const int64_t p = list[q];
    const T* x = X + (size_t)p * d;
    double best = INFINITY;
    int a = 0x7fffffff;
    for (int j = lane; j < k; j += 64) {
      double D = dist2_canon<T>(x, C64 + (size_t)j * d, d);
      if (D < best) { best = D; a = j; }
    }
    for (int off = 32; off > 0; off >>= 1) {
      double ob = __shfl_xor(best, off);
      int oa = __shfl_xor(a, off);
      if (ob < best || (ob == best && oa < a)) { best = ob; a = oa; }
    }
    if (lane == 0) {
      int32_t old = labels[p];
      labels[p] = a;
      if (old != a) atomicAdd(&ctr[CNT_CHANGED], 1ull);
      if (ub) ub[p] = f32_up(sqrt(best) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
    }
  }
}

hipError_t launch_assign(const CentroidOps& o, const AssignJob& j,
                         hipStream_t s) {
  if (j.dt == KNOR_F64) {
    int64_t blocks = (j.n + 255) / 256;
    int grid = (int)(blocks < 4096 ? (blocks < 1 ? 1 : blocks) : 4096);
    hipLaunchKernelGGL(exact_assign_lane<double>, dim3(grid), dim3(256), 0, s,
                       (const double*)j.X, j.n, j.d, o.C64, o.k, j.list,
                       j.list_len, j.labels, j.u, j.ctr, j.done, j.dist2);
    return hipGetLastError();
  }
  if (j.dt == KNOR_F32) {
    switch (o.dp) {
      case 8: return launch_mfma_dp<8>(o, j, s);
      case 16: return launch_mfma_dp<16>(o, j, s);
      case 32: return launch_mfma_dp<32>(o, j, s);
      case 64: return launch_mfma_dp<64>(o, j, s);
      case 128: return launch_mfma_dp<128>(o, j, s);
      case 256: return launch_mfma_dp<256>(o, j, s);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorNotSupported;
}

hipError_t launch_recheck(const CentroidOps& o, const AssignJob& j,
                          hipStream_t s) {
  // the list length lives on the device; size the grid for the worst case
  // and let surplus waves exit
  int64_t waves = j.n;
  int64_t blocks = (waves + 3) / 4;
  int grid = (int)(blocks < 2048 ? (blocks < 1 ? 1 : blocks) : 2048);
  const unsigned long long* len = &j.ctr[CNT_RECHECKED];
  switch (j.dt) {
    case KNOR_F32:
      hipLaunchKernelGGL(exact_recheck_wave<float>, dim3(grid), dim3(256), 0, s,
                         (const float*)j.X, j.d, o.C64, o.k, j.flags, len,
                         j.labels, j.u, j.ctr, j.done);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(exact_recheck_wave<uint16_t>, dim3(grid), dim3(256), 0,
                         s, (const uint16_t*)j.X, j.d, o.C64, o.k, j.flags, len,
                         j.labels, j.u, j.ctr, j.done);
      break;
    default:
      return hipSuccess;   // FP64 data never uses the recheck list
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exact per-point distance to the assigned centroid, and the canonical sum
// ---------------------------------------------------------------------------

template <typename T>
__global__ __launch_bounds__(256) void exact_dist2_kernel(
    const T* __restrict__ X, int64_t n, int d, const double* __restrict__ C64,
    const int32_t* __restrict__ labels, double* __restrict__ out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  out[p] = dist2_canon<T>(X + (size_t)p * d, C64 + (size_t)labels[p] * d, d);
}

hipError_t launch_exact_dist2(const void* X, knor_dtype dt, int64_t n, int d,
                              const double* C64, const int32_t* labels,
                              double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  switch (dt) {
    case KNOR_F64:
      hipLaunchKernelGGL(exact_dist2_kernel<double>, dim3(blocks), dim3(256), 0,
                         s, (const double*)X, n, d, C64, labels, out);
      break;
    case KNOR_F32:
      hipLaunchKernelGGL(exact_dist2_kernel<float>, dim3(blocks), dim3(256), 0,
                         s, (const float*)X, n, d, C64, labels, out);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(exact_dist2_kernel<uint16_t>, dim3(blocks), dim3(256),
                         0, s, (const uint16_t*)X, n, d, C64, labels, out);
      break;
  }
  return hipGetLastError();
}

// Leaf sums of the canonical order: 64 consecutive values, left to right,
// starting from the first.
__global__ __launch_bounds__(256) void leaf_sum_scalar(const double* __restrict__ v,
                                                       int64_t n,
                                                       double* __restrict__ out) {
  int64_t L = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t m0 = L * kLeaf;
  if (m0 >= n) return;
  int64_t m1 = m0 + kLeaf < n ? m0 + kLeaf : n;
  double s = v[m0];
  for (int64_t m = m0 + 1; m < m1; ++m) s = __dadd_rn(s, v[m]);
  out[L] = s;
}

// Pairwise tree over the leaf sums, bottom-up: at stride s, node a (a a
// multiple of 2s) absorbs node a+s when it exists.  This equals splitting
// each range at the largest power of two below its length.
__global__ __launch_bounds__(1024) void tree_scalar(double* __restrict__ t,
                                                    int64_t m,
                                                    double* __restrict__ out) {
  for (int64_t s = 1; s < m; s <<= 1) {
    for (int64_t i = threadIdx.x; i * 2 * s + s < m; i += blockDim.x) {
      int64_t a = i * 2 * s;
      t[a] = __dadd_rn(t[a], t[a + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = m > 0 ? t[0] : 0.0;
}

hipError_t launch_canonical_sum(const double* v, int64_t n, double* tmp,
                                double* out, hipStream_t s) {
  int64_t leaves = (n + kLeaf - 1) / kLeaf;
  if (leaves > 0) {
    hipLaunchKernelGGL(leaf_sum_scalar, dim3((leaves + 255) / 256), dim3(256),
                       0, s, v, n, tmp);
  }
  hipLaunchKernelGGL(tree_scalar, dim3(1), dim3(1024), 0, s, tmp, leaves, out);
  return hipGetLastError();
}

}  // namespace knor
