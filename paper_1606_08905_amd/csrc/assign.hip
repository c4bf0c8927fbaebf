// Assignment step: nearest centroid of every point (Mhembere et al., HPDC'17,
// Algorithm 1, the nearest-centroid loop with a strict "<").
//
// This file holds the centroid operands, the exact FP64 assignment (the
// definition itself, used for FP64 data), the FP64 recheck of the points the
// FP32 tile (tile_f32.hip) could not decide, and the canonical FP64 objective.
#include <float.h>
#include <math.h>

#include "recheck.h"

namespace knor {

// ---------------------------------------------------------------------------
// centroid operands
// ---------------------------------------------------------------------------

// One wave per centroid row.  Cm2 = -2 * RNE_fp32(c) (exact scaling), zero
// padded to dp columns; for the BF16 tile Chi = RNE_bf16(-2c) and
// Clo = RNE_bf16(-2c - Chi) (the difference is exact in FP64), zero padded
// to dpb columns; cn = RNE_fp32(|c|^2) with the sum in FP64 index order;
// CT = transposed FP64 copy.  Rows k..kpad-1 are padding: operands 0,
// cn = +inf (they can never be chosen).
__global__ __launch_bounds__(256) void prep_centroids_kernel(
    const double* __restrict__ C64, int k, int kpad, int d, int dp, int dpb,
    float* __restrict__ Cm2, float* __restrict__ cn, double* __restrict__ CT,
    uint16_t* __restrict__ Chi, uint16_t* __restrict__ Clo) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (j >= kpad) return;
  const int wmax = dp > dpb ? dp : dpb;
  for (int i = lane; i < wmax; i += 64) {
    double c = (j < k && i < d) ? C64[(size_t)j * d + i] : 0.0;
    if (Cm2 && i < dp) Cm2[(size_t)j * dp + i] = -2.0f * (float)c;
    if (Chi && i < dpb) {
      uint16_t h, l;
      bf16_split_m2(c, h, l);
      Chi[(size_t)j * dpb + i] = h;
      Clo[(size_t)j * dpb + i] = l;
    }
    if (j < k && i < d && CT) CT[(size_t)i * k + j] = c;
  }
  if (lane == 0) {
    double ss = 0.0;
    if (j < k)
      for (int i = 0; i < d; ++i) {
        double c = C64[(size_t)j * d + i];
        ss = __dadd_rn(ss, __dmul_rn(c, c));
      }
    cn[j] = (j < k) ? (float)ss : INFINITY;
  }
}

hipError_t launch_prep_centroids(const CentroidOps& o, hipStream_t s) {
  int blocks = (o.kpad + 3) / 4;
  hipLaunchKernelGGL(prep_centroids_kernel, dim3(blocks), dim3(256), 0, s,
                     o.C64, o.k, o.kpad, o.d, o.dp, o.dpb, o.Cm2, o.cn, o.CT,
                     o.Chi, o.Clo);
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
    int k, const int* __restrict__ list, const int* __restrict__ seg_cnt,
    int nseg, int32_t* __restrict__ labels, float* __restrict__ ub,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int* __restrict__ dirty) {
  if (*conv < iter) return;
  // dense: q over [0, n); segmented: q over nseg * kSeg slots
  const int64_t m = seg_cnt ? (int64_t)nseg * kSeg : n;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q0 = (int64_t)blockIdx.x * blockDim.x; q0 < m; q0 += stride) {
    int64_t q = q0 + threadIdx.x;
    bool valid = q < m;
    int64_t p = q;
    if (valid && seg_cnt) {
      int s = (int)(q / kSeg);
      int r = (int)(q - (int64_t)s * kSeg);
      valid = r < seg_cnt[s];
      p = valid ? (int64_t)list[q] : 0;
    }
    bool changed = false;
    if (valid) {
      const T* x = X + (size_t)p * d;
      double best = INFINITY;
      int a = 0;
      for (int j = 0; j < k; ++j) {
        double D = dist2_canon<T>(x, C64 + (size_t)j * d, d);
        if (D < best) { best = D; a = j; }
      }
      int32_t old = labels[p];
      if (old != a) {                        // unchanged labels are not rewritten
        labels[p] = a;
        changed = true;
        mark_dirty(dirty, old, a);
      }
      if (ub) ub[p] = f32_up(sqrt(best) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
    }
    wave_count_changed(changed, row, (int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  }
}

// The FP64 recheck kernel.  Workgroup b takes the recheck slices
// [b*S, b*S + S) (one slice per tile workgroup; slices the tile workgroup
// already rechecked itself have count 0) as one list of nf near-tie points:
// the throughput path when nf is large, else the latency path (recheck.h).
constexpr int kRecheckSlices = 4;     // at most

template <typename T, bool LDSC>
__global__ __launch_bounds__(256) void exact_recheck_unit(
    const T* __restrict__ X, int d, int vec, const double* __restrict__ C64,
    const double* __restrict__ CT, int k,
    int tpf_max, const int* __restrict__ flags, const int* __restrict__ ucnt,
    int nslices, int S, int64_t cap, int32_t* __restrict__ labels,
    float* __restrict__ ub, unsigned long long* __restrict__ row,
    const int* __restrict__ conv, int iter, int* __restrict__ dirty) {
  extern __shared__ __attribute__((aligned(16))) double sC[];
  // this workgroup's slices and the start of each within its list (read
  // together with the convergence flag: one round trip)
  const int s0 = blockIdx.x * S;
  int cnt[kRecheckSlices];
#pragma unroll
  for (int i = 0; i < kRecheckSlices; ++i)
    cnt[i] = (i < S && s0 + i < nslices) ? ucnt[s0 + i] : 0;
  if (*conv < iter) return;
  int sstart[kRecheckSlices + 1];
  sstart[0] = 0;
#pragma unroll
  for (int i = 0; i < kRecheckSlices; ++i) sstart[i + 1] = sstart[i] + cnt[i];
  const int nf = sstart[kRecheckSlices];     // uniform over the workgroup
  if (nf == 0) return;
  auto point_of = [&](int f) {
    int si = 0;
#pragma unroll
    for (int i = 1; i < kRecheckSlices; ++i) si += (f >= sstart[i]) ? 1 : 0;
    return flags[(int64_t)(s0 + si) * cap + (f - sstart[si])];
  };
  if (nf >= kRecheckBlockedMin) {
    const unsigned long long ch =
        recheck_blocked<T>(X, d, C64, k, nf, point_of, labels, ub, dirty);
    const int q1[1] = {SLOT_CHANGED};
    const unsigned long long v1[1] = {ch};
    block_add_slots<1>(row, q1, v1);
    return;
  }
  const unsigned long long changes = recheck_small<T, LDSC>(
      X, d, vec, C64, CT, sC, k, tpf_max, nf, point_of, labels, ub, dirty);
  const int q[1] = {SLOT_CHANGED};
  const unsigned long long v[1] = {changes};
  block_add_slots<1>(row, q, v);
}

hipError_t launch_assign(const CentroidOps& o, const AssignJob& j,
                         hipStream_t s) {
  if (j.dt == KNOR_F64) {
    int64_t m = j.seg_cnt ? (int64_t)j.nseg * kSeg : j.n;
    int64_t blocks = (m + 255) / 256;
    int grid = (int)(blocks < 4096 ? (blocks < 1 ? 1 : blocks) : 4096);
    hipLaunchKernelGGL(exact_assign_lane<double>, dim3(grid), dim3(256), 0, s,
                       (const double*)j.X, j.n, j.d, o.C64, o.k, j.list,
                       j.seg_cnt, j.nseg, j.labels, j.u, j.row, j.conv, j.iter,
                       j.dirty);
    return hipGetLastError();
  }
  if (j.dt == KNOR_F32) return launch_tile_f32(o, j, s);
  if (j.dt == KNOR_BF16) return launch_tile_bf16(o, j, s);
  return hipErrorNotSupported;
}

constexpr size_t kRecheckLds = 65536;

template <typename T>
static void launch_recheck_t(const CentroidOps& o, const AssignJob& j,
                             const TileGeom& g, int tpf, hipStream_t s) {
  const int vec = (int)(((uintptr_t)j.X & 15) == 0 &&
                        ((size_t)j.d * sizeof(T)) % 16 == 0);
  const size_t lds = (size_t)o.k * (j.d + 1) * sizeof(double);
  // several slices per workgroup when the tile grid alone fills the device
  const int S = g.grid >= 1024 ? kRecheckSlices : 1;
  const int grid = (g.grid + S - 1) / S;
  if (lds <= kRecheckLds)
    hipLaunchKernelGGL((exact_recheck_unit<T, true>), dim3(grid), dim3(256),
                       lds, s, (const T*)j.X, j.d, vec, o.C64, o.CT, o.k, tpf,
                       j.flags, j.ucnt, g.grid, S, g.cap, j.labels, j.u, j.row, j.conv,
                       j.iter, j.dirty);
  else
    hipLaunchKernelGGL((exact_recheck_unit<T, false>), dim3(grid), dim3(256),
                       0, s, (const T*)j.X, j.d, vec, o.C64, o.CT, o.k, tpf,
                       j.flags, j.ucnt, g.grid, S, g.cap, j.labels, j.u, j.row, j.conv,
                       j.iter, j.dirty);
}

hipError_t launch_recheck(const CentroidOps& o, const AssignJob& j,
                          hipStream_t s) {
  const TileGeom g = tile_geometry(o, j.dt, j.n, j.seg_cnt != nullptr, j.nseg);
  int tpf = 1;
  while (tpf < o.k && tpf < 256) tpf *= 2;
  switch (j.dt) {
    case KNOR_F32: launch_recheck_t<float>(o, j, g, tpf, s); break;
    case KNOR_BF16: launch_recheck_t<uint16_t>(o, j, g, tpf, s); break;
    default:
      return hipSuccess;   // FP64 data never uses the recheck list
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// exact per-point distance to the assigned centroid, and the canonical sum
// ---------------------------------------------------------------------------

// dist2_canon of each point and its centroid, its operations in its order;
// the operands of 8 dimensions are loaded together before they are summed
// (every load in range: the last dimension stands in past d).  VEC: d is a
// multiple of 8 and both rows start on 16 bytes, so the 8 dimensions come
// in 16-byte pieces.
constexpr int kDist2Dims = 8;

template <typename T, bool VEC>
__global__ __launch_bounds__(256) void exact_dist2_kernel(
    const T* __restrict__ X, int64_t n, int d, const double* __restrict__ C64,
    const int32_t* __restrict__ labels, double* __restrict__ out) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const T* x = X + (size_t)p * d;
  const double* c = C64 + (size_t)labels[p] * d;
  double acc = 0.0;
  for (int d0 = 0; d0 < d; d0 += kDist2Dims) {
    double xv[kDist2Dims], cv[kDist2Dims];
    if constexpr (VEC) {
      constexpr int XE = 16 / (int)sizeof(T);          // elements per 16-byte piece
      static_assert(kDist2Dims % XE == 0 || XE > kDist2Dims, "piece size");
      if constexpr (XE <= kDist2Dims) {
#pragma unroll
        for (int q = 0; q < kDist2Dims / XE; ++q) {
          const uint4 w = *reinterpret_cast<const uint4*>(x + d0 + q * XE);
          const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
          for (int r = 0; r < XE; ++r) xv[q * XE + r] = to_f64<T>(e[r]);
        }
      } else {
        // 8 BF16 values are one 16-byte piece
        const uint4 w = *reinterpret_cast<const uint4*>(x + d0);
        const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
        for (int r = 0; r < kDist2Dims; ++r) xv[r] = to_f64<T>(e[r]);
      }
#pragma unroll
      for (int q = 0; q < kDist2Dims / 2; ++q) {
        const double2 w = *reinterpret_cast<const double2*>(c + d0 + 2 * q);
        cv[2 * q] = w.x;
        cv[2 * q + 1] = w.y;
      }
    } else {
#pragma unroll
      for (int e = 0; e < kDist2Dims; ++e) {
        const int i = d0 + e < d ? d0 + e : d - 1;
        xv[e] = to_f64<T>(x[i]);
        cv[e] = c[i];
      }
    }
#pragma unroll
    for (int e = 0; e < kDist2Dims; ++e)
      if (d0 + e < d) {
        const double t = __dsub_rn(xv[e], cv[e]);
        acc = __dadd_rn(acc, __dmul_rn(t, t));
      }
  }
  out[p] = acc;
}

template <typename T>
static void launch_dist2_t(const T* X, int64_t n, int d, const double* C64,
                           const int32_t* labels, double* out, bool vec, hipStream_t s) {
  const int64_t blocks = (n + 255) / 256;
  auto kern = vec ? exact_dist2_kernel<T, true> : exact_dist2_kernel<T, false>;
  hipLaunchKernelGGL(kern, dim3(blocks), dim3(256), 0, s, X, n, d, C64, labels, out);
}

hipError_t launch_exact_dist2(const void* X, knor_dtype dt, int64_t n, int d,
                              const double* C64, const int32_t* labels,
                              double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const bool vec = d % kDist2Dims == 0 && ((uintptr_t)X & 15) == 0 && ((uintptr_t)C64 & 15) == 0;
  switch (dt) {
    case KNOR_F64:
      launch_dist2_t<double>((const double*)X, n, d, C64, labels, out, vec, s);
      break;
    case KNOR_F32:
      launch_dist2_t<float>((const float*)X, n, d, C64, labels, out, vec, s);
      break;
    case KNOR_BF16:
      launch_dist2_t<uint16_t>((const uint16_t*)X, n, d, C64, labels, out, vec, s);
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
// each range at the largest power of two below its length.  Strides below
// kTreeRun stay inside aligned runs of kTreeRun nodes: tree_runs takes them,
// one workgroup per run in LDS, and leaves each run's node at its first
// position; tree_scalar takes the strides from s0 on.
constexpr int kTreeRun = 1024;

__global__ __launch_bounds__(kTreeRun / 2) void tree_runs(double* __restrict__ t, int64_t m) {
  __shared__ double sv[kTreeRun];
  const int64_t b0 = (int64_t)blockIdx.x * kTreeRun;
  for (int i = threadIdx.x; i < kTreeRun; i += blockDim.x) sv[i] = b0 + i < m ? t[b0 + i] : 0.0;
  __syncthreads();
  for (int s = 1; s < kTreeRun; s <<= 1) {
    for (int i = threadIdx.x; i * 2 * s + s < kTreeRun; i += blockDim.x) {
      const int a = i * 2 * s;
      if (b0 + a + s < m) sv[a] = __dadd_rn(sv[a], sv[a + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) t[b0] = sv[0];
}

__global__ __launch_bounds__(1024) void tree_scalar(double* __restrict__ t,
                                                    int64_t m, int64_t s0,
                                                    double* __restrict__ out) {
  for (int64_t s = s0; s < m; s <<= 1) {
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
  int64_t s0 = 1;
  if (leaves > kTreeRun) {
    hipLaunchKernelGGL(tree_runs, dim3((unsigned)((leaves + kTreeRun - 1) / kTreeRun)),
                       dim3(kTreeRun / 2), 0, s, tmp, leaves);
    s0 = kTreeRun;
  }
  hipLaunchKernelGGL(tree_scalar, dim3(1), dim3(1024), 0, s, tmp, leaves, s0, out);
  return hipGetLastError();
}

}  // namespace knor
