// Assignment step: nearest centroid of every point (Mhembere et al., HPDC'17,
// Algorithm 1, the nearest-centroid loop with a strict "<").
//
// This file holds the centroid operands, the exact FP64 assignment (the
// definition itself, used for FP64 data), the FP64 recheck of the points the
// FP32 tile (tile_f32.hip) could not decide, and the canonical FP64 objective.
#include <float.h>
#include <math.h>

#include "common.h"

namespace knor {

// ---------------------------------------------------------------------------
// centroid operands
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t bf16_rne(double c) {
  uint64_t b = (uint64_t)__double_as_longlong(c);
  double a = fabs(c);
  uint16_t out = 0;
  if (a != 0.0) {
    int e = ilogb(a);
    if (e < -126) e = -126;
    double r = rint(ldexp(a, 7 - e));
    float y = (float)ldexp(r, e - 7);
    out = (uint16_t)(__float_as_uint(y) >> 16);
  }
  return out | (uint16_t)((b >> 48) & 0x8000u);
}

// One wave per centroid row: Cm2 = -2 * RNE_fp32(c) (exact scaling), zero
// padded to dp columns; cn = RNE_fp32(|c|^2) with the sum in FP64 index
// order; CT = transposed FP64 copy.  Rows k..kpad-1 are padding: Cm2 = 0,
// cn = +inf (they can never be chosen).
__global__ __launch_bounds__(256) void prep_centroids_kernel(
    const double* __restrict__ C64, int k, int kpad, int d, int dp,
    float* __restrict__ Cm2, float* __restrict__ cn, double* __restrict__ CT,
    uint16_t* __restrict__ Cbf) {
  int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (j >= kpad) return;
  for (int i = lane; i < dp; i += 64) {
    double c = (j < k && i < d) ? C64[(size_t)j * d + i] : 0.0;
    Cm2[(size_t)j * dp + i] = -2.0f * (float)c;
    if (Cbf) Cbf[(size_t)j * dp + i] = bf16_rne(c);
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
                     o.C64, o.k, o.kpad, o.d, o.dp, o.Cm2, o.cn, o.CT, o.Cbf);
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
      labels[p] = a;
      if (old != a) {
        changed = true;
        mark_dirty(dirty, old, a);
      }
      if (ub) ub[p] = f32_up(sqrt(best) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
    }
    wave_count_changed(changed, row, (int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
  }
}

// The FP64 recheck.  One workgroup per recheck slice (one slice per tile
// workgroup); its 256 threads are split into groups of tpf threads
// (tpf = min(256, pow2 >= k)), each group takes one of the slice's near-tie
// points and its threads split the centroids, so all (point, centroid)
// distances of a slice are in flight at once.  Each distance is the
// canonical FP64 form; the transposed centroid copy makes the threads' reads
// contiguous.  The lexicographic (D, j) minimum is the lowest-index argmin.
template <typename T>
__global__ __launch_bounds__(256) void exact_recheck_unit(
    const T* __restrict__ X, int d, const double* __restrict__ CT, int k,
    int tpf, const int* __restrict__ flags, const int* __restrict__ ucnt,
    int64_t cap, int32_t* __restrict__ labels,
    float* __restrict__ ub, unsigned long long* __restrict__ row,
    const int* __restrict__ conv, int iter, int* __restrict__ dirty) {
  __shared__ double red_d[4];
  __shared__ int red_j[4];
  if (*conv < iter) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int G = 256 / tpf;                   // points per pass
  const int gsel = threadIdx.x / tpf, t = threadIdx.x % tpf;
  unsigned long long changes = 0;
  {
    const int64_t unit = blockIdx.x;
    const int nf = ucnt[unit];               // uniform over the workgroup
    for (int f0 = 0; f0 < nf; f0 += G) {
      const int f = f0 + gsel;
      const bool live_f = f < nf;
      const int p = live_f ? flags[unit * cap + f] : 0;
      const T* x = X + (size_t)p * d;
      double best = INFINITY;
      int a = 0x7fffffff;
      constexpr int kC = 16;                 // dimensions loaded together
      for (int j = t; live_f && j < k; j += tpf) {
        double acc = 0.0;
        for (int i0 = 0; i0 < d; i0 += kC) {
          double cv[kC], xv[kC];
#pragma unroll
          for (int q = 0; q < kC; ++q) {
            const bool in = i0 + q < d;
            cv[q] = in ? CT[(size_t)(i0 + q) * k + j] : 0.0;
            xv[q] = in ? to_f64<T>(x[i0 + q]) : 0.0;
          }
#pragma unroll
          for (int q = 0; q < kC; ++q)
            if (i0 + q < d) {
              const double dd = __dsub_rn(xv[q], cv[q]);
              acc = __dadd_rn(acc, __dmul_rn(dd, dd));
            }
        }
        if (acc < best) { best = acc; a = j; }
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
        const int32_t old = labels[p];
        labels[p] = a;
        if (old != a) {
          ++changes;
          mark_dirty(dirty, old, a);
        }
        if (ub) ub[p] = f32_up(sqrt(best) * (1.0 + (double)(d + 4) * 2.220446049250313e-16));
      }
    }
  }
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
  return hipErrorNotSupported;
}

hipError_t launch_recheck(const CentroidOps& o, const AssignJob& j,
                          hipStream_t s) {
  const TileGeom g = tile_f32_geometry(o.dp, o.kpad, j.n, j.seg_cnt != nullptr,
                                       j.nseg);
  int tpf = 1;
  while (tpf < o.k && tpf < 256) tpf *= 2;
  switch (j.dt) {
    case KNOR_F32:
      hipLaunchKernelGGL(exact_recheck_unit<float>, dim3(g.grid), dim3(256), 0, s,
                         (const float*)j.X, j.d, o.CT, o.k, tpf, j.flags, j.ucnt,
                         g.cap, j.labels, j.u, j.row, j.conv, j.iter,
                         j.dirty);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(exact_recheck_unit<uint16_t>, dim3(g.grid), dim3(256), 0,
                         s, (const uint16_t*)j.X, j.d, o.CT, o.k, tpf, j.flags,
                         j.ucnt, g.cap, j.labels, j.u, j.row, j.conv,
                         j.iter, j.dirty);
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
