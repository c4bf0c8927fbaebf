// Minimal triangle inequality (MTI) pruning (Mhembere et al., HPDC'17,
// Section "Minimal Triangle Inequality (MTI) Pruning").
//
// State: one upper bound u(x) >= d(x, c_a(x)) per point (FP32, rounded up),
// the centroid drift f(c) = d(c^t, c^{t-1}) (rounded up), and
// s(c) = 1/2 min_{j != c} d(c, j) (rounded down) -- the paper's
// centroid-to-centroid distance term with Elkan's factor 1/2.
//
// Per iteration t >= 1, for every point (mti_filter):
//   Clause 1:  u <- u + f(c_a); if u (1 + eta) < s(c_a) the point keeps its
//              centroid and no distance is evaluated.
//   Clause 3:  otherwise tighten u to d(x, c_a) (FP64, rounded up) and test
//              Clause 1 again with the tight bound.
//   Survivors are appended (wave ballot + one atomic per wave) to a list that
//   the assignment tile scans against every centroid.
// The strict test with margin eta keeps every pruned centroid farther than
// the kept one by a relative gap of about 4 eta, far above FP64 rounding, so
// the labels equal the unpruned FP64 argmin.
#include <math.h>

#include "common.h"

namespace knor {

// s_bits[i] <- min over j != i of the rounded-down 1/2 d(c_i, c_j), as the
// bit pattern of a non-negative float (so integer atomicMin orders them).
// Block = one wave of 64 centroids i; blockIdx.y selects a segment of j.
__global__ __launch_bounds__(64) void cc_bounds_kernel(
    const double* __restrict__ C64, int k, int d, int jseg,
    unsigned int* __restrict__ s_bits) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  const int j0 = blockIdx.y * jseg;
  const int j1 = j0 + jseg < k ? j0 + jseg : k;
  if (i >= k) return;
  const double* ci = C64 + (size_t)i * d;
  double best = INFINITY;
  for (int j = j0; j < j1; ++j) {
    if (j == i) continue;
    double D = dist2_canon<double>(ci, C64 + (size_t)j * d, d);
    best = D < best ? D : best;
  }
  if (best < INFINITY) {
    float v = f32_down(0.5 * sqrt(best) * (1.0 - (double)(d + 8) * 2.220446049250313e-16));
    atomicMin(&s_bits[i], __float_as_uint(v));
  }
}

__global__ void fill_u32(unsigned int* p, int n, unsigned int v) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_cc_bounds(const double* C64, int k, int d, float* s_half,
                            hipStream_t s) {
  unsigned int* bits = reinterpret_cast<unsigned int*>(s_half);
  hipLaunchKernelGGL(fill_u32, dim3((k + 255) / 256), dim3(256), 0, s, bits, k,
                     0x7f800000u /* +inf */);
  const int jseg = 128;
  dim3 grid((k + 63) / 64, (k + jseg - 1) / jseg);
  hipLaunchKernelGGL(cc_bounds_kernel, grid, dim3(64), 0, s, C64, k, d, jseg,
                     bits);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(256) void mti_filter_kernel(
    const T* __restrict__ X, int64_t n, int d, const double* __restrict__ C64,
    const int32_t* __restrict__ labels, float* __restrict__ u,
    const float* __restrict__ drift, const float* __restrict__ s_half,
    int* __restrict__ survivors, unsigned long long* __restrict__ ctr,
    const int* __restrict__ done) {
  if (*done) return;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x; p0 < n; p0 += stride) {
    const int64_t p = p0 + threadIdx.x;
    const bool valid = p < n;
    bool pa = false, pb = false, surv = false;
    if (valid) {
      const int a = labels[p];
      const double s = (double)s_half[a];
      // Clause 1 with the drift-updated bound
      double ub = f32_up(((double)u[p] + (double)drift[a]) * (1.0 + 8.881784197001252e-16));
      if (ub * (1.0 + kEta) < s) {
        pa = true;
      } else {
        // Clause 3: tighten to the exact distance, then Clause 1 again
        double D = dist2_canon<T>(X + (size_t)p * d, C64 + (size_t)a * d, d);
        ub = f32_up(sqrt(D) * (1.0 + (double)(d + 8) * 2.220446049250313e-16));
        if (ub * (1.0 + kEta) < s) pb = true; else surv = true;
      }
      u[p] = (float)ub;
    }
    wave_count(pa, &ctr[CNT_PRUNED_A]);
    wave_count(pb, &ctr[CNT_PRUNED_B]);
    wave_append(surv, (int)p, &ctr[CNT_SURVIVORS], survivors);
  }
}

hipError_t launch_mti_filter(const void* X, knor_dtype dt, int64_t n, int d,
                             const double* C64, const int32_t* labels,
                             float* u, const float* drift, const float* s_half,
                             int* survivors, unsigned long long* ctr,
                             const int* done, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  int grid = (int)(blocks < 8192 ? (blocks < 1 ? 1 : blocks) : 8192);
  switch (dt) {
    case KNOR_F64:
      hipLaunchKernelGGL(mti_filter_kernel<double>, dim3(grid), dim3(256), 0, s,
                         (const double*)X, n, d, C64, labels, u, drift, s_half,
                         survivors, ctr, done);
      break;
    case KNOR_F32:
      hipLaunchKernelGGL(mti_filter_kernel<float>, dim3(grid), dim3(256), 0, s,
                         (const float*)X, n, d, C64, labels, u, drift, s_half,
                         survivors, ctr, done);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(mti_filter_kernel<uint16_t>, dim3(grid), dim3(256), 0,
                         s, (const uint16_t*)X, n, d, C64, labels, u, drift,
                         s_half, survivors, ctr, done);
      break;
  }
  return hipGetLastError();
}

}  // namespace knor
