// Pieces shared by the two centroid updates (the canonical sum and the exact
// mean): the leaf lookup, the close of an iteration and the write of one
// centroid with the operands derived from it.
#pragma once

#include "common.h"

namespace knor {

// Largest j with leaf_off[j] <= g (leaves are numbered cluster by cluster).
__device__ __forceinline__ int cluster_of_leaf(const int* leaf_off, int k, int g) {
  int lo = 0, hi = k - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (leaf_off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// The iteration's bookkeeping, run by every thread of one workgroup: totals
// of the spread counter slots, the MTI counters, and the stopping rule
// (#changed <= tol * n).
__device__ __forceinline__ void close_iteration(const IterCtl& ctl, int iter) {
  // fold the spread slots: thread (q, i) loads slot i of quantity q
  __shared__ unsigned long long slot[NSLOTQ * kChgSlots];
  unsigned long long* row = ctl.row;
  if (threadIdx.x < NSLOTQ * kChgSlots) slot[threadIdx.x] = row[threadIdx.x * kSlotStride];
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot[NSLOTQ];
    for (int q = 0; q < NSLOTQ; ++q) {
      unsigned long long s = 0;
      for (int i = 0; i < kChgSlots; ++i) s += slot[q * kChgSlots + i];
      tot[q] = s;
    }
    row[ROW_CHANGED] = tot[SLOT_CHANGED];
    row[ROW_FLAG_HEAD] = tot[SLOT_FLAGGED];
    row[ROW_CERTIFIED] = tot[SLOT_CERTIFIED];
    row[ROW_DISTS] = tot[SLOT_DISTS];
    if (ctl.segmented) {
      row[ROW_SURVIVED] = tot[SLOT_SURV];
      row[ROW_SCANNED] = tot[SLOT_SURV] - tot[SLOT_CERTIFIED];
      row[ROW_PRUNED_A] = (unsigned long long)ctl.n - tot[SLOT_CAND];
      row[ROW_PRUNED_B] = tot[SLOT_CAND] - tot[SLOT_SURV];
      // keep tightening while it prunes at least 1/16 of its candidates
      row[ROW_TIGHTEN_NEXT] =
          row[ROW_TIGHTEN] && 16 * (tot[SLOT_CAND] - tot[SLOT_SURV]) >= tot[SLOT_CAND];
    } else {
      row[ROW_SCANNED] = (unsigned long long)ctl.n;
    }
    if ((double)tot[SLOT_CHANGED] <= ctl.tol_n) *ctl.conv = iter;
  }
}

// Centroid j of a dirty cluster, by every thread of a 256-thread workgroup:
// mean_of(dim) when the cluster has members, else the previous value; then
// the FP64 copy (row- and dimension-major), the drift bound f(c), the
// squared norm and the FP32 / BF16 operands of the distance tiles, and the
// dirty flag is cleared.
template <class MeanOf>
__device__ __forceinline__ void write_centroid(
    int j, int k, int d, int cntj, MeanOf mean_of, const double* C_prev,
    double* C_out, double* __restrict__ CT, float* __restrict__ Cm2,
    float* __restrict__ cn, int dp, uint16_t* __restrict__ Chi,
    uint16_t* __restrict__ Clo, int dpb, float* __restrict__ drift,
    int* __restrict__ dirty) {
  __shared__ double red[256];
  __shared__ double cval[kMaxD];
  double diff2 = 0.0;
  for (int dim = threadIdx.x; dim < d; dim += blockDim.x) {
    double old = C_prev[(size_t)j * d + dim];
    double c = cntj > 0 ? mean_of(dim) : old;
    C_out[(size_t)j * d + dim] = c;
    if (CT) CT[(size_t)dim * k + j] = c;
    cval[dim] = c;
    double t = __dsub_rn(c, old);
    diff2 = __dadd_rn(diff2, __dmul_rn(t, t));
  }
  red[threadIdx.x] = diff2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = __dadd_rn(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (drift)
      drift[j] = f32_up(sqrt(red[0]) * (1.0 + (double)(d + 8) * 2.220446049250313e-16));
    if (cn) {
      double ss = 0.0;
      for (int dim = 0; dim < d; ++dim) ss = __dadd_rn(ss, __dmul_rn(cval[dim], cval[dim]));
      cn[j] = (float)ss;
    }
    if (dirty) dirty[j] = 0;
  }
  if (Cm2)
    for (int dim = threadIdx.x; dim < dp; dim += blockDim.x)
      Cm2[(size_t)j * dp + dim] = dim < d ? -2.0f * (float)cval[dim] : 0.0f;
  if (Chi)
    for (int dim = threadIdx.x; dim < dpb; dim += blockDim.x) {
      uint16_t h, l;
      bf16_split_m2(dim < d ? cval[dim] : 0.0, h, l);
      Chi[(size_t)j * dpb + dim] = h;
      Clo[(size_t)j * dpb + dim] = l;
    }
}

}  // namespace knor
