// Shared device helpers and host-side launch interfaces of the k-means library.
//
// Numerical conventions (Mhembere et al., HPDC'17, Section "Nomenclature":
// Euclidean distance; Algorithm 1: strict "<" nearest-centroid scan):
//  * dist2_canon() is THE definition of a point-centroid squared distance:
//    FP64, index order, one rounding per subtract/multiply/add, no FMA
//    (this library is compiled with -ffp-contract=off).
//  * Faster, lower-precision distance forms are only used together with a
//    proven error bound; whatever the bound cannot decide is recomputed with
//    dist2_canon().
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "knor.h"

namespace knor {

constexpr int kWave = 64;
constexpr int kLeaf = 64;          // members per leaf of the canonical sum
constexpr double kEta = 9.5367431640625e-07;   // 2^-20: relative pruning margin
constexpr int kMaxD = 256;
constexpr int kMaxK = 16384;

// per-iteration device counters (unsigned long long each), one row per
// iteration; columns 0..4 mirror KNOR_CNT_*; the rest are list heads.
enum {
  CNT_CHANGED = KNOR_CNT_CHANGED,
  CNT_SCANNED = KNOR_CNT_SCANNED,
  CNT_PRUNED_A = KNOR_CNT_PRUNED_A,
  CNT_PRUNED_B = KNOR_CNT_PRUNED_B,
  CNT_RECHECKED = KNOR_CNT_RECHECKED,  // = length of the FP64 recheck list
  CNT_SURVIVORS = 5,                   // = length of the survivor list
  CNT_ROWS = 8
};

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

#if defined(__HIP_DEVICE_COMPILE__)
#pragma clang fp contract(off)
#endif

template <typename T>
__device__ __forceinline__ double to_f64(T v);
template <>
__device__ __forceinline__ double to_f64<double>(double v) { return v; }
template <>
__device__ __forceinline__ double to_f64<float>(float v) { return (double)v; }
template <>
__device__ __forceinline__ double to_f64<uint16_t>(uint16_t v) {
  return (double)__uint_as_float(((uint32_t)v) << 16);   // BF16 bit pattern
}

// The canonical squared distance (FP64, index order, no contraction).
template <typename T>
__device__ __forceinline__ double dist2_canon(const T* __restrict__ x,
                                              const double* __restrict__ c,
                                              int d) {
  double acc = 0.0;
  for (int i = 0; i < d; ++i) {
    double t = __dsub_rn(to_f64<T>(x[i]), c[i]);
    double t2 = __dmul_rn(t, t);
    acc = __dadd_rn(acc, t2);
  }
  return acc;
}

// Smallest float >= v (v >= 0 finite, or +inf).
__device__ __forceinline__ float f32_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
  return f;
}

// Largest float <= v (v >= 0).
__device__ __forceinline__ float f32_down(double v) {
  float f = (float)v;
  if ((double)f > v) f = __uint_as_float(__float_as_uint(f) - 1u);
  return f;
}

__device__ __forceinline__ int lane_id() {
  return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0));
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Append the calling lanes whose `want` is true to list[], in an order that
// does not matter to any result; head is the list length counter.
__device__ __forceinline__ void wave_append(bool want, int value,
                                            unsigned long long* head,
                                            int* list) {
  uint64_t m = __ballot(want);
  if (m == 0) return;
  int cnt = __popcll(m);
  int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if (lane_id() == leader) base = atomicAdd(head, (unsigned long long)cnt);
  base = __shfl(base, leader);
  if (want) list[base + __popcll(m & lanemask_lt())] = value;
}

// Add a per-lane 0/1 predicate count of the whole wave to *ctr.
__device__ __forceinline__ void wave_count(bool pred, unsigned long long* ctr) {
  uint64_t m = __ballot(pred);
  if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
    atomicAdd(ctr, (unsigned long long)__popcll(m));
}

}  // namespace knor

// ---------------------------------------------------------------------------
// host-side launch interfaces (each implemented next to its kernels)
// ---------------------------------------------------------------------------
namespace knor {

// Centroid operands derived from the FP64 centroids.
struct CentroidOps {
  double* C64;     // k x d canonical centroids
  float* Cm2;      // kpad x dp: -2 * fp32(c), zero-padded; pad rows zero
  float* cn;       // kpad: fp32(|c|^2) (pad rows +inf)
  uint16_t* Cbf;   // kpad x dp BF16 rounding of c (BF16 path only) or null
  int k, kpad, d, dp;
};

// Arguments of one assignment pass over a point set.
struct AssignJob {
  const void* X;
  knor_dtype dt;
  int64_t n;
  int d;
  const int* list;                   // survivor indices, or null = all points
  const unsigned long long* list_len;// device length of `list` (if list)
  int32_t* labels;                   // in: previous labels; out: new labels
  float* u;                          // MTI upper bounds (or null)
  int* flags;                        // FP64 recheck list (n entries)
  unsigned long long* ctr;           // this iteration's counter row
  const int* done;                   // skip all work when *done != 0
  int recheck_all;                   // 2 = send every point to the recheck
  double* dist2;                     // optional per-point exact D (or null)
};

hipError_t launch_prep_centroids(const CentroidOps& ops, hipStream_t s);
hipError_t launch_assign(const CentroidOps& ops, const AssignJob& job,
                         hipStream_t s);
hipError_t launch_recheck(const CentroidOps& ops, const AssignJob& job,
                          hipStream_t s);
hipError_t launch_exact_dist2(const void* X, knor_dtype dt, int64_t n, int d,
                              const double* C64, const int32_t* labels,
                              double* dist2, hipStream_t s);
hipError_t launch_canonical_sum(const double* v, int64_t n, double* tmp,
                                double* out, hipStream_t s);

// Optional GPU timing of kernel groups with HIP events on the launch stream.
struct Prof {
  hipStream_t stream = nullptr;
  bool on = false;
  std::vector<int> groups;
  std::vector<hipEvent_t> starts, ends;
  void begin(int g);
  void end();
  // adds elapsed milliseconds and launch counts per group (stream synced)
  void collect(double* ms, int64_t* launches);
  ~Prof();
};

// Two-pass segmented update.
struct UpdatePlan {
  int64_t n;
  int k, d;
  int B;              // points per histogram block
  int nb;             // number of blocks
  // device workspace
  int* blockcnt;      // nb x k (block-major)
  int* nj;            // k: members per cluster
  int* off;           // k+1: first member slot of each cluster
  int* leaf_off;      // k+1: first leaf of each cluster
  int* perm;          // n: point indices sorted by (label, index)
  double* leafsum;    // (n/64 + k) x d
  int64_t max_leaves;
};
size_t update_workspace_bytes(int64_t n, int k, int d);
void update_plan_init(UpdatePlan* p, int64_t n, int k, int d, void* ws);
hipError_t launch_update(const UpdatePlan& p, const void* X, knor_dtype dt,
                         const int32_t* labels, const double* C_prev,
                         double* C_out, int64_t* counts_out,
                         CentroidOps* ops /* may be null */,
                         float* drift /* may be null */, const int* done,
                         hipStream_t s, Prof* prof = nullptr);

// MTI.
hipError_t launch_cc_bounds(const double* C64, int k, int d, float* s_half,
                            hipStream_t s);
hipError_t launch_mti_filter(const void* X, knor_dtype dt, int64_t n, int d,
                             const double* C64, const int32_t* labels,
                             float* u, const float* drift, const float* s_half,
                             int* survivors, unsigned long long* ctr,
                             const int* done, hipStream_t s);

// Misc.
hipError_t launch_check_finite(const void* p, knor_dtype dt, int64_t count,
                               int* bad, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v,
                           const int* done, hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t count,
                           const int* done, hipStream_t s);
hipError_t launch_converge(const unsigned long long* ctr, double tol_n,
                           int t, int* done, int* iters, hipStream_t s);
hipError_t launch_gather_rows(const void* X, knor_dtype dt, int d,
                              const int64_t* rows, int k, double* C64,
                              hipStream_t s);

inline int pad_dim(int d) {
  int p = 8;
  while (p < d) p *= 2;
  return p;
}

}  // namespace knor
