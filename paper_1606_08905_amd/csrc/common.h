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
constexpr int kSeg = 4096;         // points per MTI filter block / list segment

// Per-iteration device counter row (unsigned long long entries).  Partial
// counts are added by workgroups into kChgSlots slots per quantity, one slot
// per 128-byte line, so that concurrent atomic adds do not serialise on one
// address; the iteration's last kernel folds them into the totals.
constexpr int kChgSlots = 32;
constexpr int kSlotStride = 16;
enum {
  SLOT_CHANGED = 0,                          // labels changed
  SLOT_FLAGGED = 1,                          // points sent to the FP64 recheck
  SLOT_CAND = 2,                             // MTI stage-A candidates
  SLOT_SURV = 3,                             // MTI survivors
  SLOT_CERTIFIED = 4,                        // survivors certified by a proposal
  SLOT_DISTS = 5,                            // distances of the candidate-list tile
  NSLOTQ = 6,
  ROW_CHANGED = NSLOTQ * kChgSlots * kSlotStride,   // totals
  ROW_SCANNED = ROW_CHANGED + 1,
  ROW_PRUNED_A = ROW_CHANGED + 2,
  ROW_PRUNED_B = ROW_CHANGED + 3,
  ROW_FLAG_HEAD = ROW_CHANGED + 4,           // FP64 rechecked points
  ROW_TIGHTEN = ROW_CHANGED + 5,             // 1 if stage B ran
  ROW_TIGHTEN_NEXT = ROW_CHANGED + 6,        // 1: run stage B next iteration
  ROW_CERTIFIED = ROW_CHANGED + 7,           // survivors decided by a proposal
  ROW_SURVIVED = ROW_CHANGED + 8,            // survivors of the MTI filter
  ROW_DISTS = ROW_CHANGED + 9,               // distances of the candidate-list tile
  ROW_STRIDE = ROW_CHANGED + 16
};

__device__ __forceinline__ unsigned long long* row_slot(unsigned long long* row,
                                                        int q, int salt) {
  return &row[(q * kChgSlots + (salt & (kChgSlots - 1))) * kSlotStride];
}

constexpr int kNotConverged = 0x7fffffff;

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

// The same value for FP32 rows with d % 4 == 0 (x 16-byte aligned, c
// 16-byte aligned): four dimensions per step from 16-byte loads, issued
// ahead of the FP64 chain, which still runs in index order.
__device__ __forceinline__ double dist2_canon_f32x4(const float* __restrict__ x,
                                                    const double* __restrict__ c, int d) {
  double acc = 0.0;
#pragma unroll 4
  for (int i = 0; i < d; i += 4) {
    const float4 xv = *reinterpret_cast<const float4*>(x + i);
    const double2 c01 = *reinterpret_cast<const double2*>(c + i);
    const double2 c23 = *reinterpret_cast<const double2*>(c + i + 2);
    const double t0 = __dsub_rn((double)xv.x, c01.x);
    acc = __dadd_rn(acc, __dmul_rn(t0, t0));
    const double t1 = __dsub_rn((double)xv.y, c01.y);
    acc = __dadd_rn(acc, __dmul_rn(t1, t1));
    const double t2 = __dsub_rn((double)xv.z, c23.x);
    acc = __dadd_rn(acc, __dmul_rn(t2, t2));
    const double t3 = __dsub_rn((double)xv.w, c23.y);
    acc = __dadd_rn(acc, __dmul_rn(t3, t3));
  }
  return acc;
}

// Smallest float >= v (v >= 0 finite, or +inf).
__device__ __forceinline__ float f32_up(double v) {
  float f = (float)v;
  if ((double)f < v) f = __uint_as_float(__float_as_uint(f) + 1u);
  return f;
}

// MTI Clause 1 with the drift-updated bound (Section "Minimal Triangle
// Inequality (MTI) Pruning"): *ub = u + f(c_a), rounded up; true when
// ub (1 + eta) < s(c_a), i.e. the point keeps its centroid without any
// distance.  The filter and the streamed fetch both decide through this.
__device__ __forceinline__ bool clause1_keeps(float u, float drift, float s_half, float* ub) {
  const double b = f32_up(((double)u + (double)drift) * (1.0 + 8.881784197001252e-16));
  *ub = (float)b;
  return b * (1.0 + kEta) < (double)s_half;
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

// Append the calling lanes whose `want` is true to list[] (used only for the
// rare near-tie points); head is the list length counter.
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

// Add the wave's count of `pred` to one of the spread changed-label slots.
__device__ __forceinline__ void wave_count_changed(bool pred,
                                                   unsigned long long* row,
                                                   int salt) {
  uint64_t m = __ballot(pred);
  if (m && lane_id() == __ffsll((unsigned long long)m) - 1)
    atomicAdd(row_slot(row, SLOT_CHANGED, salt), (unsigned long long)__popcll(m));
}

// Workgroup-wide sums of up to four per-thread counters, added once per
// workgroup into the spread slots q0..q0+nq-1 of `row` (all threads call).
// Workgroup copy of `count` elements: thread t handles elements t, t + nt,
// ... in batches of B, issuing a batch's B loads before its first store, so
// a batch costs one memory round trip (a plain strided loop waits on each
// load before the next).  ld(e) returns element e; st(e, v) stores it.
template <int B, typename V, typename Ld, typename St>
__device__ __forceinline__ void stage_batched(int count, Ld ld, St st) {
  const int nt = (int)blockDim.x;
  for (int e0 = (int)threadIdx.x; e0 < count; e0 += B * nt) {
    V v[B];
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + u * nt;
      if (e < count) v[u] = ld(e);
    }
#pragma unroll
    for (int u = 0; u < B; ++u) {
      const int e = e0 + u * nt;
      if (e < count) st(e, v[u]);
    }
  }
}

template <int NQ>
__device__ __forceinline__ void block_add_slots(unsigned long long* row,
                                                const int (&q)[NQ],
                                                const unsigned long long (&v)[NQ]) {
  __shared__ unsigned long long part[NQ][16];
  const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  unsigned long long s[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    s[i] = v[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s[i] += __shfl_xor(s[i], off);
  }
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < NQ; ++i) part[i][wave] = s[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NQ; ++i) {
      unsigned long long t = 0;
      for (int w = 0; w < nw; ++w) t += part[i][w];
      if (t) atomicAdd(row_slot(row, q[i], blockIdx.x), t);
    }
}

// BF16 round-to-nearest-even of an FP64 value in one rounding (no detour
// through FP32): scale to an 8-bit integer significand at the value's binade
// (binade -126 below the normal range), rint, scale back; the result has at
// most 8 significant bits, so its FP32 image is exact and its upper half is
// the BF16 pattern.
__device__ __forceinline__ uint16_t bf16_rne(double c) {
  const uint64_t b = (uint64_t)__double_as_longlong(c);
  const double a = fabs(c);
  uint16_t out = 0;
  if (a != 0.0) {
    int e = ilogb(a);
    if (e < -126) e = -126;
    const double r = rint(ldexp(a, 7 - e));
    const float y = (float)ldexp(r, e - 7);
    out = (uint16_t)(__float_as_uint(y) >> 16);
  }
  return out | (uint16_t)((b >> 48) & 0x8000u);
}

// The two BF16 terms of -2c used by the BF16 tile: hi = bf16(-2c),
// lo = bf16(-2c - hi) (the difference is exact in FP64).
__device__ __forceinline__ void bf16_split_m2(double c, uint16_t& hi, uint16_t& lo) {
  const double m2 = -2.0 * c;
  hi = bf16_rne(m2);
  const double hv = (double)__uint_as_float(((uint32_t)hi) << 16);
  lo = bf16_rne(m2 - hv);
}

// Record a label change: both clusters lose/gain a member.
__device__ __forceinline__ void mark_dirty(int* dirty, int old_lab, int new_lab) {
  if (!dirty) return;
  dirty[new_lab] = 1;
  if (old_lab >= 0) dirty[old_lab] = 1;
}

}  // namespace knor

// ---------------------------------------------------------------------------
// host-side launch interfaces (each implemented next to its kernels)
// ---------------------------------------------------------------------------
namespace knor {

// Centroid operands derived from the FP64 centroids.
struct CentroidOps {
  double* C64;     // k x d canonical centroids
  double* CT;      // d x k transposed copy (coalesced per-centroid lanes)
  float* Cm2;      // kpad x dp: -2 * fp32(c), zero-padded; pad rows zero
  float* cn;       // kpad: fp32(|c|^2) (pad rows +inf)
  uint16_t* Chi;   // kpad x dpb BF16 bf16(-2c), zero-padded (BF16 path) or null
  uint16_t* Clo;   // kpad x dpb BF16 bf16(-2c - Chi) (BF16 path) or null
  int k, kpad, d, dp, dpb;
  int tpb, tres;   // FP32 tile schedule: point blocks of 16 per wave, resident
};

// The point set one assignment pass covers.
//  dense:      all n points (seg_cnt == null)
//  segmented:  segment b holds seg_cnt[b] point indices at list[b*kSeg ...]
// The FP32 tile runs a grid of TileGeom::grid workgroups; workgroup b writes
// its near-tie points to flags[b*cap ...] and their number to ucnt[b], and
// the FP64 recheck reads the same slices.  Counts of changed labels go to
// the spread slots of `row`.
struct AssignJob {
  const void* X;
  knor_dtype dt;
  int64_t n;
  int d;
  const int* list;
  const int* seg_cnt;
  int nseg;
  int32_t* labels;                   // in: previous labels; out: new labels
  float* u;                          // MTI upper bounds (or null)
  int* flags;                        // per-workgroup recheck slices
  int* ucnt;                         // per workgroup: recheck slice length
  unsigned long long* row;           // this iteration's counter row
  const int* conv;                   // skip when *conv < iter
  int iter;
  int* dirty;                        // clusters whose membership changed
  int recheck_all;                   // 1 = send every point to the recheck
};

// Launch geometry of the FP32 tile (padded dimension dp, padded centroid
// count kpad) for a dense pass over n points or a segmented pass over nseg
// segments: grid size and per-workgroup recheck slice capacity.
constexpr int kTileMaxGrid = 2048;
struct TileGeom {
  int grid;
  int64_t cap;
  bool resident;
};
bool tile_f32_resident(int dp, int kpad);
bool tile_f32_pb_ok(int dp, int pb);
void tile_f32_default(int dp, int kpad, int* pb, int* resident);
TileGeom tile_f32_geometry(int dp, int kpad, int pb, int resident, int64_t n,
                           bool segmented, int nseg);
bool tile_bf16_resident(int dpb, int kpad);
TileGeom tile_bf16_geometry(int dpb, int kpad, int64_t n, bool segmented, int nseg);
// the geometry of the tile that serves points of type dt
TileGeom tile_geometry(const CentroidOps& o, knor_dtype dt, int64_t n,
                       bool segmented, int nseg);
// entries the flags array needs for either kind of pass
int64_t tile_flag_capacity(const CentroidOps& o, knor_dtype dt, int64_t n,
                           int nseg);
hipError_t launch_tile_f32(const CentroidOps& o, const AssignJob& j,
                           hipStream_t s);
hipError_t launch_tile_bf16(const CentroidOps& o, const AssignJob& j,
                            hipStream_t s);
// The tiles' FP32 values and bounds (for checking the bound): Y (n x k),
// E (n); operands as prepared by launch_prep_centroids.
hipError_t launch_tile_values_f32(const CentroidOps& o, const float* X, int64_t n, int d,
                                  float* Y, double* E, hipStream_t s);
hipError_t launch_tile_values_bf16(const CentroidOps& o, const uint16_t* X, int64_t n,
                                   int d, float* Y, double* E, hipStream_t s);
// The survivor pass with Clause 2 per block of survivors (tile_cand.hip):
// FP32 points, k <= kCandMaxK; the job's segmented list holds the
// survivors, each with a set sign bit in u; rows: the neighbour rows of
// launch_cc_bounds; ws: cand_workspace_bytes(n, k).
constexpr int kCandMaxK = 8192;
constexpr int kCandMinK = 1024;      // default use from this many centroids
size_t cand_workspace_bytes(int64_t n, int k);
hipError_t launch_tile_cand(const CentroidOps& o, const AssignJob& j, const float* rows,
                            void* ws, hipStream_t s);

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
  int mask = ~0;
  int every = 1, iter = 0;   // time only iterations with iter % every == 0
  bool open = false;
  std::vector<int> groups;
  std::vector<hipEvent_t> starts, ends;
  void begin(int g);
  void end();
  // adds elapsed milliseconds and launch counts per group (stream synced)
  void collect(double* ms, int64_t* launches);
  ~Prof();
};

// Two-pass segmented update.
// first tree stage: blocks of TB leaves (a power of two), TB x d doubles
// within kTreeBlockDoubles of LDS
constexpr int kTreeBlockDoubles = 4096;
inline int tree_block_leaves(int d) {
  int tb = 64;
  while (tb > 1 && tb * d > kTreeBlockDoubles) tb >>= 1;
  return tb;
}

struct UpdatePlan {
  int64_t n;
  int k, d;
  int B;              // points per histogram block
  int nb;             // number of blocks
  int seglen;         // blocks per column-scan segment
  int nsegc;          // column-scan segments
  int* blockcnt;      // nb x k (block-major) label counts
  int* segsum;        // nsegc x k: exclusive prefix over segments
  int* ticket;        // last-block-done counter of the segment scan
  int* nj;            // k: members per cluster
  int* off;           // k+1: first member slot of each cluster
  int* leaf_off;      // k+1: first leaf of each cluster
  int* rpre;          // nb x k: exclusive prefix over ranges (fused sort)
  int* perm;          // n: point indices sorted by (label, index)
  double* leafsum;    // (n/64 + k) x d
  int64_t max_leaves;
  int tb;             // leaves per block of the first tree stage
};
size_t update_workspace_bytes(int64_t n, int k, int d);
void update_plan_init(UpdatePlan* p, int64_t n, int k, int d, void* ws);
hipError_t update_plan_reset(const UpdatePlan& p, hipStream_t s);

// Iteration bookkeeping that rides on the update's last kernel.
struct IterCtl {
  unsigned long long* row = nullptr;  // counter row of this iteration
  int* conv = nullptr;                // iteration that converged (or max int)
  int iter = 0;
  double tol_n = 0.0;
  int segmented = 0;                  // MTI survivors were scanned
  int64_t n = 0;
  // MTI survivors of this iteration (every point whose label may have
  // changed): list[s * kSeg + i] for i < seg_cnt[s], s < nseg; null: all
  const int* list = nullptr;
  const int* seg_cnt = nullptr;
  int nseg = 0;
  int delta_only = 0;                 // exact update: moved points only
};

hipError_t launch_update(const UpdatePlan& p, const void* X, knor_dtype dt,
                         const int32_t* labels, const double* C_prev,
                         double* C_out, int64_t* counts_out,
                         CentroidOps* ops /* may be null */,
                         float* drift /* may be null */,
                         int* dirty /* may be null: all clusters */,
                         const IterCtl* ctl /* may be null */, hipStream_t s,
                         Prof* prof = nullptr);

// Pass 1 of the update alone: the stable counting sort (perm, nj, off,
// leaf_off), skipped when *conv < iter.  early = 1: every kernel tests that
// before its first load (for a gate that often skips the sort); early = 0:
// the test overlaps the first loads.
hipError_t launch_sort(const UpdatePlan& p, const int32_t* labels, int* dirty,
                       const int* conv, int iter, hipStream_t s, int early);

// Exact update (FP32 and BF16 points): per (cluster, dimension) kXD signed
// 64-bit digits of weight 2^(16 s - 149); centroids are the exact member
// means rounded once.  Inside a fit (ctl->row set, dirty required) only the
// points whose label changed move between clusters when few do; outside a
// fit (ctl->row null, dirty null) every cluster is summed from scratch.
constexpr int kXD = 20;
struct ExactPlan {
  int64_t n;
  int k, d;
  unsigned long long* slots;   // k x kXD x d digits
  int32_t* prev;               // n: labels at the last update (-1 at start)
  int* gate;                   // this iteration's mode (kNotConverged: full)
  int delta_max;               // most changed labels moved one by one
};
size_t exact_workspace_bytes(int64_t n, int k, int d);
// The pieces of an exact update, for callers that see an iteration's points
// in several passes: enter moves the changed points of one pass (labels and
// prev are that pass's views; rows of X are the pass's rows) into their new
// clusters' digits (and out of the old ones), never choosing the full pass;
// split = 1 whenever the iteration as a whole may move 2^23 or more points.
// finalize divides every dirty cluster's digits once all passes are in.
hipError_t launch_exact_enter(const ExactPlan& xp, int* nj, const void* X, knor_dtype dt,
                              int64_t n, const int* list, const int* seg_cnt, int nseg,
                              const int32_t* labels, int32_t* prev, const int* dirty,
                              const unsigned long long* row, const int* conv, int iter,
                              int split, hipStream_t s);
hipError_t launch_exact_finalize(const ExactPlan& xp, const int* nj, const double* C_prev,
                                 double* C_out, int64_t* counts_out, CentroidOps* ops,
                                 float* drift, int* dirty, const IterCtl& ctl, hipStream_t s);
void exact_plan_init(ExactPlan* p, int64_t n, int k, int d, void* ws);
hipError_t launch_update_exact(const UpdatePlan& p, const ExactPlan& xp, const void* X,
                               knor_dtype dt, const int32_t* labels, const double* C_prev,
                               double* C_out, int64_t* counts_out,
                               CentroidOps* ops /* may be null */,
                               float* drift /* may be null */, int* dirty,
                               const IterCtl* ctl, hipStream_t s, Prof* prof = nullptr);

// MTI.
// rows (optional, k x k): row i lists every centroid j (i included) by
// increasing 1/2 d(c_i, c_j) as float keys: the half distance rounded down,
// its low cc_rows_bits(k) mantissa bits replaced by j; key & ~mask is a
// lower bound of the half distance, key & mask the index.
int cc_rows_bits(int k);
hipError_t launch_cc_bounds(const CentroidOps& ops, float* s_half, float* rows,
                            const int* conv, int iter, hipStream_t s);
// mark = 1: survivors leave the pass with the sign bit of their bound set
// (the candidate-list tile finds them by it), and Clause 3 runs every time.
hipError_t launch_mti_filter(const void* X, knor_dtype dt, int64_t n, int d,
                             const double* C64, const int32_t* labels,
                             float* u, const float* drift, const float* s_half,
                             int* list, int* seg_cnt,
                             const unsigned long long* prev_row,
                             unsigned long long* row, const int* conv,
                             int iter, int mark, hipStream_t s);

// Misc.
hipError_t launch_check_finite(const void* p, knor_dtype dt, int64_t count,
                               int* bad, hipStream_t s, int* kill = nullptr);
hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v,
                           hipStream_t s);
hipError_t launch_copy_i32(const int32_t* src, int32_t* dst, int64_t count,
                           const int* conv, int iter, hipStream_t s);
hipError_t launch_gather_rows(const void* X, knor_dtype dt, int d,
                              const int64_t* rows, int k, double* C64,
                              hipStream_t s);

// k-means++ seeding (init.hip): rnd holds k SplitMix64 outputs, C receives
// k x d FP64 centroids; ws has kmeanspp_workspace_bytes(n, k) bytes.
size_t kmeanspp_workspace_bytes(int64_t n, int k);
hipError_t launch_kmeanspp(const void* X, knor_dtype dt, int64_t n, int d, int k,
                           const unsigned long long* rnd, double* C, void* ws,
                           hipStream_t s);

// Matrix product on the BF16 matrix cores (learned.hip):
// C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]) (ReLU) (masked by
// mask > 0); op = transpose when the flag is set; FP32 in memory, operands
// rounded to BF16 (nearest even), FP32 sums.  Mdev: rows = min(M, *Mdev).
struct GemmArgs {
  const float* A; int lda; int transA;
  const float* B; int ldb; int transB;
  float* C; int ldc;
  int M, N, K;
  const int* Mdev;
  const float* bias;
  int relu;
  const float* mask; int ldm;
};
// part: FP32 workspace of gemm_split_floats(M, N, K) floats for split-K
// partials, or null (no split)
hipError_t launch_gemm_bf16(const GemmArgs& g, float* part, hipStream_t s);
size_t gemm_split_floats(int M, int N, int K);

// The proposal MLP d -> h -> h -> k: offsets of W1 (d x h), b1, W2 (h x h),
// b2, W3 (h x k), b3 in the flat FP32 parameter vector of P entries.
struct MlpLayout {
  int d, h, k;
  int64_t W1, b1, W2, b2, W3, b3, P;
};
MlpLayout mlp_layout(int d, int h, int k);
size_t mlp_train_workspace(int d, int h, int k, int B);
hipError_t mlp_train_step(float* th, float* am, float* av, int64_t step,
                          const MlpLayout& L, const float* Xs, const int32_t* y,
                          int B, float lr, float* grad, void* ws, double* loss_dev,
                          hipStream_t s);
// The forward pass with the top-16 epilogue (BF16 copies of the weights in
// the layout mlp_pack_layout describes, packed by launch_mlp_pack).
struct MlpPacked {
  int d, h, k, kpad, KP1;
  uint16_t *W1b, *W2b, *W3b;
  float* b3p;
  int *fl_rows, *fl_pos, *fl_cnt;   // points the short-list pass defers (<= mmax)
  float* keys;                      // per point and class slice: its 16 largest keys
};
int mlp_kpad(int k);
size_t mlp_pack_bytes(int d, int h, int k, int64_t mmax);
MlpPacked mlp_pack_layout(int d, int h, int k, int64_t mmax, void* ws);
hipError_t launch_mlp_pack(const float* th, const MlpLayout& L, const MlpPacked& P,
                           hipStream_t s);
// cand (m x 16): points rows[q] (or q) of X standardized by mean / istd
// (or taken as they are when null); m = min(m, *mdev) when mdev is given.
hipError_t launch_mlp_forward(const void* X, knor_dtype dt, int d, const int* rows, int m,
                              const int* mdev, const double* mean, const double* istd,
                              const float* th, const MlpLayout& L, const MlpPacked& P,
                              int32_t* cand, const int* outpos, hipStream_t s);
size_t standardize_workspace(int d);
hipError_t launch_standardize_stats(const void* X, knor_dtype dt, int64_t n, int d,
                                    double* mean, double* istd, double* part, hipStream_t s);
hipError_t launch_gather_std(const void* X, knor_dtype dt, int d, const int* rows,
                             int64_t count, const int* cdev, const double* mean,
                             const double* istd, float* Xs, hipStream_t s);
constexpr int kMlpTop = 16;          // candidates per point
// Inside a fit the proposals are kept per point: row p of cand (16 ints)
// starts as kUnproposed and holds p's candidates once p has been through the
// forward pass (the trained network and p's input are fixed from then on).
constexpr int32_t kUnproposed = -2;
// Survivors without a proposal yet: cnt_new (per segment), seg_off (their
// exclusive prefix, total at seg_off[nseg]) and their point indices in dense.
// prop: one byte per point, zero until the point is listed here (the
// caller then runs the forward pass over dense).  rows (or null): the
// neighbour rows; survivors that the certificate will not test
// (launch_mlp_certify with tight: u, labels) are left out.
hipError_t launch_seg_unproposed(const int* list, const int* seg_cnt, int nseg,
                                 uint8_t* prop, int* cnt_new, int* seg_off, int* dense,
                                 const int* conv, int iter, const float* u,
                                 const int32_t* labels, const float* rows, int k,
                                 hipStream_t s);
// nrows: the k x k neighbour rows of launch_cc_bounds.  tight: every
// listed survivor's |u| is its distance to its centroid rounded up (the
// filter's Clause 3); the certificate is then skipped where it cannot pass
// with c* = the survivor's centroid.
hipError_t launch_mlp_certify(const void* X, knor_dtype dt, int d, const double* C64,
                              int k, const float* nrows, const int* list,
                              const int* seg_cnt, int nseg,
                              const int32_t* cand, int32_t* labels, float* u, int* dirty,
                              int* list2, int* seg_cnt2, unsigned long long* row,
                              const int* conv, int iter, bool tight, hipStream_t s);
constexpr int kMlpHidden = 256;      // hidden width inside knor_fit
constexpr int kMlpBatch = 4096;      // training minibatch inside knor_fit
constexpr float kMlpLr = 1e-3f;
std::vector<float> mlp_init_host(int d, int h, int k, uint64_t seed);

// padded row length of the BF16 tile: a power of two, at least one K-step
inline int pad_dim_bf16(int d) {
  int p = 32;
  while (p < d) p *= 2;
  return p;
}
inline int pad_dim(int d) {
  int p = 8;
  while (p < d) p *= 2;
  return p;
}

inline int nseg_of_n(int64_t n) { return (int)((n + kSeg - 1) / kSeg); }

// One fetch pass of a streamed fit over a batch of rows (stream.hip).  All
// per-point arrays are views of the batch (point 0 = the batch's first row).
struct StreamFetch {
  const void* Xh = nullptr;            // the batch's rows in host memory (device-visible)
  knor_dtype dt = KNOR_F32;
  int64_t n = 0;                       // points in the batch
  int d = 0;
  const int32_t* labels = nullptr;
  const float* u = nullptr;
  const float* drift = nullptr;        // per cluster
  const float* s_half = nullptr;       // per cluster
  int all = 0;                         // 1: every point is a candidate
  const int* pslot = nullptr;          // point -> cache slot (-1: not cached), or null
  const void* cache = nullptr;         // rows of the current cache region
  void* stage = nullptr;               // out: row of point p at p
  void* adm_rows = nullptr;            // refresh: rows of the new cache region, or null
  int* adm_pts = nullptr;              // refresh: global point index of each new slot
  const int64_t* adm_base = nullptr;   // refresh: first new slot of each segment
  int64_t adm_cap = 0;                 // cache capacity in rows
  int64_t gid0 = 0;                    // global index of the batch's point 0
  int* seg_count = nullptr;            // count mode: candidates per segment (no copies)
  unsigned long long* io = nullptr;    // this iteration's I/O counters
  const int* conv = nullptr;
  int iter = 0;
};
hipError_t launch_stream_fetch(const StreamFetch& f, hipStream_t s);
hipError_t launch_stream_scan(const int* cnt, int nseg, int64_t* base, const int* conv,
                              int iter, hipStream_t s);
hipError_t launch_stream_remap(int* pslot, const int* old_pts, const int64_t* old_cnt,
                               const int* new_pts, const int64_t* total, int64_t cap,
                               int64_t* new_cnt, const int* conv, int iter, hipStream_t s);

}  // namespace knor
