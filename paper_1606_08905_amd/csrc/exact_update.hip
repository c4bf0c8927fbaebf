// Exact centroid update: each centroid is the exact mean of its members'
// values, rounded once to the nearest double (ties to even).  This takes the
// member mean of Phase II (Section "Parallel Lloyd's Algorithm") as an exact
// quantity: no summation order can change it, so sums may be kept across
// iterations and moved point by point, the "running totals" of the paper's
// merge and its no-I/O-for-pruned-rows idea (Section "Minimal Triangle
// Inequality (MTI) Pruning", semi-external memory).
//
// Representation.  Every FP32 or BF16 value is m 2^(sh - 149) with m < 2^24
// and 0 <= sh <= 253, an integer in units of 2^-149 below 2^277.  The sum of
// a cluster's values in one dimension is kept as kXD = 20 signed 64-bit
// digits of weight 2^(16 s) in those units (carry-save: a digit may leave
// [0, 2^16) between normalisations).  A value adds m << (sh mod 16), below
// 2^39, to digit sh/16 with the value's sign: one add per value when fewer
// than 2^23 points move in an iteration (below 2^62 per digit), else two
// pieces below 2^32 on digits sh/16 and sh/16 + 2.  The full pass adds
// pieces below 2^32, at most one per digit per value or per flushed sum, so
// a digit stays below n 2^32 < 2^63.  Each update normalises the dirty
// clusters' digits.
//
// The mode is chosen on the device each iteration (the full pass is gated
// by a word the delta kernel writes); once the caller has seen an iteration
// with few changes it stops launching the full pass, and every later
// iteration moves points (both modes give the same centroids).
//
// Per iteration of a fit (labels of the previous update in `prev`):
//   exact_delta    counts this iteration's changed labels and chooses the
//                  mode in a gate word; it visits every point, or under MTI
//                  only the survivors (no other label can change), and
//                  copies changed labels to prev.  Delta mode (few changes):
//                  each changed point leaves the old cluster's digits and
//                  enters the new one's (64-bit atomic adds, order-free) and
//                  the member counts move by one.  Full mode: the digits of
//                  every dirty cluster are cleared.
//   sort           the canonical counting sort (full mode only, via the gate)
//   exact_leaf     full mode: a wave walks a run of leaves (64 members of one
//                  cluster each), sums each dimension in FP64 (exact under a
//                  bound checked per lane, else digit by digit) and adds the
//                  sums to the cluster's digits when the cluster ends
//   exact_finalize every dirty cluster: normalise the digits (through LDS),
//                  divide by the member count with one rounding, write the
//                  centroid and its derived operands; close the iteration.
#include <math.h>

#include "common.h"
#include "update_common.h"

namespace knor {

constexpr int kExactWavesTarget = 16384; // full pass: waves wanted (runs of 4..32 leaves)
constexpr int kExactWaves = 4;
constexpr int kDeltaAtomics = 1 << 20; // delta mode up to about this many digit adds

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t exact_workspace_bytes(int64_t n, int k, int d) {
  return al256((size_t)k * kXD * d * sizeof(unsigned long long)) +
         al256((size_t)n * sizeof(int32_t)) + al256(sizeof(int) * 4);
}

void exact_plan_init(ExactPlan* p, int64_t n, int k, int d, void* ws) {
  char* c = (char*)ws;
  p->n = n;
  p->k = k;
  p->d = d;
  p->slots = (unsigned long long*)c;
  c += al256((size_t)k * kXD * d * sizeof(unsigned long long));
  p->prev = (int32_t*)c;
  c += al256((size_t)n * sizeof(int32_t));
  p->gate = (int*)c;
  // each moved point costs 2 d digit adds (old and new cluster) at about
  // 15 G adds/s, while the full pass re-sums every member of the dirty
  // clusters at about 10^12 values/s: moving points pays up to about n / 128
  // changes, and at least up to kDeltaAtomics / (4 d); at most 2^22 (single
  // adds stay below 2^62 per digit)
  int64_t dm = kDeltaAtomics / (4 * d);
  if (n / 128 > dm) dm = n / 128;
  if (dm > (1 << 22)) dm = 1 << 22;
  p->delta_max = dm < 256 ? 256 : (int)dm;
}

template <typename T>
__device__ __forceinline__ uint32_t f32_bits(T v);
template <>
__device__ __forceinline__ uint32_t f32_bits<float>(float v) { return __float_as_uint(v); }
template <>
__device__ __forceinline__ uint32_t f32_bits<uint16_t>(uint16_t v) { return (uint32_t)v << 16; }

// The value with FP32 bit pattern u as one digit add: v to digit idx, with
// the value's sign (two's complement in 64 bits).
struct FixedAdd {
  int idx;
  unsigned long long v;
};
__device__ __forceinline__ FixedAdd fixed_of(uint32_t u) {
  const uint32_t ef = (u >> 23) & 255u;
  const uint32_t m = (u & 0x7fffffu) | (ef ? 0x800000u : 0u);
  const int sh = ef ? (int)ef - 1 : 0;
  const unsigned long long v = (unsigned long long)m << (sh & 15);
  FixedAdd f;
  f.idx = sh >> 4;                              // <= 15
  f.v = (u >> 31) ? 0ull - v : v;
  return f;
}

// Add the signed amount w (|w| < 2^62) to digit idx of (cluster jc,
// dimension dim) in two pieces below 2^32, on digits idx and idx + 2 (so
// that no digit takes more than one piece per value or flush).
__device__ __forceinline__ void add_split(unsigned long long* slots, int jc, int d, int dim,
                                          int idx, long long w) {
  if (w == 0) return;
  const bool neg = w < 0;
  const unsigned long long m = neg ? 0ull - (unsigned long long)w : (unsigned long long)w;
  unsigned long long* p = slots + ((size_t)jc * kXD + idx) * d + dim;
  const unsigned long long pc[2] = {m & 0xffffffffull, m >> 32};
#pragma unroll
  for (int t = 0; t < 2; ++t)
    if (pc[t] && idx + 2 * t < kXD) atomicAdd(p + (size_t)(2 * t) * d, neg ? 0ull - pc[t] : pc[t]);
}

// ---------------------------------------------------------------------------
// mode choice, delta moves, prev labels
// ---------------------------------------------------------------------------

// Every point whose label may have changed: all n, or the MTI survivors
// list[s * kSeg + i] for i < seg_cnt[s].
struct DeltaSrc {
  int64_t n;
  const int* list;
  const int* seg_cnt;
  int nseg;
};

// Block b takes block b of points: survivor segment b, or points
// [b kSeg, (b + 1) kSeg); each thread loads its kSeg / 256 points at once.
// In delta mode each wave then moves its changed points: two at a time when
// d <= 32 (one per half wave), one dimension per lane, with order-free
// 64-bit atomic adds to the digits of the new (+x) and old (-x) cluster.
constexpr int kDeltaPer = kSeg / 256;
// exact_delta's choice of mode: full pass at t = 0 and after many changes;
// full pass at t = 0 only; never (the points of a streamed pass enter their
// clusters one by one, starting from digits the caller cleared)
constexpr int kDeltaAuto = 0, kDeltaOnly = 1, kDeltaStream = 2;

template <typename T>
__global__ __launch_bounds__(256) void exact_delta(
    const T* __restrict__ X, DeltaSrc src, const int32_t* __restrict__ labels,
    int32_t* __restrict__ prev, int k, int d, unsigned long long* __restrict__ slots,
    int* __restrict__ nj, const int* __restrict__ dirty,
    const unsigned long long* __restrict__ row, int* __restrict__ gate, int delta_max,
    int mode, int force_split, const int* __restrict__ conv, int iter) {
  const int cv = *conv;
  const int lane = threadIdx.x & 63;
  // this iteration's changed labels, from the spread counter slots
  unsigned long long c =
      lane < kChgSlots ? row[(SLOT_CHANGED * kChgSlots + lane) * kSlotStride] : 0ull;
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  const bool full = mode != kDeltaStream &&
                    (iter == 0 || (mode == kDeltaAuto && c > (unsigned long long)delta_max));
  // with the full pass not launched, many moves are possible: a digit then
  // takes two pieces below 2^32 per value instead of one add below 2^39.
  // A streamed pass sees the iteration in pieces, so its caller decides
  // from a bound on the iteration's moves.
  const bool split = mode == kDeltaStream ? force_split != 0 : c >= (1ull << 23);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    *gate = cv < iter ? cv : (full ? kNotConverged : -1);
  if (cv < iter) return;
  if (full) {
    const int64_t ns = (int64_t)k * kXD * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ns;
         e += (int64_t)gridDim.x * blockDim.x)
      if (dirty[e / ((int64_t)kXD * d)]) slots[e] = 0ull;
  }
  const bool two = d <= 32;
  const int half = two ? lane >> 5 : 0;
  const int dl = two ? (lane & 31) : lane;
  const int dstep = two ? 32 : 64;
  const int nblk = src.list ? src.nseg : (int)((src.n + kSeg - 1) / kSeg);
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int64_t b0 = (int64_t)b * kSeg;
    const int cnt = src.list ? src.seg_cnt[b]
                             : (int)(src.n - b0 < kSeg ? src.n - b0 : kSeg);
    int pt[kDeltaPer], a[kDeltaPer], o[kDeltaPer];
#pragma unroll
    for (int q = 0; q < kDeltaPer; ++q) {
      const int i = q * (int)blockDim.x + (int)threadIdx.x;
      pt[q] = i < cnt ? (src.list ? src.list[(size_t)b * kSeg + i] : (int)(b0 + i)) : -1;
    }
#pragma unroll
    for (int q = 0; q < kDeltaPer; ++q) {
      a[q] = pt[q] >= 0 ? labels[pt[q]] : 0;
      o[q] = pt[q] >= 0 ? prev[pt[q]] : 0;
    }
    uint32_t mv = 0;
#pragma unroll
    for (int q = 0; q < kDeltaPer; ++q)
      if (pt[q] >= 0 && a[q] != o[q]) {
        prev[pt[q]] = a[q];
        mv |= 1u << q;
      }
    if (full) continue;                         // uniform over the grid
#pragma unroll
    for (int q = 0; q < kDeltaPer; ++q) {
      uint64_t mask = __ballot((mv >> q) & 1u);
      while (mask) {
        const int l0 = __builtin_ctzll(mask);
        mask &= mask - 1;
        int l1 = -1;
        if (two && mask) {
          l1 = __builtin_ctzll(mask);
          mask &= mask - 1;
        }
        const int l = half ? l1 : l0;
        const int ls = l < 0 ? l0 : l;
        const int pq = __shfl(pt[q], ls);
        const int32_t na = __shfl(a[q], ls), oa = __shfl(o[q], ls);
        if (l < 0) continue;                    // second half without a point
        if (dl == 0) {
          atomicAdd(&nj[na], 1);
          if (oa >= 0) atomicSub(&nj[oa], 1);
        }
        for (int dim = dl; dim < d; dim += dstep) {
          const FixedAdd f = fixed_of(f32_bits<T>(X[(size_t)pq * d + dim]));
          if (!f.v) continue;
          if (split) {
            add_split(slots, na, d, dim, f.idx, (long long)f.v);
            if (oa >= 0) add_split(slots, oa, d, dim, f.idx, -(long long)f.v);
          } else {
            atomicAdd(slots + ((size_t)na * kXD + f.idx) * d + dim, f.v);
            if (oa >= 0) atomicAdd(slots + ((size_t)oa * kXD + f.idx) * d + dim, 0ull - f.v);
          }
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// full pass: runs of leaves
// ---------------------------------------------------------------------------

// Add the FP64 value s (exact, an integer multiple of 2^-149 below 2^285)
// to the digits of (cluster jc, dimension dim): its 53-bit significand, in
// 32-bit pieces, lands on digits idx, idx + 2 and idx + 4 (idx <= 14).
__device__ __forceinline__ void add_f64_digits(unsigned long long* slots, int jc, int d, int dim,
                                               double s) {
  if (s == 0.0) return;
  const unsigned long long u = (unsigned long long)__double_as_longlong(s);
  const int e = (int)((u >> 52) & 0x7ff);                 // |s| >= 2^-149: normal
  unsigned long long mant = (u & 0xfffffffffffffull) | (1ull << 52);
  int shift = e - 1075 + 149;                              // |s| = mant 2^shift units
  if (shift < 0) {                                         // low bits are zero
    mant >>= -shift;
    shift = 0;
  }
  // mant 2^off (off < 16) in 32-bit pieces on digits idx, idx + 2, idx + 4
  const int idx = shift >> 4, off = shift & 15;
  const unsigned long long lo = mant << off;
  const unsigned long long hi = off ? mant >> (64 - off) : 0ull;
  const bool neg = (u >> 63) != 0;
  const unsigned long long dg[3] = {lo & 0xffffffffull, lo >> 32, hi};
  unsigned long long* p = slots + ((size_t)jc * kXD + idx) * d + dim;
#pragma unroll
  for (int t = 0; t < 3; ++t)
    if (dg[t]) atomicAdd(p + (size_t)(2 * t) * d, neg ? 0ull - dg[t] : dg[t]);
}

// Wave w of block b walks leaves [g0, g0 + run) of the canonical leaf
// list (consecutive leaves, cluster by cluster), skipping clean clusters.
// For each chunk of DC dimensions, lane m copies member m's row piece into
// the wave's LDS tile (16-byte pieces when rows allow), then each lane takes
// one dimension: for chunks of at most 32 dimensions lane (r, i) =
// (lane / 32, lane mod 32) takes dimension i of every second member
// starting at r, otherwise lane i takes dimension i of every member.  Each
// lane sums its values of a cluster in FP64 and tracks the lowest set bit L
// and the top bit bound M of those values (units of 2^-149).  Every value
// is a multiple of 2^L and every partial sum is below count 2^M, so when
// M - L + ceil(log2 count) <= 53 each partial sum is a double and the FP64
// sum is exact; it then goes to the cluster's digits as one 53-bit
// significand.  Otherwise the lane's values of that cluster are walked
// again and added digit by digit.
template <typename T>
struct ExactCfg {
  static constexpr int DC = 128 / (int)sizeof(T);      // dimensions per chunk
  static constexpr int LD = DC + 16 / (int)sizeof(T);  // row stride in the tile
};

template <typename T>
__global__ __launch_bounds__(64 * kExactWaves) void exact_leaf(
    const T* __restrict__ X, int d, const int* __restrict__ perm,
    const int* __restrict__ nj, const int* __restrict__ off,
    const int* __restrict__ leaf_off, int k, const int* __restrict__ dirty,
    unsigned long long* __restrict__ slots, const int* __restrict__ gate, int iter,
    int vec, int run) {
  constexpr int DC = ExactCfg<T>::DC, LD = ExactCfg<T>::LD;
  __shared__ __attribute__((aligned(16))) T tile[kExactWaves][kLeaf * LD];
  if (*gate < iter) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int total = leaf_off[k];
  const int g0 = (blockIdx.x * kExactWaves + wave) * run;
  if (g0 >= total) return;                     // per wave; no block barrier below
  const int g1 = g0 + run < total ? g0 + run : total;
  const int j0 = cluster_of_leaf(leaf_off, k, g0);
  T* tl = tile[wave];
  for (int c0 = 0; c0 < d; c0 += DC) {
    const int dc = d - c0 < DC ? d - c0 : DC;
    const bool two = dc <= 32;
    const int r = two ? lane >> 5 : 0;         // member offset of this lane
    const int step = two ? 2 : 1;
    const int dl = two ? (lane & 31) : lane;
    const int dim = c0 + dl;
    const bool on = dl < dc;
    // the lane's values of leaf g of cluster j: fn(u) for each (every lane
    // of the wave calls this together)
    auto walk_leaf = [&](int j, int g, auto&& fn) {
      const int L = g - leaf_off[j];
      const int m0 = off[j] + L * kLeaf;
      int cnt = nj[j] - L * kLeaf;
      if (cnt > kLeaf) cnt = kLeaf;
      if (lane < cnt) {
        const T* xr = X + (size_t)perm[m0 + lane] * d + c0;
        uint4* dst = reinterpret_cast<uint4*>(tl + lane * LD);
        const uint4* src = reinterpret_cast<const uint4*>(xr);
        constexpr int NV = DC * (int)sizeof(T) / 16;
        if (vec && dc == DC) {
          // a full chunk: all loads in flight before the first store
          uint4 t0 = src[0], t1 = src[1], t2 = src[2], t3 = src[3];
          uint4 t4 = src[4], t5 = src[5], t6 = src[6], t7 = src[7];
          static_assert(NV == 8, "128-byte chunks");
          dst[0] = t0; dst[1] = t1; dst[2] = t2; dst[3] = t3;
          dst[4] = t4; dst[5] = t5; dst[6] = t6; dst[7] = t7;
        } else if (vec) {
          const int nv = dc * (int)sizeof(T) / 16;
          for (int v = 0; v < nv; ++v) dst[v] = src[v];
        } else {
          for (int i = 0; i < dc; ++i) tl[lane * LD + i] = xr[i];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (on)
        for (int m = r; m < cnt; m += step) {
          const uint32_t u = f32_bits<T>(tl[m * LD + dl]);
          if ((u << 1) != 0u) fn(u);           // +-0 adds nothing
        }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    int j = j0, cur = -1, gs = g0;
    double sacc = 0.0;
    int Lm = 1 << 30, Mm = -1, cntv = 0;
    auto bound_ok = [](int L, int M, int c) {
      int lg = 0;
      while ((1 << lg) < c) ++lg;
      return c == 0 || M - L + lg <= 53;
    };
    auto flush = [&](int jc, int gend) {       // leaves [gs, gend) of cluster jc
      // the two lanes of a dimension merge their sums when the merged
      // bound still holds (the FP64 sum of the two is then exact too)
      bool merged = false;
      if (two) {
        const double so = __shfl_xor(sacc, 32);
        const int Lo = __shfl_xor(Lm, 32), Mo = __shfl_xor(Mm, 32), co = __shfl_xor(cntv, 32);
        const int L2 = Lo < Lm ? Lo : Lm, M2 = Mo > Mm ? Mo : Mm;
        if (bound_ok(L2, M2, cntv + co)) {
          merged = true;
          if (on && r == 0 && cntv + co > 0) add_f64_digits(slots, jc, d, dim, sacc + so);
        }
      }
      const bool has = on && cntv > 0 && !merged;
      const bool need = has && !bound_ok(Lm, Mm, cntv);
      if (has && !need) add_f64_digits(slots, jc, d, dim, sacc);
      // rare: lanes whose sum may have rounded add their values digit by
      // digit; the walk runs on the whole wave (it stages rows for every
      // lane), and only those lanes accumulate
      if (__ballot(need)) {
        unsigned long long w0 = 0, w1 = 0;
        int base = -1;
        const int gl = leaf_off[jc + 1] < gend ? leaf_off[jc + 1] : gend;
        for (int g = gs; g < gl; ++g)
          walk_leaf(jc, g, [&](uint32_t u) {
            if (!need) return;
            const FixedAdd f = fixed_of(u);
            if (base < 0) base = f.idx;        // idx <= 15: base + 1 < kXD
            const bool in0 = f.idx == base, in1 = f.idx == base + 1;
            w0 += in0 ? f.v : 0ull;
            w1 += in1 ? f.v : 0ull;
            if (!in0 && !in1) add_split(slots, jc, d, dim, f.idx, (long long)f.v);
          });
        if (need && base >= 0) {
          add_split(slots, jc, d, dim, base, (long long)w0);
          add_split(slots, jc, d, dim, base + 1, (long long)w1);
        }
      }
      sacc = 0.0;
      Lm = 1 << 30;
      Mm = -1;
      cntv = 0;
    };
    for (int g = g0; g < g1; ++g) {
      while (leaf_off[j + 1] <= g) ++j;        // uniform over the wave
      if (dirty && !dirty[j]) continue;
      if (j != cur) {
        if (cur >= 0) flush(cur, g);
        cur = j;
        gs = g;
      }
      walk_leaf(j, g, [&](uint32_t u) {
        const uint32_t ef = (u >> 23) & 255u;
        const uint32_t m = (u & 0x7fffffu) | (ef ? 0x800000u : 0u);
        const int sh = ef ? (int)ef - 1 : 0;
        const int lo = sh + __builtin_ctz(m);
        Lm = lo < Lm ? lo : Lm;
        Mm = sh + 24 > Mm ? sh + 24 : Mm;
        ++cntv;
        sacc += (double)__uint_as_float(u);
      });
    }
    if (cur >= 0) flush(cur, g1);
  }
}

// ---------------------------------------------------------------------------
// finalize
// ---------------------------------------------------------------------------

// Normalise the kXD digits at p (stride d) in place: digits 0..kXD-2 in
// [0, 2^16), the top digit signed.  Returns the value as kQ - 1 digits of
// 32 bits (dig) and a signed top of weight 2^(32 (kQ - 1)).
constexpr int kQ = kXD / 2;
__device__ __forceinline__ void normalise_digits(unsigned long long* p, int d, uint32_t* dig,
                                                 long long& top) {
  long long carry = 0;
  uint32_t h[kXD - 1];
#pragma unroll
  for (int s = 0; s < kXD - 1; ++s) {
    const long long v = (long long)p[(size_t)s * d] + carry;
    h[s] = (uint32_t)((unsigned long long)v & 0xffffull);
    carry = v >> 16;                            // arithmetic shift: floor
  }
  const long long t16 = (long long)p[(size_t)(kXD - 1) * d] + carry;
#pragma unroll
  for (int s = 0; s < kXD - 1; ++s) p[(size_t)s * d] = h[s];
  p[(size_t)(kXD - 1) * d] = (unsigned long long)t16;
#pragma unroll
  for (int t = 0; t < kQ - 1; ++t) dig[t] = h[2 * t] | (h[2 * t + 1] << 16);
  top = t16 * 65536 + (long long)h[kXD - 2];    // |V| < 2^308: no overflow
}

// RN(V / cnt) for V = sum_s dig[s] 2^(32 s - 149) + top 2^(32 (kQ-1) - 149),
// cnt >= 1: the magnitude's long division by cnt with three 32-bit guard
// digits, then 53 bits, a round bit and a sticky bit (remainder included).
// Every mean of FP32 values lies in [2^-180, 2^128]: a normal double.
__device__ __forceinline__ double exact_quotient(const uint32_t* dig, long long top,
                                                 int cnt) {
  constexpr int G = 3;                          // guard digits
  constexpr int W = kQ + G;
  uint32_t a[W];
  const bool neg = top < 0;
  // magnitude digits (two's complement negation when negative)
#pragma unroll
  for (int s = 0; s < G; ++s) a[s] = 0u;
  unsigned long long borrow = neg ? 1ull : 0ull;   // ~x + 1
#pragma unroll
  for (int s = 0; s < kQ - 1; ++s) {
    const unsigned long long v = (unsigned long long)(neg ? ~dig[s] : dig[s]) + borrow;
    a[G + s] = (uint32_t)v;
    borrow = v >> 32;
  }
  const unsigned long long tmag = neg ? (unsigned long long)(~top) + borrow
                                      : (unsigned long long)top;
  a[W - 1] = (uint32_t)tmag;                    // |V| < 2^308: the top fits
  // long division, most significant digit first.  Each quotient digit is
  // cur / cnt < 2^32; the FP64 estimate cur * (1 / cnt) has relative error
  // below 2^-50, so its truncation is off by at most one, fixed from the
  // sign and size of the remainder.
  const unsigned long long n = (unsigned long long)cnt;
  const double rn = 1.0 / (double)cnt;
  unsigned long long rem = 0;
  uint32_t q[W];
#pragma unroll
  for (int s = W - 1; s >= 0; --s) {
    const unsigned long long cur = (rem << 32) | a[s];
    unsigned long long qd = (unsigned long long)((double)cur * rn);
    long long r = (long long)(cur - qd * n);
    if (r < 0) { qd -= 1; r += (long long)n; }
    else if (r >= (long long)n) { qd += 1; r -= (long long)n; }
    q[s] = (uint32_t)qd;
    rem = (unsigned long long)r;
  }
  int t = W - 1;
  while (t > 0 && q[t] == 0u) --t;
  if (q[t] == 0u) return 0.0;                   // V == 0
  // t >= 2 whenever V != 0: |V| 2^96 / cnt >= 2^65
  const int lz = __clz((int)q[t]);
  const unsigned long long hi64 = ((unsigned long long)q[t] << 32) | q[t - 1];
  const uint32_t lo32 = q[t - 2];
  const unsigned long long w = lz ? (hi64 << lz) | ((unsigned long long)lo32 >> (32 - lz)) : hi64;
  unsigned long long mant = w >> 11;            // 53 bits, leading one at bit 52
  const unsigned long long rbit = (w >> 10) & 1ull;
  bool sticky = (w & 0x3ffull) != 0ull || rem != 0ull ||
                (lz ? (uint32_t)(lo32 << lz) != 0u : lo32 != 0u);
  for (int s = t - 3; s >= 0 && !sticky; --s) sticky = q[s] != 0u;
  if (rbit && (sticky || (mant & 1ull))) mant += 1ull;
  // the leading one sits at bit b = 32 t + 31 - lz of q, in units of
  // 2^-(149 + 32 G); mant's last bit has weight 2^(b - 52)
  const int b = 32 * t + 31 - lz;
  const double r = ldexp((double)mant, b - 52 - 149 - 32 * G);
  return neg ? -r : r;
}

__global__ __launch_bounds__(256) void exact_finalize(
    unsigned long long* __restrict__ slots, const int* __restrict__ nj, int k, int d,
    const double* C_prev, double* C_out, int64_t* __restrict__ counts_out,
    float* __restrict__ Cm2, float* __restrict__ cn, double* __restrict__ CT, int dp,
    uint16_t* __restrict__ Chi, uint16_t* __restrict__ Clo, int dpb,
    float* __restrict__ drift, int* __restrict__ dirty, IterCtl ctl,
    const int* __restrict__ conv, int iter) {
  __shared__ double mean[kMaxD];
  __shared__ unsigned long long sdig[kXD * kMaxD];
  const int cv = *conv;
  const int j = blockIdx.x;
  const int cntj = nj[j];
  const int dj = dirty ? dirty[j] : 1;
  if (cv < iter) return;
  if (j == 0 && ctl.row) close_iteration(ctl, iter);
  if (counts_out && threadIdx.x == 0) counts_out[j] = cntj;
  if (!dj) {
    if (drift && threadIdx.x == 0) drift[j] = 0.0f;     // centroid unchanged
    return;
  }
  // the cluster's kXD x d digits (contiguous) through LDS: loaded and
  // stored back by the whole workgroup; normalise and divide per dimension
  unsigned long long* base = slots + (size_t)j * kXD * d;
  const int nd = kXD * d;
  stage_batched<8, unsigned long long>(
      nd, [&](int e) { return base[e]; }, [&](int e, unsigned long long v) { sdig[e] = v; });
  __syncthreads();
  for (int dim = threadIdx.x; dim < d; dim += blockDim.x) {
    uint32_t dig[kQ - 1];
    long long top;
    normalise_digits(sdig + dim, d, dig, top);
    mean[dim] = cntj > 0 ? exact_quotient(dig, top, cntj) : 0.0;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nd; e += blockDim.x) base[e] = sdig[e];
  write_centroid(j, k, d, cntj, [&](int dim) { return mean[dim]; }, C_prev, C_out, CT,
                 Cm2, cn, dp, Chi, Clo, dpb, drift, dirty);
}

// ---------------------------------------------------------------------------
// launch
// ---------------------------------------------------------------------------

hipError_t launch_update_exact(const UpdatePlan& p, const ExactPlan& xp, const void* X,
                               knor_dtype dt, const int32_t* labels, const double* C_prev,
                               double* C_out, int64_t* counts_out, CentroidOps* ops,
                               float* drift, int* dirty, const IterCtl* ctl, hipStream_t s,
                               Prof* prof) {
  if (dt != KNOR_F32 && dt != KNOR_BF16) return hipErrorInvalidValue;
  const int k = p.k, d = p.d;
  const int* conv = ctl->conv;
  const int iter = ctl->iter;
  // one update outside a fit (no counter row): every cluster from scratch
  const bool one_shot = ctl->row == nullptr;
  const int* gate = conv;
  if (prof) prof->begin(KNOR_PROF_SORT);
  if (one_shot) {
    if (dirty) return hipErrorInvalidValue;
    hipError_t e = launch_fill_i32((int32_t*)xp.slots, (int64_t)k * kXD * d * 2, 0, s);
    if (e != hipSuccess) return e;
  } else {
    if (!dirty) return hipErrorInvalidValue;
    DeltaSrc src{p.n, ctl->list, ctl->seg_cnt, ctl->nseg};
    int64_t blocks = ctl->list ? ctl->nseg : (p.n + kSeg - 1) / kSeg;
    if (blocks > (1 << 20)) blocks = 1 << 20;
    if (blocks < 1) blocks = 1;
    const int mode = ctl->delta_only && iter > 0 ? kDeltaOnly : kDeltaAuto;
    if (dt == KNOR_F32)
      hipLaunchKernelGGL(exact_delta<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                         (const float*)X, src, labels, xp.prev, k, d, xp.slots, p.nj, dirty,
                         ctl->row, xp.gate, xp.delta_max, mode, 0, conv, iter);
    else
      hipLaunchKernelGGL(exact_delta<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                         (const uint16_t*)X, src, labels, xp.prev, k, d, xp.slots, p.nj,
                         dirty, ctl->row, xp.gate, xp.delta_max, mode, 0, conv, iter);
    gate = xp.gate;
  }
  // the full pass: gated on the device, or not launched at all once the
  // caller knows that only moved points remain (delta_only)
  const bool full_pass = one_shot || !(ctl->delta_only && iter > 0);
  if (full_pass)
    if (hipError_t e = launch_sort(p, labels, dirty, gate, iter, s, one_shot ? 0 : 1)) return e;
  if (prof) { prof->end(); prof->begin(KNOR_PROF_LEAF); }
  // longer runs at large n: fewer flushes of partial digits (global adds)
  int64_t run = p.max_leaves / kExactWavesTarget;
  run = run < 4 ? 4 : (run > 32 ? 32 : run);
  const int64_t waves = (p.max_leaves + run - 1) / run;
  const int64_t lblocks = (waves + kExactWaves - 1) / kExactWaves;
  const size_t esz = dt == KNOR_F32 ? 4 : 2;
  const int vec = (int)(((size_t)d * esz) % 16 == 0 && ((uintptr_t)X & 15) == 0);
  if (!full_pass) {
    // nothing to launch
  } else if (dt == KNOR_F32)
    hipLaunchKernelGGL(exact_leaf<float>, dim3((unsigned)lblocks), dim3(64 * kExactWaves), 0, s,
                       (const float*)X, d, p.perm, p.nj, p.off, p.leaf_off, k, dirty, xp.slots,
                       gate, iter, vec, (int)run);
  else
    hipLaunchKernelGGL(exact_leaf<uint16_t>, dim3((unsigned)lblocks), dim3(64 * kExactWaves), 0,
                       s, (const uint16_t*)X, d, p.perm, p.nj, p.off, p.leaf_off, k, dirty,
                       xp.slots, gate, iter, vec, (int)run);
  if (prof) { prof->end(); prof->begin(KNOR_PROF_TREE); }
  hipError_t e = launch_exact_finalize(xp, p.nj, C_prev, C_out, counts_out, ops, drift, dirty,
                                       *ctl, s);
  if (prof) prof->end();
  return e;
}

hipError_t launch_exact_finalize(const ExactPlan& xp, const int* nj, const double* C_prev,
                                 double* C_out, int64_t* counts_out, CentroidOps* ops,
                                 float* drift, int* dirty, const IterCtl& ctl, hipStream_t s) {
  hipLaunchKernelGGL(exact_finalize, dim3(xp.k), dim3(256), 0, s, xp.slots, nj, xp.k, xp.d,
                     C_prev, C_out, counts_out, ops ? ops->Cm2 : nullptr,
                     ops ? ops->cn : nullptr, ops ? ops->CT : nullptr, ops ? ops->dp : 0,
                     ops ? ops->Chi : nullptr, ops ? ops->Clo : nullptr, ops ? ops->dpb : 0,
                     drift, dirty, ctl, ctl.conv, ctl.iter);
  return hipGetLastError();
}

hipError_t launch_exact_enter(const ExactPlan& xp, int* nj, const void* X, knor_dtype dt,
                              int64_t n, const int* list, const int* seg_cnt, int nseg,
                              const int32_t* labels, int32_t* prev, const int* dirty,
                              const unsigned long long* row, const int* conv, int iter,
                              int split, hipStream_t s) {
  if (dt != KNOR_F32 && dt != KNOR_BF16) return hipErrorInvalidValue;
  DeltaSrc src{n, list, seg_cnt, nseg};
  int64_t blocks = list ? nseg : (n + kSeg - 1) / kSeg;
  if (blocks > (1 << 20)) blocks = 1 << 20;
  if (blocks < 1) blocks = 1;
  if (dt == KNOR_F32)
    hipLaunchKernelGGL(exact_delta<float>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const float*)X, src, labels, prev, xp.k, xp.d, xp.slots, nj, dirty, row,
                       xp.gate, xp.delta_max, kDeltaStream, split, conv, iter);
  else
    hipLaunchKernelGGL(exact_delta<uint16_t>, dim3((unsigned)blocks), dim3(256), 0, s,
                       (const uint16_t*)X, src, labels, prev, xp.k, xp.d, xp.slots, nj, dirty,
                       row, xp.gate, xp.delta_max, kDeltaStream, split, conv, iter);
  return hipGetLastError();
}

}  // namespace knor
