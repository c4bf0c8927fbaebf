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
// Each filter block owns one segment of kSeg consecutive points and writes
// its survivors to its own slice of the list (no global atomics); the
// assignment tile then scans the survivors against every centroid.  With
// mark, Clause 3 runs every iteration and a survivor's tightened bound is
// stored negated (sign bit set) for the candidate-list tile, which finds
// the survivors of a cluster through it and writes a positive bound back.
// The strict test with margin eta keeps every pruned centroid farther than
// the kept one by a relative gap of about 4 eta, far above FP64 rounding, so
// the labels equal the unpruned FP64 argmin.
#include <math.h>

#include "common.h"

namespace knor {

// Half of sqrt(D) rounded down to FP32, D a squared distance summed in FP64
// (any order: relative error below (d + 2) 2^-53, covered with room).
__device__ __forceinline__ float half_dist_down(double D, int d) {
  return f32_down(0.5 * sqrt(D) * (1.0 - (double)(d + 8) * 2.220446049250313e-16));
}

// s_half[i] = rounded-down 1/2 min_{j != i} d(c_i, c_j).  One block per i;
// threads over j read the transposed copy CT (contiguous across lanes).
// With rows, row i of the neighbour table as well: for every j (i itself
// included, at half distance 0) the key 1/2 d(c_i, c_j), rounded down, with
// its low ib mantissa bits replaced by j (2^ib >= k), sorted in increasing
// order.  Keys order by the half distance rounded down to its leading
// 23 - ib mantissa bits, then by index, and the value of a key with its low
// ib bits cleared is still a lower bound of the half distance.  The row is
// sorted in LDS (bitonic, padded with +inf to kp2 = the next power of two).
constexpr int kCcDims = 16;   // CT loads issued before their dimensions are summed

__global__ __launch_bounds__(256) void cc_bounds_kernel(
    const double* __restrict__ C64, const double* __restrict__ CT, int k,
    int d, float* __restrict__ s_half, float* __restrict__ rows, int ib, int kp2,
    const int* __restrict__ conv, int iter) {
  extern __shared__ float sKey[];                    // kp2 keys (rows only)
  __shared__ double red[256];
  if (*conv < iter) return;
  const int i = blockIdx.x;
  const double* ci = C64 + (size_t)i * d;
  const uint32_t mask = (1u << ib) - 1u;
  double best = INFINITY;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    if (j == i) {
      if (rows) sKey[j] = __uint_as_float((uint32_t)j);   // half distance 0
      continue;
    }
    double acc = 0.0;
    for (int d0 = 0; d0 < d; d0 += kCcDims) {
      double c[kCcDims];                               // loads in flight together
#pragma unroll
      for (int e = 0; e < kCcDims; ++e)
        c[e] = d0 + e < d ? CT[(size_t)(d0 + e) * k + j] : 0.0;
#pragma unroll
      for (int e = 0; e < kCcDims; ++e)
        if (d0 + e < d) {
          const double t = __dsub_rn(ci[d0 + e], c[e]);
          acc = __dadd_rn(acc, __dmul_rn(t, t));
        }
    }
    if (rows)
      sKey[j] = __uint_as_float((__float_as_uint(half_dist_down(acc, d)) & ~mask) | (uint32_t)j);
    best = acc < best ? acc : best;
  }
  red[threadIdx.x] = best;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s && red[threadIdx.x + s] < red[threadIdx.x])
      red[threadIdx.x] = red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double m = red[0];
    s_half[i] = m < INFINITY ? half_dist_down(m, d) : INFINITY;
  }
  if (!rows) return;                                 // uniform
  for (int j = k + (int)threadIdx.x; j < kp2; j += blockDim.x) sKey[j] = INFINITY;
  __syncthreads();
  for (int size = 2; size <= kp2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (kp2 >> 1); t += blockDim.x) {
        // stride is a power of two: (t / stride) 2 stride + t mod stride
        const int lo = 2 * t - (t & (stride - 1)), hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const float x = sKey[lo], y = sKey[hi];
        if ((x > y) == asc) { sKey[lo] = y; sKey[hi] = x; }
      }
      __syncthreads();
    }
  for (int j = threadIdx.x; j < k; j += blockDim.x) rows[(size_t)i * k + j] = sKey[j];
}

// With rows and 256 <= kp2 <= 4096 (KPL = kp2 / 64 keys per lane): four
// rows per workgroup.  Each thread computes, for its centroids j, the
// squared distances to the centroids i0 .. i0 + 3 from one read of CT (the
// FP64 operations of cc_bounds_kernel in its order, so keys and s_half are
// the same) and stores the keys in LDS (one pad word per KPL keys: the
// reads below are free of bank conflicts).  Wave w then sorts row i0 + w in
// registers, lane l holding keys l KPL .. l KPL + KPL - 1, and writes it.
// The network is bitonic in its direction-free form: a merge of size s
// first compares i with i xor (s - 1), then i with i + t for t = s/4 .. 1,
// the smaller key always going to the lower index.  Merges within a lane
// are unrolled; across lanes the partner comes by a lane shuffle.  Keys are
// non-negative floats or +inf, so their integer order is their float order.
constexpr int kRowsPerBlock = 4;

__device__ __forceinline__ void cmpx(uint32_t& a, uint32_t& b) {
  const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}

// lane keeps the smaller (low) or the larger of its key and the partner's
__device__ __forceinline__ uint32_t keep(uint32_t a, uint32_t p, bool low) {
  const uint32_t lo = a < p ? a : p, hi = a < p ? p : a;
  return low ? lo : hi;
}

template <int KPL>
__device__ __forceinline__ void lane_half_cleaners(uint32_t (&v)[KPL]) {
#pragma unroll
  for (int st = KPL >> 1; st > 0; st >>= 1)
#pragma unroll
    for (int r = 0; r < KPL; ++r)
      if ((r & st) == 0) cmpx(v[r], v[r + st]);
}

template <int KPL>
__device__ void wave_bitonic(uint32_t (&v)[KPL], int lane) {
  // merges of size 2 .. KPL, within each lane
#pragma unroll
  for (int size = 2; size <= KPL; size <<= 1) {
#pragma unroll
    for (int r = 0; r < KPL; ++r)
      if ((r & (size >> 1)) == 0) cmpx(v[r], v[r ^ (size - 1)]);
#pragma unroll
    for (int st = size >> 2; st > 0; st >>= 1)
#pragma unroll
      for (int r = 0; r < KPL; ++r)
        if ((r & st) == 0) cmpx(v[r], v[r + st]);
  }
  // merges of size lsz KPL, lsz = 2 .. 64 lanes
  for (int lsz = 2; lsz <= 64; lsz <<= 1) {
    // key r of lane l pairs with key KPL - 1 - r of lane l xor (lsz - 1)
    const bool low = (lane & (lsz >> 1)) == 0;
#pragma unroll
    for (int r = 0; r < KPL / 2; ++r) {
      const int q = KPL - 1 - r;
      const uint32_t pr = (uint32_t)__shfl_xor((int)v[q], lsz - 1);
      const uint32_t pq = (uint32_t)__shfl_xor((int)v[r], lsz - 1);
      v[r] = keep(v[r], pr, low);
      v[q] = keep(v[q], pq, low);
    }
    for (int ls = lsz >> 2; ls > 0; ls >>= 1) {
      const bool lo = (lane & ls) == 0;
#pragma unroll
      for (int r = 0; r < KPL; ++r) v[r] = keep(v[r], (uint32_t)__shfl_xor((int)v[r], ls), lo);
    }
    lane_half_cleaners<KPL>(v);
  }
}

template <int KPL>
__global__ __launch_bounds__(64 * kRowsPerBlock) void cc_rows_kernel(
    const double* __restrict__ C64, const double* __restrict__ CT, int k, int d,
    float* __restrict__ s_half, float* __restrict__ rows, int ib,
    const int* __restrict__ conv, int iter) {
  constexpr int KP2 = 64 * KPL, RS = KP2 + 64;       // LDS row stride (words)
  constexpr int R = kRowsPerBlock;
  extern __shared__ uint32_t sK[];                    // R x RS
  __shared__ double red[R][R];                        // [wave][row]
  if (*conv < iter) return;
  const int i0 = blockIdx.x * R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint32_t mask = (1u << ib) - 1u;
  const double* ci[R];
#pragma unroll
  for (int w = 0; w < R; ++w) ci[w] = C64 + (size_t)(i0 + w < k ? i0 + w : k - 1) * d;
  double best[R];
#pragma unroll
  for (int w = 0; w < R; ++w) best[w] = INFINITY;
  for (int j = threadIdx.x; j < KP2; j += blockDim.x) {
    const int a = j + j / KPL;
    if (j >= k) {
#pragma unroll
      for (int w = 0; w < R; ++w) sK[w * RS + a] = 0x7f800000u;   // +inf
      continue;
    }
    double acc[R];
#pragma unroll
    for (int w = 0; w < R; ++w) acc[w] = 0.0;
    for (int d0 = 0; d0 < d; d0 += kCcDims) {
      double c[kCcDims];                               // loads in flight together
#pragma unroll
      for (int e = 0; e < kCcDims; ++e)
        c[e] = d0 + e < d ? CT[(size_t)(d0 + e) * k + j] : 0.0;
#pragma unroll
      for (int e = 0; e < kCcDims; ++e)
        if (d0 + e < d)
#pragma unroll
          for (int w = 0; w < R; ++w) {
            const double t = __dsub_rn(ci[w][d0 + e], c[e]);
            acc[w] = __dadd_rn(acc[w], __dmul_rn(t, t));
          }
    }
#pragma unroll
    for (int w = 0; w < R; ++w) {
      uint32_t key = (uint32_t)j;                      // i itself: half distance 0
      if (j != i0 + w) {
        key = (__float_as_uint(half_dist_down(acc[w], d)) & ~mask) | (uint32_t)j;
        best[w] = acc[w] < best[w] ? acc[w] : best[w];
      }
      sK[w * RS + a] = key;
    }
  }
#pragma unroll
  for (int w = 0; w < R; ++w) {
    double b = best[w];
    for (int o = 32; o > 0; o >>= 1) {
      const double x = __shfl_xor(b, o);
      b = x < b ? x : b;
    }
    if (lane == 0) red[wave][w] = b;
  }
  __syncthreads();
  if (threadIdx.x < R && i0 + (int)threadIdx.x < k) {
    double m = red[0][threadIdx.x];
#pragma unroll
    for (int v = 1; v < R; ++v) m = red[v][threadIdx.x] < m ? red[v][threadIdx.x] : m;
    s_half[i0 + threadIdx.x] = m < INFINITY ? half_dist_down(m, d) : INFINITY;
  }
  const int i = i0 + wave;
  if (i >= k) return;                                 // uniform per wave; no barrier follows
  uint32_t v[KPL];
#pragma unroll
  for (int r = 0; r < KPL; ++r) v[r] = sK[wave * RS + lane * (KPL + 1) + r];
  wave_bitonic<KPL>(v, lane);
  float* out = rows + (size_t)i * k;
  const int base = lane * KPL;
  if ((k & 3) == 0) {
    // base + 4q < k implies base + 4q + 3 < k
#pragma unroll
    for (int q = 0; q < KPL / 4; ++q)
      if (base + 4 * q < k)
        *reinterpret_cast<float4*>(out + base + 4 * q) =
            make_float4(__uint_as_float(v[4 * q]), __uint_as_float(v[4 * q + 1]),
                        __uint_as_float(v[4 * q + 2]), __uint_as_float(v[4 * q + 3]));
  } else {
#pragma unroll
    for (int r = 0; r < KPL; ++r)
      if (base + r < k) out[base + r] = __uint_as_float(v[r]);
  }
}

template <int KPL>
static hipError_t launch_cc_rows(const CentroidOps& o, float* s_half, float* rows, int ib,
                                 const int* conv, int iter, hipStream_t s) {
  const size_t lds = sizeof(uint32_t) * (size_t)kRowsPerBlock * (64 * KPL + 64);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&cc_rows_kernel<KPL>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cc_rows_kernel<KPL>, dim3((o.k + kRowsPerBlock - 1) / kRowsPerBlock),
                     dim3(64 * kRowsPerBlock), lds, s, o.C64, o.CT, o.k, o.d, s_half, rows, ib,
                     conv, iter);
  return hipGetLastError();
}

int cc_rows_bits(int k) {
  int ib = 0;
  while ((1 << ib) < k) ++ib;
  return ib;
}

hipError_t launch_cc_bounds(const CentroidOps& o, float* s_half, float* rows,
                            const int* conv, int iter, hipStream_t s) {
  int kp2 = 1;
  while (kp2 < o.k) kp2 <<= 1;
  if (rows) {
    const int ib = cc_rows_bits(o.k);
    switch (kp2) {
      case 256: return launch_cc_rows<4>(o, s_half, rows, ib, conv, iter, s);
      case 512: return launch_cc_rows<8>(o, s_half, rows, ib, conv, iter, s);
      case 1024: return launch_cc_rows<16>(o, s_half, rows, ib, conv, iter, s);
      case 2048: return launch_cc_rows<32>(o, s_half, rows, ib, conv, iter, s);
      case 4096: return launch_cc_rows<64>(o, s_half, rows, ib, conv, iter, s);
      default: break;
    }
  }
  const size_t lds = rows ? sizeof(float) * (size_t)kp2 : 0;
  if (lds) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&cc_bounds_kernel),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(cc_bounds_kernel, dim3(o.k), dim3(256), lds, s, o.C64, o.CT,
                     o.k, o.d, s_half, rows, cc_rows_bits(o.k), kp2, conv, iter);
  return hipGetLastError();
}

constexpr int kFilterThreads = 1024;
constexpr int kTightenLanes = 8;     // lanes cooperating on one point's distance

// Clause 3 (tightening) pays off only while it still prunes: it runs in the
// first iterations, every 8th iteration, and whenever the previous run
// pruned at least 1/16 of its candidates (decided on the device).  Skipping
// it is always exact: the candidates are then scanned in full.
__device__ __forceinline__ bool tighten_now(const unsigned long long* prev_row,
                                            int iter) {
  return iter <= 2 || (iter & 7) == 0 ||
         (prev_row && prev_row[ROW_TIGHTEN_NEXT] != 0);
}

template <typename T>
__global__ __launch_bounds__(kFilterThreads) void mti_filter_kernel(
    const T* __restrict__ X, int64_t n, int d, const double* __restrict__ C64,
    const int32_t* __restrict__ labels, float* __restrict__ u,
    const float* __restrict__ drift, const float* __restrict__ s_half,
    int* __restrict__ list, int* __restrict__ seg_cnt,
    const unsigned long long* __restrict__ prev_row,
    unsigned long long* __restrict__ row, const int* __restrict__ conv,
    int iter, int vec, int mark) {
  // stage-A candidates: point, its label and s(label) (stage B reads the
  // last two from here instead of global memory)
  __shared__ int candA[kSeg];
  __shared__ int candL[kSeg];
  __shared__ float candS[kSeg];
  __shared__ int nA, nB;
  const int cv = *conv;
  const int seg = blockIdx.x;
  const int64_t p0 = (int64_t)seg * kSeg;
  const bool tighten = mark || tighten_now(prev_row, iter);

  // Clause 1 with the drift-updated bound, for every point of the segment:
  // thread t owns points 4t .. 4t + 3 of the segment (16-byte loads of
  // labels and bounds, issued with the convergence test, then the per-label
  // gathers, then one 16-byte store)
  static_assert(kSeg == 4 * kFilterThreads, "four points per thread");
  const int64_t pb = p0 + 4 * threadIdx.x;
  int lab[4];
  float uu[4];
  // the caller's label array may be only 4-byte aligned
  const bool full = pb + 3 < n && (((uintptr_t)labels & 15) == 0);
  if (full) {
    const int4 l4 = *reinterpret_cast<const int4*>(labels + pb);
    const float4 u4 = *reinterpret_cast<const float4*>(u + pb);
    lab[0] = l4.x; lab[1] = l4.y; lab[2] = l4.z; lab[3] = l4.w;
    uu[0] = u4.x; uu[1] = u4.y; uu[2] = u4.z; uu[3] = u4.w;
  } else {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      lab[e] = pb + e < n ? labels[pb + e] : 0;
      uu[e] = pb + e < n ? u[pb + e] : 0.0f;
    }
  }
  if (cv < iter) return;
  if (threadIdx.x == 0) { nA = 0; nB = 0; }
  if (tighten && seg == 0 && threadIdx.x == 0) row[ROW_TIGHTEN] = 1;
  __syncthreads();
  {
    float dr[4], sh[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) { dr[e] = drift[lab[e]]; sh[e] = s_half[lab[e]]; }
    bool cand[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      cand[e] = false;
      if (pb + e < n) {
        float ub;
        if (clause1_keeps(uu[e], dr[e], sh[e], &ub)) uu[e] = ub;
        else cand[e] = true;
      }
    }
    if (full) {
      *reinterpret_cast<float4*>(u + pb) = make_float4(uu[0], uu[1], uu[2], uu[3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (pb + e < n) u[pb + e] = uu[e];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint64_t m = __ballot(cand[e]);
      if (m) {
        int base = 0;
        if (lane_id() == __ffsll((unsigned long long)m) - 1)
          base = atomicAdd(&nA, __popcll(m));          // LDS atomic
        base = __shfl(base, __ffsll((unsigned long long)m) - 1);
        if (cand[e]) {
          const int slot = base + __popcll(m & lanemask_lt());
          candA[slot] = (int)(pb + e);
          candL[slot] = lab[e];
          candS[slot] = sh[e];
        }
      }
    }
  }
  __syncthreads();
  const int na = nA;
  if (!tighten) {
    // every candidate survives to the full scan (in index order of candA's
    // slots; the order does not affect any result)
    for (int c = threadIdx.x; c < na; c += kFilterThreads) list[p0 + c] = candA[c];
    if (threadIdx.x == 0) seg_cnt[seg] = na;
    const int q[2] = {SLOT_CAND, SLOT_SURV};
    const unsigned long long v[2] = {threadIdx.x == 0 ? (unsigned long long)na : 0ull,
                                     threadIdx.x == 0 ? (unsigned long long)na : 0ull};
    block_add_slots<2>(row, q, v);
    return;
  }

  // Clause 3: tighten to d(x, c_a) for the candidates, kTightenLanes lanes
  // per point, then Clause 1 again with the tight bound
  const int r = threadIdx.x % kTightenLanes;
  const int slot = threadIdx.x / kTightenLanes;
  constexpr int per_pass = kFilterThreads / kTightenLanes;
  for (int c0 = 0; c0 < na; c0 += per_pass) {
    const int c = c0 + slot;
    const bool live = c < na;
    const int p = live ? candA[c] : 0;
    const int a = live ? candL[c] : 0;
    double part = 0.0;
    if (live) {
      const T* x = X + (size_t)p * d;
      const double* ca = C64 + (size_t)a * d;
      constexpr int kE = 16 / (int)sizeof(T);      // elements per 16 bytes
      if (vec) {
        // lane r takes the 16-byte pieces r, r + 8, ... of the row
        for (int v = r; v * kE < d; v += kTightenLanes) {
          const uint4 w = reinterpret_cast<const uint4*>(x)[v];
          const T* e = reinterpret_cast<const T*>(&w);
#pragma unroll
          for (int q = 0; q < kE; ++q) {
            const double t = to_f64<T>(e[q]) - ca[v * kE + q];
            part = part + t * t;
          }
        }
      } else {
        for (int dim = r; dim < d; dim += kTightenLanes) {
          const double t = to_f64<T>(x[dim]) - ca[dim];
          part = part + t * t;
        }
      }
    }
#pragma unroll
    for (int off = 1; off < kTightenLanes; off <<= 1) part += __shfl_xor(part, off);
    bool surv = false;
    if (live && r == 0) {
      // any summation order of d non-negative terms: relative error below
      // (d + 2) 2^-53; inflate to an upper bound of the exact distance
      const double ub = f32_up(sqrt(part * (1.0 + (double)(d + 8) * 2.220446049250313e-16)) *
                               (1.0 + 8.881784197001252e-16));
      surv = !(ub * (1.0 + kEta) < (double)candS[c]);
      u[p] = (mark && surv) ? -(float)ub : (float)ub;
    }
    uint64_t m = __ballot(surv);
    if (m) {
      int base = 0;
      if (lane_id() == __ffsll((unsigned long long)m) - 1)
        base = atomicAdd(&nB, __popcll(m));
      base = __shfl(base, __ffsll((unsigned long long)m) - 1);
      if (surv) list[p0 + base + __popcll(m & lanemask_lt())] = p;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) seg_cnt[seg] = nB;
  const int q[2] = {SLOT_CAND, SLOT_SURV};
  const unsigned long long v[2] = {threadIdx.x == 0 ? (unsigned long long)na : 0ull,
                                   threadIdx.x == 0 ? (unsigned long long)nB : 0ull};
  block_add_slots<2>(row, q, v);
}

hipError_t launch_mti_filter(const void* X, knor_dtype dt, int64_t n, int d,
                             const double* C64, const int32_t* labels,
                             float* u, const float* drift, const float* s_half,
                             int* list, int* seg_cnt,
                             const unsigned long long* prev_row,
                             unsigned long long* row, const int* conv,
                             int iter, int mark, hipStream_t s) {
  const int nseg = nseg_of_n(n);
  const size_t esz = dt == KNOR_F64 ? 8 : (dt == KNOR_F32 ? 4 : 2);
  const int vec = (int)(((size_t)d * esz) % 16 == 0 && ((uintptr_t)X & 15) == 0);
  switch (dt) {
    case KNOR_F64:
      hipLaunchKernelGGL(mti_filter_kernel<double>, dim3(nseg),
                         dim3(kFilterThreads), 0, s, (const double*)X, n, d,
                         C64, labels, u, drift, s_half, list, seg_cnt,
                         prev_row, row, conv, iter, vec, mark);
      break;
    case KNOR_F32:
      hipLaunchKernelGGL(mti_filter_kernel<float>, dim3(nseg),
                         dim3(kFilterThreads), 0, s, (const float*)X, n, d, C64,
                         labels, u, drift, s_half, list, seg_cnt, prev_row, row,
                         conv, iter, vec, mark);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(mti_filter_kernel<uint16_t>, dim3(nseg),
                         dim3(kFilterThreads), 0, s, (const uint16_t*)X, n, d,
                         C64, labels, u, drift, s_half, list, seg_cnt,
                         prev_row, row, conv, iter, vec, mark);
      break;
  }
  return hipGetLastError();
}

}  // namespace knor
