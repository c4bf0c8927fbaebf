// Initial centroids chosen by k-means++ seeding on the device
// (KNOR_INIT_KMEANSPP).  The paper does not fix an initialisation; this is
// Arthur and Vassilvitskii's D^2 seeding made a deterministic function of a
// seed and of the data, independent of launch shape and summation order:
//
//  * D(p) is the canonical FP64 squared distance (index order, no FMA) from
//    point p to its nearest centroid chosen so far.
//  * Sampling weights are integers: with M = max_p D(p), e the exponent with
//    M < 2^e, and B = 63 - ceil(log2 n), w(p) = floor(D(p) 2^(B - e)), so
//    that w(p) < 2^B and the total W < 2^63.  Integer sums do not depend on
//    their order, so any grid computes the same W and the same prefix sums.
//  * Draw t (t >= 1) takes the SplitMix64 output r_t, the target
//    q = floor(r_t W / 2^64), and selects the point p with
//    sum_{p' < p} w(p') <= q < sum_{p' <= p} w(p').  If W = 0 (every point
//    coincides with a chosen centroid) p = floor(r_t n / 2^64) instead.
//  * The first centroid is point floor(r_0 n / 2^64).
// Row p of X, upcast to FP64 exactly, becomes the next centroid.
#include <math.h>

#include "common.h"

namespace knor {

constexpr int kPPThreads = 256;
constexpr int kPPPoints = 1024;          // points per block of the passes
constexpr int kPPPick = 1024;            // threads of the selection kernel
static_assert(kPPPoints == kPPPick, "one selection thread per point of a block");

// D(p) <- min(D(p), dist2(x_p, c)) for the block's points (first: D(p) <-
// dist2); the block's largest D joins Mbits by an integer max (non-negative
// doubles order like their bit patterns).
template <typename T>
__global__ __launch_bounds__(kPPThreads) void pp_min_kernel(
    const T* __restrict__ X, int64_t n, int d, const double* __restrict__ c,
    double* __restrict__ dmin, unsigned long long* __restrict__ Mbits, int first) {
  __shared__ double sc[kMaxD];
  __shared__ unsigned long long smax;
  for (int i = threadIdx.x; i < d; i += kPPThreads) sc[i] = c[i];
  if (threadIdx.x == 0) smax = 0ull;
  __syncthreads();
  unsigned long long mine = 0ull;
  const int64_t p0 = (int64_t)blockIdx.x * kPPPoints;
  for (int e = threadIdx.x; e < kPPPoints; e += kPPThreads) {
    const int64_t p = p0 + e;
    if (p >= n) break;
    const double D = dist2_canon<T>(X + (size_t)p * d, sc, d);
    const double m = first ? D : (D < dmin[p] ? D : dmin[p]);
    dmin[p] = m;
    const unsigned long long b = (unsigned long long)__double_as_longlong(m);
    mine = b > mine ? b : mine;
  }
  atomicMax(&smax, mine);
  __syncthreads();
  if (threadIdx.x == 0) atomicMax(Mbits, smax);
}

__device__ __forceinline__ int pp_shift(unsigned long long mbits, int B) {
  const double M = __longlong_as_double((long long)mbits);
  return B - (ilogb(M) + 1);          // M < 2^(ilogb(M) + 1)
}

__device__ __forceinline__ unsigned long long pp_weight(double D, int shift) {
  return (unsigned long long)floor(ldexp(D, shift));
}

// bsum[b] = sum of the weights of block b's points (M > 0).
__global__ __launch_bounds__(kPPThreads) void pp_wsum_kernel(
    const double* __restrict__ dmin, int64_t n, int B,
    const unsigned long long* __restrict__ Mbits,
    unsigned long long* __restrict__ bsum) {
  __shared__ unsigned long long part[kPPThreads / 64];
  const unsigned long long mb = *Mbits;
  const int shift = mb ? pp_shift(mb, B) : 0;
  unsigned long long s = 0ull;
  const int64_t p0 = (int64_t)blockIdx.x * kPPPoints;
  if (mb)
    for (int e = threadIdx.x; e < kPPPoints; e += kPPThreads) {
      const int64_t p = p0 + e;
      if (p < n) s += pp_weight(dmin[p], shift);
    }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0ull;
    for (int w = 0; w < kPPThreads / 64; ++w) t += part[w];
    bsum[blockIdx.x] = t;
  }
}

// Inclusive scan of v over the workgroup (kPPPick threads); returns the
// thread's inclusive prefix and leaves the total in *tot.
__device__ unsigned long long pp_scan(unsigned long long v, unsigned long long* buf,
                                      unsigned long long* tot) {
  buf[threadIdx.x] = v;
  __syncthreads();
  for (int s = 1; s < kPPPick; s <<= 1) {
    const unsigned long long t = threadIdx.x >= (unsigned)s ? buf[threadIdx.x - s] : 0ull;
    __syncthreads();
    buf[threadIdx.x] += t;
    __syncthreads();
  }
  const unsigned long long r = buf[threadIdx.x];
  *tot = buf[kPPPick - 1];
  __syncthreads();
  return r;
}

// Draw `slot` (r = its SplitMix64 output): uniform when `uniform` or when
// the total weight is zero, else D^2-weighted through the block sums.  The
// chosen row becomes centroid `slot` of C (FP64).
template <typename T>
__global__ __launch_bounds__(kPPPick) void pp_pick_kernel(
    const T* __restrict__ X, int64_t n, int d, int B, const double* __restrict__ dmin,
    const unsigned long long* __restrict__ Mbits, const unsigned long long* __restrict__ bsum,
    int nb, const unsigned long long* __restrict__ rnd, int slot, int uniform,
    double* __restrict__ C) {
  __shared__ unsigned long long buf[kPPPick];
  __shared__ long long s_pick, s_blk;
  __shared__ unsigned long long s_rem;
  const unsigned long long r = rnd[slot];
  const unsigned long long mb = uniform ? 0ull : *Mbits;
  if (threadIdx.x == 0) { s_pick = -1; s_blk = -1; s_rem = 0ull; }
  // block sums in contiguous ranges per thread, then a scan of the ranges
  const int per = (nb + kPPPick - 1) / kPPPick;
  const int b0 = threadIdx.x * per;
  unsigned long long loc = 0ull;
  if (mb)
    for (int b = b0; b < b0 + per && b < nb; ++b) loc += bsum[b];
  unsigned long long W = 0ull;
  const unsigned long long incl = pp_scan(loc, buf, &W);
  if (W == 0ull) {
    if (threadIdx.x == 0) s_pick = (long long)__umul64hi(r, (unsigned long long)n);
  } else {
    const unsigned long long q = __umul64hi(r, W);       // 0 <= q < W
    const unsigned long long excl = incl - loc;
    if (loc && excl <= q && q < incl) {                  // exactly one thread
      unsigned long long run = excl;
      for (int b = b0; b < b0 + per && b < nb; ++b) {
        if (q < run + bsum[b]) { s_blk = b; s_rem = q - run; break; }
        run += bsum[b];
      }
    }
    __syncthreads();
    const long long blk = s_blk;
    const unsigned long long rem = s_rem;
    const int shift = pp_shift(mb, B);
    const int64_t p = (int64_t)blk * kPPPoints + threadIdx.x;
    const unsigned long long w = (blk >= 0 && p < n) ? pp_weight(dmin[p], shift) : 0ull;
    unsigned long long tot = 0ull;
    const unsigned long long wi = pp_scan(w, buf, &tot);
    if (w && wi - w <= rem && rem < wi) s_pick = p;
  }
  __syncthreads();
  int64_t p = s_pick;
  if (p < 0 || p >= n) p = 0;          // unreachable: the scans above agree
  for (int i = threadIdx.x; i < d; i += kPPPick)
    C[(size_t)slot * d + i] = to_f64<T>(X[(size_t)p * d + i]);
}

size_t kmeanspp_workspace_bytes(int64_t n, int k) {
  const int64_t nb = (n + kPPPoints - 1) / kPPPoints;
  return sizeof(double) * (size_t)n + sizeof(unsigned long long) * (size_t)nb + 256 +
         sizeof(unsigned long long) * (size_t)k + 256;
}

template <typename T>
static hipError_t kmeanspp_t(const T* X, int64_t n, int d, int k,
                             const unsigned long long* rnd, double* C, void* ws,
                             hipStream_t s) {
  const int64_t nb64 = (n + kPPPoints - 1) / kPPPoints;
  const int nb = (int)nb64;
  char* w = (char*)ws;
  double* dmin = (double*)w;
  w += (sizeof(double) * (size_t)n + 255) & ~(size_t)255;
  unsigned long long* bsum = (unsigned long long*)w;
  w += (sizeof(unsigned long long) * (size_t)nb + 255) & ~(size_t)255;
  unsigned long long* Mslot = (unsigned long long*)w;   // one maximum per draw
  int lg = 0;
  while (((int64_t)1 << lg) < n) ++lg;
  const int B = 63 - lg;
  hipError_t e = hipMemsetAsync(Mslot, 0, sizeof(unsigned long long) * (size_t)k, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pp_pick_kernel<T>, dim3(1), dim3(kPPPick), 0, s, X, n, d, B, dmin,
                     Mslot, bsum, nb, rnd, 0, 1, C);
  for (int t = 1; t < k; ++t) {
    hipLaunchKernelGGL(pp_min_kernel<T>, dim3(nb), dim3(kPPThreads), 0, s, X, n, d,
                       C + (size_t)(t - 1) * d, dmin, Mslot + t, t == 1 ? 1 : 0);
    hipLaunchKernelGGL(pp_wsum_kernel, dim3(nb), dim3(kPPThreads), 0, s, dmin, n, B,
                       Mslot + t, bsum);
    hipLaunchKernelGGL(pp_pick_kernel<T>, dim3(1), dim3(kPPPick), 0, s, X, n, d, B, dmin,
                       Mslot + t, bsum, nb, rnd, t, 0, C);
  }
  return hipGetLastError();
}

hipError_t launch_kmeanspp(const void* X, knor_dtype dt, int64_t n, int d, int k,
                           const unsigned long long* rnd, double* C, void* ws,
                           hipStream_t s) {
  switch (dt) {
    case KNOR_F64: return kmeanspp_t((const double*)X, n, d, k, rnd, C, ws, s);
    case KNOR_F32: return kmeanspp_t((const float*)X, n, d, k, rnd, C, ws, s);
    case KNOR_BF16: return kmeanspp_t((const uint16_t*)X, n, d, k, rnd, C, ws, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace knor
