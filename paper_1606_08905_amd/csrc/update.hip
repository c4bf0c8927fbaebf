// Centroid update: the mean of each cluster's members (Mhembere et al.,
// HPDC'17, Section "Parallel Lloyd's Algorithm", Phase II; Algorithm 1 merges
// per-thread partial centroids with a tree-shaped reduction).
//
// Here the merge is an atomic-free, two-pass segmented reduction whose FP64
// summation order is fixed and independent of the launch configuration:
//   pass 1  stable counting sort of point indices by label (perm), with
//           per-block histograms, column scans and an in-order scatter that
//           ranks equal labels inside a wave with per-bit ballots;
//   pass 2  leaf sums: each leaf = 64 consecutive members of one cluster in
//           increasing point index, summed left to right from the first;
//           then per cluster a pairwise tree over its leaves (bottom-up,
//           node a absorbs node a+s at stride s), one correctly rounded
//           division by the member count, and the derived operands.
// A cluster without members keeps its previous centroid.
#include <math.h>

#include "common.h"

namespace knor {

// ---------------------------------------------------------------------------
// plan / workspace
// ---------------------------------------------------------------------------

static int choose_block(int64_t n, int k) {
  int64_t B = 4096;
  int64_t cap = n > (1 << 24) ? n : (1 << 24);
  while (((n + B - 1) / B) * (int64_t)k > cap && B < (1 << 22)) B *= 2;
  return (int)B;
}

static int nseg_of(int nb) { return (nb + 31) / 32; }

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t update_workspace_bytes(int64_t n, int k, int d) {
  int B = choose_block(n, k);
  int64_t nb = (n + B - 1) / B;
  int64_t maxleaves = n / kLeaf + k + 1;
  int nseg = nseg_of((int)nb);
  size_t b = 0;
  b += align256(sizeof(int) * (size_t)nb * k);          // blockcnt
  b += align256(sizeof(int) * (size_t)nseg * k);        // segment sums
  b += align256(sizeof(int) * (size_t)k);               // nj
  b += align256(sizeof(int) * (size_t)(k + 1));         // off
  b += align256(sizeof(int) * (size_t)(k + 1));         // leaf_off
  b += align256(sizeof(int) * (size_t)n);               // perm
  b += align256(sizeof(double) * (size_t)maxleaves * d);// leafsum
  return b;
}

void update_plan_init(UpdatePlan* p, int64_t n, int k, int d, void* ws) {
  p->n = n;
  p->k = k;
  p->d = d;
  p->B = choose_block(n, k);
  p->nb = (int)((n + p->B - 1) / p->B);
  p->max_leaves = n / kLeaf + k + 1;
  char* c = (char*)ws;
  p->blockcnt = (int*)c; c += align256(sizeof(int) * (size_t)p->nb * k);
  // segment sums follow blockcnt; addressed through blockcnt + nb*k rounded
  c += align256(sizeof(int) * (size_t)nseg_of(p->nb) * k);
  p->nj = (int*)c; c += align256(sizeof(int) * (size_t)k);
  p->off = (int*)c; c += align256(sizeof(int) * (size_t)(k + 1));
  p->leaf_off = (int*)c; c += align256(sizeof(int) * (size_t)(k + 1));
  p->perm = (int*)c; c += align256(sizeof(int) * (size_t)n);
  p->leafsum = (double*)c;
}

static int* segsum_ptr(const UpdatePlan& p) {
  return (int*)((char*)p.blockcnt + align256(sizeof(int) * (size_t)p.nb * p.k));
}

// ---------------------------------------------------------------------------
// pass 1: stable counting sort by label
// ---------------------------------------------------------------------------

// Per-block label histogram; blockcnt is block-major [b][j].
__global__ __launch_bounds__(256) void hist_kernel(const int32_t* __restrict__ labels,
                                                   int64_t n, int k, int B,
                                                   int* __restrict__ blockcnt,
                                                   const int* __restrict__ done) {
  extern __shared__ int sh[];
  if (*done) return;
  const int b = blockIdx.x;
  for (int j = threadIdx.x; j < k; j += blockDim.x) sh[j] = 0;
  __syncthreads();
  int64_t p0 = (int64_t)b * B, p1 = p0 + B < n ? p0 + B : n;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    unsigned lab = (unsigned)labels[p];
    if (lab < (unsigned)k) atomicAdd(&sh[lab], 1);   // out-of-range: ignored
  }
  __syncthreads();
  int* row = blockcnt + (size_t)b * k;
  for (int j = threadIdx.x; j < k; j += blockDim.x) row[j] = sh[j];
}

// Column scan, phase A: per (segment of 32 blocks, cluster) sum.
__global__ __launch_bounds__(256) void colscan_a(const int* __restrict__ blockcnt,
                                                 int nb, int k,
                                                 int* __restrict__ segsum,
                                                 const int* __restrict__ done) {
  if (*done) return;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int seg = blockIdx.y;
  if (j >= k) return;
  int b0 = seg * 32, b1 = b0 + 32 < nb ? b0 + 32 : nb;
  int s = 0;
  for (int b = b0; b < b1; ++b) s += blockcnt[(size_t)b * k + j];
  segsum[(size_t)seg * k + j] = s;
}

// Phase B: per cluster, exclusive scan over segments; nj = total.
__global__ __launch_bounds__(256) void colscan_b(int* __restrict__ segsum,
                                                 int nseg, int k,
                                                 int* __restrict__ nj,
                                                 const int* __restrict__ done) {
  if (*done) return;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  int run = 0;
  for (int s = 0; s < nseg; ++s) {
    int v = segsum[(size_t)s * k + j];
    segsum[(size_t)s * k + j] = run;
    run += v;
  }
  nj[j] = run;
}

// Phase C: per (segment, cluster), exclusive prefix of blockcnt in place.
__global__ __launch_bounds__(256) void colscan_c(int* __restrict__ blockcnt,
                                                 int nb, int k,
                                                 const int* __restrict__ segsum,
                                                 const int* __restrict__ done) {
  if (*done) return;
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  int seg = blockIdx.y;
  if (j >= k) return;
  int b0 = seg * 32, b1 = b0 + 32 < nb ? b0 + 32 : nb;
  int run = segsum[(size_t)seg * k + j];
  for (int b = b0; b < b1; ++b) {
    int v = blockcnt[(size_t)b * k + j];
    blockcnt[(size_t)b * k + j] = run;
    run += v;
  }
}

// Exclusive scans over clusters: off (members) and leaf_off (leaves of 64).
__global__ __launch_bounds__(1024) void cluster_scan(const int* __restrict__ nj,
                                                     int k, int* __restrict__ off,
                                                     int* __restrict__ leaf_off,
                                                     const int* __restrict__ done) {
  __shared__ int sa[1024], sb[1024];
  if (*done) return;
  const int per = (k + 1023) / 1024;
  const int j0 = threadIdx.x * per;
  int a = 0, l = 0;
  for (int j = j0; j < j0 + per && j < k; ++j) {
    a += nj[j];
    l += (nj[j] + kLeaf - 1) / kLeaf;
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = l;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    int va = threadIdx.x >= s ? sa[threadIdx.x - s] : 0;
    int vb = threadIdx.x >= s ? sb[threadIdx.x - s] : 0;
    __syncthreads();
    sa[threadIdx.x] += va;
    sb[threadIdx.x] += vb;
    __syncthreads();
  }
  int ra = sa[threadIdx.x] - a, rb = sb[threadIdx.x] - l;   // exclusive
  for (int j = j0; j < j0 + per && j < k; ++j) {
    off[j] = ra;
    leaf_off[j] = rb;
    ra += nj[j];
    rb += (nj[j] + kLeaf - 1) / kLeaf;
  }
  if (threadIdx.x == 1023) {
    off[k] = sa[1023];
    leaf_off[k] = sb[1023];
  }
}

// In-order scatter: one wave per block walks its points in chunks of 64.
// Lanes holding the same label find each other with one ballot per label
// bit; a lane's rank among them is the count of such lanes below it.
__global__ __launch_bounds__(64) void scatter_kernel(
    const int32_t* __restrict__ labels, int64_t n, int k, int B, int bits,
    const int* __restrict__ blockcnt, const int* __restrict__ off,
    int* __restrict__ perm, const int* __restrict__ done) {
  extern __shared__ int run[];
  if (*done) return;
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int* row = blockcnt + (size_t)b * k;
  for (int j = lane; j < k; j += 64) run[j] = off[j] + row[j];
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  int64_t p0 = (int64_t)b * B, p1 = p0 + B < n ? p0 + B : n;
  for (int64_t c = p0; c < p1; c += 64) {
    int64_t p = c + lane;
    int lab = p < p1 ? labels[p] : 0;
    bool valid = p < p1 && (unsigned)lab < (unsigned)k;
    if (!valid) lab = 0;
    uint64_t mask = __ballot(valid);
    for (int bit = 0; bit < bits; ++bit) {
      bool on = (lab >> bit) & 1;
      uint64_t bb = __ballot(on);
      mask &= on ? bb : ~bb;
    }
    int rank = __popcll(mask & lt);
    int cnt = __popcll(mask);
    int pos = 0;
    if (valid) pos = run[lab] + rank;
    __builtin_amdgcn_wave_barrier();
    if (valid) {
      perm[pos] = (int)p;
      if (rank == cnt - 1) run[lab] = pos + 1;
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------------------
// pass 2: leaf sums, tree, finalize
// ---------------------------------------------------------------------------

__device__ __forceinline__ int cluster_of_leaf(const int* __restrict__ leaf_off,
                                               int k, int g) {
  int lo = 0, hi = k - 1;      // largest j with leaf_off[j] <= g
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (leaf_off[mid] <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// G lanes per leaf (G = power of two >= d, at most 64); lane t of a group
// owns dimensions t, t+G, ...  Each leaf is summed left to right.
template <typename T>
__global__ __launch_bounds__(256) void leaf_kernel(
    const T* __restrict__ X, int d, int G, const int* __restrict__ perm,
    const int* __restrict__ nj, const int* __restrict__ off,
    const int* __restrict__ leaf_off, int k, double* __restrict__ leafsum,
    const int* __restrict__ done) {
  if (*done) return;
  const int total = leaf_off[k];
  const int per_block = blockDim.x / G;
  const int g = blockIdx.x * per_block + threadIdx.x / G;
  const int t = threadIdx.x % G;
  if (g >= total) return;
  const int j = cluster_of_leaf(leaf_off, k, g);
  const int L = g - leaf_off[j];
  const int m0 = off[j] + L * kLeaf;
  int cnt = nj[j] - L * kLeaf;
  if (cnt > kLeaf) cnt = kLeaf;
  for (int i = t; i < d; i += G) {
    double s = to_f64<T>(X[(size_t)perm[m0] * d + i]);
    for (int m = 1; m < cnt; ++m)
      s = __dadd_rn(s, to_f64<T>(X[(size_t)perm[m0 + m] * d + i]));
    leafsum[(size_t)g * d + i] = s;
  }
}

// One workgroup per cluster: tree over its leaves, mean, operands, drift.
__global__ __launch_bounds__(256) void tree_finalize(
    double* __restrict__ leafsum, const int* __restrict__ nj,
    const int* __restrict__ leaf_off, int k, int d,
    const double* C_prev, double* C_out, int64_t* __restrict__ counts_out,
    float* __restrict__ Cm2, float* __restrict__ cn, int dp,
    float* __restrict__ drift, const int* __restrict__ done) {
  __shared__ double red[256];
  __shared__ double cval[kMaxD];
  if (*done) return;
  const int j = blockIdx.x;
  const int cntj = nj[j];
  const int m = leaf_off[j + 1] - leaf_off[j];
  double* base = leafsum + (size_t)leaf_off[j] * d;
  for (int s = 1; s < m; s <<= 1) {
    const int pairs = (m - s - 1) / (2 * s) + 1;
    for (int e = threadIdx.x; e < pairs * d; e += blockDim.x) {
      int i = e / d, dim = e - i * d;
      int a = i * 2 * s;
      base[(size_t)a * d + dim] =
          __dadd_rn(base[(size_t)a * d + dim], base[(size_t)(a + s) * d + dim]);
    }
    __syncthreads();
  }
  double diff2 = 0.0;
  for (int dim = threadIdx.x; dim < d; dim += blockDim.x) {
    double old = C_prev[(size_t)j * d + dim];
    double c = cntj > 0 ? __ddiv_rn(base[dim], (double)cntj) : old;
    C_out[(size_t)j * d + dim] = c;
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
    if (counts_out) counts_out[j] = cntj;
    if (drift)
      drift[j] = f32_up(sqrt(red[0]) * (1.0 + (double)(d + 8) * 2.220446049250313e-16));
    if (cn) {
      double ss = 0.0;
      for (int dim = 0; dim < d; ++dim) ss = __dadd_rn(ss, __dmul_rn(cval[dim], cval[dim]));
      cn[j] = (float)ss;
    }
  }
  if (Cm2)
    for (int dim = threadIdx.x; dim < dp; dim += blockDim.x)
      Cm2[(size_t)j * dp + dim] = dim < d ? -2.0f * (float)cval[dim] : 0.0f;
}

hipError_t launch_update(const UpdatePlan& p, const void* X, knor_dtype dt,
                         const int32_t* labels, const double* C_prev,
                         double* C_out, int64_t* counts_out, CentroidOps* ops,
                         float* drift, const int* done, hipStream_t s,
                         Prof* prof) {
  const int k = p.k, d = p.d;
  const size_t lds_k = sizeof(int) * (size_t)k;
  if (prof) prof->begin(KNOR_PROF_SORT);
  hipLaunchKernelGGL(hist_kernel, dim3(p.nb), dim3(256), lds_k, s, labels, p.n,
                     k, p.B, p.blockcnt, done);
  int* seg = segsum_ptr(p);
  int nseg = nseg_of(p.nb);
  dim3 g2((k + 255) / 256, nseg);
  hipLaunchKernelGGL(colscan_a, g2, dim3(256), 0, s, p.blockcnt, p.nb, k, seg,
                     done);
  hipLaunchKernelGGL(colscan_b, dim3((k + 255) / 256), dim3(256), 0, s, seg,
                     nseg, k, p.nj, done);
  hipLaunchKernelGGL(colscan_c, g2, dim3(256), 0, s, p.blockcnt, p.nb, k, seg,
                     done);
  hipLaunchKernelGGL(cluster_scan, dim3(1), dim3(1024), 0, s, p.nj, k, p.off,
                     p.leaf_off, done);
  int bits = 0;
  while ((1 << bits) < k) ++bits;
  hipLaunchKernelGGL(scatter_kernel, dim3(p.nb), dim3(64), lds_k, s, labels,
                     p.n, k, p.B, bits, p.blockcnt, p.off, p.perm, done);
  if (prof) { prof->end(); prof->begin(KNOR_PROF_LEAF); }
  int G = 1;
  while (G < d && G < 64) G *= 2;
  const int per_block = 256 / G;
  const int64_t lblocks = (p.max_leaves + per_block - 1) / per_block;
  switch (dt) {
    case KNOR_F64:
      hipLaunchKernelGGL(leaf_kernel<double>, dim3(lblocks), dim3(256), 0, s,
                         (const double*)X, d, G, p.perm, p.nj, p.off,
                         p.leaf_off, k, p.leafsum, done);
      break;
    case KNOR_F32:
      hipLaunchKernelGGL(leaf_kernel<float>, dim3(lblocks), dim3(256), 0, s,
                         (const float*)X, d, G, p.perm, p.nj, p.off,
                         p.leaf_off, k, p.leafsum, done);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(leaf_kernel<uint16_t>, dim3(lblocks), dim3(256), 0, s,
                         (const uint16_t*)X, d, G, p.perm, p.nj, p.off,
                         p.leaf_off, k, p.leafsum, done);
      break;
  }
  if (prof) { prof->end(); prof->begin(KNOR_PROF_TREE); }
  hipLaunchKernelGGL(tree_finalize, dim3(k), dim3(256), 0, s, p.leafsum, p.nj,
                     p.leaf_off, k, d, C_prev, C_out, counts_out,
                     ops ? ops->Cm2 : nullptr, ops ? ops->cn : nullptr,
                     ops ? ops->dp : 0, drift, done);
  if (prof) prof->end();
  return hipGetLastError();
}

}  // namespace knor
