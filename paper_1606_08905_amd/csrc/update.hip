// Centroid update: the mean of each cluster's members (Mhembere et al.,
// HPDC'17, Section "Parallel Lloyd's Algorithm", Phase II; Algorithm 1 merges
// per-thread partial centroids with a tree-shaped reduction).
//
// Here the merge is an atomic-free, two-pass segmented reduction whose FP64
// summation order is fixed and independent of the launch configuration:
//   pass 1  stable counting sort of point indices by label (perm): per-range
//           label histograms, prefix sums over ranges and clusters, and an
//           in-order scatter that ranks equal labels inside a wave with
//           per-bit ballots;
//   pass 2  leaf sums: each leaf = 64 consecutive members of one cluster in
//           increasing point index, summed left to right from the first;
//           then per cluster a pairwise tree over its leaves (bottom-up,
//           node a absorbs node a+s at stride s), one correctly rounded
//           division by the member count, and the derived operands.
// A cluster without members keeps its previous centroid.  Inside a fit, a
// cluster whose member set did not change since the last update ("clean")
// has the same canonical sum, so pass 2 skips it and keeps its centroid.
//
// Pass 1 has two schedules.  For k <= kFusedMaxK, one workgroup of 16 waves
// owns a range of points; each wave owns a sub-range and a private running
// table in LDS, and every workgroup derives its own offsets from the range
// totals (two kernels, or three when the table of range totals is too large
// for the scatter to take its own prefix).  For larger k, per-block counts
// go through a segmented column scan (four kernels).
#include <math.h>

#include "common.h"
#include "update_common.h"

namespace knor {

constexpr int kFusedMaxK = 768;            // 16 x k running tables within 48 KB
constexpr int kFusedWaves = 16;
constexpr int kFusedMaxRanges = 1024;

// ---------------------------------------------------------------------------
// plan / workspace
// ---------------------------------------------------------------------------

static bool fused_sort(int k) { return k <= kFusedMaxK; }

// The scatter computes the prefix over ranges itself when each of its
// threads sums at most kScatterPrefix range totals (the 1024 threads split
// as floor(1024 / k) parts per cluster); otherwise range_scan runs first.
constexpr int kScatterPrefix = 32;
static bool scatter_prefix(int nb, int k) {
  const int parts = 1024 / k;
  return (nb + parts - 1) / parts <= kScatterPrefix;
}

static int choose_block(int64_t n, int k) {
  if (fused_sort(k)) {
    // sub-range per wave (a multiple of 64 points, about 256, so that a
    // million points spread over all CUs); a workgroup covers kFusedWaves
    // sub-ranges; up to kFusedMaxRanges workgroups
    int64_t ranges = (n + kFusedWaves * 256 - 1) / (kFusedWaves * 256);
    if (ranges > kFusedMaxRanges) ranges = kFusedMaxRanges;
    if (ranges < 1) ranges = 1;
    int64_t sb = (n + kFusedWaves * ranges - 1) / (kFusedWaves * ranges);
    sb = (sb + 63) / 64 * 64;
    if (sb < 64) sb = 64;
    return (int)sb;
  }
  // one wave per block: enough blocks to occupy the GPU, while the nb x k
  // count matrix stays within max(n, 2^24) entries
  int64_t B = 1024;
  while (n / B > 4096 && B < 4096) B *= 2;
  int64_t cap = n > (1 << 24) ? n : (1 << 24);
  while (((n + B - 1) / B) * (int64_t)k > cap && B < (1 << 22)) B *= 2;
  return (int)B;
}

// blocks per column-scan segment: the scatter re-adds at most seglen-1 rows
static int choose_seglen(int k) {
  int s = 16384 / k;
  return s < 1 ? 1 : (s > 32 ? 32 : s);
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static void plan_dims(int64_t n, int k, int* B, int* nb, int* seglen,
                      int* nsegc) {
  *B = choose_block(n, k);
  if (fused_sort(k)) {
    const int64_t range = (int64_t)*B * kFusedWaves;
    *nb = (int)((n + range - 1) / range);    // workgroup ranges
    *seglen = 1;
    *nsegc = 0;
  } else {
    *nb = (int)((n + *B - 1) / *B);
    *seglen = choose_seglen(k);
    *nsegc = (*nb + *seglen - 1) / *seglen;
  }
}

size_t update_workspace_bytes(int64_t n, int k, int d) {
  int B, nb, seglen, nsegc;
  plan_dims(n, k, &B, &nb, &seglen, &nsegc);
  const int64_t maxleaves = n / kLeaf + k + 1;
  const size_t cnt_entries = fused_sort(k) ? (size_t)nb * (kFusedWaves + 1) * k
                                           : (size_t)nb * k;
  size_t b = 0;
  b += align256(sizeof(int) * cnt_entries);                  // blockcnt
  b += align256(sizeof(int) * (size_t)(nsegc > 0 ? nsegc : 1) * k);  // segsum
  b += align256(sizeof(int) * 64);                           // ticket
  b += align256(sizeof(int) * (size_t)k);                    // nj
  b += align256(sizeof(int) * (size_t)(k + 1));              // off
  b += align256(sizeof(int) * (size_t)(k + 1));              // leaf_off
  b += align256(sizeof(int) * (size_t)(fused_sort(k) ? nb : 1) * k);  // rpre
  b += align256(sizeof(int) * (size_t)n);                    // perm
  b += align256(sizeof(double) * (size_t)maxleaves * d);     // leafsum
  return b;
}

void update_plan_init(UpdatePlan* p, int64_t n, int k, int d, void* ws) {
  p->n = n;
  p->k = k;
  p->d = d;
  plan_dims(n, k, &p->B, &p->nb, &p->seglen, &p->nsegc);
  p->max_leaves = n / kLeaf + k + 1;
  p->tb = tree_block_leaves(d);
  const size_t cnt_entries = fused_sort(k) ? (size_t)p->nb * (kFusedWaves + 1) * k
                                           : (size_t)p->nb * k;
  char* c = (char*)ws;
  p->blockcnt = (int*)c; c += align256(sizeof(int) * cnt_entries);
  p->segsum = (int*)c; c += align256(sizeof(int) * (size_t)(p->nsegc > 0 ? p->nsegc : 1) * k);
  p->ticket = (int*)c; c += align256(sizeof(int) * 64);
  p->nj = (int*)c; c += align256(sizeof(int) * (size_t)k);
  p->off = (int*)c; c += align256(sizeof(int) * (size_t)(k + 1));
  p->leaf_off = (int*)c; c += align256(sizeof(int) * (size_t)(k + 1));
  p->rpre = (int*)c; c += align256(sizeof(int) * (size_t)(fused_sort(k) ? p->nb : 1) * k);
  p->perm = (int*)c; c += align256(sizeof(int) * (size_t)n);
  p->leafsum = (double*)c;
}

hipError_t update_plan_reset(const UpdatePlan& p, hipStream_t s) {
  return hipMemsetAsync(p.ticket, 0, sizeof(int) * 64, s);
}

#define SKIP_IF_CONVERGED \
  if (*conv < iter) return;

// Rank of each lane among the lanes holding the same label (one ballot per
// label bit); returns the mask of those lanes.
__device__ __forceinline__ uint64_t same_label_mask(bool valid, int lab,
                                                    int bits) {
  uint64_t mask = __ballot(valid);
  for (int bit = 0; bit < bits; ++bit) {
    const bool on = (lab >> bit) & 1;
    const uint64_t bb = __ballot(on);
    mask &= on ? bb : ~bb;
  }
  return mask;
}

// Exclusive scans over clusters of per-cluster totals: off (members) and
// leaf_off (leaves of 64).  Run by one block of 1024 threads.
__device__ void cluster_scan_block(const int* __restrict__ nj, int k,
                                   int* __restrict__ off,
                                   int* __restrict__ leaf_off, int* sa,
                                   int* sb) {
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

// ---------------------------------------------------------------------------
// pass 1, fused schedule (k <= kFusedMaxK): two kernels
// ---------------------------------------------------------------------------
//
// cnt layout per range r: kFusedWaves rows of per-wave counts, then one row
// of range totals: cnt[(r * (W + 1) + w) * k + j].

template <bool EARLY>
__global__ __launch_bounds__(1024) void hist_fused(const int32_t* __restrict__ labels,
                                                   int64_t n, int k, int SB,
                                                   int* __restrict__ cnt,
                                                   const int* __restrict__ conv,
                                                   int iter) {
  extern __shared__ int tab[];               // kFusedWaves x k
  const int cv = *conv;
  if (EARLY && cv < iter) return;            // gated: nothing loaded yet
  const int r = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t p0 = ((int64_t)r * kFusedWaves + wave) * SB;
  const int64_t p1 = p0 + SB < n ? p0 + SB : n;
  // the labels of kAhead chunks of 64 are loaded together (the first batch
  // before the convergence test, so the two waits overlap)
  constexpr int kAhead = 16;
  int labs[kAhead];
#pragma unroll
  for (int q = 0; q < kAhead; ++q) {
    const int64_t p = p0 + q * 64 + lane;
    labs[q] = p < p1 ? labels[p] : -1;
  }
  for (int e = threadIdx.x; e < kFusedWaves * k; e += blockDim.x) tab[e] = 0;
  if (cv < iter) return;
  __syncthreads();
  int* t = tab + wave * k;
  for (int64_t c0 = p0; c0 < p1; c0 += 64 * kAhead) {
    if (c0 != p0)
#pragma unroll
      for (int q = 0; q < kAhead; ++q) {
        const int64_t p = c0 + q * 64 + lane;
        labs[q] = p < p1 ? labels[p] : -1;
      }
#pragma unroll
    for (int q = 0; q < kAhead; ++q)
      if ((unsigned)labs[q] < (unsigned)k) atomicAdd(&t[labs[q]], 1);   // LDS; order-free
  }
  __syncthreads();
  int* out = cnt + (size_t)r * (kFusedWaves + 1) * k;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    int s = 0;
    for (int w = 0; w < kFusedWaves; ++w) {
      const int v = tab[w * k + j];
      out[(size_t)w * k + j] = v;
      s += v;
    }
    out[(size_t)kFusedWaves * k + j] = s;
  }
}

// Per cluster j (one workgroup each): exclusive prefix over the ranges of
// the range totals, rpre[r * k + j], and the cluster total nj[j].
template <bool EARLY>
__global__ __launch_bounds__(256) void range_scan(const int* __restrict__ cnt,
                                                  int nr, int k,
                                                  int* __restrict__ rpre,
                                                  int* __restrict__ nj,
                                                  const int* __restrict__ conv,
                                                  int iter) {
  __shared__ int part[256];
  const int cv = *conv;
  if (EARLY && cv < iter) return;
  const int j = blockIdx.x;
  const int per = (nr + 255) / 256;
  const int r0 = threadIdx.x * per;
  int v[4];
  int local = 0;
  for (int q = 0; q < per; q += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + q + u;
      v[u] = (q + u < per && r < nr)
                 ? cnt[((size_t)r * (kFusedWaves + 1) + kFusedWaves) * k + j] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) local += v[u];
  }
  if (cv < iter) return;
  part[threadIdx.x] = local;
  __syncthreads();
  for (int s = 1; s < 256; s <<= 1) {
    const int t = threadIdx.x >= s ? part[threadIdx.x - s] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int run = part[threadIdx.x] - local;
  for (int q = 0; q < per; ++q) {
    const int r = r0 + q;
    if (r >= nr) break;
    rpre[(size_t)r * k + j] = run;
    run += cnt[((size_t)r * (kFusedWaves + 1) + kFusedWaves) * k + j];
  }
  if (threadIdx.x == 255) nj[j] = part[255];
}

// Exclusive prefix over ranges of the range totals: from range_scan (rpre
// and nj), or, with in_prefix, computed here: thread (q, c) = (t / k, t % k)
// sums the totals of cluster c over ranges q, q + Q, ... (Q = 1024 / k
// parts), over all ranges and over the ranges before this one, and range 0
// stores the cluster totals in nj.
template <bool EARLY>
__global__ __launch_bounds__(1024) void scatter_fused(
    const int32_t* __restrict__ labels, int64_t n, int k, int SB,
    int bits, const int* __restrict__ cnt, const int* __restrict__ rpre,
    int* __restrict__ nj, int in_prefix, int lab_lds, const int* __restrict__ dirty,
    int* __restrict__ perm, int* __restrict__ off_out,
    int* __restrict__ leaf_off_out, const int* __restrict__ conv, int iter) {
  extern __shared__ int run[];               // kFusedWaves x k (+ the range's labels)
  __shared__ int sa[1024], sb[1024];
  __shared__ int sDirty[kFusedMaxK];         // the dirty flags, read per point
  const int cv = *conv;
  if (EARLY && cv < iter) return;
  const int r = blockIdx.x, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int j = threadIdx.x;                 // k <= 1024: one cluster per thread
  int tot = 0, pre = 0;
  int part_all = 0, part_before = 0;
  if (in_prefix) {
    const int Q = 1024 / k, q = threadIdx.x / k, c = threadIdx.x - q * k;
    if (q < Q) {
      int v[kScatterPrefix];
#pragma unroll
      for (int u = 0; u < kScatterPrefix; ++u) {
        const int rr = q + u * Q;
        v[u] = rr < (int)gridDim.x
                   ? cnt[((size_t)rr * (kFusedWaves + 1) + kFusedWaves) * k + c] : 0;
      }
#pragma unroll
      for (int u = 0; u < kScatterPrefix; ++u) {
        part_all += v[u];
        if (q + u * Q < r) part_before += v[u];
      }
    }
  } else if (j < k) {
    tot = nj[j];
    pre = rpre[(size_t)r * k + j];
  }
  // this range's per-wave counts
  int wcnt[kFusedWaves];
  const int* mine = cnt + (size_t)r * (kFusedWaves + 1) * k;
#pragma unroll
  for (int w = 0; w < kFusedWaves; ++w) wcnt[w] = j < k ? mine[(size_t)w * k + j] : 0;
  if (j < k) sDirty[j] = dirty ? dirty[j] : 1;
  const int64_t p0 = ((int64_t)r * kFusedWaves + wave) * SB;
  const int64_t p1 = p0 + SB < n ? p0 + SB : n;
  // with lab_lds the range's labels are staged in LDS here (their loads
  // overlap the loads above), so the walk below waits only on LDS
  int* sLab = run + kFusedWaves * k;
  if (lab_lds) {
    const int64_t r0 = (int64_t)r * kFusedWaves * SB;
    const int64_t rn = n - r0 < (int64_t)kFusedWaves * SB ? n - r0 : (int64_t)kFusedWaves * SB;
    stage_batched<4, int>(
        (int)(rn > 0 ? rn : 0), [&](int e) { return labels[r0 + e]; },
        [&](int e, int v) { sLab[e] = v; });
  }
  if (cv < iter) return;
  if (in_prefix) {
    sa[threadIdx.x] = part_all;
    sb[threadIdx.x] = part_before;
    __syncthreads();
    if (j < k)
      for (int q = 0; q < 1024 / k; ++q) {
        tot += sa[q * k + j];
        pre += sb[q * k + j];
      }
    if (r == 0 && j < k) nj[j] = tot;
    __syncthreads();
  }
  // exclusive prefix over clusters of the totals (members and leaves)
  const int lv = (tot + kLeaf - 1) / kLeaf;
  sa[threadIdx.x] = tot;
  sb[threadIdx.x] = lv;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    const int va = threadIdx.x >= s ? sa[threadIdx.x - s] : 0;
    const int vb = threadIdx.x >= s ? sb[threadIdx.x - s] : 0;
    __syncthreads();
    sa[threadIdx.x] += va;
    sb[threadIdx.x] += vb;
    __syncthreads();
  }
  const int off = sa[threadIdx.x] - tot;
  if (r == 0) {
    if (j < k) {
      off_out[j] = off;
      leaf_off_out[j] = sb[threadIdx.x] - lv;
    }
    if (threadIdx.x == 1023) {
      off_out[k] = sa[1023];
      leaf_off_out[k] = sb[1023];
    }
  }
  if (j < k) {
    int base = off + pre;
#pragma unroll
    for (int w = 0; w < kFusedWaves; ++w) {
      run[w * k + j] = base;
      base += wcnt[w];
    }
  }
  __syncthreads();
  // each wave walks its sub-range in chunks of 64 with its own table; the
  // labels of 16 chunks are loaded ahead so the walk only waits on LDS
  int* t = run + wave * k;
  const uint64_t lt = lanemask_lt();
  constexpr int kAhead = 16;
  for (int64_t c0 = p0; c0 < p1; c0 += 64 * kAhead) {
    int labs[kAhead];
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
      const int64_t p = c0 + q * 64 + lane;
      labs[q] = p < p1 ? (lab_lds ? sLab[p - (int64_t)r * kFusedWaves * SB] : labels[p]) : -1;
    }
#pragma unroll
    for (int q = 0; q < kAhead; ++q) {
      const int64_t p = c0 + q * 64 + lane;
      int lab = labs[q];
      const bool valid = p < p1 && (unsigned)lab < (unsigned)k;
      if (!valid) lab = 0;
      const uint64_t mask = same_label_mask(valid, lab, bits);
      const int rank = __popcll(mask & lt);
      const int cntl = __popcll(mask);
      int pos = 0;
      if (valid) pos = t[lab] + rank;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        if (sDirty[lab]) perm[pos] = (int)p;
        if (rank == cntl - 1) t[lab] = pos + 1;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// ---------------------------------------------------------------------------
// pass 1, large-k schedule: four kernels
// ---------------------------------------------------------------------------

// Per-block label histogram; blockcnt is block-major [b][j].  Labels outside
// [0, k) are ignored by every pass.
__global__ __launch_bounds__(256) void hist_kernel(const int32_t* __restrict__ labels,
                                                   int64_t n, int k, int B,
                                                   int* __restrict__ blockcnt,
                                                   const int* __restrict__ conv,
                                                   int iter) {
  extern __shared__ int sh[];
  SKIP_IF_CONVERGED
  const int b = blockIdx.x;
  for (int j = threadIdx.x; j < k; j += blockDim.x) sh[j] = 0;
  __syncthreads();
  int64_t p0 = (int64_t)b * B, p1 = p0 + B < n ? p0 + B : n;
  for (int64_t p = p0 + threadIdx.x; p < p1; p += blockDim.x) {
    unsigned lab = (unsigned)labels[p];
    if (lab < (unsigned)k) atomicAdd(&sh[lab], 1);   // LDS; order-free count
  }
  __syncthreads();
  int* row = blockcnt + (size_t)b * k;
  for (int j = threadIdx.x; j < k; j += blockDim.x) row[j] = sh[j];
}

// Column scan, phase A: per (segment of seglen blocks, cluster) sum.
__global__ __launch_bounds__(256) void colscan_a(const int* __restrict__ blockcnt,
                                                 int nb, int k, int seglen,
                                                 int* __restrict__ segsum,
                                                 const int* __restrict__ conv,
                                                 int iter) {
  SKIP_IF_CONVERGED
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int seg = blockIdx.y;
  if (j >= k) return;
  const int b0 = seg * seglen, b1 = b0 + seglen < nb ? b0 + seglen : nb;
  int s = 0;
  for (int b = b0; b < b1; ++b) s += blockcnt[(size_t)b * k + j];
  segsum[(size_t)seg * k + j] = s;
}

// Phase B: per cluster, exclusive scan over segments (in place) and the
// cluster total nj.  The last block to finish (a ticket taken after a device
// fence; nobody waits on it) runs the scans over clusters.
__global__ __launch_bounds__(1024) void colscan_b(int* __restrict__ segsum,
                                                  int nsegc, int k,
                                                  int* __restrict__ nj,
                                                  int* __restrict__ off,
                                                  int* __restrict__ leaf_off,
                                                  int* __restrict__ ticket,
                                                  const int* __restrict__ conv,
                                                  int iter) {
  __shared__ int sa[1024], sb[1024];
  __shared__ int last;
  SKIP_IF_CONVERGED
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < k) {
    // 64 segments' loads in flight before their stores (one memory round
    // trip per 64 segments, not per segment)
    constexpr int U = 64;
    int run = 0;
    for (int s0 = 0; s0 < nsegc; s0 += U) {
      int v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = s0 + u < nsegc ? segsum[(size_t)(s0 + u) * k + j] : 0;
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (s0 + u < nsegc) {
          segsum[(size_t)(s0 + u) * k + j] = run;
          run += v[u];
        }
    }
    nj[j] = run;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(ticket, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  cluster_scan_block(nj, k, off, leaf_off, sa, sb);
  if (threadIdx.x == 0) *ticket = 0;     // ready for the next iteration
}

// In-order scatter: one wave per block walks its points in chunks of 64,
// starting from off[j] + the segment prefix + the counts of the earlier
// blocks of its segment.  Members of clean clusters are ranked but not
// written (pass 2 skips them).
__global__ __launch_bounds__(64) void scatter_kernel(
    const int32_t* __restrict__ labels, int64_t n, int k, int B, int bits,
    int seglen, const int* __restrict__ blockcnt,
    const int* __restrict__ segsum, const int* __restrict__ off,
    const int* __restrict__ dirty, int* __restrict__ perm,
    const int* __restrict__ conv, int iter) {
  extern __shared__ int run[];
  SKIP_IF_CONVERGED
  const int b = blockIdx.x;
  const int lane = threadIdx.x;
  const int seg = b / seglen;
  const int* sp = segsum + (size_t)seg * k;
#pragma unroll 8
  for (int j = lane; j < k; j += 64) {
    int r = off[j] + sp[j];
    for (int bb = seg * seglen; bb < b; ++bb) r += blockcnt[(size_t)bb * k + j];
    run[j] = r;
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt();
  int64_t p0 = (int64_t)b * B, p1 = p0 + B < n ? p0 + B : n;
  // eight chunks of 64 labels (and their clusters' dirty flags) are loaded
  // before the first of them is placed: one memory round trip per eight
  // chunks instead of per chunk
  constexpr int U = 8;
  for (int64_t c0 = p0; c0 < p1; c0 += 64 * U) {
    int labv[U], dv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t p = c0 + 64 * u + lane;
      labv[u] = p < p1 ? labels[p] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      dv[u] = (!dirty || (unsigned)labv[u] >= (unsigned)k) ? 1 : dirty[labv[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t c = c0 + 64 * u;
      if (c >= p1) break;                       // uniform
      const int64_t p = c + lane;
      int lab = labv[u];
      bool valid = p < p1 && (unsigned)lab < (unsigned)k;
      if (!valid) lab = 0;
      const uint64_t mask = same_label_mask(valid, lab, bits);
      int rank = __popcll(mask & lt);
      int cnt = __popcll(mask);
      int pos = 0;
      if (valid) pos = run[lab] + rank;
      __builtin_amdgcn_wave_barrier();
      if (valid) {
        if (dv[u]) perm[pos] = (int)p;
        if (rank == cnt - 1) run[lab] = pos + 1;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
}

// ---------------------------------------------------------------------------
// pass 2: leaf sums, tree, finalize
// ---------------------------------------------------------------------------

// One wave per leaf.  Lane m loads member m's row (a chunk of DC dimensions
// at a time) into the wave's LDS tile, then lane i sums dimension i over the
// members in order (left to right, starting from the first member).  For
// k <= kLeafStageK the workgroup first stages the leaf offsets and the dirty
// flags (one bit per cluster) in LDS, so a wave finds its cluster by a
// binary search in LDS instead of a chain of dependent global reads.
constexpr int kLeafWaves = 4;
constexpr int kLeafStageK = 4096;

// k + 1 offsets, rounded up to an even count (8-byte alignment of the bits)
__host__ __device__ constexpr int leaf_stage_ints(int k) { return (k + 2) & ~1; }
static size_t leaf_stage_bytes(int k) {
  return k <= kLeafStageK
             ? sizeof(int) * (size_t)leaf_stage_ints(k) + sizeof(uint64_t) * (size_t)((k + 63) / 64)
             : 0;
}

template <typename T>
struct LeafCfg {
  static constexpr int DC = 128 / (int)sizeof(T);      // dims per chunk
  static constexpr int LD = DC + 16 / (int)sizeof(T);  // row stride: 16-byte
                                                       // rows, spread banks
};

template <typename T>
__global__ __launch_bounds__(64 * kLeafWaves) void leaf_kernel(
    const T* __restrict__ X, int d, const int* __restrict__ perm,
    const int* __restrict__ nj, const int* __restrict__ off,
    const int* __restrict__ leaf_off, int k, const int* __restrict__ dirty,
    double* __restrict__ leafsum, const int* __restrict__ conv, int iter, int vec) {
  constexpr int DC = LeafCfg<T>::DC, LD = LeafCfg<T>::LD;
  __shared__ __attribute__((aligned(16))) T tile[kLeafWaves][kLeaf * LD];
  // dynamic: leaf_stage_bytes(k) when k <= kLeafStageK
  extern __shared__ __attribute__((aligned(16))) int sLo[];
  uint64_t* sDm = reinterpret_cast<uint64_t*>(sLo + leaf_stage_ints(k));
  const int cv = *conv;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool staged = k <= kLeafStageK;
  if (staged) {
    // dirty bits: wave w packs the 64-cluster words w, w + 4, ...
    if (k < (int)blockDim.x) {
      if ((int)threadIdx.x <= k) sLo[threadIdx.x] = leaf_off[threadIdx.x];
      const int e = wave * 64 + lane;
      const uint64_t m = __ballot(e < k && (!dirty || dirty[e]));
      if (wave * 64 < k && lane == 0) sDm[wave] = m;
    } else {
      stage_batched<8, int>(
          k + 1, [&](int e) { return leaf_off[e]; }, [&](int e, int v) { sLo[e] = v; });
      constexpr int kB = 4;
      for (int e0 = wave * 64; e0 < k; e0 += kB * (int)blockDim.x) {
        int f[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int e = e0 + u * (int)blockDim.x + lane;
          f[u] = e < k ? (dirty ? dirty[e] : 1) : 0;
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int w0 = e0 + u * (int)blockDim.x;   // uniform over the wave
          const uint64_t m = __ballot(f[u] != 0);
          if (w0 < k && lane == 0) sDm[w0 >> 6] = m;
        }
      }
    }
  }
  if (cv < iter) return;
  if (staged) __syncthreads();
  const int* lo_tab = staged ? sLo : leaf_off;
  const int total = lo_tab[k];
  const int g = blockIdx.x * kLeafWaves + wave;
  if (g >= total) return;                    // per wave; no later block barrier
  const int j = cluster_of_leaf(lo_tab, k, g);
  if (staged ? !((sDm[j >> 6] >> (j & 63)) & 1) : (dirty && !dirty[j])) return;
  const int L = g - lo_tab[j];
  const int m0 = off[j] + L * kLeaf;
  int cnt = nj[j] - L * kLeaf;
  if (cnt > kLeaf) cnt = kLeaf;
  const int p = lane < cnt ? perm[m0 + lane] : 0;
  T* tl = tile[wave];
  for (int c0 = 0; c0 < d; c0 += DC) {
    const int dc = d - c0 < DC ? d - c0 : DC;
    if (lane < cnt) {
      const T* xr = X + (size_t)p * d + c0;
      if (vec) {                             // 16-byte pieces of the row
        const int nv = dc * (int)sizeof(T) / 16;
        const uint4* src = reinterpret_cast<const uint4*>(xr);
        uint4* dst = reinterpret_cast<uint4*>(tl + lane * LD);
        for (int v = 0; v < nv; ++v) dst[v] = src[v];
      } else {
        for (int i = 0; i < dc; ++i) tl[lane * LD + i] = xr[i];
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < dc) {
      double s = to_f64<T>(tl[lane]);
      for (int m = 1; m < cnt; ++m) s = __dadd_rn(s, to_f64<T>(tl[m * LD + lane]));
      leafsum[(size_t)g * d + c0 + lane] = s;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

constexpr int kTreeLdsDoubles = 6144;   // 48 KB: trees that fit run in LDS

// First stage of the pairwise tree.  In the bottom-up form (at stride s,
// node a with a % 2s == 0 absorbs node a + s when a + s < m) every level
// with 2s <= TB pairs leaves inside one aligned block of TB leaves, so the
// blocks reduce independently: workgroup (j, y) reduces blocks y, y + Y, ...
// of cluster j in LDS and leaves each block's sum at its first leaf.  The
// remaining levels run over the block sums in tree_finalize.
__global__ __launch_bounds__(256) void tree_block(
    double* __restrict__ leafsum, const int* __restrict__ leaf_off, int k,
    int d, int TB, const int* __restrict__ dirty, const int* __restrict__ conv,
    int iter) {
  __shared__ double node[kTreeBlockDoubles];
  const int cv = *conv;
  const int j = blockIdx.x;
  const int dj = dirty ? dirty[j] : 1;
  const int L0 = leaf_off[j], m = leaf_off[j + 1] - L0;
  if (cv < iter || !dj) return;
  const int mb = (m + TB - 1) / TB;
  for (int b = blockIdx.y; b < mb; b += gridDim.y) {
    const int cnt = m - b * TB < TB ? m - b * TB : TB;
    if (cnt <= 1) continue;                  // uniform over the workgroup
    double* base = leafsum + (size_t)(L0 + b * TB) * d;
    stage_batched<8, double>(
        cnt * d, [&](int e) { return base[e]; }, [&](int e, double v) { node[e] = v; });
    __syncthreads();
    for (int s = 1; s < cnt; s <<= 1) {
      const int pairs = (cnt - s - 1) / (2 * s) + 1;
      for (int e = threadIdx.x; e < pairs * d; e += blockDim.x) {
        const int i = e / d, dim = e - i * d;
        const int a = i * 2 * s;
        node[a * d + dim] = __dadd_rn(node[a * d + dim], node[(a + s) * d + dim]);
      }
      __syncthreads();
    }
    for (int dim = threadIdx.x; dim < d; dim += blockDim.x) base[dim] = node[dim];
    __syncthreads();
  }
}

// One workgroup per cluster: tree over its leaves, mean, operands, drift.
// Block 0 also closes the iteration: totals of the counters and the
// stopping rule (#changed <= tol * n).
__global__ __launch_bounds__(256) void tree_finalize(
    double* __restrict__ leafsum, const int* __restrict__ nj,
    const int* __restrict__ leaf_off, int k, int d, const double* C_prev,
    double* C_out, int64_t* __restrict__ counts_out, float* __restrict__ Cm2,
    float* __restrict__ cn, double* __restrict__ CT, int dp,
    uint16_t* __restrict__ Chi, uint16_t* __restrict__ Clo, int dpb,
    float* __restrict__ drift, int* __restrict__ dirty, int TB, IterCtl ctl,
    const int* __restrict__ conv, int iter) {
  __shared__ double tree[kTreeLdsDoubles];
  const int cv = *conv;
  const int j = blockIdx.x;
  const int cntj = nj[j];
  const int dj = dirty ? dirty[j] : 1;
  const int lo0 = leaf_off[j], lo1 = leaf_off[j + 1];
  if (cv < iter) return;

  if (j == 0 && ctl.row) close_iteration(ctl, iter);

  if (counts_out && threadIdx.x == 0) counts_out[j] = cntj;
  if (!dj) {
    if (drift && threadIdx.x == 0) drift[j] = 0.0f;     // centroid unchanged
    return;
  }
  // the block sums of tree_block sit at leaves 0, TB, 2 TB, ...: node b
  const int m = lo1 - lo0;
  const int mb = (m + TB - 1) / TB;
  double* base = leafsum + (size_t)lo0 * d;
  const size_t bstride = (size_t)TB * d;
  const bool in_lds = (size_t)mb * d <= (size_t)kTreeLdsDoubles;
  if (in_lds) {
    for (int e = threadIdx.x; e < mb * d; e += blockDim.x) {
      const int b = e / d, dim = e - b * d;
      tree[e] = base[(size_t)b * bstride + dim];
    }
    __syncthreads();
  }
  double* node = in_lds ? tree : base;
  const size_t nstride = in_lds ? (size_t)d : bstride;
  for (int s = 1; s < mb; s <<= 1) {
    const int pairs = (mb - s - 1) / (2 * s) + 1;
    for (int e = threadIdx.x; e < pairs * d; e += blockDim.x) {
      int i = e / d, dim = e - i * d;
      int a = i * 2 * s;
      node[(size_t)a * nstride + dim] =
          __dadd_rn(node[(size_t)a * nstride + dim], node[(size_t)(a + s) * nstride + dim]);
    }
    __syncthreads();
  }
  write_centroid(j, k, d, cntj, [&](int dim) { return __ddiv_rn(node[dim], (double)cntj); },
                 C_prev, C_out, CT, Cm2, cn, dp, Chi, Clo, dpb, drift, dirty);
}

hipError_t launch_sort(const UpdatePlan& p, const int32_t* labels, int* dirty,
                       const int* conv, int iter, hipStream_t s, int early) {
  const int k = p.k;
  int bits = 0;
  while ((1 << bits) < k) ++bits;
  if (fused_sort(k)) {
    const size_t lds = sizeof(int) * (size_t)kFusedWaves * k;
    auto hist = early ? hist_fused<true> : hist_fused<false>;
    auto rscan = early ? range_scan<true> : range_scan<false>;
    auto scat = early ? scatter_fused<true> : scatter_fused<false>;
    hipLaunchKernelGGL(hist, dim3(p.nb), dim3(1024), lds, s, labels, p.n,
                       k, p.B, p.blockcnt, conv, iter);
    const int in_prefix = scatter_prefix(p.nb, k) ? 1 : 0;
    if (!in_prefix)
      hipLaunchKernelGGL(rscan, dim3(k), dim3(256), 0, s, p.blockcnt, p.nb,
                         k, p.rpre, p.nj, conv, iter);
    // the range's labels in LDS next to the running tables, within 48 KB
    const int lab_lds = (size_t)kFusedWaves * (k + p.B) * sizeof(int) <= 49152 ? 1 : 0;
    const size_t lds_s = lds + (lab_lds ? sizeof(int) * (size_t)kFusedWaves * p.B : 0);
    hipLaunchKernelGGL(scat, dim3(p.nb), dim3(1024), lds_s, s, labels,
                       p.n, k, p.B, bits, p.blockcnt, p.rpre, p.nj, in_prefix,
                       lab_lds, dirty, p.perm, p.off, p.leaf_off, conv, iter);
  } else {
    const size_t lds_k = sizeof(int) * (size_t)k;
    hipLaunchKernelGGL(hist_kernel, dim3(p.nb), dim3(256), lds_k, s, labels,
                       p.n, k, p.B, p.blockcnt, conv, iter);
    hipLaunchKernelGGL(colscan_a, dim3((k + 255) / 256, p.nsegc), dim3(256), 0,
                       s, p.blockcnt, p.nb, k, p.seglen, p.segsum, conv, iter);
    hipLaunchKernelGGL(colscan_b, dim3((k + 1023) / 1024), dim3(1024), 0, s,
                       p.segsum, p.nsegc, k, p.nj, p.off, p.leaf_off, p.ticket,
                       conv, iter);
    hipLaunchKernelGGL(scatter_kernel, dim3(p.nb), dim3(64), lds_k, s, labels,
                       p.n, k, p.B, bits, p.seglen, p.blockcnt, p.segsum, p.off,
                       dirty, p.perm, conv, iter);
  }
  return hipGetLastError();
}

hipError_t launch_update(const UpdatePlan& p, const void* X, knor_dtype dt,
                         const int32_t* labels, const double* C_prev,
                         double* C_out, int64_t* counts_out, CentroidOps* ops,
                         float* drift, int* dirty, const IterCtl* ctl,
                         hipStream_t s, Prof* prof) {
  // ctl->conv must point at device memory (max int when no fit is running)
  const int k = p.k, d = p.d;
  const int* conv = ctl->conv;
  const int iter = ctl->iter;
  if (prof) prof->begin(KNOR_PROF_SORT);
  // clean clusters keep their member order (and their sums)
  if (hipError_t e = launch_sort(p, labels, dirty, conv, iter, s, 0)) return e;
  if (prof) { prof->end(); prof->begin(KNOR_PROF_LEAF); }
  const int64_t lblocks = (p.max_leaves + kLeafWaves - 1) / kLeafWaves;
  const size_t esz = dt == KNOR_F64 ? 8 : (dt == KNOR_F32 ? 4 : 2);
  const int vec = (int)(((size_t)d * esz) % 16 == 0 && ((uintptr_t)X & 15) == 0);
  switch (dt) {
    case KNOR_F64:
      hipLaunchKernelGGL(leaf_kernel<double>, dim3(lblocks), dim3(64 * kLeafWaves),
                         leaf_stage_bytes(k), s, (const double*)X, d, p.perm, p.nj, p.off,
                         p.leaf_off, k, dirty, p.leafsum, conv, iter, vec);
      break;
    case KNOR_F32:
      hipLaunchKernelGGL(leaf_kernel<float>, dim3(lblocks), dim3(64 * kLeafWaves),
                         leaf_stage_bytes(k), s, (const float*)X, d, p.perm, p.nj, p.off,
                         p.leaf_off, k, dirty, p.leafsum, conv, iter, vec);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(leaf_kernel<uint16_t>, dim3(lblocks), dim3(64 * kLeafWaves),
                         leaf_stage_bytes(k), s, (const uint16_t*)X, d, p.perm, p.nj, p.off,
                         p.leaf_off, k, dirty, p.leafsum, conv, iter, vec);
      break;
  }
  if (prof) { prof->end(); prof->begin(KNOR_PROF_TREE); }
  {
    // blocks per cluster for an even split: twice the mean, at most 256
    const int64_t blocks = (p.max_leaves + p.tb - 1) / p.tb;
    int64_t Y = 2 * ((blocks + k - 1) / k);
    Y = Y < 1 ? 1 : (Y > 256 ? 256 : Y);
    if (p.tb > 1)
      hipLaunchKernelGGL(tree_block, dim3(k, (unsigned)Y), dim3(256), 0, s,
                         p.leafsum, p.leaf_off, k, d, p.tb, dirty, conv, iter);
  }
  hipLaunchKernelGGL(tree_finalize, dim3(k), dim3(256), 0, s, p.leafsum, p.nj,
                     p.leaf_off, k, d, C_prev, C_out, counts_out,
                     ops ? ops->Cm2 : nullptr, ops ? ops->cn : nullptr,
                     ops ? ops->CT : nullptr, ops ? ops->dp : 0,
                     ops ? ops->Chi : nullptr, ops ? ops->Clo : nullptr,
                     ops ? ops->dpb : 0, drift, dirty, p.tb,
                     *ctl, conv, iter);
  if (prof) prof->end();
  return hipGetLastError();
}

}  // namespace knor
