// Assignment of the MTI survivors with the paper's Clause 2 applied at the
// granularity of a matrix-core tile (Mhembere et al., HPDC'17, Section
// "Minimal Triangle Inequality (MTI) Pruning", Clauses 2 and 3).
//
// Clause 2: a point x with current centroid a and upper bound u >= d(x, c_a)
// need not be compared with centroid j when u (1 + eta) < 1/2 d(c_a, c_j).
// Then d(x, c_j) >= d(c_a, c_j) - d(x, c_a) > u (1 + 2 eta) >= d(x, c_a)
// (1 + 2 eta): j is farther than a by a relative gap of 2 eta, far above the
// FP64 evaluation error of the canonical distance, so j is neither the FP64
// argmin nor tied with it.  Every centroid that can be the argmin is
// therefore in C(x) = {j : !(u (1 + eta) < h(a, j))}, h(a, j) any lower
// bound of 1/2 d(c_a, c_j); C(x) always holds a (h(a, a) = 0).
//
// The centroid-pair pass of the previous update leaves, for every centroid
// a, its neighbour row: all centroids in increasing order of a lower bound
// h(a, j) (a float key that also carries j), so C(x) is a prefix of a's row.
//
// The survivors still to assign (the segmented list; their bounds carry a
// set sign bit, Clause 3 having tightened them to the exact distance
// rounded up) are first grouped by cluster without global atomics: each
// grouping workgroup counts the survivors of its segments per cluster in
// LDS (one row of a count table), a column scan turns the rows into
// offsets, one workgroup scans the cluster totals and writes the task
// table, and each grouping workgroup then places its survivors from its own
// offsets with LDS cursors.  The order within a cluster is not fixed; it
// decides no label.  A task holds at most kTaskMembers survivors of one cluster;
// the sort pass sorts them by bound in LDS and cuts them into blocks of
// BLOCK in increasing bound: the members of a block share the prefix of
// a's row that the largest of their bounds needs.  Each block goes to a global list
// (long prefixes first) with its cluster, its sorted members and its
// prefix length.  The tile pass is persistent: each workgroup takes blocks
// from the list with an atomic counter, so the work of one cluster spreads
// over the whole GPU instead of serialising in one workgroup.
//
// For each block the FP32 tile runs over the gathered candidate rows,
// keeping each point's smallest values and the index of the smallest; a
// point is decided by the dense tile's rounding-bound test (its R^2 taken
// over the candidates, the only centroids whose values it compares).  The
// order in which candidates are visited decides no label: a decided point
// has a strict gap to every other value, and every other point is resolved
// from canonical FP64 distances with the lowest-index rule over the block's
// whole candidate list, which contains the FP64 argmin and every centroid
// tied with it.
#include <math.h>

#include <atomic>

#include "tile_f32.h"

namespace knor {

constexpr int kTaskMembers = 2048;  // members per task (all may survive)
constexpr int kCandBlockMax = 128;  // survivors per candidate prefix, at most
constexpr int kSlotBits = 11;       // survivor slot in a sort key
// the largest finite float on the grid of rounded bounds; a bound that
// rounds up to it or beyond is taken as unbounded (every centroid competes)
constexpr uint32_t kTopKey = 0x7f7ff800u;
static_assert((1 << kSlotBits) == kTaskMembers, "slot field holds a task's members");


// Survivors per candidate prefix: 4 waves of PB blocks of 16 points; two
// blocks per wave (two independent MFMA chains) where the rows are narrow
// enough for the registers, one otherwise.
template <int DP>
struct CandTile {
  static constexpr int PB = DP <= 64 ? 2 : 1;
  static constexpr int BLOCK = 64 * PB;
  using T = F32Tile<DP, PB>;
  static constexpr int CK = (4096 / DP) < 16 ? 16 : ((4096 / DP) > 128 ? 128 : (4096 / DP));
  static constexpr int Q = T::KS;                           // 16-byte pieces per row
  static constexpr int PER = (CK * Q + kTileThreads - 1) / kTileThreads;
};

// Workspace: a header of ints (task count, long and short block counts,
// the block counter of the tile pass), the task table, the block list
// (long blocks from the front, short ones from the back), the members of
// every task in bound order, and the grouping: survivors per cluster,
// cluster offsets, the count table (one row of k per grouping workgroup)
// and the survivors by cluster.
constexpr int kHdrTasks = 0, kHdrLong = 1, kHdrShort = 2, kHdrNext = 3;
// a block whose prefix is at least this long goes to the front of the list
constexpr int kLongPrefix = 512;
// grouping: workgroups (rows of the count table), their threads, the
// entries of a segment per thread, segments in flight per workgroup
constexpr int kGroupBlocks = 256;
constexpr int kGroupThreads = 1024;
constexpr int kGroupPer = kSeg / kGroupThreads;
constexpr int kGroupSegs = 2;

struct CandWs {
  int* hdr;
  int2* tasks;
  int4* blocks;
  int* sorted;
  int* gcnt;   // k
  int* goff;   // k + 1
  int* table;  // kGroupBlocks x k
  int* gperm;  // n
  int cap;     // block list entries
};

static int64_t cand_task_cap(int64_t n, int k) { return n / kTaskMembers + k + 1; }
static int64_t cand_block_cap(int64_t n, int k) { return n / 64 + cand_task_cap(n, k) + 1; }
static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

static CandWs cand_ws(void* ws, int64_t n, int k) {
  CandWs w;
  char* c = (char*)ws;
  w.hdr = (int*)c;
  c += 256;
  w.tasks = (int2*)c;
  c += al256(sizeof(int2) * (size_t)cand_task_cap(n, k));
  w.blocks = (int4*)c;
  w.cap = (int)cand_block_cap(n, k);
  c += al256(sizeof(int4) * (size_t)w.cap);
  w.sorted = (int*)c;
  c += al256(sizeof(int) * (size_t)n);
  w.gcnt = (int*)c;
  c += al256(sizeof(int) * (size_t)k);
  w.goff = (int*)c;
  c += al256(sizeof(int) * (size_t)(k + 1));
  w.table = (int*)c;
  c += al256(sizeof(int) * (size_t)kGroupBlocks * k);
  w.gperm = (int*)c;
  return w;
}

size_t cand_workspace_bytes(int64_t n, int k) {
  return 256 + al256(sizeof(int2) * (size_t)cand_task_cap(n, k)) +
         al256(sizeof(int4) * (size_t)cand_block_cap(n, k)) + al256(sizeof(int) * (size_t)n) +
         al256(sizeof(int) * (size_t)k) + al256(sizeof(int) * (size_t)(k + 1)) +
         al256(sizeof(int) * (size_t)kGroupBlocks * k) + sizeof(int) * (size_t)n;
}

// Grouping, count and scatter passes.  Workgroup g visits the segments b =
// g, g + G, ... (G = gridDim.x, the same in both passes) of the list,
// kGroupSegs of them at a time (all list loads, then all label loads, then
// LDS atomics).  SCATTER = false counts the survivors of each cluster in LDS
// and writes the counts as row g of the table; true starts a cursor per
// cluster at its offset plus row g's exclusive prefix (written by the
// column scan) and puts each survivor in the next slot of its cluster.
template <bool SCATTER>
__global__ __launch_bounds__(kGroupThreads) void cand_group_kernel(
    const int* __restrict__ list, const int* __restrict__ seg_cnt, int nseg,
    const int32_t* __restrict__ labels, int k, int* __restrict__ table,
    const int* __restrict__ goff, int* __restrict__ gperm, const int* __restrict__ conv,
    int iter) {
  extern __shared__ int sH[];                                    // k
  if (*conv < iter) return;                                      // uniform
  int* trow = table + (size_t)blockIdx.x * k;
  for (int a = threadIdx.x; a < k; a += kGroupThreads) sH[a] = SCATTER ? goff[a] + trow[a] : 0;
  __syncthreads();
  const int G = (int)gridDim.x;
  for (int b0 = blockIdx.x; b0 < nseg; b0 += G * kGroupSegs) {
    int cnt[kGroupSegs];
#pragma unroll
    for (int q = 0; q < kGroupSegs; ++q) {
      const int b = b0 + q * G;
      cnt[q] = b < nseg ? seg_cnt[b] : 0;
    }
    int p[kGroupSegs * kGroupPer], a[kGroupSegs * kGroupPer];
#pragma unroll
    for (int q = 0; q < kGroupSegs; ++q)
#pragma unroll
      for (int e = 0; e < kGroupPer; ++e) {
        const int i = (int)threadIdx.x + e * kGroupThreads;
        p[q * kGroupPer + e] = i < cnt[q] ? list[(size_t)(b0 + q * G) * kSeg + i] : -1;
      }
#pragma unroll
    for (int e = 0; e < kGroupSegs * kGroupPer; ++e) a[e] = p[e] >= 0 ? labels[p[e]] : 0;
#pragma unroll
    for (int e = 0; e < kGroupSegs * kGroupPer; ++e) {
      if (p[e] < 0) continue;
      if (SCATTER)
        gperm[atomicAdd(&sH[a[e]], 1)] = p[e];
      else
        atomicAdd(&sH[a[e]], 1);
    }
  }
  if (!SCATTER) {
    __syncthreads();
    for (int a = threadIdx.x; a < k; a += kGroupThreads) trow[a] = sH[a];
  }
}

// Column scan of the count table: for each cluster (one thread), the
// exclusive prefix over the rows replaces each count, and the total is the
// cluster's survivor count.
constexpr int kScanRows = 64;   // table loads in flight per thread
__global__ __launch_bounds__(256) void cand_colscan_kernel(int* __restrict__ table, int rows,
                                                           int k, int* __restrict__ gcnt,
                                                           const int* __restrict__ conv,
                                                           int iter) {
  if (*conv < iter) return;
  const int a = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (a >= k) return;
  int run = 0;
  for (int r0 = 0; r0 < rows; r0 += kScanRows) {
    int v[kScanRows];
#pragma unroll
    for (int e = 0; e < kScanRows; ++e)
      v[e] = r0 + e < rows ? table[(size_t)(r0 + e) * k + a] : 0;
#pragma unroll
    for (int e = 0; e < kScanRows; ++e)
      if (r0 + e < rows) {
        table[(size_t)(r0 + e) * k + a] = run;
        run += v[e];
      }
  }
  gcnt[a] = run;
}

// Offsets and task table, one workgroup of 1024 threads: exclusive scans of
// the per-cluster survivor and task counts, then each thread writes the
// offsets and tasks of its clusters.  Task c of cluster a covers its
// survivors [c kTaskMembers, ...), c < ceil(n_a / kTaskMembers); tasks are
// numbered cluster by cluster.  It also clears the block counts and the
// block counter of this iteration.
__global__ __launch_bounds__(1024) void cand_tasks_kernel(int k, CandWs ws,
                                                          const int* __restrict__ conv,
                                                          int iter) {
  __shared__ int part[1024], tpart[1024];
  if (*conv < iter) return;
  const int per = (k + 1023) / 1024;
  const int a0 = threadIdx.x * per;
  int mem = 0, loc = 0;
  for (int a = a0; a < a0 + per && a < k; ++a) {
    const int c = ws.gcnt[a];
    mem += c;
    loc += (c + kTaskMembers - 1) / kTaskMembers;
  }
  part[threadIdx.x] = mem;
  tpart[threadIdx.x] = loc;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    const int m = threadIdx.x >= (unsigned)s ? part[threadIdx.x - s] : 0;
    const int t = threadIdx.x >= (unsigned)s ? tpart[threadIdx.x - s] : 0;
    __syncthreads();
    part[threadIdx.x] += m;
    tpart[threadIdx.x] += t;
    __syncthreads();
  }
  int m = part[threadIdx.x] - mem;
  int t = tpart[threadIdx.x] - loc;
  for (int a = a0; a < a0 + per && a < k; ++a) {
    const int c = ws.gcnt[a];
    ws.goff[a] = m;
    m += c;
    const int nt = (c + kTaskMembers - 1) / kTaskMembers;
    for (int q = 0; q < nt; ++q) ws.tasks[t++] = make_int2(a, q);
  }
  if (threadIdx.x == 1023) {
    ws.goff[k] = part[1023];
    ws.hdr[kHdrTasks] = tpart[1023];
  }
  if (threadIdx.x < 3) ws.hdr[kHdrLong + threadIdx.x] = 0;
}

// The sort pass: one workgroup per task.  The task's survivors are
// written to sorted[m0 + i] in increasing rounded bound, and each block of
// BLOCK of them becomes one record (a, first member slot, count, prefix
// length L) of the block list.
template <int BLOCK>
__global__ __launch_bounds__(kTileThreads) void cand_sort_kernel(
    int k, const float* __restrict__ rows, int ib, const float* __restrict__ u, CandWs ws,
    const int* __restrict__ conv, int iter) {
  const int* __restrict__ perm = ws.gperm;
  const int* __restrict__ off = ws.goff;
  extern __shared__ __attribute__((aligned(16))) float sRow[];   // a's neighbour row
  __shared__ int sP[kTaskMembers];
  __shared__ float sKey[kTaskMembers];
  __shared__ int sCnt;
  if (*conv < iter || (int)blockIdx.x >= ws.hdr[kHdrTasks]) return;     // uniform
  const int2 tk = ws.tasks[blockIdx.x];
  const int a = tk.x;
  const int m0 = off[a] + tk.y * kTaskMembers;
  const int m1 = off[a + 1] < m0 + kTaskMembers ? off[a + 1] : m0 + kTaskMembers;
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  const uint32_t mask = (1u << ib) - 1u;
  if (threadIdx.x == 0) sCnt = 0;
  // a's neighbour row into LDS (its loads overlap the member walk below)
  stage_batched<8, float>(
      k, [&](int e) { return rows[(size_t)a * k + e]; }, [&](int e, float v) { sRow[e] = v; });
  __syncthreads();
  // the task's survivors (a set sign bit, checked again): all indices
  // first, then all their bounds (two memory round trips)
  {
    constexpr int E = kTaskMembers / kTileThreads;
    int p[E];
    float uu[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = m0 + (int)threadIdx.x + e * kTileThreads;
      p[e] = i < m1 ? perm[i] : 0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = m0 + (int)threadIdx.x + e * kTileThreads;
      uu[e] = i < m1 ? u[p[e]] : 0.0f;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = m0 + (int)threadIdx.x + e * kTileThreads;
      const bool surv = i < m1 && (__float_as_uint(uu[e]) >> 31) != 0u;
      const uint64_t m = __ballot(surv);
      if (m) {
        const int leader = __ffsll((unsigned long long)m) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&sCnt, __popcll(m));   // LDS
        base = __shfl(base, leader);
        if (surv) {
          const int slot = base + __popcll(m & lt);
          sP[slot] = p[e];
          // the bound rounded up to 12 significant bits, then the slot
          const uint32_t ub = __float_as_uint(-uu[e]);
          uint32_t up = (ub + ((1u << kSlotBits) - 1u)) & ~((1u << kSlotBits) - 1u);
          if (up > kTopKey) up = kTopKey;           // stands for "unbounded"
          sKey[slot] = __uint_as_float(up | (uint32_t)slot);
        }
      }
    }
  }
  __syncthreads();
  const int nS = sCnt;
  if (nS == 0) return;                                        // uniform
  // sort the survivors by rounded bound (bitonic, padded with +inf)
  int N2 = 1;
  while (N2 < nS) N2 <<= 1;
  for (int i = nS + (int)threadIdx.x; i < N2; i += kTileThreads) sKey[i] = INFINITY;
  __syncthreads();
  for (int size = 2; size <= N2; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < (N2 >> 1); i += kTileThreads) {
        // stride is a power of two: (i / stride) 2 stride + i mod stride
        const int lo = 2 * i - (i & (stride - 1)), hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const float x = sKey[lo], y = sKey[hi];
        if ((x > y) == asc) { sKey[lo] = y; sKey[hi] = x; }
      }
      __syncthreads();
    }
  const uint32_t smask = (1u << kSlotBits) - 1u;
  for (int i = threadIdx.x; i < nS; i += kTileThreads)
    ws.sorted[m0 + i] = sP[__float_as_uint(sKey[i]) & smask];
  // one record per block: the prefix of a's row that its largest bound
  // (rounded up) needs, the number of entries whose lower bound h passes
  // !(thr < h)
  const int nb = (nS + BLOCK - 1) / BLOCK;
  for (int bl = threadIdx.x; bl < nb; bl += kTileThreads) {
    const int b0 = bl * BLOCK;
    const int last = b0 + BLOCK - 1 < nS ? b0 + BLOCK - 1 : nS - 1;
    const uint32_t tb = __float_as_uint(sKey[last]) & ~smask;
    const double thr = tb >= kTopKey ? (double)INFINITY
                                     : (double)__uint_as_float(tb) * (1.0 + kEta);
    int lo = 0, hi = k;                         // first entry with h > thr
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const double h = (double)__uint_as_float(__float_as_uint(sRow[mid]) & ~mask);
      if (thr < h) hi = mid; else lo = mid + 1;
    }
    // lo >= 1: a itself has h = 0
    const int cnt = nS - b0 < BLOCK ? nS - b0 : BLOCK;
    const int pos = lo >= kLongPrefix ? atomicAdd(&ws.hdr[kHdrLong], 1)
                                      : ws.cap - 1 - atomicAdd(&ws.hdr[kHdrShort], 1);
    ws.blocks[pos] = make_int4(a, m0 + b0, cnt, lo);
  }
}

// The tile pass: a persistent grid; each workgroup takes the next block of
// the list (long ones first) until the list is exhausted.  Rows up to 32
// wide fit three waves per SIMD in the register file (the LDS holds four
// workgroups), which hides more of each block's load latency.
template <int DP>
__global__ __launch_bounds__(kTileThreads)
__attribute__((amdgpu_waves_per_eu(DP <= 32 ? 3 : 1))) void tile_f32_cand_kernel(
    const float* __restrict__ X, int d, const float* __restrict__ Cm2,
    const float* __restrict__ cn, const double* __restrict__ C64, int k,
    const float* __restrict__ rows, int ib, CandWs ws, float* __restrict__ u,
    int32_t* __restrict__ labels, int* __restrict__ dirty, unsigned long long* __restrict__ row,
    const int* __restrict__ conv, int iter, int vec, int vec4) {
  using G = CandTile<DP>;
  using T = typename G::T;
  constexpr int LDA = T::LDA, CK = G::CK, KS = T::KS, Q = G::Q, PB = G::PB, BLOCK = G::BLOCK;
  static_assert(BLOCK <= kCandBlockMax, "flag slots");
  extern __shared__ __attribute__((aligned(16))) float sRow[];   // the block's prefix
  __shared__ __attribute__((aligned(16))) float sC[CK * LDA];
  __shared__ __attribute__((aligned(16))) float sN[CK];
  __shared__ int sFl[kCandBlockMax];
  __shared__ int sFlN, sBlk;
  __shared__ float sWmax[kTileThreads / 64];   // per wave: largest candidate norm
  if (*conv < iter) return;                                   // uniform
  const int nlong = ws.hdr[kHdrLong];
  const int nblk = nlong + ws.hdr[kHdrShort];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const uint32_t mask = (1u << ib) - 1u;
  if (threadIdx.x == 0) sFlN = 0;
  unsigned long long chg = 0, nflag = 0, ndist = 0;
  auto cand_in = [&](int pos, int Lb) {
    return pos < Lb ? (int)(__float_as_uint(sRow[pos]) & mask) : -1;
  };
  // candidate rows, CK at a time: a chunk's loads are issued before the
  // previous chunk's matrix work
  float4 pre[G::PER];
  float pn = INFINITY;
  float tmax = 0.0f;
  auto load_chunk = [&](int c0, int Lb) {
    const int Lp = (Lb + 15) / 16 * 16;
    const int cc = (Lp - c0) < CK ? (Lp - c0) : CK;
#pragma unroll
    for (int i = 0; i < G::PER; ++i) {
      const int e = threadIdx.x + i * kTileThreads;
      const int r = e / Q, q4 = e - r * Q;
      const int j = (e < cc * Q) ? cand_in(c0 + r, Lb) : -1;
      pre[i] = j >= 0 ? *reinterpret_cast<const float4*>(Cm2 + (size_t)j * DP + q4 * 4)
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int jn = (int)threadIdx.x < cc ? cand_in(c0 + threadIdx.x, Lb) : -1;
    pn = jn >= 0 ? cn[jn] : INFINITY;
  };
  auto store_chunk = [&](int c0, int Lb) {
    const int Lp = (Lb + 15) / 16 * 16;
    const int cc = (Lp - c0) < CK ? (Lp - c0) : CK;
#pragma unroll
    for (int i = 0; i < G::PER; ++i) {
      const int e = threadIdx.x + i * kTileThreads;
      const int r = e / Q, q4 = e - r * Q;
      if (e < cc * Q) *reinterpret_cast<float4*>(&sC[r * LDA + q4 * 4]) = pre[i];
    }
    if ((int)threadIdx.x < cc) {
      sN[threadIdx.x] = pn;
      // the rounding bound takes the largest norm over the block's
      // candidates: each thread keeps the largest it stored, reduced once
      // per block after the sweep
      if (pn < INFINITY) tmax = fmax_nc(tmax, pn);
    }
  };
  for (;;) {
    if (threadIdx.x == 0) sBlk = atomicAdd(&ws.hdr[kHdrNext], 1);
    __syncthreads();                          // also: the previous block is done
    const int bi = sBlk;
    if (bi >= nblk) break;                    // uniform
    const int4 rec = ws.blocks[bi < nlong ? bi : ws.cap - 1 - (bi - nlong)];
    const int a = rec.x, s0 = rec.y, nv = rec.z, L = rec.w;
    const int Lpad = (L + 15) / 16 * 16;
    auto cand_of = [&](int pos) { return cand_in(pos, L); };
    // the wave's 16 PB points and their rows; a's row prefix into LDS
    WaveState<T> w;
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      const int q = wave * 16 * PB + pb * 16 + col;
      w.valid[pb] = q < nv;
      w.pid[pb] = w.valid[pb] ? ws.sorted[s0 + q] : 0;
      w.old[pb] = a;
    }
    stage_batched<8, float>(
        L, [&](int e) { return rows[(size_t)a * k + e]; }, [&](int e, float v) { sRow[e] = v; });
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      T::load_row(w.bx[pb], X, w.pid[pb], d, grp, vec, w.valid[pb]);
      double acc = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < KS; ++s2) {
        const double v = (double)w.bx[pb][s2];
        acc = acc + v * v;
      }
      w.xs[pb] = acc;
      top3_reset(w.b1[pb], w.b2[pb], w.b3[pb], w.i1[pb], w.i2[pb]);
    }
    __syncthreads();                          // the prefix is staged
    load_chunk(0, L);
    tmax = 0.0f;
    for (int c0 = 0; c0 < Lpad; c0 += CK) {
      const int cc = (Lpad - c0) < CK ? (Lpad - c0) : CK;
      __syncthreads();                        // the previous chunk is consumed
      store_chunk(c0, L);
      __syncthreads();
      if (c0 + CK < Lpad) load_chunk(c0 + CK, L);
      tile_sweep<T, false, true>(w, sC, sN, cc, c0, col, grp);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) tmax = fmax_nc(tmax, __shfl_xor(tmax, o));
    if (lane == 0) sWmax[wave] = tmax;
    __syncthreads();
    float cmax = sWmax[0];
#pragma unroll
    for (int v = 1; v < kTileThreads / 64; ++v) cmax = fmax_nc(cmax, sWmax[v]);
    // one index kept per point: a two-candidate point is recomputed in FP64
    // with the undecided ones
    merge_groups<T, false>(w);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) w.i1[pb] = cand_of(w.i1[pb]);
    bool flag, changed;
    int fp;
    finalize_points<T, false>(w, cmax, d, grp, 0, false, nullptr, nullptr, labels, u, dirty,
                              flag, fp, changed);
    chg += changed ? 1 : 0;
    if (flag) sFl[atomicAdd(&sFlN, 1)] = fp;   // at most one per point of the block
    __syncthreads();
    const int nfl = sFlN;
    // near-tie points: canonical FP64 distances to every candidate, one
    // wave per point, lowest index among equal distances
    for (int f = wave; f < nfl; f += 4) {
      const int p = sFl[f];
      double best = INFINITY;
      int bj = 0x7fffffff;
      for (int q = lane; q < L; q += 64) {
        const int j = cand_of(q);
        const double D = vec4 ? dist2_canon_f32x4(X + (size_t)p * d, C64 + (size_t)j * d, d)
                              : dist2_canon<float>(X + (size_t)p * d, C64 + (size_t)j * d, d);
        if (D < best || (D == best && j < bj)) { best = D; bj = j; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o);
        const int oj = __shfl_xor(bj, o);
        if (ob < best || (ob == best && oj < bj)) { best = ob; bj = oj; }
      }
      if (lane == 0)
        chg += commit_label(p, a, bj, pair_bound(best, d), labels, u, dirty) ? 1 : 0;
    }
    if (threadIdx.x == 0) {
      ndist += (unsigned long long)(nv + nfl) * (unsigned long long)L;
      nflag += (unsigned long long)nfl;
    }
    __syncthreads();
    if (threadIdx.x == 0) sFlN = 0;
  }
  const int qs[3] = {SLOT_CHANGED, SLOT_FLAGGED, SLOT_DISTS};
  const unsigned long long v[3] = {chg, nflag, ndist};
  block_add_slots<3>(row, qs, v);
}

// Workgroups of the persistent tile pass: as many as are resident at once.
template <int DP>
static int cand_grid(size_t lds) {
  static std::atomic<int> cached{0};
  const int c = cached.load(std::memory_order_relaxed);
  if (c) return c;
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per, reinterpret_cast<const void*>(&tile_f32_cand_kernel<DP>), kTileThreads,
          lds) != hipSuccess ||
      cus <= 0 || per <= 0)
    return 1024;
  cached.store(cus * per, std::memory_order_relaxed);
  return cus * per;
}

template <int DP>
static hipError_t launch_cand_dp(const CentroidOps& o, const AssignJob& j, const float* rows,
                                 void* ws_, hipStream_t s) {
  const int vec = (int)(j.d == DP && ((uintptr_t)j.X & 15) == 0);
  const int vec4 = (int)(j.d % 4 == 0 && ((uintptr_t)j.X & 15) == 0 &&
                         ((uintptr_t)o.C64 & 15) == 0);
  const size_t lds = sizeof(float) * (size_t)o.k;
  // with the static arrays the totals can pass the default 64 KB
  hipError_t e = hipFuncSetAttribute(
      reinterpret_cast<const void*>(&tile_f32_cand_kernel<DP>),
      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&cand_sort_kernel<CandTile<DP>::BLOCK>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const CandWs ws = cand_ws(ws_, j.n, o.k);
  const int ib = cc_rows_bits(o.k);
  // the count and scatter passes take the same segments per workgroup
  const int gg = j.nseg < kGroupBlocks ? (j.nseg > 0 ? j.nseg : 1) : kGroupBlocks;
  const size_t glds = sizeof(int) * (size_t)o.k;
  hipLaunchKernelGGL(cand_group_kernel<false>, dim3(gg), dim3(kGroupThreads), glds, s, j.list,
                     j.seg_cnt, j.nseg, (const int32_t*)j.labels, o.k, ws.table, ws.goff,
                     ws.gperm, j.conv, j.iter);
  hipLaunchKernelGGL(cand_colscan_kernel, dim3((o.k + 255) / 256), dim3(256), 0, s, ws.table,
                     gg, o.k, ws.gcnt, j.conv, j.iter);
  hipLaunchKernelGGL(cand_tasks_kernel, dim3(1), dim3(1024), 0, s, o.k, ws, j.conv, j.iter);
  hipLaunchKernelGGL(cand_group_kernel<true>, dim3(gg), dim3(kGroupThreads), glds, s, j.list,
                     j.seg_cnt, j.nseg, (const int32_t*)j.labels, o.k, ws.table, ws.goff,
                     ws.gperm, j.conv, j.iter);
  const int64_t tgrid = cand_task_cap(j.n, o.k);           // >= the number of tasks
  hipLaunchKernelGGL((cand_sort_kernel<CandTile<DP>::BLOCK>), dim3((unsigned)tgrid),
                     dim3(kTileThreads), lds, s, o.k, rows, ib, (const float*)j.u, ws, j.conv,
                     j.iter);
  hipLaunchKernelGGL((tile_f32_cand_kernel<DP>), dim3((unsigned)cand_grid<DP>(lds)),
                     dim3(kTileThreads), lds, s, (const float*)j.X, j.d, o.Cm2, o.cn, o.C64,
                     o.k, rows, ib, ws, j.u, j.labels, j.dirty, j.row, j.conv, j.iter, vec,
                     vec4);
  return hipGetLastError();
}

hipError_t launch_tile_cand(const CentroidOps& o, const AssignJob& j, const float* rows,
                            void* ws, hipStream_t s) {
  if (j.dt != KNOR_F32 || o.k > kCandMaxK || !j.list) return hipErrorInvalidValue;
  switch (o.dp) {
    case 8: return launch_cand_dp<8>(o, j, rows, ws, s);
    case 16: return launch_cand_dp<16>(o, j, rows, ws, s);
    case 32: return launch_cand_dp<32>(o, j, rows, ws, s);
    case 64: return launch_cand_dp<64>(o, j, rows, ws, s);
    case 128: return launch_cand_dp<128>(o, j, rows, ws, s);
    case 256: return launch_cand_dp<256>(o, j, rows, ws, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace knor
