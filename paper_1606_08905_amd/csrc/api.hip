// C ABI of the k-means library: argument validation, stream-ordered device
// workspace, and the Lloyd iteration driver (Mhembere et al., HPDC'17,
// Sections "Parallel Lloyd's Algorithm" and "Minimal Triangle Inequality
// (MTI) Pruning").  Every arithmetic step runs in the kernels of this
// library; the host only validates, allocates, enqueues and polls.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <map>
#include <memory>
#include <math.h>
#include <mutex>
#include <string.h>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.h"

namespace knor {

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

// Non-finite test on the bit pattern (exponent all ones).
template <typename T>
__device__ __forceinline__ bool nonfinite_bits(T v);
template <>
__device__ __forceinline__ bool nonfinite_bits<double>(double v) {
  return ((unsigned long long)__double_as_longlong(v) & 0x7ff0000000000000ull) ==
         0x7ff0000000000000ull;
}
template <>
__device__ __forceinline__ bool nonfinite_bits<float>(float v) {
  return (__float_as_uint(v) & 0x7f800000u) == 0x7f800000u;
}
template <>
__device__ __forceinline__ bool nonfinite_bits<uint16_t>(uint16_t v) {
  return (v & 0x7f80u) == 0x7f80u;
}

// bad |= some element of p[0, count) is NaN or Inf; with kill, a hit also
// sets *kill = -1 (the convergence word: every later kernel of the fit then
// returns at once).  16-byte loads, four in flight per thread, when p is
// aligned.
template <typename T>
__global__ __launch_bounds__(256) void check_finite_kernel(const T* __restrict__ p,
                                                           int64_t count,
                                                           int* __restrict__ bad,
                                                           int* __restrict__ kill) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool b = false;
  int64_t done = 0;
  if (((uintptr_t)p & 15) == 0) {
    constexpr int E = 16 / (int)sizeof(T);
    const int64_t nv = count / E;
    const uint4* q = reinterpret_cast<const uint4*>(p);
    for (int64_t i = tid; i < nv; i += 4 * stride) {
      uint4 w[4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
        w[r] = i + r * stride < nv ? q[i + r * stride] : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const T* e = reinterpret_cast<const T*>(&w[r]);
#pragma unroll
        for (int j = 0; j < E; ++j) b |= nonfinite_bits<T>(e[j]);
      }
    }
    done = nv * E;
  }
  for (int64_t i = done + tid; i < count; i += stride) b |= nonfinite_bits<T>(p[i]);
  if (__ballot(b) && lane_id() == 0) {
    atomicOr(bad, 1);
    if (kill) atomicExch(kill, -1);
  }
}

hipError_t launch_check_finite(const void* p, knor_dtype dt, int64_t count,
                               int* bad, hipStream_t s, int* kill) {
  int64_t blocks = (count + 1023) / 1024;
  int grid = (int)(blocks < 1024 ? (blocks < 1 ? 1 : blocks) : 1024);
  switch (dt) {
    case KNOR_F64:
      hipLaunchKernelGGL(check_finite_kernel<double>, dim3(grid), dim3(256), 0,
                         s, (const double*)p, count, bad, kill);
      break;
    case KNOR_F32:
      hipLaunchKernelGGL(check_finite_kernel<float>, dim3(grid), dim3(256), 0,
                         s, (const float*)p, count, bad, kill);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(check_finite_kernel<uint16_t>, dim3(grid), dim3(256), 0,
                         s, (const uint16_t*)p, count, bad, kill);
      break;
  }
  return hipGetLastError();
}

__global__ void fill_i32_kernel(int32_t* p, int64_t count, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((count + 255) / 256), dim3(256), 0,
                     s, p, count, v);
  return hipGetLastError();
}

__global__ void copy_i32_kernel(const int32_t* __restrict__ a,
                                int32_t* __restrict__ b, int64_t count,
                                const int* conv, int iter) {
  if (*conv < iter) return;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) b[i] = a[i];
}

hipError_t launch_copy_i32(const int32_t* a, int32_t* b, int64_t count,
                           const int* conv, int iter, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(copy_i32_kernel, dim3((count + 255) / 256), dim3(256), 0,
                     s, a, b, count, conv, iter);
  return hipGetLastError();
}

__global__ void gather_i32_kernel(const int32_t* __restrict__ a,
                                  const int* __restrict__ rows, int64_t count,
                                  int32_t* __restrict__ out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = a[rows[i]];
}

static hipError_t launch_gather_i32(const int32_t* a, const int* rows, int64_t count,
                                    int32_t* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(gather_i32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, a,
                     rows, count, out);
  return hipGetLastError();
}

template <typename T>
__global__ void gather_rows_kernel(const T* __restrict__ X, int d,
                                   const int64_t* __restrict__ rows, int k,
                                   double* __restrict__ C) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * d) return;
  int j = (int)(e / d), i = (int)(e - (int64_t)j * d);
  C[e] = to_f64<T>(X[(size_t)rows[j] * d + i]);
}

hipError_t launch_gather_rows(const void* X, knor_dtype dt, int d,
                              const int64_t* rows, int k, double* C,
                              hipStream_t s) {
  int64_t tot = (int64_t)k * d;
  dim3 g((tot + 255) / 256);
  switch (dt) {
    case KNOR_F64:
      hipLaunchKernelGGL(gather_rows_kernel<double>, g, dim3(256), 0, s,
                         (const double*)X, d, rows, k, C);
      break;
    case KNOR_F32:
      hipLaunchKernelGGL(gather_rows_kernel<float>, g, dim3(256), 0, s,
                         (const float*)X, d, rows, k, C);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(gather_rows_kernel<uint16_t>, g, dim3(256), 0, s,
                         (const uint16_t*)X, d, rows, k, C);
      break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// kernel-group timing
// ---------------------------------------------------------------------------

void Prof::begin(int g) {
  open = false;
  if (!on || !((mask >> g) & 1) || iter % every != 0) return;
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
    (void)hipGetLastError();
    on = false;
    return;
  }
  (void)hipEventRecord(a, stream);
  groups.push_back(g);
  starts.push_back(a);
  ends.push_back(b);
  open = true;
}

void Prof::end() {
  if (!on || !open) return;
  (void)hipEventRecord(ends.back(), stream);
  open = false;
}

void Prof::collect(double* ms, int64_t* launches) {
  if (groups.empty()) return;
  (void)hipEventSynchronize(ends.back());
  for (size_t i = 0; i < groups.size(); ++i) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, starts[i], ends[i]) != hipSuccess) {
      (void)hipGetLastError();
      continue;
    }
    if (ms) ms[groups[i]] += t;
    if (launches) launches[groups[i]] += 1;
  }
}

Prof::~Prof() {
  for (auto e : starts) (void)hipEventDestroy(e);
  for (auto e : ends) (void)hipEventDestroy(e);
}

// ---------------------------------------------------------------------------
// workspace: one stream-ordered allocation carved into aligned pieces
// ---------------------------------------------------------------------------

struct Arena {
  static constexpr int kMaxPieces = 64;
  size_t bytes = 0;
  int npieces = 0;
  void** slot[kMaxPieces];
  size_t size[kMaxPieces];
  bool overflow = false;
  void add(void** s, size_t b) {
    if (npieces == kMaxPieces) { overflow = true; return; }
    slot[npieces] = s;
    size[npieces++] = b;
    bytes += (b + 255) & ~(size_t)255;
  }
  char* base = nullptr;
  bool owned = false;
  hipStream_t stream = nullptr;
  void place(char* c) {
    for (int i = 0; i < npieces; ++i) {
      *slot[i] = c;
      c += (size[i] + 255) & ~(size_t)255;
    }
  }
  // one stream-ordered allocation, freed (stream-ordered) with the arena
  knor_status alloc(hipStream_t s, size_t cap) {
    stream = s;
    if (overflow) return KNOR_ERR_INVALID_ARG;
    if (cap && bytes > cap) return KNOR_ERR_OUT_OF_MEMORY;
    if (bytes == 0) return KNOR_OK;
    if (hipMallocAsync((void**)&base, bytes, s) != hipSuccess) {
      (void)hipGetLastError();
      base = nullptr;
      return KNOR_ERR_OUT_OF_MEMORY;
    }
    owned = true;
    place(base);
    return KNOR_OK;
  }
  // the pieces carved from caller-provided device memory (no allocation)
  knor_status within(void* mem, size_t cap) {
    if (overflow) return KNOR_ERR_INVALID_ARG;
    if (bytes > cap) return KNOR_ERR_SCRATCH;
    base = (char*)mem;
    place(base);
    return KNOR_OK;
  }
  ~Arena() {
    if (owned && base) (void)hipFreeAsync(base, stream);
  }
};

struct Opts {
  int prune = 1, recheck = 1, check_numeric = 1, poll_every = 8;
  uint64_t seed = 0;
  hipStream_t stream = nullptr;
  size_t cap = 0;
  int32_t* label_history = nullptr;
  int64_t* iter_counters = nullptr;
  double* profile_ms = nullptr;
  int64_t* profile_launches = nullptr;
  int profile_mask = 0, profile_every = 1;
  int tile_blocks = 0, tile_resident = 0, autotune = 0;
  int learned = 0, train_iters = 5, train_batches = 16;
  int update = 0;
  double* centroid_history = nullptr;
  int clause2 = 0;
  int batch_graph = 0;
  double* objective_history = nullptr;
};

static knor_status read_opts(const knor_opts* o, Opts* out) {
  if (!o || o->struct_size == 0) return KNOR_OK;
  if (o->struct_size != sizeof(knor_opts)) return KNOR_ERR_INVALID_ARG;
  if (o->prune < 0 || o->prune > 1) return KNOR_ERR_INVALID_ARG;
  if (o->recheck < 1 || o->recheck > 2) return KNOR_ERR_INVALID_ARG;
  if (o->check_numeric < 0 || o->check_numeric > 1) return KNOR_ERR_INVALID_ARG;
  if (o->poll_every < 0) return KNOR_ERR_INVALID_ARG;
  out->prune = o->prune;
  out->recheck = o->recheck;
  out->check_numeric = o->check_numeric;
  out->seed = o->seed;
  out->stream = (hipStream_t)o->stream;
  out->cap = o->workspace_cap;
  out->label_history = o->label_history;
  out->iter_counters = o->iter_counters;
  out->profile_ms = o->profile_ms;
  out->profile_launches = o->profile_launches;
  out->profile_mask = o->profile_mask;
  if (o->profile_every < 0) return KNOR_ERR_INVALID_ARG;
  if (o->profile_every > 0) out->profile_every = o->profile_every;
  if (o->poll_every > 0) out->poll_every = o->poll_every;
  if (o->tile_blocks != 0 && o->tile_blocks != 1 && o->tile_blocks != 2 &&
      o->tile_blocks != 4)
    return KNOR_ERR_INVALID_ARG;
  if (o->tile_resident < 0 || o->tile_resident > 2) return KNOR_ERR_INVALID_ARG;
  if (o->autotune < 0 || o->autotune > 1) return KNOR_ERR_INVALID_ARG;
  if (o->learned < 0 || o->learned > 1 || o->train_iters < 0 ||
      o->train_batches < 0)
    return KNOR_ERR_INVALID_ARG;
  out->learned = o->learned;
  if (o->train_iters > 0) out->train_iters = o->train_iters;
  if (o->train_batches > 0) out->train_batches = o->train_batches;
  if (o->update < 0 || o->update > 1) return KNOR_ERR_INVALID_ARG;
  out->update = o->update;
  out->centroid_history = o->centroid_history;
  if (o->clause2 < 0 || o->clause2 > 2) return KNOR_ERR_INVALID_ARG;
  out->clause2 = o->clause2;
  out->objective_history = o->objective_history;
  if (o->batch_graph < 0 || o->batch_graph > 1) return KNOR_ERR_INVALID_ARG;
  out->batch_graph = o->batch_graph;
  out->tile_blocks = o->tile_blocks;
  out->tile_resident = o->tile_resident;
  out->autotune = o->autotune;
  return KNOR_OK;
}

static bool dtype_ok(knor_dtype dt) {
  return dt == KNOR_F64 || dt == KNOR_F32 || dt == KNOR_BF16;
}

#define HIPCHK(x)                                   \
  do {                                              \
    if ((x) != hipSuccess) {                        \
      (void)hipGetLastError();                      \
      return KNOR_ERR_HIP;                          \
    }                                               \
  } while (0)

// SplitMix64 (Steele, Lea, Flood 2014).
static uint64_t splitmix64(uint64_t* state) {
  uint64_t z = (*state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// The last k slots of a Fisher-Yates pass over 0..n-1 (i = n-1 down to n-k).
static std::vector<int64_t> forgy_rows(int64_t n, int k, uint64_t seed) {
  std::unordered_map<int64_t, int64_t> swapped;
  auto at = [&](int64_t i) {
    auto it = swapped.find(i);
    return it == swapped.end() ? i : it->second;
  };
  uint64_t st = seed;
  std::vector<int64_t> rows(k);
  for (int r = 0; r < k; ++r) {
    int64_t i = n - 1 - r;
    int64_t j = (int64_t)(splitmix64(&st) % (uint64_t)(i + 1));
    int64_t vi = at(i), vj = at(j);
    swapped[i] = vj;
    swapped[j] = vi;
    rows[r] = vj;
  }
  return rows;
}

// The first k entries of a front-to-back Fisher-Yates shuffle of 0..n-1:
// for i = 0 .. k-1, j = i + next() % (n - i), swap slots i and j.
static std::vector<int64_t> shuffle_first_k(int64_t n, int k, uint64_t seed) {
  std::unordered_map<int64_t, int64_t> swapped;
  auto at = [&](int64_t i) {
    auto it = swapped.find(i);
    return it == swapped.end() ? i : it->second;
  };
  uint64_t st = seed;
  std::vector<int64_t> rows(k);
  for (int i = 0; i < k; ++i) {
    const int64_t j = i + (int64_t)(splitmix64(&st) % (uint64_t)(n - i));
    const int64_t vi = at(i), vj = at(j);
    swapped[i] = vj;
    swapped[j] = vi;
    rows[i] = vj;
  }
  return rows;
}

// Centroid operands of the tile that serves points of type dt: FP32 -2c for
// FP32 points, the BF16 hi/lo terms of -2c for BF16 points (FP64 points use
// the canonical centroids directly); FP32 norms for both.
static void add_operands(Arena& ar, CentroidOps& ops, knor_dtype dt) {
  if (dt == KNOR_F32)
    ar.add((void**)&ops.Cm2, sizeof(float) * (size_t)ops.kpad * ops.dp);
  if (dt == KNOR_BF16) {
    ar.add((void**)&ops.Chi, sizeof(uint16_t) * (size_t)ops.kpad * ops.dpb);
    ar.add((void**)&ops.Clo, sizeof(uint16_t) * (size_t)ops.kpad * ops.dpb);
  }
  ar.add((void**)&ops.cn, sizeof(float) * (size_t)ops.kpad);
}

static int64_t flag_capacity(const CentroidOps& ops, knor_dtype dt, int64_t n,
                             int nseg) {
  return dt == KNOR_F64 ? 1 : tile_flag_capacity(ops, dt, n, nseg);
}

// ---------------------------------------------------------------------------
// FP32 tile schedule: default, tuned, or forced
// ---------------------------------------------------------------------------
//
// Every schedule computes the same FP32 values in the same order for every
// (point, centroid) pair, and undecided points go to the FP64 recheck, so
// the schedule changes speed only, never labels.  The tune table is the
// library's only process-wide mutable state; a mutex guards it.

static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, std::pair<int, int>> g_tune;   // (dp, kpad) -> (pb, resident)

static bool tune_lookup(int dp, int kpad, int* pb, int* res) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find({dp, kpad});
  if (it == g_tune.end()) return false;
  *pb = it->second.first;
  *res = it->second.second;
  return true;
}

static void tune_store(int dp, int kpad, int pb, int res) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[{dp, kpad}] = {pb, res};
}

// schedule candidates of a (dp, kpad) class
static std::vector<std::pair<int, int>> tile_candidates(int dp, int kpad) {
  std::vector<std::pair<int, int>> c;
  for (int res = 1; res >= 0; --res) {
    if (res && !tile_f32_resident(dp, kpad)) continue;
    for (int pb : {1, 2, 4})
      if (tile_f32_pb_ok(dp, pb)) c.push_back({pb, res});
  }
  return c;
}

// Times every candidate schedule of the dense FP32 tile on the first ns
// points of X against centroids C (k x d FP64, device) and stores the
// fastest in the table.  Writes only its own scratch.
static knor_status tune_tile(const float* X, int64_t n, int d, const double* C,
                             int k, hipStream_t s) {
  const int kpad = (k + 15) / 16 * 16, dp = pad_dim(d);
  const int64_t ns = n < (1 << 17) ? n : (1 << 17);
  const auto cand = tile_candidates(dp, kpad);
  CentroidOps ops{};
  ops.k = k; ops.kpad = kpad; ops.d = d; ops.dp = dp; ops.dpb = pad_dim_bf16(d);
  ops.C64 = const_cast<double*>(C);
  int64_t fcap = 1;
  for (auto& c : cand) {
    const TileGeom g = tile_f32_geometry(dp, kpad, c.first, c.second, ns, false, 1);
    fcap = std::max(fcap, (int64_t)g.grid * g.cap);
  }
  int32_t* lab = nullptr;
  int *flags = nullptr, *ucnt = nullptr, *conv = nullptr;
  unsigned long long* row = nullptr;
  double* Cs = nullptr;
  int64_t* rows_dev = nullptr;
  Arena ar;
  if (!C) {                                  // centroids: the first k rows
    ar.add((void**)&Cs, sizeof(double) * (size_t)k * d);
    ar.add((void**)&rows_dev, sizeof(int64_t) * (size_t)k);
  }
  ar.add((void**)&ops.Cm2, sizeof(float) * (size_t)kpad * dp);
  ar.add((void**)&ops.cn, sizeof(float) * (size_t)kpad);
  ar.add((void**)&lab, sizeof(int32_t) * (size_t)ns);
  ar.add((void**)&flags, sizeof(int) * (size_t)fcap);
  ar.add((void**)&ucnt, sizeof(int) * (size_t)kTileMaxGrid);
  ar.add((void**)&row, sizeof(unsigned long long) * ROW_STRIDE);
  ar.add((void**)&conv, sizeof(int) * 4);
  if (knor_status r = ar.alloc(s, 0)) return r;
  if (!C) {
    std::vector<int64_t> rows(k);
    for (int i = 0; i < k; ++i) rows[i] = i;
    HIPCHK(hipMemcpyAsync(rows_dev, rows.data(), sizeof(int64_t) * k,
                          hipMemcpyHostToDevice, s));
    HIPCHK(launch_gather_rows(X, KNOR_F32, d, rows_dev, k, Cs, s));
    HIPCHK(hipStreamSynchronize(s));        // `rows` leaves scope
    ops.C64 = Cs;
  }
  HIPCHK(launch_prep_centroids(ops, s));
  HIPCHK(launch_fill_i32(conv, 1, kNotConverged, s));
  HIPCHK(launch_fill_i32(lab, ns, -1, s));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  float best_ms = 1e30f;
  std::pair<int, int> best = cand.front();
  for (auto& c : cand) {
    ops.tpb = c.first;
    ops.tres = c.second;
    AssignJob job{};
    job.X = X; job.dt = KNOR_F32; job.n = ns; job.d = d;
    job.labels = lab; job.flags = flags; job.ucnt = ucnt; job.row = row;
    job.conv = conv; job.iter = 0;
    float tmin = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {     // the first is a warm-up
      HIPCHK(hipEventRecord(e0, s));
      HIPCHK(launch_tile_f32(ops, job, s));
      HIPCHK(hipEventRecord(e1, s));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      if (rep > 0) tmin = std::min(tmin, ms);
    }
    if (tmin < best_ms) { best_ms = tmin; best = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(hipStreamSynchronize(s));
  tune_store(dp, kpad, best.first, best.second);
  return KNOR_OK;
}

// The FP32 tile schedule of one call: forced by the options, else tuned
// (table), else the default.
static knor_status select_tile(CentroidOps& ops, const Opts& o) {
  int pb, res;
  tile_f32_default(ops.dp, ops.kpad, &pb, &res);
  int tpb, tres;
  if (tune_lookup(ops.dp, ops.kpad, &tpb, &tres)) { pb = tpb; res = tres; }
  if (o.tile_resident == 1) {
    if (!tile_f32_resident(ops.dp, ops.kpad)) return KNOR_ERR_UNSUPPORTED;
    res = 1;
  } else if (o.tile_resident == 2) {
    res = 0;
  }
  if (o.tile_blocks) pb = o.tile_blocks;
  if (!tile_f32_pb_ok(ops.dp, pb)) {
    if (o.tile_blocks) return KNOR_ERR_UNSUPPORTED;
    tile_f32_default(ops.dp, ops.kpad, &pb, &tres);   // keep res, fix pb
  }
  ops.tpb = pb;
  ops.tres = res;
  return KNOR_OK;
}

// ---------------------------------------------------------------------------
// fit
// ---------------------------------------------------------------------------

// Whether a fit's survivor passes use the Clause-2 candidate-list tile:
// MTI on FP32 points with k <= kCandMaxK, by default from kCandMinK
// centroids on (below that a survivor's scan of all k is short already).
static bool cand_enabled(const Opts& o, knor_dtype dt, int k) {
  if (o.prune != 1 || dt != KNOR_F32 || k > kCandMaxK || o.clause2 == 1) return false;
  return o.clause2 == 2 || k >= kCandMinK;
}

// Per-iteration counters (iter_counters) and their sums (st) from the
// device's counter rows of the first hiters iterations.  Distances
// evaluated in iteration i: the tiles and FP64 rechecks (all k per point,
// or the candidate lists), and Clause-3 tightening.
static void report_counters(const std::vector<unsigned long long>& hc, int hiters, int64_t n,
                            int k, bool mti, const std::vector<char>& cand_used,
                            const std::vector<char>& proposed,
                            const std::vector<int64_t>& forwarded, int64_t* iter_counters,
                            knor_stats* st) {
  // survivors that took a proposal: every survivor of a proposal iteration
  auto queried = [&](int i) {
    return proposed[(size_t)i] ? (int64_t)hc[(size_t)i * ROW_STRIDE + ROW_SURVIVED] : 0;
  };
  auto dists_of = [&](int i) {
    const unsigned long long* r = &hc[(size_t)i * ROW_STRIDE];
    const int64_t tighten = (mti && i > 0) ? (n - (int64_t)r[ROW_PRUNED_A]) : 0;
    if (cand_used[(size_t)i]) return (int64_t)r[ROW_DISTS] + tighten;
    return ((int64_t)r[ROW_SCANNED] + (int64_t)r[ROW_FLAG_HEAD]) * k + tighten;
  };
  if (iter_counters)
    for (int i = 0; i < hiters; ++i) {
      const unsigned long long* r = &hc[(size_t)i * ROW_STRIDE];
      int64_t* dst = iter_counters + (size_t)i * KNOR_NCOUNTERS;
      dst[KNOR_CNT_CHANGED] = (int64_t)r[ROW_CHANGED];
      dst[KNOR_CNT_SCANNED] = (int64_t)r[ROW_SCANNED];
      dst[KNOR_CNT_PRUNED_A] = (int64_t)r[ROW_PRUNED_A];
      dst[KNOR_CNT_PRUNED_B] = (int64_t)r[ROW_PRUNED_B];
      dst[KNOR_CNT_RECHECKED] = (int64_t)r[ROW_FLAG_HEAD];
      dst[KNOR_CNT_CERTIFIED] = (int64_t)r[ROW_CERTIFIED];
      dst[KNOR_CNT_QUERIED] = queried(i);
      dst[KNOR_CNT_DISTS] = dists_of(i);
      dst[KNOR_CNT_FORWARD] = forwarded[(size_t)i];
    }
  if (st) {
    memset(st, 0, sizeof(*st));
    st->iters = hiters;
    st->changed_last = (int64_t)hc[(size_t)(hiters - 1) * ROW_STRIDE + ROW_CHANGED];
    for (int i = 0; i < hiters; ++i) {
      const unsigned long long* r = &hc[(size_t)i * ROW_STRIDE];
      st->scanned += (int64_t)r[ROW_SCANNED];
      st->pruned_a += (int64_t)r[ROW_PRUNED_A];
      st->pruned_b += (int64_t)r[ROW_PRUNED_B];
      st->rechecked += (int64_t)r[ROW_FLAG_HEAD];
      st->certified += (int64_t)r[ROW_CERTIFIED];
      st->dists_computed += dists_of(i);
      st->mlp_queries += queried(i);
      st->mlp_forward_rows += forwarded[(size_t)i];
    }
  }
}

// One fit in phases: setup (workspace and initial state; may synchronize),
// iteration t (enqueues the iteration's kernels on the fit's stream; only
// the learned proposal synchronizes inside it), poll (reads the convergence
// word every poll_every iterations), finish (objective, counters, stats).
// knor_fit runs them in order; the batched form can record the iterations
// of every problem into one graph between setup and finish.  Not movable
// once set up (the workspace pieces point at its members).
struct FitRun {
  const void* X = nullptr;
  knor_dtype dt = KNOR_F32;
  int64_t n = 0;
  int d = 0, k = 0;
  knor_init init = KNOR_INIT_GIVEN;
  const double* C_init = nullptr;
  int max_iters = 0;
  double tol = 0.0;
  Opts o;
  double* C_out = nullptr;
  int32_t* labels_out = nullptr;
  knor_stats* st = nullptr;

  std::chrono::steady_clock::time_point t0;
  hipStream_t s = nullptr;
  int kpad = 0, dp = 0, nseg = 0;
  bool mti = false, use_cand = false, exact = false, learned = false, need_rows = false;
  CentroidOps ops{};
  UpdatePlan plan{};
  ExactPlan xplan{};
  void* upd_ws = nullptr;
  float *u = nullptr, *drift = nullptr, *s_half = nullptr;
  int *list = nullptr, *seg_cnt = nullptr, *flags = nullptr, *ucnt = nullptr;
  int *flagbuf = nullptr, *dirty = nullptr, *conv = nullptr, *bad = nullptr;
  unsigned long long* ctr = nullptr;
  size_t ctr_bytes = 0;
  int64_t* rows_dev = nullptr;
  double *dist2 = nullptr, *sumtmp = nullptr, *objective = nullptr;
  double* obj_hist = nullptr;                   // J_t per iteration (opt-in)
  void* exact_ws = nullptr;
  float* ccrows = nullptr;
  void* cand_ws = nullptr;
  int hM = kMlpHidden, Bt = 0;
  MlpLayout ML{};
  MlpPacked MP{};
  float *th = nullptr, *am = nullptr, *av = nullptr, *grad = nullptr, *Xs_tr = nullptr;
  int32_t *y_tr = nullptr, *cand = nullptr;
  int *rows_tr = nullptr, *dense = nullptr, *seg_off = nullptr, *list2 = nullptr,
      *seg_cnt2 = nullptr;
  void *mlp_ws = nullptr, *pack_ws = nullptr;
  double *mean = nullptr, *istd = nullptr, *loss_dev = nullptr, *stat_part = nullptr;
  void* pp_ws = nullptr;
  unsigned long long* pp_rnd = nullptr;
  int64_t mlp_step = 0;
  std::vector<char> proposed;                   // survivors took a proposal
  std::vector<int64_t> forwarded;               // rows through the forward pass
  std::vector<char> cand_used;                  // candidate-list tile ran
  int* seg_new = nullptr;                       // per segment: unproposed survivors
  uint8_t* prop = nullptr;                      // per point: sent to the network
  bool packed = false;
  Prof prof;
  Prof* pp = nullptr;
  double tol_n = 0.0;
  int hconv = kNotConverged;
  int ctl_delta_only = 0;
  Arena ar;

  FitRun() = default;
  FitRun(const FitRun&) = delete;
  FitRun& operator=(const FitRun&) = delete;

  knor_status setup() {
    t0 = std::chrono::steady_clock::now();
    s = o.stream;
    kpad = (k + 15) / 16 * 16;
    dp = pad_dim(d);
    mti = o.prune == 1;
    nseg = nseg_of_n(n);
    // Clause 2 per block of survivors (FP32 points, large k by default)
    use_cand = cand_enabled(o, dt, k);

    ops.k = k; ops.kpad = kpad; ops.d = d; ops.dp = dp; ops.dpb = pad_dim_bf16(d);
    ops.C64 = C_out;                 // the output buffer is the working copy
    if (knor_status r = select_tile(ops, o)) return r;
    add_operands(ar, ops, dt);
    ar.add((void**)&ops.CT, sizeof(double) * (size_t)k * d);
    ar.add((void**)&drift, sizeof(float) * (size_t)k);
    ar.add((void**)&s_half, sizeof(float) * (size_t)k);
    ar.add((void**)&dirty, sizeof(int) * (size_t)k);
    ar.add((void**)&flags, sizeof(int) * (size_t)flag_capacity(ops, dt, n, nseg));
    ar.add((void**)&ucnt, sizeof(int) * (size_t)kTileMaxGrid);
    if (mti) {
      ar.add((void**)&u, sizeof(float) * (size_t)n);
      ar.add((void**)&list, sizeof(int) * (size_t)nseg * kSeg);
      ar.add((void**)&seg_cnt, sizeof(int) * (size_t)nseg);
    }
    ctr_bytes = sizeof(unsigned long long) * ROW_STRIDE * (size_t)max_iters;
    ar.add((void**)&ctr, ctr_bytes);
    ar.add((void**)&flagbuf, sizeof(int) * 8);   // conv, bad
    ar.add((void**)&rows_dev, sizeof(int64_t) * (size_t)k);
    ar.add(&upd_ws, update_workspace_bytes(n, k, d));
    exact = o.update == 1;
    if (exact && dt == KNOR_F64) return KNOR_ERR_UNSUPPORTED;
    if (exact) ar.add(&exact_ws, exact_workspace_bytes(n, k, d));
    // learned proposal (MTI survivors only)
    learned = o.learned && mti;
    // the centroids' neighbour rows: the candidate lists and the certificate
    need_rows = use_cand || learned;
    if (need_rows) ar.add((void**)&ccrows, sizeof(float) * (size_t)k * k);
    if (use_cand) ar.add(&cand_ws, cand_workspace_bytes(n, k));
    ar.add((void**)&dist2, sizeof(double) * (size_t)n);
    ar.add((void**)&sumtmp, sizeof(double) * (size_t)(n / kLeaf + 2));
    ar.add((void**)&objective, sizeof(double));
    if (o.objective_history) ar.add((void**)&obj_hist, sizeof(double) * (size_t)max_iters);
    Bt = n < kMlpBatch ? (int)n : kMlpBatch;
    if (learned) {
      ML = mlp_layout(d, hM, k);
      for (float** q : {&th, &am, &av, &grad}) ar.add((void**)q, sizeof(float) * (size_t)ML.P);
      ar.add(&mlp_ws, mlp_train_workspace(d, hM, k, Bt));
      ar.add((void**)&Xs_tr, sizeof(float) * (size_t)Bt * d);
      ar.add((void**)&y_tr, sizeof(int32_t) * (size_t)Bt);
      ar.add((void**)&rows_tr, sizeof(int) * (size_t)Bt * o.train_batches);
      ar.add((void**)&mean, sizeof(double) * (size_t)d);
      ar.add((void**)&istd, sizeof(double) * (size_t)d);
      ar.add((void**)&loss_dev, sizeof(double));
      ar.add((void**)&stat_part, standardize_workspace(d));
      ar.add(&pack_ws, mlp_pack_bytes(d, hM, k, n));
      ar.add((void**)&dense, sizeof(int) * (size_t)n);
      ar.add((void**)&seg_off, sizeof(int) * (size_t)(nseg + 1));
      ar.add((void**)&list2, sizeof(int) * (size_t)nseg * kSeg);
      ar.add((void**)&seg_cnt2, sizeof(int) * (size_t)nseg);
      ar.add((void**)&cand, sizeof(int32_t) * (size_t)n * kMlpTop);
      ar.add((void**)&seg_new, sizeof(int) * (size_t)nseg);
      ar.add((void**)&prop, sizeof(int32_t) * (size_t)((n + 3) / 4));
    }
    if (init == KNOR_INIT_KMEANSPP) {
      ar.add(&pp_ws, kmeanspp_workspace_bytes(n, k));
      ar.add((void**)&pp_rnd, sizeof(unsigned long long) * (size_t)k);
    }
    knor_status rs = ar.alloc(s, o.cap);
    if (rs != KNOR_OK) return rs;
    update_plan_init(&plan, n, k, d, upd_ws);
    if (learned) MP = mlp_pack_layout(d, hM, k, n, pack_ws);
    if (exact) exact_plan_init(&xplan, n, k, d, exact_ws);
    conv = flagbuf;
    bad = flagbuf + 1;
    HIPCHK(update_plan_reset(plan, s));

    HIPCHK(hipMemsetAsync(flagbuf, 0, sizeof(int) * 8, s));
    HIPCHK(launch_fill_i32(conv, 1, kNotConverged, s));
    HIPCHK(hipMemsetAsync(ctr, 0, ctr_bytes, s));

    // numeric check of the inputs before anything is written to the outputs
    if (o.check_numeric) {
      HIPCHK(launch_check_finite(X, dt, n * (int64_t)d, bad, s));
      if (init == KNOR_INIT_GIVEN)
        HIPCHK(launch_check_finite(C_init, KNOR_F64, (int64_t)k * d, bad, s));
      int hbad = 0;
      HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (hbad) return KNOR_ERR_NUMERIC;
    }

    // initial centroids into the working buffer C_out
    if (init == KNOR_INIT_GIVEN) {
      if (C_init != C_out)
        HIPCHK(hipMemcpyAsync(C_out, C_init, sizeof(double) * (size_t)k * d,
                              hipMemcpyDeviceToDevice, s));
    } else if (init == KNOR_INIT_KMEANSPP) {
      std::vector<unsigned long long> rnd(k);
      uint64_t st_r = o.seed;
      for (auto& r : rnd) r = splitmix64(&st_r);
      HIPCHK(hipMemcpyAsync(pp_rnd, rnd.data(), sizeof(unsigned long long) * k,
                            hipMemcpyHostToDevice, s));
      HIPCHK(launch_kmeanspp(X, dt, n, d, k, pp_rnd, C_out, pp_ws, s));
      HIPCHK(hipStreamSynchronize(s));   // `rnd` leaves scope
    } else {
      std::vector<int64_t> rows = init == KNOR_INIT_FORGY ? forgy_rows(n, k, o.seed)
                                                          : shuffle_first_k(n, k, o.seed);
      HIPCHK(hipMemcpyAsync(rows_dev, rows.data(), sizeof(int64_t) * k,
                            hipMemcpyHostToDevice, s));
      HIPCHK(launch_gather_rows(X, dt, d, rows_dev, k, C_out, s));
      HIPCHK(hipStreamSynchronize(s));   // `rows` leaves scope
    }
    HIPCHK(launch_prep_centroids(ops, s));
    HIPCHK(launch_fill_i32(labels_out, n, -1, s));   // every label changes at t = 0
    HIPCHK(launch_fill_i32(dirty, k, 1, s));         // every cluster is summed at t = 0
    if (exact) HIPCHK(launch_fill_i32(xplan.prev, n, -1, s));
    if (learned) {
      HIPCHK(launch_standardize_stats(X, dt, n, d, mean, istd, stat_part, s));
      std::vector<float> th0 = mlp_init_host(d, hM, k, o.seed);
      HIPCHK(hipMemcpyAsync(th, th0.data(), sizeof(float) * th0.size(),
                            hipMemcpyHostToDevice, s));
      HIPCHK(hipMemsetAsync(am, 0, sizeof(float) * (size_t)ML.P, s));
      HIPCHK(hipMemsetAsync(av, 0, sizeof(float) * (size_t)ML.P, s));
      HIPCHK(launch_fill_i32(cand, n * kMlpTop, kUnproposed, s));
      HIPCHK(launch_fill_i32(reinterpret_cast<int32_t*>(prop), (n + 3) / 4, 0, s));
      HIPCHK(hipStreamSynchronize(s));          // `th0` leaves scope
    }
    proposed.assign((size_t)max_iters, 0);
    forwarded.assign((size_t)max_iters, 0);
    cand_used.assign((size_t)max_iters, 0);

    prof.stream = s;
    prof.on = o.profile_ms != nullptr || o.profile_launches != nullptr;
    prof.mask = o.profile_mask ? o.profile_mask : ~0;
    prof.every = o.profile_every;
    pp = prof.on ? &prof : nullptr;
    tol_n = tol * (double)n;
    return KNOR_OK;
  }

  knor_status iteration(int t) {
    prof.iter = t;
    unsigned long long* row = ctr + (size_t)t * ROW_STRIDE;
    if (o.centroid_history)
      HIPCHK(hipMemcpyAsync(o.centroid_history + (size_t)t * k * d, C_out,
                            sizeof(double) * (size_t)k * d, hipMemcpyDeviceToDevice, s));
    AssignJob job{};
    job.X = X; job.dt = dt; job.n = n; job.d = d;
    job.labels = labels_out; job.u = mti ? u : nullptr;
    job.flags = flags; job.row = row; job.conv = conv; job.iter = t;
    job.ucnt = ucnt;
    job.dirty = dirty; job.recheck_all = o.recheck == 2;
    const bool seg = mti && t > 0;
    if (seg) {
      prof.begin(KNOR_PROF_FILTER);
      HIPCHK(launch_mti_filter(X, dt, n, d, C_out, labels_out, u, drift, s_half,
                               list, seg_cnt, row - ROW_STRIDE, row, conv, t,
                               use_cand ? 1 : 0, s));
      prof.end();
      job.list = list;
      job.seg_cnt = seg_cnt;
      job.nseg = nseg;
    }
    if (learned && seg && t > o.train_iters) {
      prof.begin(KNOR_PROF_LEARNED);
      if (!packed) {                          // training is over
        HIPCHK(launch_mlp_pack(th, ML, MP, s));
        packed = true;
      }
      // only survivors that were never proposed for go through the network:
      // a point's candidates do not change once training is over
      HIPCHK(launch_seg_unproposed(list, seg_cnt, nseg, prop, seg_new, seg_off, dense, conv,
                                   t, u, labels_out, use_cand ? ccrows : nullptr, k, s));
      int hm[2] = {0, 0};
      HIPCHK(hipMemcpyAsync(&hm[0], seg_off + nseg, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipMemcpyAsync(&hm[1], conv, sizeof(int), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (hm[1] == kNotConverged) {
        const int m_new = hm[0];
        proposed[t] = 1;
        forwarded[t] = m_new;
        HIPCHK(launch_mlp_forward(X, dt, d, dense, m_new, nullptr, mean, istd, th, ML, MP,
                                  cand, dense, s));
        prof.end();
        prof.begin(KNOR_PROF_CERTIFY);
        HIPCHK(launch_mlp_certify(X, dt, d, C_out, k, ccrows, list, seg_cnt, nseg, cand,
                                  labels_out, u, dirty, list2, seg_cnt2, row, conv, t,
                                  use_cand, s));
        job.list = list2;
        job.seg_cnt = seg_cnt2;
      }
      prof.end();
    }
    const bool cand_t = seg && use_cand;
    cand_used[t] = cand_t ? 1 : 0;
    prof.begin(seg ? KNOR_PROF_ASSIGN_LIST : KNOR_PROF_ASSIGN_DENSE);
    if (cand_t)
      HIPCHK(launch_tile_cand(ops, job, ccrows, cand_ws, s));
    else
      HIPCHK(launch_assign(ops, job, s));
    prof.end();
    if (dt != KNOR_F64 && !cand_t) {
      prof.begin(KNOR_PROF_RECHECK);
      HIPCHK(launch_recheck(ops, job, s));
      prof.end();
    }
    if (learned && t >= 1 && t <= o.train_iters) {
      // one pass of train_batches minibatches on (x, this iteration's label)
      prof.begin(KNOR_PROF_LEARNED);
      std::vector<int> rows((size_t)Bt * o.train_batches);
      uint64_t st_r = o.seed ^ (0x9e3779b97f4a7c15ull * (uint64_t)(t + 1));
      for (auto& r : rows) r = (int)(splitmix64(&st_r) % (uint64_t)n);
      HIPCHK(hipMemcpyAsync(rows_tr, rows.data(), sizeof(int) * rows.size(),
                            hipMemcpyHostToDevice, s));
      for (int b = 0; b < o.train_batches; ++b) {
        const int* rb = rows_tr + (size_t)b * Bt;
        HIPCHK(launch_gather_std(X, dt, d, rb, Bt, nullptr, mean, istd, Xs_tr, s));
        HIPCHK(launch_gather_i32(labels_out, rb, Bt, y_tr, s));
        HIPCHK(mlp_train_step(th, am, av, ++mlp_step, ML, Xs_tr, y_tr, Bt, kMlpLr, grad,
                              mlp_ws, loss_dev, s));
      }
      HIPCHK(hipStreamSynchronize(s));        // `rows` leaves scope
      prof.end();
    }
    if (o.label_history)
      HIPCHK(launch_copy_i32(labels_out, o.label_history + (size_t)t * n, n,
                             conv, t, s));
    if (obj_hist) {
      // J_t under the centroids this assignment used (the update follows)
      HIPCHK(launch_exact_dist2(X, dt, n, d, C_out, labels_out, dist2, s));
      HIPCHK(launch_canonical_sum(dist2, n, sumtmp, obj_hist + t, s));
    }
    IterCtl ctl;
    ctl.row = row; ctl.conv = conv; ctl.iter = t; ctl.tol_n = tol_n;
    ctl.segmented = seg; ctl.n = n;
    if (seg) { ctl.list = list; ctl.seg_cnt = seg_cnt; ctl.nseg = nseg; }
    ctl.delta_only = ctl_delta_only;
    if (exact)
      HIPCHK(launch_update_exact(plan, xplan, X, dt, labels_out, C_out, C_out, nullptr, &ops,
                                 mti ? drift : nullptr, dirty, &ctl, s, pp));
    else
      HIPCHK(launch_update(plan, X, dt, labels_out, C_out, C_out, nullptr, &ops,
                           mti ? drift : nullptr, dirty, &ctl, s, pp));
    if (mti) {
      prof.begin(KNOR_PROF_CC);
      HIPCHK(launch_cc_bounds(ops, s_half, need_rows ? ccrows : nullptr, conv, t, s));
      prof.end();
    }
    return KNOR_OK;
  }

  knor_status poll(int t, bool* stop) {
    const unsigned long long* row = ctr + (size_t)t * ROW_STRIDE;
    if ((t + 1) % o.poll_every == 0 || t + 1 == max_iters) {
      unsigned long long hch = 0;
      HIPCHK(hipMemcpyAsync(&hconv, conv, sizeof(int), hipMemcpyDeviceToHost, s));
      if (exact && !ctl_delta_only)
        HIPCHK(hipMemcpyAsync(&hch, row + ROW_CHANGED, sizeof(hch), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (hconv != kNotConverged) {
        *stop = true;
        return KNOR_OK;
      }
      // the exact update: once few labels change, stop launching the full
      // pass (both modes give the same centroids; this only saves launches)
      if (exact && !ctl_delta_only && hch <= (unsigned long long)xplan.delta_max)
        ctl_delta_only = 1;
    }
    return KNOR_OK;
  }

  knor_status finish() {
    // final objective: sum over points of D(x, C_out[label]) in the canonical order
    HIPCHK(launch_exact_dist2(X, dt, n, d, C_out, labels_out, dist2, s));
    HIPCHK(launch_canonical_sum(dist2, n, sumtmp, objective, s));

    std::vector<unsigned long long> hc((size_t)ROW_STRIDE * max_iters);
    double hobj = 0.0;
    HIPCHK(hipMemcpyAsync(&hconv, conv, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(hc.data(), ctr, ctr_bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hobj, objective, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    prof.collect(o.profile_ms, o.profile_launches);
    const int converged = hconv != kNotConverged;
    const int hiters = converged ? hconv + 1 : max_iters;
    if (obj_hist) {
      HIPCHK(hipMemcpyAsync(o.objective_history, obj_hist, sizeof(double) * (size_t)hiters,
                            hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }

    report_counters(hc, hiters, n, k, mti, cand_used, proposed, forwarded, o.iter_counters, st);
    if (st) {
      st->converged = converged;
      st->objective = hobj;
      st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    return KNOR_OK;
  }
};

static knor_status fit_impl(const void* X, knor_dtype dt, int64_t n, int d,
                            int k, knor_init init, const double* C_init,
                            int max_iters, double tol, const Opts& o,
                            double* C_out, int32_t* labels_out,
                            knor_stats* st) {
  FitRun r;
  r.X = X; r.dt = dt; r.n = n; r.d = d; r.k = k; r.init = init; r.C_init = C_init;
  r.max_iters = max_iters; r.tol = tol; r.o = o; r.C_out = C_out;
  r.labels_out = labels_out; r.st = st;
  if (knor_status e = r.setup()) return e;
  for (int t = 0; t < max_iters; ++t) {
    if (knor_status e = r.iteration(t)) return e;
    bool stop = false;
    if (knor_status e = r.poll(t, &stop)) return e;
    if (stop) break;
  }
  return r.finish();
}

// ---------------------------------------------------------------------------
// assignment (knor_assign and its allocation-free form)
// ---------------------------------------------------------------------------

// One assignment.  mem == null and cap == 0: workspace from a stream-ordered
// allocation; mem != null: carved from mem (cap bytes, KNOR_ERR_SCRATCH if
// too small) with no allocation and no memset; mem == null and cap != 0:
// validate only (no device work).
static knor_status assign_impl(const void* X, knor_dtype dt, int64_t n, int32_t d,
                               const double* C, int32_t k, const knor_opts* opts,
                               int32_t* labels_out, double* dist2_out, void* mem,
                               size_t cap) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  // X and labels_out may be NULL when n == 0
  if ((n > 0 && (!X || !labels_out)) || !C || !dtype_ok(dt)) return KNOR_ERR_INVALID_ARG;
  if (n < 0 || n >= (int64_t)1 << 31 || d < 1 || d > kMaxD || k < 1 || k > kMaxK)
    return KNOR_ERR_INVALID_ARG;
  if (n == 0 || (!mem && cap)) return KNOR_OK;
  hipStream_t s = o.stream;
  CentroidOps ops{};
  ops.k = k; ops.kpad = (k + 15) / 16 * 16; ops.d = d; ops.dp = pad_dim(d);
  ops.dpb = pad_dim_bf16(d);
  ops.C64 = const_cast<double*>(C);
  if (knor_status r = select_tile(ops, o)) return r;
  int* flags = nullptr;
  int* conv = nullptr;
  int* ucnt = nullptr;
  unsigned long long* ctr = nullptr;
  Arena ar;
  add_operands(ar, ops, dt);
  ar.add((void**)&ops.CT, sizeof(double) * (size_t)k * d);
  ar.add((void**)&flags, sizeof(int) * (size_t)flag_capacity(ops, dt, n, nseg_of_n(n)));
  ar.add((void**)&ucnt, sizeof(int) * (size_t)kTileMaxGrid);
  ar.add((void**)&ctr, sizeof(unsigned long long) * ROW_STRIDE);
  ar.add((void**)&conv, sizeof(int) * 4);
  if (knor_status r = mem ? ar.within(mem, cap) : ar.alloc(s, o.cap)) return r;
  // fill kernels rather than memset: callers may capture this in a graph
  HIPCHK(launch_fill_i32((int32_t*)ctr, 2 * (int64_t)ROW_STRIDE, 0, s));
  HIPCHK(launch_fill_i32(conv, 1, kNotConverged, s));
  HIPCHK(launch_fill_i32(labels_out, n, -1, s));
  HIPCHK(launch_prep_centroids(ops, s));
  AssignJob job{};
  job.X = X; job.dt = dt; job.n = n; job.d = d;
  job.labels = labels_out; job.flags = flags; job.row = ctr; job.conv = conv;
  job.ucnt = ucnt;
  job.iter = 0; job.recheck_all = o.recheck == 2;
  HIPCHK(launch_assign(ops, job, s));
  HIPCHK(launch_recheck(ops, job, s));
  if (dist2_out)
    HIPCHK(launch_exact_dist2(X, dt, n, d, C, labels_out, dist2_out, s));
  return KNOR_OK;
}

// ---------------------------------------------------------------------------
// the allocation-free assignment's scratch
// ---------------------------------------------------------------------------

// Device memory of knor_assign_noalloc: one array per device for the life
// of the process.  In host code `scratch` names a host-side stand-in, never
// the device memory: every use goes through the address hipGetSymbolAddress
// returns for the current device, looked up once per device.
constexpr size_t kScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kScratchDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kScratchDevices];

static knor_status scratch_of_device(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return KNOR_ERR_HIP;
  }
  if (dev < 0 || dev >= kScratchDevices) return KNOR_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return KNOR_ERR_HIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KNOR_OK;
}

}  // namespace knor

using namespace knor;

extern "C" {

static bool mlp_sizes_ok(int32_t d, int32_t h, int32_t k) {
  return d >= 1 && d <= kMaxD && (h == 32 || h == 64 || h == 128 || h == 256) &&
         k >= 1 && k <= kMaxK;
}

int64_t knor_mlp_param_count(int32_t d, int32_t h, int32_t k) {
  return mlp_sizes_ok(d, h, k) ? mlp_layout(d, h, k).P : -1;
}

knor_status knor_mlp_init(float* params, int32_t d, int32_t h, int32_t k,
                          uint64_t seed, const knor_opts* opts) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  if (!params || !mlp_sizes_ok(d, h, k)) return KNOR_ERR_INVALID_ARG;
  std::vector<float> th = mlp_init_host(d, h, k, seed);
  HIPCHK(hipMemcpyAsync(params, th.data(), sizeof(float) * th.size(),
                        hipMemcpyHostToDevice, o.stream));
  HIPCHK(hipStreamSynchronize(o.stream));
  return KNOR_OK;
}

knor_status knor_mlp_train_step(float* params, float* adam_m, float* adam_v,
                                int64_t step, int32_t d, int32_t h, int32_t k,
                                const float* Xs, const int32_t* y, int32_t B,
                                float lr, float* grad_out, double* loss_out,
                                const knor_opts* opts) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  if (!params || !Xs || !y || !mlp_sizes_ok(d, h, k) || B < 1 || !(lr >= 0.0f))
    return KNOR_ERR_INVALID_ARG;
  if (lr > 0.0f && (!adam_m || !adam_v || step < 1)) return KNOR_ERR_INVALID_ARG;
  const MlpLayout L = mlp_layout(d, h, k);
  hipStream_t s = o.stream;
  float* grad = grad_out;
  void* ws = nullptr;
  double* loss_dev = nullptr;
  Arena ar;
  if (!grad) ar.add((void**)&grad, sizeof(float) * (size_t)L.P);
  ar.add(&ws, mlp_train_workspace(d, h, k, B));
  ar.add((void**)&loss_dev, sizeof(double));
  if (knor_status r = ar.alloc(s, o.cap)) return r;
  HIPCHK(mlp_train_step(params, adam_m, adam_v, step, L, Xs, y, B, lr, grad, ws,
                        loss_dev, s));
  if (loss_out) {
    HIPCHK(hipMemcpyAsync(loss_out, loss_dev, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  return KNOR_OK;
}

knor_status knor_mlp_propose(const float* params, int32_t d, int32_t h,
                             int32_t k, const float* Xs, int64_t m,
                             int32_t* cand_out, const knor_opts* opts) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  if (!params || !Xs || !cand_out || !mlp_sizes_ok(d, h, k) || m < 0 ||
      m >= ((int64_t)1 << 31))
    return KNOR_ERR_INVALID_ARG;
  if (m == 0) return KNOR_OK;
  const MlpLayout L = mlp_layout(d, h, k);
  hipStream_t s = o.stream;
  void* pack_ws = nullptr;
  Arena ar;
  ar.add(&pack_ws, mlp_pack_bytes(d, h, k, m));
  if (knor_status r = ar.alloc(s, o.cap)) return r;
  const MlpPacked P = mlp_pack_layout(d, h, k, m, pack_ws);
  HIPCHK(launch_mlp_pack(params, L, P, s));
  // Xs is already standardized: no row list, no mean / scale
  HIPCHK(launch_mlp_forward(Xs, KNOR_F32, d, nullptr, (int)m, nullptr, nullptr, nullptr,
                            params, L, P, cand_out, nullptr, s));
  return KNOR_OK;
}

const char* knor_status_string(knor_status s) {
  switch (s) {
    case KNOR_OK: return "ok";
    case KNOR_ERR_INVALID_ARG: return "invalid argument";
    case KNOR_ERR_OUT_OF_MEMORY: return "out of device memory or over workspace cap";
    case KNOR_ERR_HIP: return "HIP runtime error";
    case KNOR_ERR_NUMERIC: return "NaN or Inf in the input";
    case KNOR_ERR_UNSUPPORTED: return "unsupported by this build";
    case KNOR_ERR_SCRATCH:
      return "request needs more than the fixed scratch of the allocation-free entry point";
  }
  return "unknown status";
}

int32_t knor_version(void) { return 400; }

knor_status knor_fit(const void* X, knor_dtype dt, int64_t n, int32_t d,
                     int32_t k, knor_init init, const double* C_init,
                     int32_t max_iters, double tol, const knor_opts* opts,
                     double* C_out, int32_t* labels_out, knor_stats* st) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  if (!X || !C_out || !labels_out || !dtype_ok(dt)) return KNOR_ERR_INVALID_ARG;
  if (n < 1 || n >= (int64_t)1 << 31 || d < 1 || d > kMaxD || k < 1 ||
      k > kMaxK || (int64_t)k > n || max_iters < 1 || !(tol >= 0.0 && tol < 1.0))
    return KNOR_ERR_INVALID_ARG;
  if (init == KNOR_INIT_GIVEN) {
    if (!C_init) return KNOR_ERR_INVALID_ARG;
  } else if (init != KNOR_INIT_FORGY && init != KNOR_INIT_SHUFFLE_FIRSTK &&
             init != KNOR_INIT_KMEANSPP) {
    return KNOR_ERR_INVALID_ARG;
  }
  if (o.update == 1 && dt == KNOR_F64) return KNOR_ERR_UNSUPPORTED;
  if (o.clause2 == 2 && (o.prune != 1 || dt != KNOR_F32 || k > kCandMaxK))
    return KNOR_ERR_UNSUPPORTED;
  if (o.autotune && dt == KNOR_F32 && !o.tile_blocks && !o.tile_resident) {
    int pb, res;
    if (!tune_lookup(pad_dim(d), (k + 15) / 16 * 16, &pb, &res))
      if (knor_status r = tune_tile((const float*)X, n, d,
                                    init == KNOR_INIT_GIVEN ? C_init : nullptr, k,
                                    o.stream))
        return r;
  }
  return fit_impl(X, dt, n, d, k, init, C_init, max_iters, tol, o, C_out,
                  labels_out, st);
}

// The batched form: independent fits of many problems, run concurrently on
// kBatchStreams streams (the device's hardware queues) by as many host
// threads, largest work (n k d) first.  Each FP32 shape class is tuned once
// (unless the options force a schedule); the results of every problem are
// those of knor_fit on it alone.
constexpr int kBatchStreams = 4;

// The batched form as one graph: every problem is set up on its chain's
// stream, then one capture records each problem's max_iters iterations on
// one of kBatchStreams parallel chains (largest work first, each problem on
// the chain with the least work so far), the graph is launched once, and
// every problem is finished.  A problem's iterations after its convergence
// return at once (its convergence word).
struct GraphRes {
  hipStream_t cs[kBatchStreams] = {};
  hipEvent_t ev[kBatchStreams + 1] = {};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~GraphRes() {
    for (hipStream_t x : cs)
      if (x) (void)hipStreamSynchronize(x);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t x : cs)
      if (x) (void)hipStreamDestroy(x);
    (void)hipGetLastError();
  }
};

static knor_status fit_batched_graph(const knor_problem* probs, int count, const Opts& o,
                                     const std::vector<int>& order, knor_stats* st) {
  GraphRes g;
  for (int w = 0; w < kBatchStreams; ++w)
    HIPCHK(hipStreamCreateWithFlags(&g.cs[w], hipStreamNonBlocking));
  for (hipEvent_t& e : g.ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  // the chains follow everything already on opts->stream
  HIPCHK(hipEventRecord(g.ev[0], o.stream));
  for (hipStream_t x : g.cs) HIPCHK(hipStreamWaitEvent(x, g.ev[0], 0));
  std::vector<int> chain(count, 0);
  double load[kBatchStreams] = {};
  for (int q : order) {
    int w = 0;
    for (int v = 1; v < kBatchStreams; ++v)
      if (load[v] < load[w]) w = v;
    chain[q] = w;
    load[w] += (double)probs[q].n * probs[q].k * probs[q].d * probs[q].max_iters;
  }
  std::vector<std::unique_ptr<FitRun>> runs(count);
  for (int q : order) {
    const knor_problem& p = probs[q];
    runs[q].reset(new FitRun());
    FitRun& r = *runs[q];
    r.X = p.X; r.dt = p.dt; r.n = p.n; r.d = p.d; r.k = p.k;
    r.init = p.C_init ? KNOR_INIT_GIVEN : KNOR_INIT_FORGY;
    r.C_init = p.C_init; r.max_iters = p.max_iters; r.tol = p.tol;
    r.o = o;
    r.o.stream = g.cs[chain[q]];
    r.o.seed = o.seed + (uint64_t)q;
    r.C_out = p.C_out; r.labels_out = p.labels_out; r.st = st ? &st[q] : nullptr;
    if (knor_status e = r.setup()) return e;
  }
  // record: a fork from chain 0, each chain's problems in order, a join
  HIPCHK(hipStreamBeginCapture(g.cs[0], hipStreamCaptureModeRelaxed));
  knor_status rec = KNOR_OK;
  if (hipEventRecord(g.ev[1], g.cs[0]) != hipSuccess) rec = KNOR_ERR_HIP;
  for (int w = 1; w < kBatchStreams && rec == KNOR_OK; ++w)
    if (hipStreamWaitEvent(g.cs[w], g.ev[1], 0) != hipSuccess) rec = KNOR_ERR_HIP;
  for (int w = 0; w < kBatchStreams && rec == KNOR_OK; ++w)
    for (int q : order) {
      if (chain[q] != w || rec != KNOR_OK) continue;
      for (int t = 0; t < probs[q].max_iters && rec == KNOR_OK; ++t)
        rec = runs[q]->iteration(t);
    }
  for (int w = 1; w < kBatchStreams && rec == KNOR_OK; ++w)
    if (hipEventRecord(g.ev[1 + w], g.cs[w]) != hipSuccess ||
        hipStreamWaitEvent(g.cs[0], g.ev[1 + w], 0) != hipSuccess)
      rec = KNOR_ERR_HIP;
  if (hipStreamEndCapture(g.cs[0], &g.graph) != hipSuccess) rec = KNOR_ERR_HIP;
  if (rec != KNOR_OK) {
    (void)hipGetLastError();
    return rec;
  }
  HIPCHK(hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0));
  HIPCHK(hipGraphLaunch(g.exec, g.cs[0]));
  HIPCHK(hipStreamSynchronize(g.cs[0]));
  knor_status first = KNOR_OK;
  for (int q = 0; q < count; ++q) {
    const knor_status e = runs[q]->finish();
    if (e != KNOR_OK && first == KNOR_OK) first = e;
  }
  return first;
}

knor_status knor_fit_batched(const knor_problem* probs, int32_t count,
                             const knor_opts* opts, knor_stats* st) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  if (count < 0 || (count > 0 && !probs)) return KNOR_ERR_INVALID_ARG;
  if (o.label_history || o.iter_counters || o.profile_ms || o.profile_launches ||
      o.centroid_history || o.objective_history)
    return KNOR_ERR_INVALID_ARG;           // per-call arrays: single fits only
  for (int i = 0; i < count; ++i) {
    const knor_problem& p = probs[i];
    if (!p.X || !p.C_out || !p.labels_out || !dtype_ok(p.dt)) return KNOR_ERR_INVALID_ARG;
    if (p.n < 1 || p.n >= (int64_t)1 << 31 || p.d < 1 || p.d > kMaxD || p.k < 1 ||
        p.k > kMaxK || (int64_t)p.k > p.n || p.max_iters < 1 ||
        !(p.tol >= 0.0 && p.tol < 1.0))
      return KNOR_ERR_INVALID_ARG;
  }
  if (o.update == 1)
    for (int i = 0; i < count; ++i)
      if (probs[i].dt == KNOR_F64) return KNOR_ERR_UNSUPPORTED;
  if (o.clause2 == 2)
    for (int i = 0; i < count; ++i)
      if (o.prune != 1 || probs[i].dt != KNOR_F32 || probs[i].k > kCandMaxK)
        return KNOR_ERR_UNSUPPORTED;
  if (count == 0) return KNOR_OK;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  // tune each FP32 class once, on its largest problem
  if (!o.tile_blocks && !o.tile_resident) {
    std::map<std::pair<int, int>, int> rep;
    for (int i = 0; i < count; ++i) {
      const knor_problem& p = probs[i];
      if (p.dt != KNOR_F32) continue;
      const std::pair<int, int> key{pad_dim(p.d), (p.k + 15) / 16 * 16};
      auto it = rep.find(key);
      if (it == rep.end() || probs[it->second].n < p.n) rep[key] = i;
    }
    for (auto& kv : rep) {
      int pb, res;
      if (tune_lookup(kv.first.first, kv.first.second, &pb, &res)) continue;
      const knor_problem& p = probs[kv.second];
      if (knor_status r = tune_tile((const float*)p.X, p.n, p.d, p.C_init, p.k, o.stream))
        return r;
    }
  }
  // work on the worker streams follows everything already on opts->stream
  hipEvent_t ready;
  HIPCHK(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
  if (hipEventRecord(ready, o.stream) != hipSuccess) {
    (void)hipEventDestroy(ready);
    return KNOR_ERR_HIP;
  }
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return probs[a].n * (int64_t)probs[a].k * probs[a].d >
           probs[b].n * (int64_t)probs[b].k * probs[b].d;
  });
  if (o.batch_graph && !o.learned) {
    const knor_status r = fit_batched_graph(probs, count, o, order, st);
    (void)hipEventDestroy(ready);
    return r;
  }
  std::vector<knor_status> res(count, KNOR_OK);
  std::atomic<int> next{0};
  const int nw = count < kBatchStreams ? count : kBatchStreams;
  auto worker = [&]() {
    hipStream_t sw = nullptr;
    if (hipSetDevice(dev) != hipSuccess ||
        hipStreamCreateWithFlags(&sw, hipStreamNonBlocking) != hipSuccess ||
        hipStreamWaitEvent(sw, ready, 0) != hipSuccess) {
      for (int i = next++; i < count; i = next++) res[order[i]] = KNOR_ERR_HIP;
      if (sw) (void)hipStreamDestroy(sw);
      return;
    }
    for (int i = next++; i < count; i = next++) {
      const int q = order[i];
      const knor_problem& p = probs[q];
      Opts oi = o;
      oi.stream = sw;
      oi.seed = o.seed + (uint64_t)q;
      res[q] = fit_impl(p.X, p.dt, p.n, p.d, p.k,
                        p.C_init ? KNOR_INIT_GIVEN : KNOR_INIT_FORGY, p.C_init,
                        p.max_iters, p.tol, oi, p.C_out, p.labels_out,
                        st ? &st[q] : nullptr);
    }
    if (hipStreamSynchronize(sw) != hipSuccess) res[order[0]] = KNOR_ERR_HIP;
    (void)hipStreamDestroy(sw);
  };
  std::vector<std::thread> th;
  for (int w = 0; w < nw; ++w) th.emplace_back(worker);
  for (auto& t : th) t.join();
  (void)hipEventDestroy(ready);
  for (int i = 0; i < count; ++i)
    if (res[i] != KNOR_OK) return res[i];
  return KNOR_OK;
}

// ---------------------------------------------------------------------------
// streamed fit: rows in host memory
// ---------------------------------------------------------------------------

// The row cache's refresh iterations: I, then each gap twice the previous
// one (I, 3I, 7I, 15I, ...).
static bool cache_refresh_at(int t, int I) {
  int64_t r = I, gap = 2 * (int64_t)I;
  while (r < t) {
    r += gap;
    gap *= 2;
  }
  return r == t;
}

// The device's address of page-locked host memory X.
static knor_status host_rows_on_device(const void* X, const void** xd) {
  hipPointerAttribute_t a{};
  if (hipPointerGetAttributes(&a, X) != hipSuccess) {
    (void)hipGetLastError();
    return KNOR_ERR_INVALID_ARG;
  }
  if (a.type != hipMemoryTypeHost) return KNOR_ERR_INVALID_ARG;
  void* p = nullptr;
  if (hipHostGetDevicePointer(&p, const_cast<void*>(X), 0) != hipSuccess || !p) {
    (void)hipGetLastError();
    return KNOR_ERR_INVALID_ARG;
  }
  *xd = p;
  return KNOR_OK;
}

// The transfer stream and its events.  Declared after the workspace, so it
// is drained before the workspace is released.
struct CopyLane {
  hipStream_t cs = nullptr;
  hipEvent_t ready[2] = {nullptr, nullptr}, done[2] = {nullptr, nullptr};
  hipEvent_t start = nullptr;
  hipError_t init() {
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    for (int i = 0; i < 2 && e == hipSuccess; ++i) {
      e = hipEventCreateWithFlags(&ready[i], hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&done[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&start, hipEventDisableTiming);
    return e;
  }
  ~CopyLane() {
    if (cs) (void)hipStreamSynchronize(cs);
    for (hipEvent_t e : {ready[0], ready[1], done[0], done[1], start})
      if (e) (void)hipEventDestroy(e);
    if (cs) (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
  }
};

struct StreamCfg {
  int64_t batch = 0;       // rows per batch (multiple of kSeg)
  int64_t cache = 0;       // cache capacity in rows
  int interval = 5;
  int skip_objective = 0;
  int64_t* io_out = nullptr;
};

// One iteration of the streamed fit visits the batches in order.  Batch b's
// rows go to staging buffer b mod 2 on the transfer stream (a DMA copy of
// the whole batch, or the fetch kernel for the points that fail Clause 1)
// while the compute stream works on batch b - 1 from the other buffer; the
// compute stream then runs the in-memory iteration's kernels on the batch's
// views (filter, tile, recheck, and the exact update's moves).  After the
// last batch: the exact update's division, the cache switch (refresh
// iterations), s(c), and the convergence poll.
static knor_status fit_streamed_impl(const void* X, const void* Xd, knor_dtype dt, int64_t n,
                                     int d, int k, knor_init init, const double* C_init,
                                     int max_iters, double tol, const Opts& o,
                                     const StreamCfg& sc, double* C_out, int32_t* labels_out,
                                     knor_stats* st) {
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = o.stream;
  const int kpad = (k + 15) / 16 * 16;
  const bool mti = o.prune == 1;
  const bool use_cache = mti && sc.cache > 0;
  const size_t rb = (size_t)d * (dt == KNOR_F32 ? 4 : 2);
  const int64_t B = sc.batch;
  const int nsegB = nseg_of_n(B);
  const int nseg = nseg_of_n(n);
  const int nbat = (int)((n + B - 1) / B);
  const bool need_obj = st && !sc.skip_objective;

  CentroidOps ops{};
  ops.k = k; ops.kpad = kpad; ops.d = d; ops.dp = pad_dim(d); ops.dpb = pad_dim_bf16(d);
  ops.C64 = C_out;
  if (knor_status r = select_tile(ops, o)) return r;
  float *u = nullptr, *drift = nullptr, *s_half = nullptr;
  int *list = nullptr, *seg_cnt = nullptr, *flags = nullptr, *ucnt = nullptr;
  int *flagbuf = nullptr, *dirty = nullptr, *nj = nullptr;
  unsigned long long *ctr = nullptr, *io = nullptr;
  int64_t* rows_dev = nullptr;
  void* exact_ws = nullptr;
  void* stage[2] = {nullptr, nullptr};
  void* creg[2] = {nullptr, nullptr};
  int* cpts[2] = {nullptr, nullptr};
  int *pslot = nullptr, *segc = nullptr;
  int64_t *abase = nullptr, *rcnt = nullptr;
  double *dist2 = nullptr, *sumtmp = nullptr, *objective = nullptr;

  Arena ar;
  add_operands(ar, ops, dt);
  ar.add((void**)&ops.CT, sizeof(double) * (size_t)k * d);
  ar.add((void**)&drift, sizeof(float) * (size_t)k);
  ar.add((void**)&s_half, sizeof(float) * (size_t)k);
  ar.add((void**)&dirty, sizeof(int) * (size_t)k);
  ar.add((void**)&nj, sizeof(int) * (size_t)k);
  ar.add((void**)&flags, sizeof(int) * (size_t)flag_capacity(ops, dt, B, nsegB));
  ar.add((void**)&ucnt, sizeof(int) * (size_t)kTileMaxGrid);
  if (mti) {
    ar.add((void**)&u, sizeof(float) * (size_t)n);
    ar.add((void**)&list, sizeof(int) * (size_t)nsegB * kSeg);
    ar.add((void**)&seg_cnt, sizeof(int) * (size_t)nsegB);
  }
  const size_t ctr_bytes = sizeof(unsigned long long) * ROW_STRIDE * (size_t)max_iters;
  const size_t io_bytes = sizeof(unsigned long long) * KNOR_NIO * (size_t)max_iters;
  ar.add((void**)&ctr, ctr_bytes);
  ar.add((void**)&io, io_bytes);
  ar.add((void**)&flagbuf, sizeof(int) * 8);
  ar.add((void**)&rows_dev, sizeof(int64_t) * (size_t)k);
  ar.add(&exact_ws, exact_workspace_bytes(n, k, d));
  for (int i = 0; i < 2; ++i) ar.add(&stage[i], rb * (size_t)B);
  if (use_cache) {
    for (int i = 0; i < 2; ++i) {
      ar.add(&creg[i], rb * (size_t)sc.cache);
      ar.add((void**)&cpts[i], sizeof(int) * (size_t)sc.cache);
    }
    ar.add((void**)&pslot, sizeof(int) * (size_t)n);
    ar.add((void**)&segc, sizeof(int) * (size_t)nseg);
    ar.add((void**)&abase, sizeof(int64_t) * (size_t)(nseg + 1));
    ar.add((void**)&rcnt, sizeof(int64_t) * 2);
  }
  if (need_obj) {
    ar.add((void**)&dist2, sizeof(double) * (size_t)n);
    ar.add((void**)&sumtmp, sizeof(double) * (size_t)(n / kLeaf + 2));
    ar.add((void**)&objective, sizeof(double));
  }
  if (knor_status r = ar.alloc(s, o.cap)) return r;
  ExactPlan xplan{};
  exact_plan_init(&xplan, n, k, d, exact_ws);
  int* conv = flagbuf;
  int* bad = flagbuf + 1;
  HIPCHK(hipMemsetAsync(flagbuf, 0, sizeof(int) * 8, s));
  HIPCHK(launch_fill_i32(conv, 1, kNotConverged, s));
  HIPCHK(hipMemsetAsync(ctr, 0, ctr_bytes, s));
  HIPCHK(hipMemsetAsync(io, 0, io_bytes, s));

  if (init == KNOR_INIT_GIVEN) {
    if (C_init != C_out)
      HIPCHK(hipMemcpyAsync(C_out, C_init, sizeof(double) * (size_t)k * d,
                            hipMemcpyDeviceToDevice, s));
  } else {
    std::vector<int64_t> rows = init == KNOR_INIT_FORGY ? forgy_rows(n, k, o.seed)
                                                        : shuffle_first_k(n, k, o.seed);
    HIPCHK(hipMemcpyAsync(rows_dev, rows.data(), sizeof(int64_t) * k,
                          hipMemcpyHostToDevice, s));
    HIPCHK(launch_gather_rows(Xd, dt, d, rows_dev, k, C_out, s));   // k rows over the link
    HIPCHK(hipStreamSynchronize(s));   // `rows` leaves scope
  }
  // numeric check: the initial centroids now, the rows of X as they arrive
  // in iteration 0 (no pass over the link of its own)
  if (o.check_numeric) {
    HIPCHK(launch_check_finite(C_out, KNOR_F64, (int64_t)k * d, bad, s));
    int hbad = 0;
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hbad) return KNOR_ERR_NUMERIC;
  }
  HIPCHK(launch_prep_centroids(ops, s));
  HIPCHK(launch_fill_i32(labels_out, n, -1, s));
  HIPCHK(launch_fill_i32(dirty, k, 1, s));
  HIPCHK(launch_fill_i32(nj, k, 0, s));
  HIPCHK(launch_fill_i32(xplan.prev, n, -1, s));
  HIPCHK(launch_fill_i32((int32_t*)xplan.slots, (int64_t)k * kXD * d * 2, 0, s));
  if (use_cache) {
    HIPCHK(launch_fill_i32(pslot, n, -1, s));
    HIPCHK(launch_fill_i32((int32_t*)rcnt, 4, 0, s));
  }

  CopyLane cl;
  HIPCHK(cl.init());
  for (hipEvent_t e : cl.done) HIPCHK(hipEventRecord(e, s));   // both buffers free
  // the iteration's moves stay below 2^23 unless n is that large
  const int split = n >= ((int64_t)1 << 23) ? 1 : 0;
  const double tol_n = tol * (double)n;
  std::vector<int64_t> copied((size_t)max_iters, 0);
  int cur = 0;                                   // the cache region in use
  int hconv = kNotConverged;
  int t_last = 0;
  for (int t = 0; t < max_iters; ++t) {
    t_last = t;
    unsigned long long* row = ctr + (size_t)t * ROW_STRIDE;
    unsigned long long* io_t = io + (size_t)t * KNOR_NIO;
    if (o.centroid_history)
      HIPCHK(hipMemcpyAsync(o.centroid_history + (size_t)t * k * d, C_out,
                            sizeof(double) * (size_t)k * d, hipMemcpyDeviceToDevice, s));
    const bool full = !mti || t == 0;
    const bool refresh = use_cache && !full && cache_refresh_at(t, sc.interval);
    // the transfer stream starts after the previous iteration's bounds
    HIPCHK(hipEventRecord(cl.start, s));
    HIPCHK(hipStreamWaitEvent(cl.cs, cl.start, 0));
    if (refresh) {
      StreamFetch f;
      f.Xh = Xd; f.dt = dt; f.n = n; f.d = d; f.labels = labels_out; f.u = u;
      f.drift = drift; f.s_half = s_half; f.seg_count = segc; f.io = io_t;
      f.conv = conv; f.iter = t;
      HIPCHK(launch_stream_fetch(f, cl.cs));
      HIPCHK(launch_stream_scan(segc, nseg, abase, conv, t, cl.cs));
    }
    for (int b = 0; b < nbat; ++b) {
      const int64_t r0 = (int64_t)b * B;
      const int64_t nb = n - r0 < B ? n - r0 : B;
      const int nsb = nseg_of_n(nb);
      const int buf = b & 1;
      HIPCHK(hipStreamWaitEvent(cl.cs, cl.done[buf], 0));
      if (full) {
        HIPCHK(hipMemcpyAsync(stage[buf], (const char*)X + (size_t)r0 * rb, (size_t)nb * rb,
                              hipMemcpyHostToDevice, cl.cs));
        copied[(size_t)t] += nb;
      } else {
        StreamFetch f;
        f.Xh = (const char*)Xd + (size_t)r0 * rb; f.dt = dt; f.n = nb; f.d = d;
        f.labels = labels_out + r0; f.u = u + r0; f.drift = drift; f.s_half = s_half;
        if (use_cache) {
          f.pslot = pslot + r0;
          f.cache = creg[cur];
          if (refresh) {
            f.adm_rows = creg[cur ^ 1];
            f.adm_pts = cpts[cur ^ 1];
            f.adm_base = abase + r0 / kSeg;
            f.adm_cap = sc.cache;
            f.gid0 = r0;
          }
        }
        f.stage = stage[buf]; f.io = io_t; f.conv = conv; f.iter = t;
        HIPCHK(launch_stream_fetch(f, cl.cs));
      }
      HIPCHK(hipEventRecord(cl.ready[buf], cl.cs));
      HIPCHK(hipStreamWaitEvent(s, cl.ready[buf], 0));
      // a non-finite value stops every later kernel of the fit
      if (t == 0 && o.check_numeric)
        HIPCHK(launch_check_finite(stage[buf], dt, nb * (int64_t)d, bad, s, conv));
      AssignJob job{};
      job.X = stage[buf]; job.dt = dt; job.n = nb; job.d = d;
      job.labels = labels_out + r0; job.u = mti ? u + r0 : nullptr;
      job.flags = flags; job.row = row; job.conv = conv; job.iter = t;
      job.ucnt = ucnt; job.dirty = dirty; job.recheck_all = o.recheck == 2;
      if (!full) {
        HIPCHK(launch_mti_filter(stage[buf], dt, nb, d, C_out, labels_out + r0, u + r0, drift,
                                 s_half, list, seg_cnt, row - ROW_STRIDE, row, conv, t, 0, s));
        job.list = list;
        job.seg_cnt = seg_cnt;
        job.nseg = nsb;
      }
      HIPCHK(launch_assign(ops, job, s));
      HIPCHK(launch_recheck(ops, job, s));
      HIPCHK(launch_exact_enter(xplan, nj, stage[buf], dt, nb, full ? nullptr : list,
                                full ? nullptr : seg_cnt, full ? 0 : nsb, labels_out + r0,
                                xplan.prev + r0, dirty, row, conv, t, split, s));
      HIPCHK(hipEventRecord(cl.done[buf], s));
    }
    IterCtl ctl;
    ctl.row = row; ctl.conv = conv; ctl.iter = t; ctl.tol_n = tol_n;
    ctl.segmented = full ? 0 : 1; ctl.n = n;
    HIPCHK(launch_exact_finalize(xplan, nj, C_out, C_out, nullptr, &ops, mti ? drift : nullptr,
                                 dirty, ctl, s));
    if (refresh) {
      HIPCHK(launch_stream_remap(pslot, cpts[cur], rcnt + cur, cpts[cur ^ 1], abase + nseg,
                                 sc.cache, rcnt + (cur ^ 1), conv, t, s));
      cur ^= 1;
    }
    if (mti) HIPCHK(launch_cc_bounds(ops, s_half, nullptr, conv, t, s));
    if (o.label_history)
      HIPCHK(launch_copy_i32(labels_out, o.label_history + (size_t)t * n, n, conv, t, s));
    int hbad = 0;
    HIPCHK(hipMemcpyAsync(&hconv, conv, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hbad) return KNOR_ERR_NUMERIC;
    if (hconv != kNotConverged) break;
  }

  // final objective: one more pass over the rows
  double hobj = 0.0;
  if (need_obj) {
    HIPCHK(hipEventRecord(cl.start, s));
    HIPCHK(hipStreamWaitEvent(cl.cs, cl.start, 0));
    for (int b = 0; b < nbat; ++b) {
      const int64_t r0 = (int64_t)b * B;
      const int64_t nb = n - r0 < B ? n - r0 : B;
      const int buf = b & 1;
      HIPCHK(hipStreamWaitEvent(cl.cs, cl.done[buf], 0));
      HIPCHK(hipMemcpyAsync(stage[buf], (const char*)X + (size_t)r0 * rb, (size_t)nb * rb,
                            hipMemcpyHostToDevice, cl.cs));
      HIPCHK(hipEventRecord(cl.ready[buf], cl.cs));
      HIPCHK(hipStreamWaitEvent(s, cl.ready[buf], 0));
      HIPCHK(launch_exact_dist2(stage[buf], dt, nb, d, C_out, labels_out + r0, dist2 + r0, s));
      HIPCHK(hipEventRecord(cl.done[buf], s));
    }
    copied[(size_t)t_last] += n;
    HIPCHK(launch_canonical_sum(dist2, n, sumtmp, objective, s));
    HIPCHK(hipMemcpyAsync(&hobj, objective, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  std::vector<unsigned long long> hc((size_t)ROW_STRIDE * max_iters);
  std::vector<unsigned long long> hio((size_t)KNOR_NIO * max_iters);
  HIPCHK(hipMemcpyAsync(&hconv, conv, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hc.data(), ctr, ctr_bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(hio.data(), io, io_bytes, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const int converged = hconv != kNotConverged;
  const int hiters = converged ? hconv + 1 : max_iters;
  if (sc.io_out)
    for (int i = 0; i < hiters; ++i) {
      int64_t* dst = sc.io_out + (size_t)i * KNOR_NIO;
      const unsigned long long* r = &hio[(size_t)i * KNOR_NIO];
      dst[KNOR_IO_COPIED] = copied[(size_t)i];
      dst[KNOR_IO_GATHERED] = (int64_t)r[1];
      dst[KNOR_IO_CACHED] = (int64_t)r[2];
      dst[KNOR_IO_ADMITTED] = (int64_t)r[3];
    }
  std::vector<char> cand_used((size_t)max_iters, 0), proposed((size_t)max_iters, 0);
  std::vector<int64_t> forwarded((size_t)max_iters, 0);
  report_counters(hc, hiters, n, k, mti, cand_used, proposed, forwarded, o.iter_counters, st);
  if (st) {
    st->converged = converged;
    st->objective = hobj;
    st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  return KNOR_OK;
}

knor_status knor_fit_streamed(const void* X, knor_dtype dt, int64_t n, int32_t d, int32_t k,
                              knor_init init, const double* C_init, int32_t max_iters,
                              double tol, const knor_opts* opts, const knor_stream_opts* sopts,
                              double* C_out, int32_t* labels_out, knor_stats* st) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  if (!X || !C_out || !labels_out || (dt != KNOR_F32 && dt != KNOR_BF16))
    return KNOR_ERR_INVALID_ARG;
  if (n < 1 || n >= (int64_t)1 << 31 || d < 1 || d > kMaxD || k < 1 || k > kMaxK ||
      (int64_t)k > n || max_iters < 1 || !(tol >= 0.0 && tol < 1.0))
    return KNOR_ERR_INVALID_ARG;
  if (init == KNOR_INIT_GIVEN) {
    if (!C_init) return KNOR_ERR_INVALID_ARG;
  } else if (init != KNOR_INIT_FORGY && init != KNOR_INIT_SHUFFLE_FIRSTK &&
             init != KNOR_INIT_KMEANSPP) {
    return KNOR_ERR_INVALID_ARG;
  }
  StreamCfg sc;
  if (sopts && sopts->struct_size != 0) {
    if (sopts->struct_size != sizeof(knor_stream_opts)) return KNOR_ERR_INVALID_ARG;
    if (sopts->batch_rows < 0 || sopts->cache_rows < 0 || sopts->cache_interval < 0 ||
        sopts->skip_objective < 0 || sopts->skip_objective > 1)
      return KNOR_ERR_INVALID_ARG;
    sc.batch = sopts->batch_rows;
    sc.cache = sopts->cache_rows;
    if (sopts->cache_interval > 0) sc.interval = sopts->cache_interval;
    sc.skip_objective = sopts->skip_objective;
    sc.io_out = sopts->io_counters;
  }
  const int64_t nr = (n + kSeg - 1) / kSeg * kSeg;
  if (sc.batch == 0) sc.batch = (int64_t)1 << 22;
  sc.batch = (sc.batch + kSeg - 1) / kSeg * kSeg;
  if (sc.batch > nr) sc.batch = nr;
  if (sc.cache > n) sc.cache = n;
  if (o.update != 1 || o.learned || o.clause2 == 2 || o.autotune ||
      init == KNOR_INIT_KMEANSPP || o.profile_ms || o.profile_launches ||
      o.objective_history)
    return KNOR_ERR_UNSUPPORTED;
  const void* Xd = nullptr;
  if (knor_status r = host_rows_on_device(X, &Xd)) return r;
  return fit_streamed_impl(X, Xd, dt, n, d, k, init, C_init, max_iters, tol, o, sc, C_out,
                           labels_out, st);
}

knor_status knor_assign(const void* X, knor_dtype dt, int64_t n, int32_t d,
                        const double* C, int32_t k, const knor_opts* opts,
                        int32_t* labels_out, double* dist2_out) {
  return knor::assign_impl(X, dt, n, d, C, k, opts, labels_out, dist2_out, nullptr, 0);
}

knor_status knor_assign_noalloc(const void* X, knor_dtype dt, int64_t n, int32_t d,
                                const double* C, int32_t k, const knor_opts* opts,
                                int32_t* labels_out, double* dist2_out) {
  // validation first: an invalid call touches neither the device nor scratch
  if (knor_status r = knor::assign_impl(X, dt, n, d, C, k, opts, labels_out, dist2_out,
                                        nullptr, (size_t)-1))
    return r;
  if (n == 0) return KNOR_OK;
  void* mem = nullptr;
  if (knor_status r = knor::scratch_of_device(&mem)) return r;
  return knor::assign_impl(X, dt, n, d, C, k, opts, labels_out, dist2_out, mem,
                           knor::kScratchBytes);
}

knor_status knor_tile_values(const void* X, knor_dtype dt, int64_t n, int32_t d,
                             const double* C, int32_t k, const knor_opts* opts, float* Y,
                             double* E) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  if ((n > 0 && (!X || !Y || !E)) || !C || !dtype_ok(dt)) return KNOR_ERR_INVALID_ARG;
  if (n < 0 || n >= (int64_t)1 << 31 || d < 1 || d > kMaxD || k < 1 || k > kMaxK)
    return KNOR_ERR_INVALID_ARG;
  if (dt == KNOR_F64) return KNOR_ERR_UNSUPPORTED;    // FP64 points use no tile
  if (n == 0) return KNOR_OK;
  hipStream_t s = o.stream;
  CentroidOps ops{};
  ops.k = k; ops.kpad = (k + 15) / 16 * 16; ops.d = d; ops.dp = pad_dim(d);
  ops.dpb = pad_dim_bf16(d);
  ops.C64 = const_cast<double*>(C);
  Arena ar;
  add_operands(ar, ops, dt);
  if (knor_status r = ar.alloc(s, o.cap)) return r;
  HIPCHK(launch_prep_centroids(ops, s));
  if (dt == KNOR_F32)
    HIPCHK(launch_tile_values_f32(ops, (const float*)X, n, d, Y, E, s));
  else
    HIPCHK(launch_tile_values_bf16(ops, (const uint16_t*)X, n, d, Y, E, s));
  return KNOR_OK;
}

knor_status knor_update(const void* X, knor_dtype dt, int64_t n, int32_t d,
                        const int32_t* labels, int32_t k, const double* C_prev,
                        const knor_opts* opts, double* C_out,
                        int64_t* counts_out) {
  Opts o;
  if (knor_status r = read_opts(opts, &o)) return r;
  // X and labels may be NULL when n == 0
  if ((n > 0 && (!X || !labels)) || !C_prev || !C_out || !dtype_ok(dt))
    return KNOR_ERR_INVALID_ARG;
  if (n < 0 || n >= (int64_t)1 << 31 || d < 1 || d > kMaxD || k < 1 || k > kMaxK)
    return KNOR_ERR_INVALID_ARG;
  if (o.update == 1 && dt == KNOR_F64) return KNOR_ERR_UNSUPPORTED;
  hipStream_t s = o.stream;
  if (n == 0) {
    if (C_out != C_prev)
      HIPCHK(hipMemcpyAsync(C_out, C_prev, sizeof(double) * (size_t)k * d,
                            hipMemcpyDeviceToDevice, s));
    if (counts_out) HIPCHK(hipMemsetAsync(counts_out, 0, sizeof(int64_t) * k, s));
    return KNOR_OK;
  }
  void* ws = nullptr;
  void* xws = nullptr;
  int* conv = nullptr;
  const bool exact = o.update == 1;
  Arena ar;
  ar.add(&ws, update_workspace_bytes(n, k, d));
  if (exact) ar.add(&xws, exact_workspace_bytes(n, k, d));
  ar.add((void**)&conv, sizeof(int) * 4);
  if (knor_status r = ar.alloc(s, o.cap)) return r;
  UpdatePlan plan{};
  update_plan_init(&plan, n, k, d, ws);
  HIPCHK(update_plan_reset(plan, s));
  HIPCHK(launch_fill_i32(conv, 1, kNotConverged, s));
  IterCtl ctl;
  ctl.conv = conv;
  if (exact) {
    ExactPlan xplan{};
    exact_plan_init(&xplan, n, k, d, xws);
    HIPCHK(launch_update_exact(plan, xplan, X, dt, labels, C_prev, C_out, counts_out, nullptr,
                               nullptr, nullptr, &ctl, s));
  } else {
    HIPCHK(launch_update(plan, X, dt, labels, C_prev, C_out, counts_out, nullptr,
                         nullptr, nullptr, &ctl, s));
  }
  return KNOR_OK;
}

}  // extern "C"
