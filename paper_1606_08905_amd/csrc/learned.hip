// Learned candidate proposal for the assignment step.
//
// An MLP d -> h -> h -> k (ReLU hidden layers) maps a standardized point to
// k logits, one per centroid.  On the points that survive MTI pruning
// (Mhembere et al., HPDC'17, Section "Minimal Triangle Inequality (MTI)
// Pruning"), it proposes 16 candidate centroids; the nearest candidate c*
// (FP64 canonical distances, lowest index on ties) is accepted only under
// the certificate d(x, c*) (1 + eta) < 1/2 min_{j not a candidate} d(c*, j)
// (which contains the paper-style test against s(c*) = 1/2 min_{j != c*}
// d(c*, j) as a special case): every non-candidate is then farther than c*
// by a relative gap of about 2 eta, and the candidates are compared in the
// FP64 definition itself, so c* is its argmin.  Points without a
// certificate go through the full distance tile.  The network therefore never changes a
// label; it only decides which points skip the k-way scan.
//
// Every matrix product runs on v_mfma_f32_16x16x32_bf16: operands are FP32
// in memory and rounded to BF16 (nearest even) when staged into LDS, sums
// are FP32.  Training (softmax cross-entropy, Adam) uses FP32 master
// weights; gradients of the biases, softmax and Adam are FP32.
//
// Proposal rule: the 16 classes with the largest keys, where a class's key
// is its FP32 logit with the low mantissa bits replaced by a code of the
// class index (value and class in one sortable float).  Each lane of the
// output tile keeps the largest keys of its share of the point's classes in
// a sorted list (median-of-three insertion), and the four lanes of a point
// merge their lists through LDS.
#include <math.h>

#include <vector>

#include "common.h"

namespace knor {

typedef float f4l __attribute__((ext_vector_type(4)));
typedef __bf16 bf8l __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f32_bf16_rne(float f) {
  uint32_t b = __float_as_uint(f);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}

// Two values rounded to BF16 (nearest, ties to even, as f32_bf16_rne for
// finite values) by one v_cvt_pk_bf16_f32: a in the low half, b in the high.
typedef float f2l __attribute__((ext_vector_type(2)));
typedef __bf16 bf2l __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t bf16_pair(float a, float b) {
  const f2l v = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf2l));
}

// ---------------------------------------------------------------------------
// generic GEMM: C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]) (ReLU)
// (masked by mask > 0); op = transpose when the flag is set
// ---------------------------------------------------------------------------
//
// A workgroup of 4 waves computes a 128 x 128 tile of C, each wave 64 x 64
// (4 x 4 blocks of v_mfma_f32_16x16x32_bf16).  Per K-step of 32 the
// operands are read from global memory as 16-byte FP32 pieces along their
// contiguous dimension, rounded to BF16 and stored in LDS with K
// contiguous (both operands), double-buffered: the next step's pieces are
// loaded into registers while the current step's MFMAs run, one barrier per
// step.  Long K with few output tiles is split over blockIdx.z; the splits
// write FP32 partial tiles and a second kernel adds them in split order and
// applies the epilogue, so the result does not depend on scheduling.

constexpr int kGT = 128;           // output tile rows and columns
constexpr int kGK = 32;            // K-step (one MFMA K-block)
constexpr int kGLD = kGK + 8;      // LDS row stride (bf16), 16-byte aligned
constexpr int kGTargetWG = 1024;   // split K until about this many workgroups
constexpr int kGMaxSplit = 32;

// The K range of split z of ksplit (multiples of kGK).
__device__ __forceinline__ void split_range(int K, int ksplit, int z, int& kb, int& ke) {
  const int steps = (K + kGK - 1) / kGK;
  const int per = (steps + ksplit - 1) / ksplit;
  kb = z * per * kGK;
  ke = (z + 1) * per * kGK < K ? (z + 1) * per * kGK : K;
}

// four consecutive elements p[0..3] that lie in [0, lim): one 16-byte load
// when all do and p is 16-byte aligned, else element by element (zeros past
// the limit)
__device__ __forceinline__ float4 load4(const float* p, int lim, bool vec) {
  if (vec && lim >= 4) return *reinterpret_cast<const float4*>(p);
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (lim > 0) v.x = p[0];
  if (lim > 1) v.y = p[1];
  if (lim > 2) v.z = p[2];
  if (lim > 3) v.w = p[3];
  return v;
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g, int ksplit,
                                                        float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[2][kGT * kGLD];
  __shared__ __attribute__((aligned(16))) uint16_t sB[2][kGT * kGLD];
  const int M = g.Mdev ? (g.M < *g.Mdev ? g.M : *g.Mdev) : g.M;
  const int N = g.N, K = g.K;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  if (m0 >= M) return;
  int kb, ke;
  split_range(K, ksplit, blockIdx.z, kb, ke);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, col = lane & 15, grp = lane >> 4;
  const bool va = (g.lda & 3) == 0 && ((uintptr_t)g.A & 15) == 0;
  const bool vb = (g.ldb & 3) == 0 && ((uintptr_t)g.B & 15) == 0;
  // piece i of this thread: f = tid + 256 i.  Along K (A plain, B
  // transposed): row f / (kGK / 4), K offset 4 (f mod (kGK / 4)).  Along M
  // or N (A transposed, B plain), with l = f mod 64 and w = f / 64: K offset
  // 8 (w mod 4) + l mod 8, rows or columns 4 (8 (w / 4) + l / 8).  A wave's
  // load then reads 128 contiguous bytes in each of 8 K rows, and its
  // 16-bit stores into the K-contiguous LDS rows spread over 8 banks (rows 4
  // apart, as 32 consecutive lanes would take, all fall on 2 banks).
  constexpr int NP = kGT * kGK / 4 / 256;     // 16-byte pieces per operand per thread
  constexpr int QK = kGK / 4, QS = QK == 16 ? 4 : 3;
  static_assert(kGK == 32 && kGT == 128, "the transposed piece layout covers 32 x 128");
  auto tpiece = [](int f, int& kk, int& r) {
    const int l = f & 63, w = f >> 6;
    kk = 8 * (w & 3) + (l & 7);
    r = 4 * (8 * (w >> 2) + (l >> 3));
  };
  float4 ra[NP], rb[NP];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int f = tid + 256 * i;
      if (!TA) {
        const int r = f >> QS, kk = 4 * (f & (QK - 1));
        const int row = m0 + r, kx = k0 + kk;
        ra[i] = row < M ? load4(g.A + (size_t)row * g.lda + kx, ke - kx, va)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        int kk, r;
        tpiece(f, kk, r);
        const int row = m0 + r, kx = k0 + kk;
        ra[i] = kx < ke ? load4(g.A + (size_t)kx * g.lda + row, M - row, va)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
      }
      if (TB) {
        const int c = f >> QS, kk = 4 * (f & (QK - 1));
        const int cn = n0 + c, kx = k0 + kk;
        rb[i] = cn < N ? load4(g.B + (size_t)cn * g.ldb + kx, ke - kx, vb)
                       : make_float4(0.f, 0.f, 0.f, 0.f);
      } else {
        int kk, c;
        tpiece(f, kk, c);
        const int cn = n0 + c, kx = k0 + kk;
        rb[i] = kx < ke ? load4(g.B + (size_t)kx * g.ldb + cn, N - cn, vb)
                        : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
  };
  auto store = [&](int buf) {
    uint16_t* a = sA[buf];
    uint16_t* b = sB[buf];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int f = tid + 256 * i;
      const uint32_t x01 = bf16_pair(ra[i].x, ra[i].y), x23 = bf16_pair(ra[i].z, ra[i].w);
      if (!TA) {
        const int r = f >> QS, kk = 4 * (f & (QK - 1));
        *reinterpret_cast<uint2*>(&a[r * kGLD + kk]) = make_uint2(x01, x23);
      } else {
        int kk, r;
        tpiece(f, kk, r);
        a[(r + 0) * kGLD + kk] = (uint16_t)x01;
        a[(r + 1) * kGLD + kk] = (uint16_t)(x01 >> 16);
        a[(r + 2) * kGLD + kk] = (uint16_t)x23;
        a[(r + 3) * kGLD + kk] = (uint16_t)(x23 >> 16);
      }
      const uint32_t y01 = bf16_pair(rb[i].x, rb[i].y), y23 = bf16_pair(rb[i].z, rb[i].w);
      if (TB) {
        const int c = f >> QS, kk = 4 * (f & (QK - 1));
        *reinterpret_cast<uint2*>(&b[c * kGLD + kk]) = make_uint2(y01, y23);
      } else {
        int kk, c;
        tpiece(f, kk, c);
        b[(c + 0) * kGLD + kk] = (uint16_t)y01;
        b[(c + 1) * kGLD + kk] = (uint16_t)(y01 >> 16);
        b[(c + 2) * kGLD + kk] = (uint16_t)y23;
        b[(c + 3) * kGLD + kk] = (uint16_t)(y23 >> 16);
      }
    }
  };
  f4l acc[4][4];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y) acc[x][y] = f4l{0.f, 0.f, 0.f, 0.f};
  int buf = 0;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  for (int k0 = kb; k0 < ke; k0 += kGK) {
    const bool more = k0 + kGK < ke;
    if (more) load(k0 + kGK);                  // in flight during the MFMAs
#pragma unroll
    for (int kq = 0; kq < kGK; kq += 32) {
      bf8l av[4], bv[4];
#pragma unroll
      for (int x = 0; x < 4; ++x)
        av[x] = *reinterpret_cast<const bf8l*>(
            &sA[buf][(wr * 64 + x * 16 + col) * kGLD + kq + grp * 8]);
#pragma unroll
      for (int y = 0; y < 4; ++y)
        bv[y] = *reinterpret_cast<const bf8l*>(
            &sB[buf][(wc * 64 + y * 16 + col) * kGLD + kq + grp * 8]);
#pragma unroll
      for (int x = 0; x < 4; ++x)
#pragma unroll
        for (int y = 0; y < 4; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[x], bv[y], acc[x][y], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  float* out = ksplit > 1 ? part + (size_t)blockIdx.z * g.M * N : nullptr;
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 4; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * 64 + x * 16 + 4 * grp + r;
        const int cn = n0 + wc * 64 + y * 16 + col;
        if (row < M && cn < N) {
          float v = acc[x][y][r];
          if (out) {
            out[(size_t)row * N + cn] = v;
          } else {
            if (g.bias) v += g.bias[cn];
            if (g.relu) v = v > 0.0f ? v : 0.0f;
            if (g.mask) v = g.mask[(size_t)row * g.ldm + cn] > 0.0f ? v : 0.0f;
            g.C[(size_t)row * g.ldc + cn] = v;
          }
        }
      }
}

// The split partials added in split order, then the epilogue.
__global__ __launch_bounds__(256) void gemm_split_sum_kernel(GemmArgs g, int ksplit,
                                                             const float* __restrict__ part) {
  const int M = g.Mdev ? (g.M < *g.Mdev ? g.M : *g.Mdev) : g.M;
  const int64_t MN = (int64_t)M * g.N, stride = (int64_t)g.M * g.N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < MN;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int row = (int)(e / g.N), cn = (int)(e - (int64_t)row * g.N);
    float v = 0.0f;
    for (int z = 0; z < ksplit; ++z) v += part[(size_t)z * stride + e];
    if (g.bias) v += g.bias[cn];
    if (g.relu) v = v > 0.0f ? v : 0.0f;
    if (g.mask) v = g.mask[(size_t)row * g.ldm + cn] > 0.0f ? v : 0.0f;
    g.C[(size_t)row * g.ldc + cn] = v;
  }
}

// Splits of K for an M x N x K product: enough workgroups to fill the chip
// when the output has few tiles, each split at least 64 deep.
static int gemm_splits(int M, int N, int K) {
  const int tiles = ((M + kGT - 1) / kGT) * ((N + kGT - 1) / kGT);
  int sp = (kGTargetWG + tiles - 1) / tiles;
  const int kmax = K / 64 > 1 ? K / 64 : 1;
  if (sp > kmax) sp = kmax;
  if (sp > kGMaxSplit) sp = kGMaxSplit;
  return sp < 1 ? 1 : sp;
}

size_t gemm_split_floats(int M, int N, int K) {
  const int sp = gemm_splits(M, N, K);
  return sp > 1 ? (size_t)sp * M * N : 0;
}

hipError_t launch_gemm_bf16(const GemmArgs& g, float* part, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  const int sp = part ? gemm_splits(g.M, g.N, g.K) : 1;
  dim3 grid((g.N + kGT - 1) / kGT, (g.M + kGT - 1) / kGT, sp);
  if (g.transA && g.transB)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, true>), grid, dim3(256), 0, s, g, sp, part);
  else if (g.transA)
    hipLaunchKernelGGL((gemm_bf16_kernel<true, false>), grid, dim3(256), 0, s, g, sp, part);
  else if (g.transB)
    hipLaunchKernelGGL((gemm_bf16_kernel<false, true>), grid, dim3(256), 0, s, g, sp, part);
  else
    hipLaunchKernelGGL((gemm_bf16_kernel<false, false>), grid, dim3(256), 0, s, g, sp, part);
  if (sp > 1) {
    const int64_t mn = (int64_t)g.M * g.N;
    int64_t blocks = (mn + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(gemm_split_sum_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, sp,
                       part);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training pieces
// ---------------------------------------------------------------------------

// One workgroup per row b of Z (B x k): loss_row[b] = logsumexp(z) - z[y],
// and dZ = (softmax(z) - onehot(y)) / B in place.  Thread t takes the
// entries t, t + 256, ...; up to kSoftRegs of them stay in registers
// (with their exponentials) between the passes, the rest are read again.
constexpr int kSoftRegs = 16;

__global__ __launch_bounds__(256) void softmax_ce_kernel(float* __restrict__ Z,
                                                         int k,
                                                         const int32_t* __restrict__ y,
                                                         float invB,
                                                         double* __restrict__ loss_row) {
  __shared__ float red[256];
  float* z = Z + (size_t)blockIdx.x * k;
  float v[kSoftRegs];
#pragma unroll
  for (int q = 0; q < kSoftRegs; ++q) {
    const int j = threadIdx.x + 256 * q;
    v[q] = j < k ? z[j] : -INFINITY;
  }
  float mx = -INFINITY;
#pragma unroll
  for (int q = 0; q < kSoftRegs; ++q)
    if (threadIdx.x + 256 * q < k) mx = fmaxf(mx, v[q]);
  for (int j = threadIdx.x + 256 * kSoftRegs; j < k; j += 256) mx = fmaxf(mx, z[j]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  __syncthreads();
  float sum = 0.0f;
#pragma unroll
  for (int q = 0; q < kSoftRegs; ++q)
    if (threadIdx.x + 256 * q < k) {
      v[q] = expf(v[q] - mx);
      sum += v[q];
    }
  for (int j = threadIdx.x + 256 * kSoftRegs; j < k; j += 256) sum += expf(z[j] - mx);
  red[threadIdx.x] = sum;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  sum = red[0];
  const int yb = y[blockIdx.x];
  if (threadIdx.x == 0) loss_row[blockIdx.x] = (double)logf(sum) + (double)mx - (double)z[yb];
  __syncthreads();
  const float inv = 1.0f / sum;
#pragma unroll
  for (int q = 0; q < kSoftRegs; ++q) {
    const int j = threadIdx.x + 256 * q;
    if (j < k) z[j] = (v[q] * inv - (j == yb ? 1.0f : 0.0f)) * invB;
  }
  for (int j = threadIdx.x + 256 * kSoftRegs; j < k; j += 256) {
    const float p = expf(z[j] - mx) * inv;
    z[j] = (p - (j == yb ? 1.0f : 0.0f)) * invB;
  }
}

// out[c] = sum over rows of D[r][c] (FP32) in two stages: workgroup (cb, rb)
// sums rows rb, rb + kColRB, ... of 64 columns (four row lanes, added in a
// fixed order) into part[rb][c]; the kColRB partial sums of a column are
// then added in order.
constexpr int kColRB = 32;

__global__ __launch_bounds__(256) void colsum_part_kernel(const float* __restrict__ D,
                                                          int rows, int cols,
                                                          float* __restrict__ part) {
  __shared__ float red[4][64];
  const int cl = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl, rb = blockIdx.y;
  float s = 0.0f;
  if (c < cols)
    for (int r = rb + kColRB * q; r < rows; r += 4 * kColRB) s += D[(size_t)r * cols + c];
  red[q][cl] = s;
  __syncthreads();
  if (q == 0 && c < cols)
    part[(size_t)rb * cols + c] = (red[0][cl] + red[1][cl]) + (red[2][cl] + red[3][cl]);
}

__global__ __launch_bounds__(256) void colsum_final_kernel(const float* __restrict__ part,
                                                           int cols, float* __restrict__ out) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= cols) return;
  float s = 0.0f;
  for (int rb = 0; rb < kColRB; ++rb) s += part[(size_t)rb * cols + c];
  out[c] = s;
}

static void launch_colsum(const float* D, int rows, int cols, float* part, float* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(colsum_part_kernel, dim3((cols + 63) / 64, kColRB), dim3(256), 0, s, D,
                     rows, cols, part);
  hipLaunchKernelGGL(colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, s, part, cols,
                     out);
}

__global__ __launch_bounds__(256) void mean_kernel(const double* __restrict__ v, int n,
                                                   double* __restrict__ out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) s += v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / (double)n;
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ th,
                                                   float* __restrict__ m,
                                                   float* __restrict__ v,
                                                   const float* __restrict__ g,
                                                   int64_t P, float lr, float c1,
                                                   float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + 1e-8f);
}

// ---------------------------------------------------------------------------
// parameter layout and host-side pieces
// ---------------------------------------------------------------------------

MlpLayout mlp_layout(int d, int h, int k) {
  MlpLayout L{};
  L.d = d; L.h = h; L.k = k;
  L.W1 = 0;
  L.b1 = L.W1 + (int64_t)d * h;
  L.W2 = L.b1 + h;
  L.b2 = L.W2 + (int64_t)h * h;
  L.W3 = L.b2 + h;
  L.b3 = L.W3 + (int64_t)h * k;
  L.P = L.b3 + k;
  return L;
}

// He-uniform weights from one SplitMix64 stream, in parameter order; zero
// biases.  u = (z >> 11) 2^-53, W = (2u - 1) sqrt(6 / fan_in) in FP64, then
// rounded to FP32.
std::vector<float> mlp_init_host(int d, int h, int k, uint64_t seed) {
  const MlpLayout L = mlp_layout(d, h, k);
  std::vector<float> th((size_t)L.P, 0.0f);
  uint64_t st = seed;
  auto next = [&]() {
    uint64_t z = (st += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  };
  const struct { int64_t off, cnt; int fan; } W[3] = {
      {L.W1, (int64_t)d * h, d}, {L.W2, (int64_t)h * h, h}, {L.W3, (int64_t)h * k, h}};
  for (const auto& w : W) {
    const double a = sqrt(6.0 / (double)w.fan);
    for (int64_t i = 0; i < w.cnt; ++i) {
      const double u = (double)(next() >> 11) * 0x1p-53;
      th[(size_t)(w.off + i)] = (float)((2.0 * u - 1.0) * a);
    }
  }
  return th;
}

// split-K partials of the training products (the largest of them)
static size_t train_split_floats(int d, int h, int k, int B) {
  const size_t c[] = {gemm_split_floats(h, k, B), gemm_split_floats(B, h, k),
                      gemm_split_floats(h, h, B), gemm_split_floats(d, h, B),
                      gemm_split_floats(B, h, h), gemm_split_floats(B, k, h),
                      gemm_split_floats(B, h, d)};
  size_t m = 0;
  for (size_t v : c) m = v > m ? v : m;
  return m;
}

size_t mlp_train_workspace(int d, int h, int k, int B) {
  return sizeof(float) * ((size_t)B * h * 4 + (size_t)B * k) + sizeof(double) * ((size_t)B + 1) +
         sizeof(float) * (size_t)kColRB * (k > h ? k : h) +
         sizeof(float) * train_split_floats(d, h, k, B) + 8192;
}

// One minibatch: forward, softmax cross-entropy, backward into grad, Adam
// (when lr > 0).  ws: mlp_train_workspace bytes.
hipError_t mlp_train_step(float* th, float* am, float* av, int64_t step,
                          const MlpLayout& L, const float* Xs, const int32_t* y,
                          int B, float lr, float* grad, void* ws, double* loss_dev,
                          hipStream_t s) {
  const int d = L.d, h = L.h, k = L.k;
  char* c = (char*)ws;
  float* H1 = (float*)c; c += sizeof(float) * (size_t)B * h;
  float* H2 = (float*)c; c += sizeof(float) * (size_t)B * h;
  float* D2 = (float*)c; c += sizeof(float) * (size_t)B * h;
  float* D1 = (float*)c; c += sizeof(float) * (size_t)B * h;
  float* Z = (float*)c; c += sizeof(float) * (size_t)B * k;
  double* lrow = (double*)c; c += sizeof(double) * ((size_t)B + 1);
  c = (char*)(((uintptr_t)c + 255) & ~(uintptr_t)255);
  float* cpart = (float*)c;
  c += sizeof(float) * (size_t)kColRB * (k > h ? k : h);
  c = (char*)(((uintptr_t)c + 255) & ~(uintptr_t)255);
  float* gpart = train_split_floats(d, h, k, B) ? (float*)c : nullptr;
  hipError_t e;
  auto gemm = [&](const float* A, int lda, int tA, const float* Bm, int ldb, int tB,
                  float* C, int ldc, int M, int N, int K, const float* bias, int relu,
                  const float* mask, int ldm) {
    GemmArgs g{};
    g.A = A; g.lda = lda; g.transA = tA; g.B = Bm; g.ldb = ldb; g.transB = tB;
    g.C = C; g.ldc = ldc; g.M = M; g.N = N; g.K = K; g.bias = bias; g.relu = relu;
    g.mask = mask; g.ldm = ldm;
    return launch_gemm_bf16(g, gpart, s);
  };
  // forward
  if ((e = gemm(Xs, d, 0, th + L.W1, h, 0, H1, h, B, h, d, th + L.b1, 1, nullptr, 0))) return e;
  if ((e = gemm(H1, h, 0, th + L.W2, h, 0, H2, h, B, h, h, th + L.b2, 1, nullptr, 0))) return e;
  if ((e = gemm(H2, h, 0, th + L.W3, k, 0, Z, k, B, k, h, th + L.b3, 0, nullptr, 0))) return e;
  hipLaunchKernelGGL(softmax_ce_kernel, dim3(B), dim3(256), 0, s, Z, k, y,
                     1.0f / (float)B, lrow);
  if ((e = hipGetLastError())) return e;
  hipLaunchKernelGGL(mean_kernel, dim3(1), dim3(256), 0, s, lrow, B, loss_dev);
  // backward (Z now holds dZ)
  if ((e = gemm(H2, h, 1, Z, k, 0, grad + L.W3, k, h, k, B, nullptr, 0, nullptr, 0))) return e;
  launch_colsum(Z, B, k, cpart, grad + L.b3, s);
  if ((e = gemm(Z, k, 0, th + L.W3, k, 1, D2, h, B, h, k, nullptr, 0, H2, h))) return e;
  if ((e = gemm(H1, h, 1, D2, h, 0, grad + L.W2, h, h, h, B, nullptr, 0, nullptr, 0))) return e;
  launch_colsum(D2, B, h, cpart, grad + L.b2, s);
  if ((e = gemm(D2, h, 0, th + L.W2, h, 1, D1, h, B, h, h, nullptr, 0, H1, h))) return e;
  if ((e = gemm(Xs, d, 1, D1, h, 0, grad + L.W1, h, d, h, B, nullptr, 0, nullptr, 0))) return e;
  launch_colsum(D1, B, h, cpart, grad + L.b1, s);
  if ((e = hipGetLastError())) return e;
  if (lr > 0.0f) {
    const double c1 = 1.0 / (1.0 - pow(0.9, (double)step));
    const double c2 = 1.0 / (1.0 - pow(0.999, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((L.P + 255) / 256)), dim3(256), 0, s,
                       th, am, av, grad, L.P, lr, (float)c1, (float)c2);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// proposal: the whole forward pass in one kernel, top-16 in its epilogue
// ---------------------------------------------------------------------------
//
// Layout of v_mfma_f32_16x16x32_bf16 used by every layer: lane (col, g)
// (col = lane % 16, g = lane / 16) supplies row col of the A operand and
// column col of the B operand at K positions 8g .. 8g + 7 of each 32-wide
// K-step, and receives D[4g + r][col], r = 0..3.  A holds weight rows
// (output units), B the points' activations (one point per column), so a
// lane ends a layer with units 16b + 4g + r of its point for every block b.
// The next layer's B fragment of K-step s is formed in place from blocks
// 2s and 2s + 1 -- element e of lane group g is unit
//   perm_unit(32 s + 8 g + e) = 32 s + 16 (e / 4) + 4 g + (e % 4)
// -- and the BF16 copies of W2 and W3 store their K columns in that order,
// so no activation crosses lanes.  W3 streams through LDS in chunks of 64
// classes shared by the workgroup's eight waves.
//
// Top-16: a logit z of class j becomes the key z with its low B mantissa
// bits replaced by (2^B - 1 - j), 2^B >= the padded class count; keys
// compare as floats, i.e. by z rounded to its leading 23 - B mantissa bits
// (towards zero), then by the code.  Each lane keeps the 16 largest keys of
// the classes it sees (a quarter of them) in a descending list updated with
// one median-of-three per entry; the four lists of a point are merged
// through LDS into its 16 largest keys.  Candidates are their classes, in
// decreasing key order (-1 for padding past k).

__host__ __device__ constexpr int perm_unit(int pos) {
  return 32 * (pos >> 5) + 16 * ((pos & 7) >> 2) + 4 * ((pos >> 3) & 3) + (pos & 3);
}

constexpr int kFwdWaves = 8;
constexpr int kFwdPB = 2;                        // blocks of 16 points per wave
constexpr int kFwdPoints = kFwdWaves * 16 * kFwdPB;
constexpr int kFwdRows = 64;                     // weight rows per LDS chunk
constexpr float kPadLogit = -3.0e38f;            // classes past k
constexpr int kFwdList = 10;                     // keys per lane in the first pass
// Small launches split the classes: up to kFwdSplitMax slices, each a
// workgroup of its own over the same points, for at most kFwdSplitRows points
constexpr int kFwdSplitMax = 16;
constexpr int kFwdSplitRows = 8192;

// W1b (h x KP1, KP1 = 32 KD >= d; input dims in natural order, zero past d),
// W2b (h x h) and W3b (kpad x h), both with permuted K columns; b3p (kpad)
// with kPadLogit past k.
__global__ __launch_bounds__(256) void mlp_pack_kernel(
    const float* __restrict__ th, int d, int h, int k, int kpad, int KP1, int64_t oW1,
    int64_t oW2, int64_t oW3, int64_t ob3, uint16_t* __restrict__ W1b,
    uint16_t* __restrict__ W2b, uint16_t* __restrict__ W3b, float* __restrict__ b3p) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t n1 = (int64_t)h * KP1, n2 = (int64_t)h * h, n3 = (int64_t)kpad * h;
  if (e < n1) {
    const int u = (int)(e / KP1), c = (int)(e - (int64_t)u * KP1);
    W1b[e] = c < d ? f32_bf16_rne(th[oW1 + (int64_t)c * h + u]) : (uint16_t)0;
  } else if (e < n1 + n2) {
    const int64_t q = e - n1;
    const int v = (int)(q / h), pos = (int)(q - (int64_t)v * h);
    W2b[q] = f32_bf16_rne(th[oW2 + (int64_t)perm_unit(pos) * h + v]);
  } else if (e < n1 + n2 + n3) {
    const int64_t q = e - n1 - n2;
    const int cl = (int)(q / h), pos = (int)(q - (int64_t)cl * h);
    W3b[q] = cl < k ? f32_bf16_rne(th[oW3 + (int64_t)perm_unit(pos) * k + cl]) : (uint16_t)0;
  } else if (e < n1 + n2 + n3 + kpad) {
    const int cl = (int)(e - n1 - n2 - n3);
    b3p[cl] = cl < k ? th[ob3 + cl] : kPadLogit;
  }
}

// two FP32 values -> one word of two BF16 (nearest even)
__device__ __forceinline__ uint32_t bf16x2(float lo, float hi) {
  return (uint32_t)f32_bf16_rne(lo) | ((uint32_t)f32_bf16_rne(hi) << 16);
}

__device__ __forceinline__ bf8l frag_of(const uint32_t (&w)[4]) {
  const uint4 v = {w[0], w[1], w[2], w[3]};
  return __builtin_bit_cast(bf8l, v);
}

// D-layout block b of a hidden layer (values of units 16b + 4g + r, after
// bias) -> words of the next layer's B fragment (ReLU, BF16)
__device__ __forceinline__ void put_block(uint32_t (&w)[4], int half, const f4l& v) {
  const float a0 = v[0] > 0.f ? v[0] : 0.f, a1 = v[1] > 0.f ? v[1] : 0.f;
  const float a2 = v[2] > 0.f ? v[2] : 0.f, a3 = v[3] > 0.f ? v[3] : 0.f;
  w[2 * half] = bf16x2(a0, a1);
  w[2 * half + 1] = bf16x2(a2, a3);
}

// Rows [r0, r0 + 64) of a BF16 matrix with row stride H into LDS (row
// stride H + 8), through registers: load() issues the global loads, store()
// writes them; rows past nrows read as zero.
template <int KH>
struct RowStage {
  static constexpr int H = 32 * KH, LD = H + 8;
  static constexpr int PIECES = kFwdRows * H / 8;                 // 16-byte pieces
  static constexpr int PER = (PIECES + 64 * kFwdWaves - 1) / (64 * kFwdWaves);
  uint4 v[PER];
  __device__ void load(const uint16_t* __restrict__ W, int r0, int nrows) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * 64 * kFwdWaves;
      const int r = e / (H / 8), q = e - r * (H / 8);
      v[i] = (e < PIECES && r0 + r < nrows)
                 ? *reinterpret_cast<const uint4*>(W + (size_t)(r0 + r) * H + q * 8)
                 : make_uint4(0u, 0u, 0u, 0u);
    }
  }
  __device__ void store(uint16_t* buf) const {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = threadIdx.x + i * 64 * kFwdWaves;
      const int r = e / (H / 8), q = e - r * (H / 8);
      if (e < PIECES) *reinterpret_cast<uint4*>(&buf[r * LD + q * 8]) = v[i];
    }
  }
};

// descending list of the TL largest keys: insert key y (one median of three
// per entry)
template <int TL>
__device__ __forceinline__ void topk_insert(float (&L)[TL], float y) {
#pragma unroll
  for (int i = TL - 1; i >= 1; --i) L[i] = __builtin_amdgcn_fmed3f(L[i - 1], L[i], y);
  L[0] = L[0] > y ? L[0] : y;
}

// The forward pass of m points (rows[q], or q when rows is null) with the
// top-16 epilogue; point q's candidates go to row outpos[q] (or q) of cand.
// Inputs are standardized as (x - mean) istd in FP64 (mean / istd null:
// taken as they are), rounded to FP32, then to BF16.
//
// Each lane keeps the TL largest keys of its quarter of the classes.  With
// TL = 16 the merged list is the top 16 outright.  With TL < 16 it is the top
// 16 unless some quarter holds more than TL of them; then that quarter's
// whole list is in the merged top 16 (its TL-th key is not below the 16th),
// and the point is appended to (fl_rows, fl_pos) for a TL = 16 pass, which
// overwrites its row.  A quarter holds more than 10 of 16 keys for about 0.3%
// of points with classes in random order.
template <int KD, int KH, int TL, typename T>
__global__ __launch_bounds__(64 * kFwdWaves) void mlp_forward_kernel(
    const T* __restrict__ X, int d, const int* __restrict__ rows, int m,
    const int* __restrict__ mdev, const double* __restrict__ mean,
    const double* __restrict__ istd, const uint16_t* __restrict__ W1b,
    const float* __restrict__ b1, const uint16_t* __restrict__ W2b,
    const float* __restrict__ b2, const uint16_t* __restrict__ W3b,
    const float* __restrict__ b3p, int k, int kpad, int cbits,
    int32_t* __restrict__ cand, const int* __restrict__ outpos, int* __restrict__ fl_rows,
    int* __restrict__ fl_pos, int* __restrict__ fl_cnt, float* __restrict__ keys_out) {
  static_assert(TL >= 1 && TL <= 16, "list length");
  constexpr int H = 32 * KH, LD = H + 8, KP1 = 32 * KD, PB = kFwdPB;
  using RS = RowStage<KH>;
  extern __shared__ __attribute__((aligned(16))) uint16_t sW[];   // 2 x 64 x LD
  const int mm = mdev ? (m < *mdev ? m : *mdev) : m;
  const int q0 = blockIdx.x * kFwdPoints;
  if (q0 >= mm) return;                                           // uniform
  // this workgroup's classes: W3 chunks [cb, ce) of slice blockIdx.y of
  // gridDim.y (all of them when the grid has one slice)
  const int NC3 = kpad / kFwdRows;
  const int cb = (int)((int64_t)blockIdx.y * NC3 / gridDim.y);
  const int ce = (int)((int64_t)(blockIdx.y + 1) * NC3 / gridDim.y);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  uint16_t* buf0 = sW;
  uint16_t* buf1 = sW + kFwdRows * LD;

  // prefetch the first W2 chunk while the inputs and layer 1 run
  RS pre;
  pre.load(W2b, 0, H);

  // inputs: K-step s of lane group g holds dims 32 s + 8 g + e
  bf8l bx[PB][KD];
  bool valid[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int q = q0 + wave * 16 * PB + pb * 16 + col;
    valid[pb] = q < mm;
    const int p = valid[pb] ? (rows ? rows[q] : q) : 0;
    const T* xr = X + (size_t)p * d;
#pragma unroll
    for (int s = 0; s < KD; ++s) {
      uint32_t w[4];
#pragma unroll
      for (int e2 = 0; e2 < 4; ++e2) {
        float f[2];
#pragma unroll
        for (int h2 = 0; h2 < 2; ++h2) {
          const int c = 32 * s + 8 * grp + 2 * e2 + h2;
          double v = 0.0;
          if (valid[pb] && c < d) {
            v = to_f64<T>(xr[c]);
            if (mean) v = (v - mean[c]) * istd[c];
          }
          f[h2] = (float)v;
        }
        w[e2] = bf16x2(f[0], f[1]);
      }
      bx[pb][s] = frag_of(w);
    }
  }

  // layer 1: W1b rows straight from memory (small; cached)
  uint32_t h1w[PB][KH][4];
#pragma unroll
  for (int ub = 0; ub < H / 16; ++ub) {
    bf8l a[KD];
#pragma unroll
    for (int s = 0; s < KD; ++s)
      a[s] = *reinterpret_cast<const bf8l*>(W1b + (size_t)(16 * ub + col) * KP1 + 32 * s + 8 * grp);
    const f4l init = *reinterpret_cast<const f4l*>(b1 + 16 * ub + 4 * grp);
#pragma unroll
    for (int pb = 0; pb < PB; ++pb) {
      f4l acc = init;
#pragma unroll
      for (int s = 0; s < KD; ++s)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], bx[pb][s], acc, 0, 0, 0);
      put_block(h1w[pb][ub >> 1], ub & 1, acc);
    }
  }
  bf8l h1f[PB][KH];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int s = 0; s < KH; ++s) h1f[pb][s] = frag_of(h1w[pb][s]);

  // layer 2: W2b through LDS in chunks of 64 rows
  uint32_t h2w[PB][KH][4];
  pre.store(buf0);
  __syncthreads();
  constexpr int NC2 = (H + kFwdRows - 1) / kFwdRows;
#pragma unroll
  for (int c = 0; c < NC2; ++c) {
    uint16_t* cur = (c & 1) ? buf1 : buf0;
    uint16_t* nxt = (c & 1) ? buf0 : buf1;
    // the next chunk: W2b's next rows, or after the last the first W3b rows
    if (c + 1 < NC2) pre.load(W2b, (c + 1) * kFwdRows, H);
    else pre.load(W3b, cb * kFwdRows, kpad);
#pragma unroll
    for (int bb = 0; bb < kFwdRows / 16; ++bb) {
      const int vb = c * (kFwdRows / 16) + bb;             // unit block
      if (vb < H / 16) {
        bf8l a[KH];
#pragma unroll
        for (int s = 0; s < KH; ++s)
          a[s] = *reinterpret_cast<const bf8l*>(&cur[(16 * bb + col) * LD + 32 * s + 8 * grp]);
        const f4l init = *reinterpret_cast<const f4l*>(b2 + 16 * vb + 4 * grp);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          f4l acc = init;
#pragma unroll
          for (int s = 0; s < KH; ++s)
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], h1f[pb][s], acc, 0, 0, 0);
          put_block(h2w[pb][vb >> 1], vb & 1, acc);
        }
      }
    }
    pre.store(nxt);
    __syncthreads();
  }
  bf8l h2f[PB][KH];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int s = 0; s < KH; ++s) h2f[pb][s] = frag_of(h2w[pb][s]);

  // layer 3 with the top-16 epilogue; the first W3b chunk is in buffer NC2 & 1
  float L[PB][TL];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int i = 0; i < TL; ++i) L[pb][i] = -INFINITY;
  const uint32_t cmask = (1u << cbits) - 1u;
#pragma unroll 1
  for (int c = cb; c < ce; ++c) {
    const int slot = (c - cb + NC2) & 1;
    uint16_t* cur = slot ? buf1 : buf0;
    uint16_t* nxt = slot ? buf0 : buf1;
    if (c + 1 < ce) pre.load(W3b, (c + 1) * kFwdRows, kpad);
#pragma unroll 1
    for (int bb = 0; bb < kFwdRows / 16; ++bb) {
      const int cl0 = c * kFwdRows + 16 * bb;
      bf8l a[KH];
#pragma unroll
      for (int s = 0; s < KH; ++s)
        a[s] = *reinterpret_cast<const bf8l*>(&cur[(16 * bb + col) * LD + 32 * s + 8 * grp]);
      const f4l init = *reinterpret_cast<const f4l*>(b3p + cl0 + 4 * grp);
      f4l acc[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[pb] = init;
#pragma unroll
      for (int s = 0; s < KH; ++s)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
          acc[pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], h2f[pb][s], acc[pb], 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t code = cmask - (uint32_t)(cl0 + 4 * grp + r);
#pragma unroll
        for (int pb = 0; pb < PB; ++pb) {
          const float key = __uint_as_float((__float_as_uint(acc[pb][r]) & ~cmask) | code);
          topk_insert<TL>(L[pb], key);
        }
      }
    }
    if (c + 1 < ce) pre.store(nxt);
    __syncthreads();
  }

  // merge the four lane groups' lists of each point through LDS
  float* sK = reinterpret_cast<float*>(sW);      // [wave][pb][col][g][16]
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    float* dst = sK + ((((size_t)wave * PB + pb) * 16 + col) * 4 + grp) * 16;
#pragma unroll
    for (int i = 0; i < TL; ++i) dst[i] = L[pb][i];
  }
  __syncthreads();
  if (lane < 16 * PB) {
    const int pb = lane >> 4, cc = lane & 15;
    const int q = q0 + wave * 16 * PB + pb * 16 + cc;
    if (q < mm) {
      const float* src = sK + (((size_t)wave * PB + pb) * 16 + cc) * 4 * 16;
      int hd[4] = {0, 0, 0, 0};
      int32_t out[16];
      float okey[16];
      float best = -INFINITY;
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        best = -INFINITY;
        int bg = 0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const float v = hd[g] < TL ? src[g * 16 + hd[g]] : -INFINITY;
          if (v > best) { best = v; bg = g; }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) hd[g] += (g == bg) ? 1 : 0;
        const int j = (int)(cmask - (__float_as_uint(best) & cmask));
        out[i] = (best == -INFINITY || j >= k) ? -1 : j;
        okey[i] = best;
      }
      if (keys_out) {
        // a slice of the classes: its 16 largest keys, in decreasing order
        float4* k4 = reinterpret_cast<float4*>(
            keys_out + ((size_t)q * gridDim.y + blockIdx.y) * kMlpTop);
#pragma unroll
        for (int i = 0; i < 4; ++i)
          k4[i] = make_float4(okey[4 * i], okey[4 * i + 1], okey[4 * i + 2], okey[4 * i + 3]);
        return;                                  // no barrier follows
      }
      if constexpr (TL < 16) {
        // best is now the 16th largest merged key
        bool full = false;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const float lastg = src[g * 16 + TL - 1];
          full |= lastg > -INFINITY && lastg >= best;
        }
        if (full) {
          const int slot = atomicAdd(fl_cnt, 1);
          fl_rows[slot] = rows ? rows[q] : q;
          fl_pos[slot] = outpos ? outpos[q] : q;
        }
      }
      const int qo = outpos ? outpos[q] : q;
      int4* o4 = reinterpret_cast<int4*>(cand + (size_t)qo * kMlpTop);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        o4[i] = make_int4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
    }
  }
}

// Point q's 16 largest keys over the S class slices (each slice's keys in
// decreasing order, as the forward kernel writes them), decoded as the
// one-pass kernel decodes its merged list: the same candidates, in the same
// order.
__global__ __launch_bounds__(256) void mlp_merge_kernel(const float* __restrict__ keys, int m,
                                                        int S, int k, int cbits,
                                                        int32_t* __restrict__ cand,
                                                        const int* __restrict__ outpos) {
  const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (q >= m) return;
  const float* kq = keys + (size_t)q * S * kMlpTop;
  const uint32_t cmask = (1u << cbits) - 1u;
  int hd[kFwdSplitMax];
#pragma unroll
  for (int s = 0; s < kFwdSplitMax; ++s) hd[s] = 0;
  int32_t out[kMlpTop];
#pragma unroll
  for (int i = 0; i < kMlpTop; ++i) {
    float best = -INFINITY;
    int bs = 0;
#pragma unroll
    for (int s = 0; s < kFwdSplitMax; ++s) {
      const float v = (s < S && hd[s] < kMlpTop) ? kq[s * kMlpTop + hd[s]] : -INFINITY;
      if (v > best) { best = v; bs = s; }
    }
#pragma unroll
    for (int s = 0; s < kFwdSplitMax; ++s) hd[s] += (s == bs) ? 1 : 0;
    const int j = (int)(cmask - (__float_as_uint(best) & cmask));
    out[i] = (best == -INFINITY || j >= k) ? -1 : j;
  }
  const int qo = outpos ? outpos[q] : q;
  int4* o4 = reinterpret_cast<int4*>(cand + (size_t)qo * kMlpTop);
#pragma unroll
  for (int i = 0; i < 4; ++i)
    o4[i] = make_int4(out[4 * i], out[4 * i + 1], out[4 * i + 2], out[4 * i + 3]);
}

// padded class count and code bits of the proposal
int mlp_kpad(int k) { return (k + kFwdRows - 1) / kFwdRows * kFwdRows; }
static int code_bits(int kpad) {
  int b = 0;
  while ((1 << b) < kpad) ++b;
  return b;
}
static int kd_of(int d) {
  int kd = 1;
  while (32 * kd < d) kd *= 2;
  return kd;
}

size_t mlp_pack_bytes(int d, int h, int k, int64_t mmax) {
  const int kpad = mlp_kpad(k), KP1 = 32 * kd_of(d);
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  return al(sizeof(uint16_t) * (size_t)h * KP1) + al(sizeof(uint16_t) * (size_t)h * h) +
         al(sizeof(uint16_t) * (size_t)kpad * h) + al(sizeof(float) * (size_t)kpad) +
         2 * al(sizeof(int) * (size_t)mmax) + al(sizeof(int)) +
         al(sizeof(float) * (size_t)kFwdSplitRows * kFwdSplitMax * kMlpTop);
}

MlpPacked mlp_pack_layout(int d, int h, int k, int64_t mmax, void* ws) {
  MlpPacked P{};
  P.d = d; P.h = h; P.k = k; P.kpad = mlp_kpad(k); P.KP1 = 32 * kd_of(d);
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  char* c = (char*)ws;
  P.W1b = (uint16_t*)c; c += al(sizeof(uint16_t) * (size_t)h * P.KP1);
  P.W2b = (uint16_t*)c; c += al(sizeof(uint16_t) * (size_t)h * h);
  P.W3b = (uint16_t*)c; c += al(sizeof(uint16_t) * (size_t)P.kpad * h);
  P.b3p = (float*)c; c += al(sizeof(float) * (size_t)P.kpad);
  P.fl_rows = (int*)c; c += al(sizeof(int) * (size_t)mmax);
  P.fl_pos = (int*)c; c += al(sizeof(int) * (size_t)mmax);
  P.fl_cnt = (int*)c; c += al(sizeof(int));
  P.keys = (float*)c;
  return P;
}

hipError_t launch_mlp_pack(const float* th, const MlpLayout& L, const MlpPacked& P,
                           hipStream_t s) {
  const int64_t tot = (int64_t)L.h * P.KP1 + (int64_t)L.h * L.h + (int64_t)P.kpad * L.h + P.kpad;
  hipLaunchKernelGGL(mlp_pack_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     th, L.d, L.h, L.k, P.kpad, P.KP1, L.W1, L.W2, L.W3, L.b3, P.W1b, P.W2b,
                     P.W3b, P.b3p);
  return hipGetLastError();
}

template <int KD, int KH, typename T>
static hipError_t fwd_launch(const T* X, int d, const int* rows, int m, const int* mdev,
                             const double* mean, const double* istd, const float* th,
                             const MlpLayout& L, const MlpPacked& P, int32_t* cand,
                             const int* outpos, hipStream_t s) {
  constexpr int LD = 32 * KH + 8;
  const size_t lds_w = sizeof(uint16_t) * 2 * kFwdRows * LD;
  const size_t lds_k = sizeof(float) * kFwdWaves * kFwdPB * 16 * 4 * 16;
  const size_t lds = lds_w > lds_k ? lds_w : lds_k;
  for (const void* kp : {reinterpret_cast<const void*>(&mlp_forward_kernel<KD, KH, kFwdList, T>),
                         reinterpret_cast<const void*>(&mlp_forward_kernel<KD, KH, 16, T>)}) {
    hipError_t e = hipFuncSetAttribute(kp, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const int grid = (m + kFwdPoints - 1) / kFwdPoints;
  // few points: the classes are split over slices, enough workgroups to
  // cover the GPU's compute units (full lists, no second pass), and the
  // slices' lists merged per point
  int S = 1;
  if (!mdev && m <= kFwdSplitRows) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    while (S < kFwdSplitMax && grid * S < cus && 2 * S <= P.kpad / kFwdRows) S *= 2;
  }
  if (S > 1) {
    hipLaunchKernelGGL((mlp_forward_kernel<KD, KH, 16, T>), dim3(grid, S), dim3(64 * kFwdWaves),
                       lds, s, X, d, rows, m, (const int*)nullptr, mean, istd, P.W1b, th + L.b1,
                       P.W2b, th + L.b2, P.W3b, P.b3p, L.k, P.kpad, code_bits(P.kpad), cand,
                       outpos, (int*)nullptr, (int*)nullptr, (int*)nullptr, P.keys);
    hipLaunchKernelGGL(mlp_merge_kernel, dim3((m + 255) / 256), dim3(256), 0, s,
                       (const float*)P.keys, m, S, L.k, code_bits(P.kpad), cand, outpos);
    return hipGetLastError();
  }
  // first pass with short lists; the points it flags again with full lists
  // (the second grid covers every point; workgroups past the flagged count
  // return at once)
  hipError_t e = launch_fill_i32(P.fl_cnt, 1, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((mlp_forward_kernel<KD, KH, kFwdList, T>), dim3(grid), dim3(64 * kFwdWaves),
                     lds, s, X, d, rows, m, mdev, mean, istd, P.W1b, th + L.b1, P.W2b,
                     th + L.b2, P.W3b, P.b3p, L.k, P.kpad, code_bits(P.kpad), cand,
                     outpos, P.fl_rows, P.fl_pos, P.fl_cnt, (float*)nullptr);
  hipLaunchKernelGGL((mlp_forward_kernel<KD, KH, 16, T>), dim3(grid), dim3(64 * kFwdWaves),
                     lds, s, X, d, (const int*)P.fl_rows, m, (const int*)P.fl_cnt, mean, istd,
                     P.W1b, th + L.b1, P.W2b, th + L.b2, P.W3b, P.b3p, L.k, P.kpad,
                     code_bits(P.kpad), cand, (const int*)P.fl_pos, (int*)nullptr,
                     (int*)nullptr, (int*)nullptr, (float*)nullptr);
  return hipGetLastError();
}

template <int KD, typename T>
static hipError_t fwd_kh(const T* X, int d, const int* rows, int m, const int* mdev,
                         const double* mean, const double* istd, const float* th,
                         const MlpLayout& L, const MlpPacked& P, int32_t* cand,
                         const int* outpos, hipStream_t s) {
  switch (L.h) {
    case 32:
      return fwd_launch<KD, 1, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
    case 64:
      return fwd_launch<KD, 2, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
    case 128:
      return fwd_launch<KD, 4, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
    case 256:
      return fwd_launch<KD, 8, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
  }
  return hipErrorInvalidValue;
}

template <typename T>
static hipError_t fwd_kd(const T* X, int d, const int* rows, int m, const int* mdev,
                         const double* mean, const double* istd, const float* th,
                         const MlpLayout& L, const MlpPacked& P, int32_t* cand,
                         const int* outpos, hipStream_t s) {
  switch (P.KP1 / 32) {
    case 1: return fwd_kh<1, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
    case 2: return fwd_kh<2, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
    case 4: return fwd_kh<4, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
    case 8: return fwd_kh<8, T>(X, d, rows, m, mdev, mean, istd, th, L, P, cand, outpos, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_mlp_forward(const void* X, knor_dtype dt, int d, const int* rows, int m,
                              const int* mdev, const double* mean, const double* istd,
                              const float* th, const MlpLayout& L, const MlpPacked& P,
                              int32_t* cand, const int* outpos, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  switch (dt) {
    case KNOR_F32:
      return fwd_kd<float>((const float*)X, d, rows, m, mdev, mean, istd, th, L, P, cand,
                           outpos, s);
    case KNOR_F64:
      return fwd_kd<double>((const double*)X, d, rows, m, mdev, mean, istd, th, L, P, cand,
                            outpos, s);
    case KNOR_BF16:
      return fwd_kd<uint16_t>((const uint16_t*)X, d, rows, m, mdev, mean, istd, th, L, P, cand,
                              outpos, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// inputs of the proposal and the certificate
// ---------------------------------------------------------------------------

// mean and 1/std per dimension in FP64 (population std; 0 -> 1), in two
// passes over X (sum, then sum of squared deviations), each split over a
// fixed grid of row ranges: thread (rl, c) of a workgroup sums dimension c
// over rows rl, rl + RL, ... of its range; the RL partial sums of the
// workgroup, then the workgroups' sums, are added in a fixed order, so the
// result does not depend on scheduling.
constexpr int kStatBlocks = 1024;

template <typename T>
__global__ __launch_bounds__(256) void stats_partial_kernel(
    const T* __restrict__ X, int64_t n, int d, const double* __restrict__ mean,
    double* __restrict__ part) {
  __shared__ double red[256];
  const int RL = 256 / d;                      // d <= 256
  const int rl = threadIdx.x / d, c = threadIdx.x - rl * d;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * per;
  const int64_t r1 = r0 + per < n ? r0 + per : n;
  double s = 0.0;
  if (rl < RL) {
    const double mu = mean ? mean[c] : 0.0;
    for (int64_t r = r0 + rl; r < r1; r += RL) {
      const double v = to_f64<T>(X[(size_t)r * d + c]);
      s += mean ? (v - mu) * (v - mu) : v;
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < d) {
    double t = 0.0;
    for (int q = 0; q < RL; ++q) t += red[q * d + threadIdx.x];
    part[(size_t)blockIdx.x * d + threadIdx.x] = t;
  }
}

// mode 0: mean[c] = sum / n; mode 1: istd[c] = 1 / sqrt(sum / n) (1 if 0)
__global__ __launch_bounds__(256) void stats_final_kernel(const double* __restrict__ part,
                                                          int nb, int d, int64_t n, int mode,
                                                          double* __restrict__ out) {
  const int c = threadIdx.x;
  if (c >= d) return;
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += part[(size_t)b * d + c];
  if (mode == 0) {
    out[c] = t / (double)n;
  } else {
    const double sd = sqrt(t / (double)n);
    out[c] = sd > 0.0 ? 1.0 / sd : 1.0;
  }
}

size_t standardize_workspace(int d) { return sizeof(double) * (size_t)kStatBlocks * d; }

template <typename T>
static void stats_t(const T* X, int64_t n, int d, double* mean, double* istd, double* part,
                    hipStream_t s) {
  const int nb = (int)(n < kStatBlocks ? (n < 1 ? 1 : n) : kStatBlocks);
  hipLaunchKernelGGL(stats_partial_kernel<T>, dim3(nb), dim3(256), 0, s, X, n, d,
                     (const double*)nullptr, part);
  hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(256), 0, s, part, nb, d, n, 0, mean);
  hipLaunchKernelGGL(stats_partial_kernel<T>, dim3(nb), dim3(256), 0, s, X, n, d,
                     (const double*)mean, part);
  hipLaunchKernelGGL(stats_final_kernel, dim3(1), dim3(256), 0, s, part, nb, d, n, 1, istd);
}

hipError_t launch_standardize_stats(const void* X, knor_dtype dt, int64_t n, int d,
                                    double* mean, double* istd, double* part, hipStream_t s) {
  switch (dt) {
    case KNOR_F32: stats_t((const float*)X, n, d, mean, istd, part, s); break;
    case KNOR_F64: stats_t((const double*)X, n, d, mean, istd, part, s); break;
    case KNOR_BF16: stats_t((const uint16_t*)X, n, d, mean, istd, part, s); break;
  }
  return hipGetLastError();
}

// Xs[r] = (x_{rows[r]} - mean) / std in FP32 for r < count
template <typename T>
__global__ __launch_bounds__(256) void gather_std_kernel(
    const T* __restrict__ X, int d, const int* __restrict__ rows, int64_t count,
    const int* __restrict__ cdev, const double* __restrict__ mean,
    const double* __restrict__ istd, float* __restrict__ Xs) {
  const int64_t cnt = cdev ? (count < *cdev ? count : *cdev) : count;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= cnt * d) return;
  const int64_t r = e / d;
  const int i = (int)(e - r * d);
  const int p = rows[r];
  Xs[e] = (float)((to_f64<T>(X[(size_t)p * d + i]) - mean[i]) * istd[i]);
}

hipError_t launch_gather_std(const void* X, knor_dtype dt, int d, const int* rows,
                             int64_t count, const int* cdev, const double* mean,
                             const double* istd, float* Xs, hipStream_t s) {
  const int64_t tot = count * d;
  const dim3 g((unsigned)((tot + 255) / 256));
  if (tot <= 0) return hipSuccess;
  switch (dt) {
    case KNOR_F32:
      hipLaunchKernelGGL(gather_std_kernel<float>, g, dim3(256), 0, s, (const float*)X, d,
                         rows, count, cdev, mean, istd, Xs);
      break;
    case KNOR_F64:
      hipLaunchKernelGGL(gather_std_kernel<double>, g, dim3(256), 0, s, (const double*)X, d,
                         rows, count, cdev, mean, istd, Xs);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(gather_std_kernel<uint16_t>, g, dim3(256), 0, s,
                         (const uint16_t*)X, d, rows, count, cdev, mean, istd, Xs);
      break;
  }
  return hipGetLastError();
}

// Segmented survivor lists -> one dense list (segment order kept) and its
// length: seg_off[b] = survivors before segment b, dense[seg_off[b] + q] =
// list[b * kSeg + q].  One workgroup scans the counts; then one workgroup
// per segment copies.
__global__ __launch_bounds__(1024) void seg_scan_kernel(const int* __restrict__ seg_cnt,
                                                        int nseg, int* __restrict__ seg_off,
                                                        const int* __restrict__ conv,
                                                        int iter) {
  __shared__ int part[1024];
  if (*conv < iter) return;
  const int per = (nseg + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  int loc = 0;
  for (int b = b0; b < b0 + per && b < nseg; ++b) loc += seg_cnt[b];
  part[threadIdx.x] = loc;
  __syncthreads();
  for (int s = 1; s < 1024; s <<= 1) {
    const int t = threadIdx.x >= s ? part[threadIdx.x - s] : 0;
    __syncthreads();
    part[threadIdx.x] += t;
    __syncthreads();
  }
  int run = part[threadIdx.x] - loc;
  for (int b = b0; b < b0 + per && b < nseg; ++b) {
    seg_off[b] = run;
    run += seg_cnt[b];
  }
  if (threadIdx.x == 1023) seg_off[nseg] = part[1023];
}

// Survivors of segment b that have no proposal yet (cand[p][0] ==
// kUnproposed): their count (count pass) or, at seg_off[b] on, their point
// indices (order within a segment is immaterial: each output row lands at
// its point's own candidate slots).
// CertPre: the certificate's test for c* = a (see mlp_certify_kernel), to
// skip survivors that cannot pass it.  Active when rows is not null.
struct CertPre {
  const float* u;       // |u|: distance to the centroid rounded up
  const int32_t* labels;
  const float* rows;    // neighbour rows (k x k keys)
  int k, ib;
  __device__ bool can_pass(int p) const {
    if (!rows || k <= kMlpTop) return true;
    const int a = labels[p];
    const float key = rows[(size_t)a * k + kMlpTop];
    const double h16 = (double)__uint_as_float(__float_as_uint(key) & ~((1u << ib) - 1u));
    const double dlo = (double)fabsf(u[p]) * (1.0 - 9.5367431640625e-07);
    return dlo * (1.0 + kEta) < h16;
  }
};

// prop[p] != 0 once p has been sent to the network (set by the write pass,
// whose points the forward pass of the same iteration proposes for): one
// byte per point, so a segment's flags share a few cache lines.
template <bool WRITE>
__global__ __launch_bounds__(256) void seg_unproposed_kernel(
    const int* __restrict__ list, const int* __restrict__ seg_cnt,
    uint8_t* __restrict__ prop, int* __restrict__ cnt_new,
    const int* __restrict__ seg_off, int* __restrict__ dense,
    const int* __restrict__ conv, int iter, CertPre pre) {
  __shared__ int run;
  if (*conv < iter) return;
  const int b = blockIdx.x;
  const int cnt = seg_cnt[b];
  if (threadIdx.x == 0) run = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt();
  for (int q0 = 0; q0 < cnt; q0 += 256) {
    const int q = q0 + (int)threadIdx.x;
    const int p = q < cnt ? list[(size_t)b * kSeg + q] : 0;
    // survivors the certificate will not test need no proposal yet
    const bool fresh = q < cnt && prop[p] == 0 && pre.can_pass(p);
    const uint64_t m = __ballot(fresh);
    if (m) {
      const int leader = __ffsll((unsigned long long)m) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&run, __popcll(m));   // LDS
      base = __shfl(base, leader);
      if (WRITE && fresh) {
        dense[seg_off[b] + base + __popcll(m & lt)] = p;
        prop[p] = 1;
      }
    }
  }
  __syncthreads();
  if (!WRITE && threadIdx.x == 0) cnt_new[b] = run;
}

hipError_t launch_seg_unproposed(const int* list, const int* seg_cnt, int nseg,
                                 uint8_t* prop, int* cnt_new, int* seg_off, int* dense,
                                 const int* conv, int iter, const float* u,
                                 const int32_t* labels, const float* rows, int k,
                                 hipStream_t s) {
  const CertPre pre{u, labels, rows, k, rows ? cc_rows_bits(k) : 0};
  hipLaunchKernelGGL(seg_unproposed_kernel<false>, dim3(nseg), dim3(256), 0, s, list, seg_cnt,
                     prop, cnt_new, (const int*)nullptr, (int*)nullptr, conv, iter, pre);
  hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(1024), 0, s, cnt_new, nseg, seg_off,
                     conv, iter);
  hipLaunchKernelGGL(seg_unproposed_kernel<true>, dim3(nseg), dim3(256), 0, s, list, seg_cnt,
                     prop, cnt_new, (const int*)seg_off, dense, conv, iter, pre);
  return hipGetLastError();
}

// The certificate.  One workgroup per segment; a wave takes 4 survivors at a
// time, 16 lanes per survivor, one lane per candidate: each lane evaluates
// its candidate's canonical FP64 distance, the 16 lanes reduce to c* (the
// smallest distance, lowest index on ties).  c*'s neighbour row (every
// centroid by increasing lower bound of its half distance to c*, c* itself
// first or among its exact duplicates) is then read from the front: lane t
// tests entry t (lanes 0 and 1 also entries 16 and 17) against the
// candidate set, which contains c*; h = the bound of the first entry that
// is not a candidate (+inf when the row ends first: every centroid is a
// candidate).  With 16 candidates, 18 entries always reach one.  Accept iff
// ub (1 + eta) < h, ub an upper bound of d(x, c*) rounded up to FP32: every
// candidate is compared in the FP64 definition itself, and every other
// centroid j has d(x, j) >= d(c*, j) - d(x, c*) > ub (1 + 2 eta).
// Certified points take c* (and ub as their MTI bound); the others are
// appended to list2 (order within a segment is immaterial to every later
// pass).
//
// tight: with 16 candidates, the first non-candidate of a row is at
// position 16 at the latest, so with c* = a (the survivor's centroid) the
// test needs d(x, a) (1 + eta) < h(a, row_a[16]).  A survivor whose bound,
// scaled down below d(x, a), fails this is not tested (it goes to the
// fallback scan like any uncertified point); only a survivor whose c*
// would differ from a could have passed.
template <typename T>
__global__ __launch_bounds__(256) void mlp_certify_kernel(
    const T* __restrict__ X, int d, const double* __restrict__ C64,
    int k, const float* __restrict__ nrows, int ib,
    const int* __restrict__ list, const int* __restrict__ seg_cnt,
    const int32_t* __restrict__ cand,
    int32_t* __restrict__ labels, float* __restrict__ ub_out, int* __restrict__ dirty,
    int* __restrict__ list2, int* __restrict__ seg_cnt2,
    unsigned long long* __restrict__ row, const int* __restrict__ conv, int iter, int vec4,
    int tight) {
  __shared__ int run, sQn;
  __shared__ int sQ[kSeg];                   // the segment's survivors to test (tight)
  if (*conv < iter) return;
  const int b = blockIdx.x;
  const int cnt = seg_cnt[b];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int ps = lane >> 4, cs = lane & 15;
  const uint64_t lt = lanemask_lt();
  if (threadIdx.x == 0) { run = 0; sQn = 0; }
  __syncthreads();
  unsigned long long certified = 0, changes = 0;
  // tight: every listed survivor is first put through the pre-test (all of
  // the segment's loads issued in three rounds); those that can pass with
  // c* = their centroid are gathered in sQ, the others go to list2 at once
  const bool pre = tight && k > kMlpTop;
  int cnt2 = cnt;
  if (pre) {
    constexpr int E = kSeg / 256;
    static_assert(E * 256 == kSeg, "one pass of the workgroup covers a segment");
    const uint32_t tmask = (1u << ib) - 1u;
    int pp[E], aa[E];
    float uu[E], kk[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = (int)threadIdx.x + 256 * e;
      pp[e] = q < cnt ? list[(size_t)b * kSeg + q] : 0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      aa[e] = labels[pp[e]];
      uu[e] = ub_out[pp[e]];
    }
#pragma unroll
    for (int e = 0; e < E; ++e) kk[e] = nrows[(size_t)aa[e] * k + kMlpTop];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int q = (int)threadIdx.x + 256 * e;
      const bool in = q < cnt;
      // d(x, a) >= |u| (1 - 2^-20): |u| is d(x, a) rounded up to FP32
      const double h16 = (double)__uint_as_float(__float_as_uint(kk[e]) & ~tmask);
      const double dlo = (double)fabsf(uu[e]) * (1.0 - 9.5367431640625e-07);
      const bool can = in && dlo * (1.0 + kEta) < h16;
      const uint64_t mc = __ballot(can), mo = __ballot(in && !can);
      const int leader = lane == 0;
      int bc = 0, bo = 0;
      if (leader && mc) bc = atomicAdd(&sQn, __popcll(mc));   // LDS
      if (leader && mo) bo = atomicAdd(&run, __popcll(mo));
      bc = __shfl(bc, 0);
      bo = __shfl(bo, 0);
      if (can) sQ[bc + __popcll(mc & lt)] = pp[e];
      if (in && !can) list2[(size_t)b * kSeg + bo + __popcll(mo & lt)] = pp[e];
    }
    __syncthreads();
    cnt2 = sQn;
  }
  auto entry = [&](int q) { return pre ? sQ[q] : list[(size_t)b * kSeg + q]; };
  // the next step's survivor and candidate are loaded a step ahead (two
  // dependent loads off the critical path)
  int pn = 0, jn = -1;
  bool ln = false;
  auto fetch = [&](int q0) {
    const int q = q0 + ps;
    ln = q < cnt2;
    pn = ln ? entry(q) : 0;
    jn = ln ? cand[(size_t)pn * kMlpTop + cs] : -1;
  };
  fetch(wave * 4);
  for (int q0 = wave * 4; q0 < cnt2; q0 += 16) {
    const bool live = ln;
    const int p = pn;
    const int j = jn;
    if (q0 + 16 < cnt2) fetch(q0 + 16);
    double D = INFINITY;
    if (j >= 0) {
      if constexpr (sizeof(T) == 4) {
        if (vec4)
          D = dist2_canon_f32x4(reinterpret_cast<const float*>(X) + (size_t)p * d,
                                C64 + (size_t)j * d, d);
        else
          D = dist2_canon<T>(X + (size_t)p * d, C64 + (size_t)j * d, d);
      } else {
        D = dist2_canon<T>(X + (size_t)p * d, C64 + (size_t)j * d, d);
      }
    }
    double best = D;
    int bj = j >= 0 ? j : 0x7fffffff;
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      const double ob = __shfl_xor(best, off);
      const int oj = __shfl_xor(bj, off);
      if (ob < best || (ob == best && oj < bj)) { best = ob; bj = oj; }
    }
    const bool have = live && bj != 0x7fffffff;
    // entries cs and (lanes 0, 1 of the slot) 16 + cs of c*'s row:
    // status 0 = a candidate, 1 = not a candidate, 2 = past the row's end
    const uint32_t mask = (1u << ib) - 1u;
    const float* nr = nrows + (size_t)(have ? bj : 0) * k;
    const int e0 = cs, e1 = cs < 2 ? 16 + cs : -1;
    const float k0 = (have && e0 < k) ? nr[e0] : INFINITY;
    const float k1 = (have && e1 >= 0 && e1 < k) ? nr[e1] : INFINITY;
    const int nb0 = (have && e0 < k) ? (int)(__float_as_uint(k0) & mask) : -1;
    const int nb1 = (have && e1 >= 0 && e1 < k) ? (int)(__float_as_uint(k1) & mask) : -1;
    bool in0 = false, in1 = false;
#pragma unroll
    for (int u = 0; u < kMlpTop; ++u) {      // every lane takes part
      const int cu = __shfl(j, (lane & ~15) + u);
      in0 |= cu == nb0;
      in1 |= cu == nb1;
    }
    const bool end0 = !(have && e0 < k), end1 = !(have && e1 >= 0 && e1 < k);
    const int st0 = !have ? 0 : (end0 ? 2 : (in0 ? 0 : 1));
    const int st1 = !have || e1 < 0 ? 0 : (end1 ? 2 : (in1 ? 0 : 1));
    const float h0 = st0 == 1 ? __uint_as_float(__float_as_uint(k0) & ~mask) : INFINITY;
    const float h1 = st1 == 1 ? __uint_as_float(__float_as_uint(k1) & ~mask) : INFINITY;
    // the first entry in row order whose status is not "candidate": among
    // entries 0..15, else entry 16, else entry 17 (which cannot be a
    // candidate when the first 17 entries all were: rejected if it were)
    const uint64_t stop = __ballot(st0 != 0);
    const uint64_t stop1 = __ballot(st1 != 0);
    const uint32_t mine = (uint32_t)((stop >> (lane & ~15)) & 0xffffu);
    const uint32_t mine1 = (uint32_t)((stop1 >> (lane & ~15)) & 0x3u);
    const int src = mine ? (lane & ~15) + (__ffs((int)mine) - 1) : (lane & ~15);
    const int src1 = (lane & ~15) + ((mine1 & 1u) ? 0 : 1);
    const float hs0 = __shfl(h0, src);
    const float hs1 = __shfl(h1, src1);
    const float hs = mine ? hs0 : (mine1 ? hs1 : 0.0f);
    const float h = hs;                        // +inf when that entry ends the row
    bool cert = false;
    if (have && cs == 0) {
      const double ub = f32_up(sqrt(best * (1.0 + (double)(d + 8) * 2.220446049250313e-16)) *
                               (1.0 + 8.881784197001252e-16));
      cert = ub * (1.0 + kEta) < (double)h;
      if (cert) {
        const int32_t old = labels[p];
        ub_out[p] = (float)ub;
        ++certified;
        if (old != bj) {                     // unchanged labels are not rewritten
          labels[p] = bj;
          ++changes;
          mark_dirty(dirty, old, bj);
        }
      }
    }
    // uncertified survivors (one lane per point)
    const bool keep = live && cs == 0 && !cert;
    const uint64_t km = __ballot(keep);
    if (km) {
      const int leader = __ffsll((unsigned long long)km) - 1;
      int base = 0;
      if (lane == leader) base = atomicAdd(&run, __popcll(km));     // LDS
      base = __shfl(base, leader);
      if (keep) list2[(size_t)b * kSeg + base + __popcll(km & lt)] = p;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) seg_cnt2[b] = run;
  const int qs[2] = {SLOT_CERTIFIED, SLOT_CHANGED};
  const unsigned long long v[2] = {certified, changes};
  block_add_slots<2>(row, qs, v);
}

hipError_t launch_mlp_certify(const void* X, knor_dtype dt, int d, const double* C64,
                              int k, const float* nrows, const int* list,
                              const int* seg_cnt, int nseg,
                              const int32_t* cand, int32_t* labels, float* u, int* dirty,
                              int* list2, int* seg_cnt2, unsigned long long* row,
                              const int* conv, int iter, bool tight, hipStream_t s) {
  const int vec4 = (int)(d % 4 == 0 && ((uintptr_t)X & 15) == 0 && ((uintptr_t)C64 & 15) == 0);
  switch (dt) {
    case KNOR_F32:
      hipLaunchKernelGGL(mlp_certify_kernel<float>, dim3(nseg), dim3(256), 0, s,
                         (const float*)X, d, C64, k, nrows, cc_rows_bits(k), list, seg_cnt,
                         cand, labels, u, dirty, list2, seg_cnt2, row, conv, iter, vec4,
                         (int)tight);
      break;
    case KNOR_F64:
      hipLaunchKernelGGL(mlp_certify_kernel<double>, dim3(nseg), dim3(256), 0, s,
                         (const double*)X, d, C64, k, nrows, cc_rows_bits(k), list, seg_cnt,
                         cand, labels, u, dirty, list2, seg_cnt2, row, conv, iter, vec4,
                         (int)tight);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(mlp_certify_kernel<uint16_t>, dim3(nseg), dim3(256), 0, s,
                         (const uint16_t*)X, d, C64, k, nrows, cc_rows_bits(k), list, seg_cnt,
                         cand, labels, u, dirty, list2, seg_cnt2, row, conv, iter, vec4,
                         (int)tight);
      break;
  }
  return hipGetLastError();
}

}  // namespace knor
