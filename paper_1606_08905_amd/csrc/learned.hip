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
// Proposal rule: the k classes are split into 16 fixed subsets -- class j
// belongs to subset 4 ((j mod 16) div 4) + ((j div 16) mod 4) -- and the
// candidates are the 16 subset-wise largest logits, which include the
// overall largest.  Each lane of the output tile owns one subset of its
// point's classes, so the selection is one compare and two selects per
// logit in the matrix-core epilogue.
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

// ---------------------------------------------------------------------------
// generic GEMM: C[M x N] = op(A)[M x K] op(B)[K x N] (+ bias[N]) (ReLU)
// (masked by mask > 0); op = transpose when the flag is set
// ---------------------------------------------------------------------------

constexpr int kGT = 64;            // output tile rows and columns
constexpr int kGK = 32;            // K-step
constexpr int kGLD = kGK + 8;      // LDS row stride (bf16), 16-byte aligned

__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) uint16_t sA[kGT * kGLD];
  __shared__ __attribute__((aligned(16))) uint16_t sB[kGT * kGLD];
  const int M = g.Mdev ? (g.M < *g.Mdev ? g.M : *g.Mdev) : g.M;
  const int m0 = blockIdx.y * kGT, n0 = blockIdx.x * kGT;
  if (m0 >= M) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave >> 1, wc = wave & 1, col = lane & 15, grp = lane >> 4;
  f4l acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f4l{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += kGK) {
#pragma unroll
    for (int i = 0; i < (kGT * kGK) / 256; ++i) {
      const int e = tid + 256 * i;
      int r, kk;
      if (!g.transA) { r = e / kGK; kk = e % kGK; } else { kk = e / kGT; r = e % kGT; }
      const int row = m0 + r, kx = k0 + kk;
      float v = 0.0f;
      if (row < M && kx < g.K)
        v = g.transA ? g.A[(size_t)kx * g.lda + row] : g.A[(size_t)row * g.lda + kx];
      sA[r * kGLD + kk] = f32_bf16_rne(v);
    }
#pragma unroll
    for (int i = 0; i < (kGT * kGK) / 256; ++i) {
      const int e = tid + 256 * i;
      int c, kk;
      if (!g.transB) { kk = e / kGT; c = e % kGT; } else { c = e / kGK; kk = e % kGK; }
      const int cn = n0 + c, kx = k0 + kk;
      float v = 0.0f;
      if (cn < g.N && kx < g.K)
        v = g.transB ? g.B[(size_t)cn * g.ldb + kx] : g.B[(size_t)kx * g.ldb + cn];
      sB[c * kGLD + kk] = f32_bf16_rne(v);
    }
    __syncthreads();
    bf8l a[2], b[2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
      a[rb] = *reinterpret_cast<const bf8l*>(&sA[(wr * 32 + rb * 16 + col) * kGLD + grp * 8]);
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
      b[cb] = *reinterpret_cast<const bf8l*>(&sB[(wc * 32 + cb * 16 + col) * kGLD + grp * 8]);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wr * 32 + rb * 16 + 4 * grp + r;
        const int cn = n0 + wc * 32 + cb * 16 + col;
        if (row < M && cn < g.N) {
          float v = acc[rb][cb][r];
          if (g.bias) v += g.bias[cn];
          if (g.relu) v = v > 0.0f ? v : 0.0f;
          if (g.mask) v = g.mask[(size_t)row * g.ldm + cn] > 0.0f ? v : 0.0f;
          g.C[(size_t)row * g.ldc + cn] = v;
        }
      }
}

hipError_t launch_gemm_bf16(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  dim3 grid((g.N + kGT - 1) / kGT, (g.M + kGT - 1) / kGT);
  hipLaunchKernelGGL(gemm_bf16_kernel, grid, dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// training pieces
// ---------------------------------------------------------------------------

// One workgroup per row b of Z (B x k): loss_row[b] = logsumexp(z) - z[y],
// and dZ = (softmax(z) - onehot(y)) / B in place.
__global__ __launch_bounds__(256) void softmax_ce_kernel(float* __restrict__ Z,
                                                         int k,
                                                         const int32_t* __restrict__ y,
                                                         float invB,
                                                         double* __restrict__ loss_row) {
  __shared__ float red[256];
  float* z = Z + (size_t)blockIdx.x * k;
  float mx = -INFINITY;
  for (int j = threadIdx.x; j < k; j += 256) mx = fmaxf(mx, z[j]);
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  mx = red[0];
  __syncthreads();
  float sum = 0.0f;
  for (int j = threadIdx.x; j < k; j += 256) sum += expf(z[j] - mx);
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
  for (int j = threadIdx.x; j < k; j += 256) {
    const float p = expf(z[j] - mx) * inv;
    z[j] = (p - (j == yb ? 1.0f : 0.0f)) * invB;
  }
}

// out[c] = sum over rows of D[r][c] (FP32): thread (q, c) of a workgroup of
// 64 columns sums rows q, q + 4, ...; the four partial sums are then added.
__global__ __launch_bounds__(256) void colsum_kernel(const float* __restrict__ D,
                                                     int rows, int cols,
                                                     float* __restrict__ out) {
  __shared__ float part[4][64];
  const int cl = threadIdx.x & 63, q = threadIdx.x >> 6;
  const int c = blockIdx.x * 64 + cl;
  float s = 0.0f;
  if (c < cols)
    for (int r = q; r < rows; r += 4) s += D[(size_t)r * cols + c];
  part[q][cl] = s;
  __syncthreads();
  if (q == 0 && c < cols) out[c] = (part[0][cl] + part[1][cl]) + (part[2][cl] + part[3][cl]);
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

size_t mlp_train_workspace(int d, int h, int k, int B) {
  (void)d;
  return sizeof(float) * ((size_t)B * h * 4 + (size_t)B * k) + sizeof(double) * ((size_t)B + 1) +
         4096;
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
  double* lrow = (double*)c;
  hipError_t e;
  auto gemm = [&](const float* A, int lda, int tA, const float* Bm, int ldb, int tB,
                  float* C, int ldc, int M, int N, int K, const float* bias, int relu,
                  const float* mask, int ldm) {
    GemmArgs g{};
    g.A = A; g.lda = lda; g.transA = tA; g.B = Bm; g.ldb = ldb; g.transB = tB;
    g.C = C; g.ldc = ldc; g.M = M; g.N = N; g.K = K; g.bias = bias; g.relu = relu;
    g.mask = mask; g.ldm = ldm;
    return launch_gemm_bf16(g, s);
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
  hipLaunchKernelGGL(colsum_kernel, dim3((k + 63) / 64), dim3(256), 0, s, Z, B, k, grad + L.b3);
  if ((e = gemm(Z, k, 0, th + L.W3, k, 1, D2, h, B, h, k, nullptr, 0, H2, h))) return e;
  if ((e = gemm(H1, h, 1, D2, h, 0, grad + L.W2, h, h, h, B, nullptr, 0, nullptr, 0))) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((h + 63) / 64), dim3(256), 0, s, D2, B, h, grad + L.b2);
  if ((e = gemm(D2, h, 0, th + L.W2, h, 1, D1, h, B, h, h, nullptr, 0, H1, h))) return e;
  if ((e = gemm(Xs, d, 1, D1, h, 0, grad + L.W1, h, d, h, B, nullptr, 0, nullptr, 0))) return e;
  hipLaunchKernelGGL(colsum_kernel, dim3((h + 63) / 64), dim3(256), 0, s, D1, B, h, grad + L.b1);
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
// proposal: last layer on the matrix cores with the subset-argmax epilogue
// ---------------------------------------------------------------------------

// W3t[j][i] = bf16(W3[i][j]) (k x h, row stride h), classes past k zero
__global__ __launch_bounds__(256) void mlp_w3t_kernel(const float* __restrict__ W3,
                                                      int h, int k, int kpad,
                                                      uint16_t* __restrict__ W3t) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)kpad * h) return;
  const int j = (int)(e / h), i = (int)(e - (int64_t)j * h);
  W3t[e] = j < k ? f32_bf16_rne(W3[(size_t)i * k + j]) : (uint16_t)0;
}

constexpr int kPropWaves = 8;
constexpr int kPropCK = 64;        // classes per LDS chunk

// 16*PB points per wave (rows of H2, m of them); A = W3t rows (classes),
// B = the points' h2 (BF16 fragments), accumulator seeded with b3.  Lane
// (c, g) sees classes 4g + r of every block of 16; tracker t = block mod 4.
template <int KS, int PB>
__global__ __launch_bounds__(64 * kPropWaves) void mlp_propose_kernel(
    const float* __restrict__ H2, const uint16_t* __restrict__ W3t,
    const float* __restrict__ b3, int k, int kpad, int m, const int* __restrict__ mdev,
    int32_t* __restrict__ cand) {
  constexpr int H = KS * 32, LD = H + 8;
  __shared__ __attribute__((aligned(16))) uint16_t sW[kPropCK * LD];
  __shared__ float sb[kPropCK];
  const int mm = mdev ? (m < *mdev ? m : *mdev) : m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int col = lane & 15, grp = lane >> 4;
  const int64_t p0 = ((int64_t)blockIdx.x * kPropWaves + wave) * 16 * PB;
  if ((int64_t)blockIdx.x * kPropWaves * 16 * PB >= mm) return;   // uniform
  bf8l bx[PB][KS];
  bool valid[PB];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    const int64_t p = p0 + pb * 16 + col;
    valid[pb] = p < mm;
    const float* hr = H2 + (size_t)(valid[pb] ? p : 0) * H;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      uint32_t w[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float lo = valid[pb] ? hr[s * 32 + grp * 8 + 2 * e] : 0.0f;
        const float hi = valid[pb] ? hr[s * 32 + grp * 8 + 2 * e + 1] : 0.0f;
        w[e] = (uint32_t)f32_bf16_rne(lo) | ((uint32_t)f32_bf16_rne(hi) << 16);
      }
      const uint4 v4 = {w[0], w[1], w[2], w[3]};
      bx[pb][s] = __builtin_bit_cast(bf8l, v4);
    }
  }
  float best[PB][4];
  int idx[PB][4];
#pragma unroll
  for (int pb = 0; pb < PB; ++pb)
#pragma unroll
    for (int t = 0; t < 4; ++t) { best[pb][t] = -INFINITY; idx[pb][t] = -1; }
  for (int c0 = 0; c0 < kpad; c0 += kPropCK) {
    __syncthreads();
    for (int e = threadIdx.x; e < kPropCK * (H / 8); e += 64 * kPropWaves) {
      const int r = e / (H / 8), q = e - r * (H / 8);
      *reinterpret_cast<uint4*>(&sW[r * LD + q * 8]) =
          *reinterpret_cast<const uint4*>(W3t + (size_t)(c0 + r) * H + q * 8);
    }
    for (int e = threadIdx.x; e < kPropCK; e += 64 * kPropWaves)
      sb[e] = c0 + e < k ? b3[c0 + e] : -INFINITY;
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 4; ++t) {            // block t of the chunk: tracker t
      const int jb = c0 + t * 16;
      bf8l a[KS];
#pragma unroll
      for (int s = 0; s < KS; ++s)
        a[s] = *reinterpret_cast<const bf8l*>(&sW[(t * 16 + col) * LD + s * 32 + grp * 8]);
      const f4l init = *reinterpret_cast<const f4l*>(&sb[t * 16 + 4 * grp]);
      f4l acc[PB];
#pragma unroll
      for (int pb = 0; pb < PB; ++pb) acc[pb] = init;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int pb = 0; pb < PB; ++pb)
          acc[pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s], bx[pb][s], acc[pb], 0, 0, 0);
#pragma unroll
      for (int pb = 0; pb < PB; ++pb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float v = acc[pb][r];
          const bool gt = v > best[pb][t];
          best[pb][t] = gt ? v : best[pb][t];
          idx[pb][t] = gt ? jb + 4 * grp + r : idx[pb][t];
        }
    }
  }
#pragma unroll
  for (int pb = 0; pb < PB; ++pb) {
    if (!valid[pb]) continue;
    const int64_t p = p0 + pb * 16 + col;
#pragma unroll
    for (int t = 0; t < 4; ++t) cand[(size_t)p * 16 + 4 * grp + t] = idx[pb][t];
  }
}

hipError_t launch_mlp_propose(const float* H2, const uint16_t* W3t, const float* b3,
                              int h, int k, int kpad, int m, const int* mdev,
                              int32_t* cand, hipStream_t s) {
  constexpr int PB = 2;
  const int per_wg = kPropWaves * 16 * PB;
  const int grid = (m + per_wg - 1) / per_wg;
  if (grid <= 0) return hipSuccess;
  switch (h) {
    case 32: hipLaunchKernelGGL((mlp_propose_kernel<1, PB>), dim3(grid), dim3(64 * kPropWaves), 0, s, H2, W3t, b3, k, kpad, m, mdev, cand); break;
    case 64: hipLaunchKernelGGL((mlp_propose_kernel<2, PB>), dim3(grid), dim3(64 * kPropWaves), 0, s, H2, W3t, b3, k, kpad, m, mdev, cand); break;
    case 128: hipLaunchKernelGGL((mlp_propose_kernel<4, PB>), dim3(grid), dim3(64 * kPropWaves), 0, s, H2, W3t, b3, k, kpad, m, mdev, cand); break;
    case 256: hipLaunchKernelGGL((mlp_propose_kernel<8, PB>), dim3(grid), dim3(64 * kPropWaves), 0, s, H2, W3t, b3, k, kpad, m, mdev, cand); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_mlp_w3t(const float* W3, int h, int k, int kpad, uint16_t* W3t,
                          hipStream_t s) {
  const int64_t tot = (int64_t)kpad * h;
  hipLaunchKernelGGL(mlp_w3t_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s,
                     W3, h, k, kpad, W3t);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// inputs of the proposal and the certificate
// ---------------------------------------------------------------------------

// mean and 1/std per dimension in FP64 (population std; 0 -> 1): one
// workgroup per dimension.
template <typename T>
__global__ __launch_bounds__(256) void standardize_stats_kernel(
    const T* __restrict__ X, int64_t n, int d, double* __restrict__ mean,
    double* __restrict__ istd) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double s = 0.0;
  for (int64_t p = threadIdx.x; p < n; p += 256) s += to_f64<T>(X[(size_t)p * d + i]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  const double mu = red[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (int64_t p = threadIdx.x; p < n; p += 256) {
    const double t = to_f64<T>(X[(size_t)p * d + i]) - mu;
    q += t * t;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double sd = sqrt(red[0] / (double)n);
    mean[i] = mu;
    istd[i] = sd > 0.0 ? 1.0 / sd : 1.0;
  }
}

hipError_t launch_standardize_stats(const void* X, knor_dtype dt, int64_t n, int d,
                                    double* mean, double* istd, hipStream_t s) {
  switch (dt) {
    case KNOR_F32:
      hipLaunchKernelGGL(standardize_stats_kernel<float>, dim3(d), dim3(256), 0, s,
                         (const float*)X, n, d, mean, istd);
      break;
    case KNOR_F64:
      hipLaunchKernelGGL(standardize_stats_kernel<double>, dim3(d), dim3(256), 0, s,
                         (const double*)X, n, d, mean, istd);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(standardize_stats_kernel<uint16_t>, dim3(d), dim3(256), 0, s,
                         (const uint16_t*)X, n, d, mean, istd);
      break;
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

__global__ __launch_bounds__(256) void seg_dense_kernel(const int* __restrict__ list,
                                                        const int* __restrict__ seg_cnt,
                                                        const int* __restrict__ seg_off,
                                                        int* __restrict__ dense,
                                                        const int* __restrict__ conv,
                                                        int iter) {
  if (*conv < iter) return;
  const int b = blockIdx.x;
  const int cnt = seg_cnt[b], o = seg_off[b];
  for (int q = threadIdx.x; q < cnt; q += 256) dense[o + q] = list[(size_t)b * kSeg + q];
}

hipError_t launch_seg_dense(const int* list, const int* seg_cnt, int nseg, int* seg_off,
                            int* dense, const int* conv, int iter, hipStream_t s) {
  hipLaunchKernelGGL(seg_scan_kernel, dim3(1), dim3(1024), 0, s, seg_cnt, nseg, seg_off,
                     conv, iter);
  hipLaunchKernelGGL(seg_dense_kernel, dim3(nseg), dim3(256), 0, s, list, seg_cnt,
                     seg_off, dense, conv, iter);
  return hipGetLastError();
}

// Each centroid's kMlpNbr nearest other centroids, in increasing (D, j)
// order, with a rounded-down half of their distance: nbr_idx[i][t],
// nbr_half[i][t] (index -1 and +inf past the k - 1 others).  One workgroup
// per centroid: every thread keeps a sorted list of its own nearest
// kMlpNbr, then kMlpNbr rounds of a workgroup minimum over the list heads.
__global__ __launch_bounds__(256) void cc_neighbors_kernel(
    const double* __restrict__ C64, const double* __restrict__ CT, int k, int d,
    int* __restrict__ nbr_idx, float* __restrict__ nbr_half,
    const int* __restrict__ conv, int iter) {
  __shared__ double hd[256];
  __shared__ int hj[256], hw[256];
  if (*conv < iter) return;
  const int i = blockIdx.x;
  const double* ci = C64 + (size_t)i * d;
  double ld[kMlpNbr];
  int lj[kMlpNbr];
#pragma unroll
  for (int t = 0; t < kMlpNbr; ++t) { ld[t] = INFINITY; lj[t] = 0x7fffffff; }
  for (int j = threadIdx.x; j < k; j += 256) {
    if (j == i) continue;
    double acc = 0.0;
    for (int dim = 0; dim < d; ++dim) {
      const double t = __dsub_rn(ci[dim], CT[(size_t)dim * k + j]);
      acc = __dadd_rn(acc, __dmul_rn(t, t));
    }
    // insert (acc, j) into the sorted list (j increases, so ties keep order)
    if (acc < ld[kMlpNbr - 1]) {
#pragma unroll
      for (int t = kMlpNbr - 1; t >= 0; --t) {
        const bool above = t > 0 && acc < ld[t - 1];
        const bool here = acc < ld[t];
        const double nd = above ? ld[t - 1] : acc;
        const int nj = above ? lj[t - 1] : j;
        ld[t] = here ? nd : ld[t];
        lj[t] = here ? nj : lj[t];
      }
    }
  }
  int head = 0;
  for (int r = 0; r < kMlpNbr; ++r) {
    double v = INFINITY;
    int vj = 0x7fffffff;
#pragma unroll
    for (int t = 0; t < kMlpNbr; ++t)
      if (t == head) { v = ld[t]; vj = lj[t]; }
    hd[threadIdx.x] = v;
    hj[threadIdx.x] = vj;
    hw[threadIdx.x] = threadIdx.x;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
      if (threadIdx.x < st) {
        const double od = hd[threadIdx.x + st];
        const int oj = hj[threadIdx.x + st];
        if (od < hd[threadIdx.x] || (od == hd[threadIdx.x] && oj < hj[threadIdx.x])) {
          hd[threadIdx.x] = od;
          hj[threadIdx.x] = oj;
          hw[threadIdx.x] = hw[threadIdx.x + st];
        }
      }
      __syncthreads();
    }
    const double m = hd[0];
    const int mj = hj[0], mw = hw[0];
    if (threadIdx.x == 0) {
      const bool ok = m < INFINITY;
      nbr_idx[(size_t)i * kMlpNbr + r] = ok ? mj : -1;
      nbr_half[(size_t)i * kMlpNbr + r] =
          ok ? f32_down(0.5 * sqrt(m) * (1.0 - (double)(d + 8) * 2.220446049250313e-16))
             : INFINITY;
    }
    if (threadIdx.x == mw && m < INFINITY) ++head;
    __syncthreads();
  }
}

hipError_t launch_cc_neighbors(const double* C64, const double* CT, int k, int d,
                               int* nbr_idx, float* nbr_half, const int* conv, int iter,
                               hipStream_t s) {
  hipLaunchKernelGGL(cc_neighbors_kernel, dim3(k), dim3(256), 0, s, C64, CT, k, d,
                     nbr_idx, nbr_half, conv, iter);
  return hipGetLastError();
}

// The certificate.  One workgroup per segment, one lane per survivor (256
// per pass).  c* = the candidate with the smallest canonical FP64 distance
// (lowest index on ties); h = the rounded-down half distance from c* to its
// nearest centroid outside the candidate set (the first such entry of c*'s
// sorted neighbour list; +inf when every other centroid is a candidate).
// Accept iff ub (1 + eta) < h, ub an upper bound of d(x, c*) rounded up to
// FP32: every candidate is compared in the FP64 definition itself, and every
// other centroid j has d(x, j) >= d(c*, j) - d(x, c*) > ub (1 + 2 eta).
// Certified points take c* (and ub as their MTI bound); the others are
// appended, in segment order, to list2.
template <typename T>
__global__ __launch_bounds__(256) void mlp_certify_kernel(
    const T* __restrict__ X, int d, const double* __restrict__ C64,
    const int* __restrict__ nbr_idx, const float* __restrict__ nbr_half,
    const int* __restrict__ list, const int* __restrict__ seg_cnt,
    const int* __restrict__ seg_off, const int32_t* __restrict__ cand,
    int32_t* __restrict__ labels, float* __restrict__ ub_out, int* __restrict__ dirty,
    int* __restrict__ list2, int* __restrict__ seg_cnt2,
    unsigned long long* __restrict__ row, const int* __restrict__ conv, int iter) {
  __shared__ int wcnt[4];
  __shared__ int run;
  if (*conv < iter) return;
  const int b = blockIdx.x;
  const int cnt = seg_cnt[b], o = seg_off[b];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (threadIdx.x == 0) run = 0;
  __syncthreads();
  unsigned long long certified = 0, changes = 0;
  for (int q0 = 0; q0 < cnt; q0 += 256) {
    const int q = q0 + threadIdx.x;
    const bool live = q < cnt;
    bool cert = false;
    int p = 0;
    if (live) {
      p = list[(size_t)b * kSeg + q];
      int cj[kMlpTop];
      const int4* cr = reinterpret_cast<const int4*>(cand + (size_t)(o + q) * kMlpTop);
#pragma unroll
      for (int v = 0; v < kMlpTop / 4; ++v) {
        const int4 c4 = cr[v];
        cj[4 * v] = c4.x; cj[4 * v + 1] = c4.y; cj[4 * v + 2] = c4.z; cj[4 * v + 3] = c4.w;
      }
      const T* x = X + (size_t)p * d;
      double best = INFINITY;
      int bj = 0x7fffffff;
#pragma unroll 1
      for (int s = 0; s < kMlpTop; ++s) {
        const int j = cj[s];
        if (j < 0) continue;
        const double D = dist2_canon<T>(x, C64 + (size_t)j * d, d);
        if (D < best || (D == best && j < bj)) { best = D; bj = j; }
      }
      if (bj != 0x7fffffff) {
        float h = INFINITY;
        for (int t = 0; t < kMlpNbr; ++t) {
          const int nb = nbr_idx[(size_t)bj * kMlpNbr + t];
          if (nb < 0) break;                 // no further centroids
          bool in = false;
#pragma unroll
          for (int s = 0; s < kMlpTop; ++s) in |= cj[s] == nb;
          if (!in) { h = nbr_half[(size_t)bj * kMlpNbr + t]; break; }
        }
        const double ub = f32_up(sqrt(best * (1.0 + (double)(d + 8) * 2.220446049250313e-16)) *
                                 (1.0 + 8.881784197001252e-16));
        cert = ub * (1.0 + kEta) < (double)h;
        if (cert) {
          const int32_t old = labels[p];
          ub_out[p] = (float)ub;
          ++certified;
          if (old != bj) {                   // unchanged labels are not rewritten
            labels[p] = bj;
            ++changes;
            mark_dirty(dirty, old, bj);
          }
        }
      }
    }
    // uncertified survivors, in order
    const bool keep = live && !cert;
    const uint64_t km = __ballot(keep);
    if (lane == 0) wcnt[wave] = __popcll(km);
    __syncthreads();
    int base = run;
    for (int w = 0; w < wave; ++w) base += wcnt[w];
    if (keep) list2[(size_t)b * kSeg + base + __popcll(km & lanemask_lt())] = p;
    __syncthreads();
    if (threadIdx.x == 0) run += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
  if (threadIdx.x == 0) seg_cnt2[b] = run;
  const int qs[2] = {SLOT_CERTIFIED, SLOT_CHANGED};
  const unsigned long long v[2] = {certified, changes};
  block_add_slots<2>(row, qs, v);
}

hipError_t launch_mlp_certify(const void* X, knor_dtype dt, int d, const double* C64,
                              const int* nbr_idx, const float* nbr_half, const int* list,
                              const int* seg_cnt, const int* seg_off, int nseg,
                              const int32_t* cand, int32_t* labels, float* u, int* dirty,
                              int* list2, int* seg_cnt2, unsigned long long* row,
                              const int* conv, int iter, hipStream_t s) {
  switch (dt) {
    case KNOR_F32:
      hipLaunchKernelGGL(mlp_certify_kernel<float>, dim3(nseg), dim3(256), 0, s,
                         (const float*)X, d, C64, nbr_idx, nbr_half, list, seg_cnt, seg_off,
                         cand, labels, u, dirty, list2, seg_cnt2, row, conv, iter);
      break;
    case KNOR_F64:
      hipLaunchKernelGGL(mlp_certify_kernel<double>, dim3(nseg), dim3(256), 0, s,
                         (const double*)X, d, C64, nbr_idx, nbr_half, list, seg_cnt, seg_off,
                         cand, labels, u, dirty, list2, seg_cnt2, row, conv, iter);
      break;
    case KNOR_BF16:
      hipLaunchKernelGGL(mlp_certify_kernel<uint16_t>, dim3(nseg), dim3(256), 0, s,
                         (const uint16_t*)X, d, C64, nbr_idx, nbr_half, list, seg_cnt, seg_off,
                         cand, labels, u, dirty, list2, seg_cnt2, row, conv, iter);
      break;
  }
  return hipGetLastError();
}

}  // namespace knor
