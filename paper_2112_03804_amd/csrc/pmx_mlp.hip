// Kernels of the warm-start network (a small BF16 MLP, FP32 accumulation) for
// gfx950: a tiled GEMM on the matrix cores (v_mfma_f32_16x16x16_bf16), masked
// softmax cross-entropy, column sums for bias gradients, row gathers and
// Adam.  Each is a C-ABI call on caller-owned device buffers, asynchronous
// on the given stream; the network itself is orchestrated by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "pmx.h"

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

void pmx_set_error(const char* m);   // shared with the game library (pmx_last_error)

static int mfail(int code, const char* m) {
  pmx_set_error(m);
  return code;
}

#define MLP_TRY(expr)                                   \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return mfail(PMX_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

__device__ inline uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// C[M x N] = op(A)[M x K] * op(B)[K x N], FP32 accumulation on MFMA.
// op(A)(m, k) = transA ? A[k * lda + m] : A[m * lda + k]
// op(B)(k, n) = transB ? B[n * ldb + k] : B[k * ldb + n]
// Epilogue per element: + bias[n]; ReLU; zero where mask[m * ldm + n] <= 0;
// store FP32 (C) and / or BF16 (Cb).
// Workgroup: 4 wavefronts, 64 x 64 output tile; each wavefront owns a 32 x 32
// quadrant = 2 x 2 MFMA tiles; K advances 32 per LDS stage.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 32, GKP = GK + 4;   // tile, K stage, padded LDS row

__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A,
                                                   int lda, int transA, const uint16_t* __restrict__ B,
                                                   int ldb, int transB, const float* __restrict__ bias,
                                                   int relu, const float* __restrict__ mask, int ldm,
                                                   float* __restrict__ C, int ldc,
                                                   uint16_t* __restrict__ Cb, int ldcb) {
  __shared__ uint16_t As[GT][GKP];   // [m][k]
  __shared__ uint16_t Bs[GT][GKP];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nbn = (N + GT - 1) / GT;
  const int m0 = (int)(blockIdx.x / nbn) * GT, n0 = (int)(blockIdx.x % nbn) * GT;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int k0 = 0; k0 < K; k0 += GK) {
    // stage: 64 x 32 of op(A) and of op(B)^T, 8 elements per thread each
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid * 8 + e;      // 0 .. 2047
      int r, c;
      if (transA) {                      // consecutive threads walk m (contiguous in memory)
        r = idx % GT;
        c = idx / GT;
      } else {                           // consecutive threads walk k
        r = idx / GK;
        c = idx % GK;
      }
      const int m = m0 + r, k = k0 + c;
      uint16_t v = 0;
      if (m < M && k < K) v = transA ? A[(int64_t)k * lda + m] : A[(int64_t)m * lda + k];
      As[r][c] = v;
      int rn, cn;
      if (transB) {
        rn = idx / GK;
        cn = idx % GK;
      } else {
        rn = idx % GT;
        cn = idx / GT;
      }
      const int n = n0 + rn, kb = k0 + cn;
      uint16_t u = 0;
      if (n < N && kb < K) u = transB ? B[(int64_t)n * ldb + kb] : B[(int64_t)kb * ldb + n];
      Bs[rn][cn] = u;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; kk += 16) {
      const int kq = kk + 4 * (lane >> 4);
      bf16x4 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int row = wm + 16 * t + (lane & 15);
        const int col = wn + 16 * t + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[t][q] = (short)As[row][kq + q];
          b[t][q] = (short)Bs[col][kq + q];
        }
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // epilogue: lane holds D[4 * (lane / 16) + r][lane % 16] of each 16 x 16 tile
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= M || n >= N) continue;
        float v = acc[i][j][r];
        if (bias) v += bias[n];
        if (relu) v = v > 0.f ? v : 0.f;
        if (mask && !(mask[(int64_t)m * ldm + n] > 0.f)) v = 0.f;
        if (C) C[(int64_t)m * ldc + n] = v;
        if (Cb) Cb[(int64_t)m * ldcb + n] = f2bf(v);
      }
}

// Masked softmax cross-entropy per row: targets < 0 mark invalid actions.
// loss_r = w_r * sum_a -t_a log p_a ; dlogits = w_r * (p - t) on valid actions.
__global__ __launch_bounds__(256) void k_softmax_xent(int rows, int K, const float* __restrict__ z, int ldz,
                                                      const float* __restrict__ t, const float* __restrict__ wt,
                                                      float* __restrict__ dz, uint16_t* __restrict__ dzb,
                                                      float* __restrict__ partial) {
  __shared__ float red[256];
  const int r = blockIdx.x * 256 + threadIdx.x;
  float loss = 0.f;
  if (r < rows) {
    const float* zr = z + (int64_t)r * ldz;
    const float* tr = t + (int64_t)r * K;
    float mx = -INFINITY;
    for (int a = 0; a < K; ++a)
      if (tr[a] >= 0.f) mx = fmaxf(mx, zr[a]);
    float se = 0.f;
    for (int a = 0; a < K; ++a)
      if (tr[a] >= 0.f) se += __expf(zr[a] - mx);
    const float lse = mx + __logf(se);
    const float w = wt ? wt[r] : 1.f;
    for (int a = 0; a < K; ++a) {
      float g = 0.f;
      if (tr[a] >= 0.f) {
        const float lp = zr[a] - lse;
        loss -= tr[a] * lp;
        g = w * (__expf(lp) - tr[a]);
      }
      if (dz) dz[(int64_t)r * K + a] = g;
      if (dzb) dzb[(int64_t)r * K + a] = f2bf(g);
    }
    loss *= w;
  }
  red[threadIdx.x] = loss;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && partial) partial[blockIdx.x] = red[0];
}

// db[n] = sum over rows of dZ[m][n] (fixed order).
__global__ __launch_bounds__(256) void k_colsum(int rows, int cols, const float* __restrict__ dz,
                                                float* __restrict__ db) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= cols) return;
  float s = 0.f;
  for (int m = 0; m < rows; ++m) s += dz[(int64_t)m * cols + n];
  db[n] = s;
}

__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, uint16_t* __restrict__ wb, float lr, float b1, float b2,
                       float eps, float wd, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i] + wd * w[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = f2bf(wi);
  }
}

__global__ void k_gather_bf16(int64_t n, int width, const int64_t* __restrict__ idx,
                              const uint16_t* __restrict__ src, uint16_t* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * width;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / width, c = i % width;
    dst[i] = src[idx[r] * width + c];
  }
}

__global__ void k_gather_f32(int64_t n, int width, const int64_t* __restrict__ idx,
                             const float* __restrict__ src, float* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * width;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / width, c = i % width;
    dst[i] = src[idx[r] * width + c];
  }
}

__global__ void k_cast_bf16(int64_t n, const float* __restrict__ src, uint16_t* __restrict__ dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = f2bf(src[i]);
}

static int grid_for(int64_t n) { return (int)std::min<int64_t>((n + 255) / 256, 8192); }

extern "C" {

int mlp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, int32_t lda, int32_t transA,
                  const uint16_t* B, int32_t ldb, int32_t transB, const float* bias, int32_t relu,
                  const float* mask, int32_t ldm, float* C, int32_t ldc, uint16_t* Cb, int32_t ldcb,
                  void* stream) {
  if (M < 0 || N < 0 || K < 0 || !A || !B || (!C && !Cb)) return mfail(PMX_EINVAL, "bad GEMM arguments");
  if ((transA ? lda < M : lda < K) || (transB ? ldb < K : ldb < N) || (C && ldc < N) ||
      (Cb && ldcb < N) || (mask && ldm < N))
    return mfail(PMX_EINVAL, "GEMM leading dimension too small");
  if (M == 0 || N == 0) return PMX_OK;
  const int64_t tiles = (int64_t)((N + GT - 1) / GT) * ((M + GT - 1) / GT);
  if (tiles > 0x7fffffff) return mfail(PMX_EINVAL, "GEMM too large");
  dim3 grid((unsigned)tiles);
  hipLaunchKernelGGL(k_gemm_bf16, grid, dim3(256), 0, (hipStream_t)stream, M, N, K, A, lda, transA, B,
                     ldb, transB, bias, relu, mask, ldm, C, ldc, Cb, ldcb);
  MLP_TRY(hipGetLastError());
  return PMX_OK;
}

int mlp_softmax_xent(int32_t rows, int32_t K, const float* logits, int32_t ldl, const float* target,
                     const float* weight, float* dlogits, uint16_t* dlogits_bf16, float* loss_partial,
                     void* stream) {
  if (rows < 0 || K < 1 || K > 64 || !logits || !target || ldl < K) return mfail(PMX_EINVAL, "bad xent arguments");
  if (rows == 0) return PMX_OK;
  hipLaunchKernelGGL(k_softmax_xent, dim3((rows + 255) / 256), dim3(256), 0, (hipStream_t)stream, rows, K,
                     logits, ldl, target, weight, dlogits, dlogits_bf16, loss_partial);
  MLP_TRY(hipGetLastError());
  return PMX_OK;
}

int mlp_colsum(int32_t rows, int32_t cols, const float* dz, float* db, void* stream) {
  if (rows < 0 || cols < 1 || !dz || !db) return mfail(PMX_EINVAL, "bad colsum arguments");
  hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, (hipStream_t)stream, rows, cols, dz, db);
  MLP_TRY(hipGetLastError());
  return PMX_OK;
}

int mlp_adam(int64_t n, float* w, const float* g, float* m, float* v, uint16_t* w_bf16, float lr, float beta1,
             float beta2, float eps, float weight_decay, int32_t step, void* stream) {
  if (n < 0 || !w || !g || !m || !v || step < 1) return mfail(PMX_EINVAL, "bad Adam arguments");
  if (n == 0) return PMX_OK;
  const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n, w, g, m, v, w_bf16, lr,
                     beta1, beta2, eps, weight_decay, c1, c2);
  MLP_TRY(hipGetLastError());
  return PMX_OK;
}

int mlp_gather_bf16(int64_t n, int32_t width, const int64_t* idx, const uint16_t* src, uint16_t* dst,
                    void* stream) {
  if (n < 0 || width < 1 || !idx || !src || !dst) return mfail(PMX_EINVAL, "bad gather arguments");
  if (n == 0) return PMX_OK;
  hipLaunchKernelGGL(k_gather_bf16, dim3(grid_for(n * width)), dim3(256), 0, (hipStream_t)stream, n, width, idx,
                     src, dst);
  MLP_TRY(hipGetLastError());
  return PMX_OK;
}

int mlp_gather_f32(int64_t n, int32_t width, const int64_t* idx, const float* src, float* dst, void* stream) {
  if (n < 0 || width < 1 || !idx || !src || !dst) return mfail(PMX_EINVAL, "bad gather arguments");
  if (n == 0) return PMX_OK;
  hipLaunchKernelGGL(k_gather_f32, dim3(grid_for(n * width)), dim3(256), 0, (hipStream_t)stream, n, width, idx,
                     src, dst);
  MLP_TRY(hipGetLastError());
  return PMX_OK;
}

int mlp_cast_bf16(int64_t n, const float* src, uint16_t* dst, void* stream) {
  if (n < 0 || !src || !dst) return mfail(PMX_EINVAL, "bad cast arguments");
  if (n == 0) return PMX_OK;
  hipLaunchKernelGGL(k_cast_bf16, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, n, src, dst);
  MLP_TRY(hipGetLastError());
  return PMX_OK;
}

}  // extern "C"
