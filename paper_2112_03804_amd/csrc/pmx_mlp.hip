// Kernels of the warm-start network (a small BF16 MLP, FP32 accumulation) for
// gfx950: a tiled GEMM on the matrix cores (v_mfma_f32_16x16x32_bf16), masked
// softmax cross-entropy, column sums for bias gradients, row gathers and
// Adam.  Each is a C-ABI call on caller-owned device buffers, asynchronous
// on the given stream; the network itself is orchestrated by the caller.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "pmx.h"

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
// C[M x N] = op(A)[M x K] * op(B)[K x N], FP32 accumulation on the gfx950
// matrix cores (v_mfma_f32_16x16x32_bf16: a 16 x 16 tile over 32 k per
// instruction, eight BF16 values of A and of B per lane).
// op(A)(m, k) = transA ? A[k * lda + m] : A[m * lda + k]
// op(B)(k, n) = transB ? B[n * ldb + k] : B[k * ldb + n]
// Epilogue per element: + bias[n]; ReLU; zero where mask[m * ldm + n] <= 0;
// store FP32 (C) and / or BF16 (Cb).
//
// Workgroup: 4 wavefronts, 64 x 64 output tile; each wavefront owns a 32 x 32
// quadrant (2 x 2 MFMA tiles).  K advances 64 per stage; both operands sit in
// LDS as [row][k] (k contiguous, rows padded by 16 bytes), so that a lane's
// eight k values of a fragment are one 16-byte LDS read.  Global loads are
// 16 bytes per lane where the operand's layout and alignment allow: eight
// consecutive k of one row (no transpose), or eight consecutive rows of one
// k, scattered into the [row][k] layout (transpose).  Two LDS buffers: the
// next stage's global loads are in flight while the current stage's MFMAs
// run, and one barrier per stage separates them.
//
// Split K (weight gradients: K = rows of the batch, M x N small): blockIdx.y
// takes one range of K and writes its raw FP32 tile to a workspace; a second
// kernel adds the ranges in a fixed order and applies the epilogue.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int GT = 64, GK = 64, GKP = GK + 8;   // tile, K stage, padded LDS row (bf16)

struct GemmArgs {
  int M, N, K, kchunk;          // kchunk: K range per blockIdx.y (a multiple of GK)
  const uint16_t* A;
  int lda;
  const uint16_t* B;
  int ldb;
  const float* bias;
  int relu;
  const float* mask;
  int ldm;
  float* C;
  int ldc;
  uint16_t* Cb;
  int ldcb;
  float* work;                  // split K: [gridDim.y][M][N] partial sums
};

// One operand's share of a stage: two 16-byte pieces per thread (64 rows x
// 64 k = 512 pieces).  Rows count along M (for A) or N (for B); TR: the
// operand is stored row-contiguous (X[k * ld + r]), else k-contiguous
// (X[r * ld + k]); VEC: 16-byte loads are aligned.
template <bool TR, bool VEC>
struct StageLoad {
  uint4 v[2];
  __device__ inline void load(const uint16_t* __restrict__ X, int ld, int rows, int r0, int k0, int kend,
                              int tid) {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = tid + 256 * j;
      uint16_t e[8];
      if (!TR) {   // X[r * ld + k]: eight consecutive k of row r
        const int r = r0 + c / 8, k = k0 + 8 * (c % 8);
        if (VEC && r < rows && k + 8 <= kend) {
          v[j] = *(const uint4*)(X + (int64_t)r * ld + k);
          continue;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (r < rows && k + i < kend) ? X[(int64_t)r * ld + k + i] : (uint16_t)0;
      } else {     // X[k * ld + r]: eight consecutive rows at one k
        const int k = k0 + c / 8, r = r0 + 8 * (c % 8);
        if (VEC && k < kend && r + 8 <= rows) {
          v[j] = *(const uint4*)(X + (int64_t)k * ld + r);
          continue;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) e[i] = (k < kend && r + i < rows) ? X[(int64_t)k * ld + r + i] : (uint16_t)0;
      }
      v[j] = make_uint4(e[0] | (uint32_t)e[1] << 16, e[2] | (uint32_t)e[3] << 16, e[4] | (uint32_t)e[5] << 16,
                        e[6] | (uint32_t)e[7] << 16);
    }
  }
  __device__ inline void store(uint16_t (*S)[GKP], int tid) const {
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = tid + 256 * j;
      if (!TR) {
        *(uint4*)&S[c / 8][8 * (c % 8)] = v[j];
      } else {
        const int k = c / 8, r = 8 * (c % 8);
        const uint32_t w[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          S[r + 2 * i][k] = (uint16_t)(w[i] & 0xffffu);
          S[r + 2 * i + 1][k] = (uint16_t)(w[i] >> 16);
        }
      }
    }
  }
};

__device__ inline void gemm_epilogue(const GemmArgs& P, int m, int n, float v) {
  if (P.bias) v += P.bias[n];
  if (P.relu) v = v > 0.f ? v : 0.f;
  if (P.mask && !(P.mask[(int64_t)m * P.ldm + n] > 0.f)) v = 0.f;
  if (P.C) P.C[(int64_t)m * P.ldc + n] = v;
  if (P.Cb) P.Cb[(int64_t)m * P.ldcb + n] = f2bf(v);
}

template <bool TRA, bool TRB, bool VA, bool VB>
__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs P) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][GT][GKP];   // [m][k]
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][GT][GKP];   // [n][k]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nbn = (P.N + GT - 1) / GT;
  const int m0 = (int)(blockIdx.x / nbn) * GT, n0 = (int)(blockIdx.x % nbn) * GT;
  const int kb = (int)blockIdx.y * P.kchunk, ke = min(P.K, kb + P.kchunk);
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  StageLoad<TRA, VA> la;
  StageLoad<TRB, VB> lb;
  const int nst = (ke - kb + GK - 1) / GK;
  if (nst > 0) {
    la.load(P.A, P.lda, P.M, m0, kb, ke, tid);
    lb.load(P.B, P.ldb, P.N, n0, kb, ke, tid);
    la.store(As[0], tid);
    lb.store(Bs[0], tid);
  }
  __syncthreads();
  for (int s = 0; s < nst; ++s) {
    const int buf = s & 1;
    if (s + 1 < nst) {   // the next stage's loads in flight during this stage's MFMAs
      la.load(P.A, P.lda, P.M, m0, kb + (s + 1) * GK, ke, tid);
      lb.load(P.B, P.ldb, P.N, n0, kb + (s + 1) * GK, ke, tid);
    }
#pragma unroll
    for (int kk = 0; kk < GK; kk += 32) {
      const int kq = kk + 8 * (lane >> 4);
      bf16x8 a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = *(const bf16x8*)&As[buf][wm + 16 * t + (lane & 15)][kq];
        b[t] = *(const bf16x8*)&Bs[buf][wn + 16 * t + (lane & 15)][kq];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (s + 1 < nst) {
      la.store(As[buf ^ 1], tid);
      lb.store(Bs[buf ^ 1], tid);
    }
    __syncthreads();
  }
  // lane holds D[4 * (lane / 16) + r][lane % 16] of each 16 x 16 tile
  float* wk = P.work ? P.work + (int64_t)blockIdx.y * P.M * P.N : nullptr;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + wn + 16 * j + (lane & 15);
        if (m >= P.M || n >= P.N) continue;
        if (wk) wk[(int64_t)m * P.N + n] = acc[i][j][r];
        else gemm_epilogue(P, m, n, acc[i][j][r]);
      }
}

// Split K: the ranges' partial tiles added in range order, then the epilogue.
__global__ __launch_bounds__(256) void k_gemm_reduce(GemmArgs P, int splits) {
  const int64_t mn = (int64_t)P.M * P.N;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mn; i += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    for (int z = 0; z < splits; ++z) v += P.work[z * mn + i];
    gemm_epilogue(P, (int)(i / P.N), (int)(i % P.N), v);
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

// db[n] = sum over rows of dZ[m][n] (fixed order).  Without a workspace one
// thread per column walks every row; with one, blockIdx.y sums a range of
// kColRows rows into the workspace and k_colsum_reduce adds the ranges in
// order.
constexpr int kColRows = 64;
__global__ __launch_bounds__(256) void k_colsum(int rows, int cols, const float* __restrict__ dz,
                                                float* __restrict__ db, float* __restrict__ work) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= cols) return;
  const int r0 = work ? (int)blockIdx.y * kColRows : 0, r1 = work ? min(rows, r0 + kColRows) : rows;
  float s = 0.f;
  for (int m = r0; m < r1; ++m) s += dz[(int64_t)m * cols + n];
  if (work) work[(int64_t)blockIdx.y * cols + n] = s;
  else db[n] = s;
}
__global__ __launch_bounds__(256) void k_colsum_reduce(int parts, int cols, const float* __restrict__ work,
                                                       float* __restrict__ db) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= cols) return;
  float s = 0.f;
  for (int z = 0; z < parts; ++z) s += work[(int64_t)z * cols + n];
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
                  float* work, int64_t work_elems, void* stream) {
  if (M < 0 || N < 0 || K < 0 || !A || !B || (!C && !Cb) || work_elems < 0)
    return mfail(PMX_EINVAL, "bad GEMM arguments");
  if ((transA ? lda < M : lda < K) || (transB ? ldb < K : ldb < N) || (C && ldc < N) ||
      (Cb && ldcb < N) || (mask && ldm < N))
    return mfail(PMX_EINVAL, "GEMM leading dimension too small");
  if (M == 0 || N == 0) return PMX_OK;
  const int64_t tiles = (int64_t)((N + GT - 1) / GT) * ((M + GT - 1) / GT);
  if (tiles > 0x7fffffff) return mfail(PMX_EINVAL, "GEMM too large");
  // split K when the tiles alone leave the chip idle and K is long: about
  // 2048 workgroups, at least 256 of K each, as the workspace allows
  int splits = 1;
  if (work && tiles < 512 && K >= 2 * 256) {
    const int64_t want = std::min<int64_t>(K / 256, (2048 + tiles - 1) / tiles);
    const int64_t room = work_elems / ((int64_t)M * N);
    splits = (int)std::max<int64_t>(1, std::min<int64_t>({want, room, 64}));
  }
  int kchunk = (int)((((int64_t)K + splits - 1) / splits + GK - 1) / GK * GK);
  if (kchunk == 0) kchunk = GK;
  splits = (int)(((int64_t)K + kchunk - 1) / kchunk);
  if (splits < 1) splits = 1;
  GemmArgs P{M, N, K, kchunk, A, lda, B, ldb, bias, relu, mask, ldm, C, ldc, Cb, ldcb, splits > 1 ? work : nullptr};
  // 16-byte loads need 16-byte aligned rows: base and leading dimension
  const bool va = ((uintptr_t)A % 16 == 0) && (lda % 8 == 0);
  const bool vb = ((uintptr_t)B % 16 == 0) && (ldb % 8 == 0);
  const dim3 grid((unsigned)tiles, (unsigned)splits);
  hipStream_t s = (hipStream_t)stream;
  auto go = [&](auto kern) { hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, P); };
  // op(A) row-contiguous when transposed; op(B) when not (B[k * ldb + n])
  const int sel = (transA ? 8 : 0) | (transB ? 0 : 4) | (va ? 2 : 0) | (vb ? 1 : 0);
  switch (sel) {
    case 0: go(k_gemm_bf16<false, false, false, false>); break;
    case 1: go(k_gemm_bf16<false, false, false, true>); break;
    case 2: go(k_gemm_bf16<false, false, true, false>); break;
    case 3: go(k_gemm_bf16<false, false, true, true>); break;
    case 4: go(k_gemm_bf16<false, true, false, false>); break;
    case 5: go(k_gemm_bf16<false, true, false, true>); break;
    case 6: go(k_gemm_bf16<false, true, true, false>); break;
    case 7: go(k_gemm_bf16<false, true, true, true>); break;
    case 8: go(k_gemm_bf16<true, false, false, false>); break;
    case 9: go(k_gemm_bf16<true, false, false, true>); break;
    case 10: go(k_gemm_bf16<true, false, true, false>); break;
    case 11: go(k_gemm_bf16<true, false, true, true>); break;
    case 12: go(k_gemm_bf16<true, true, false, false>); break;
    case 13: go(k_gemm_bf16<true, true, false, true>); break;
    case 14: go(k_gemm_bf16<true, true, true, false>); break;
    default: go(k_gemm_bf16<true, true, true, true>); break;
  }
  if (splits > 1) {
    const int64_t mn = (int64_t)M * N;
    hipLaunchKernelGGL(k_gemm_reduce, dim3((unsigned)std::min<int64_t>((mn + 255) / 256, 4096)), dim3(256), 0, s,
                       P, splits);
  }
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

int mlp_colsum(int32_t rows, int32_t cols, const float* dz, float* db, float* work, int64_t work_elems,
               void* stream) {
  if (rows < 0 || cols < 1 || !dz || !db || work_elems < 0) return mfail(PMX_EINVAL, "bad colsum arguments");
  hipStream_t s = (hipStream_t)stream;
  const int parts = (rows + kColRows - 1) / kColRows;
  if (work && parts > 1 && (int64_t)parts * cols <= work_elems) {
    hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256, parts), dim3(256), 0, s, rows, cols, dz, db, work);
    hipLaunchKernelGGL(k_colsum_reduce, dim3((cols + 255) / 256), dim3(256), 0, s, parts, cols, work, db);
  } else {
    hipLaunchKernelGGL(k_colsum, dim3((cols + 255) / 256), dim3(256), 0, s, rows, cols, dz, db, nullptr);
  }
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
