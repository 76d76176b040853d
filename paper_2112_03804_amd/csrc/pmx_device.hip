// libpmx device code for gfx950 (CDNA4) and the C ABI.
//
// Kernels
//   k_mvc         rows of A y (or A^T x), schedules 2 and 3 and every FP64 product: one
//                 workgroup of 256 or 512 threads per chunk of output rows,
//                 one launch per hands-per-thread class, on the
//                 chunk-aligned layout (every segment starts at a thread's
//                 chunk of slots).  Per item it applies the hand factor of
//                 Prop. 1 without forming it:
//                   - fold / compatibility (eq. cf): total of the opponent's
//                     weighted vector minus its per-card sums plus the
//                     identical hand (inclusion-exclusion over shared cards);
//                   - showdown (Technique B: the inverse of the bidiagonal
//                     difference operator is a prefix sum over hands sorted
//                     by strength): exclusive prefix sums over the sorted
//                     opponent hands and inside each card's sorted sub-list,
//                     read at the tie-aware positions of each own hand.
//                 All prefix sums come from one segmented scan over LDS:
//                 FP32 sums inside a thread's chunk, FP64 carries across
//                 chunks (FP64 adds issue at the unpacked FP32 rate on
//                 CDNA4, so this costs less than compensated FP32).
//   k_mvg         rows of A y (or A^T x), the default FP32 schedule (4):
//                 groups of up to four input rows of one board context
//                 share one staged gather, one segmented scan and one set of
//                 prefix slots; every output row takes its showdown and fold
//                 terms by coefficient.
//   k_rmp         regret matching+ (or discounted CFR) on pieces of a
//                 treeplex of at most 64 sequences, one lane per hand (the
//                 paper's GPU solver updates all hands in parallel), the
//                 piece's rows resident in LDS during the walk; four
//                 wavefronts walk subtree groups of the piece concurrently.
//   k_br          FP64 best responses (bottom-up max / min) for the gap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pmx_internal.hpp"

using namespace pmx;

// ---------------------------------------------------------------------------
// error plumbing
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

void pmx_set_error(const char* m) { g_err = m; }

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(PMX_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

// ---------------------------------------------------------------------------
// structured matvec
// ---------------------------------------------------------------------------
// One direction of a launch as the host sees it: the layouts of the
// schedule in use supply the rest.
struct MvParams {
  double scale;
  int32_t nblk;              // row chunks of the direction (0: the direction is not launched)
  int32_t dir;
  const int32_t* active;     // per-instance flag (NULL: all); inactive chunks are skipped
};

__device__ inline int lo16(uint32_t v) { return (int)(int16_t)(v & 0xffffu); }
__device__ inline int hi16(uint32_t v) { return (int)(int16_t)(v >> 16); }

// ---------------------------------------------------------------------------
// chunk-aligned matvec (kernels 2 and 3; layout in McCtx)
// ---------------------------------------------------------------------------
// DPP lane moves (CDNA encodings): row_shr:n = 0x110 + n, row_bcast:15 =
// 0x142, row_bcast:31 = 0x143, wave_shr:1 = 0x138.  Lanes without a source
// (or outside the row mask) read 0.
template <int CTRL, int RM>
__device__ inline int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, RM, 0xf, false);
}
template <int CTRL, int RM>
__device__ inline double dpp_d(double v) {
  const int lo = dpp_i<CTRL, RM>(__double2loint(v));
  const int hi = dpp_i<CTRL, RM>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}
// One step of an inclusive segmented scan of (flag, a, b): the element from
// the earlier lane is added unless this lane's run already holds a flag.
template <int CTRL, int RM>
__device__ inline void seg_step(int& f, double& a, double& b) {
  const int f2 = dpp_i<CTRL, RM>(f);
  const double a2 = dpp_d<CTRL, RM>(a), b2 = dpp_d<CTRL, RM>(b);
  if (!f) {
    a += a2;
    b += b2;
  }
  f |= f2;
}

// Exclusive segmented scan over the threads of a block: thread t receives
// the sum of a (and b) over the threads from the nearest thread at or before
// t - 1 whose flag is set, up to t - 1; 0 if t's own flag is set.  One
// barrier; `scr` holds 3 doubles per wavefront and is free again after the
// caller's next barrier.
template <int NW>
__device__ inline void block_seg_scan_x(int flag, double a, double b, double* scr, double& ea, double& eb) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int f = flag;
  double ai = a, bi = b;
  seg_step<0x111, 0xf>(f, ai, bi);
  seg_step<0x112, 0xf>(f, ai, bi);
  seg_step<0x114, 0xf>(f, ai, bi);
  seg_step<0x118, 0xf>(f, ai, bi);
  seg_step<0x142, 0xa>(f, ai, bi);
  seg_step<0x143, 0xc>(f, ai, bi);
  if (lane == 63) {
    scr[3 * wid + 0] = (double)f;
    scr[3 * wid + 1] = ai;
    scr[3 * wid + 2] = bi;
  }
  __syncthreads();
  // carry into this wavefront: lane w holds wavefront w's (flag, totals),
  // a segmented scan across those lanes (three DPP steps, NW <= 8) combines
  // them, and the carry is the scan at lane wid - 1
  static_assert(NW <= 8, "wavefront totals are scanned within one DPP row");
  int fw = 0;
  double aw = 0.0, bw = 0.0;
  if (lane < NW) {
    fw = scr[3 * lane] != 0.0;
    aw = scr[3 * lane + 1];
    bw = scr[3 * lane + 2];
  }
  seg_step<0x111, 0xf>(fw, aw, bw);
  seg_step<0x112, 0xf>(fw, aw, bw);
  seg_step<0x114, 0xf>(fw, aw, bw);
  double ca = 0.0, cb = 0.0;
  if (wid > 0) {
    const int src = wid - 1;
    ca = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(aw), src),
                          __builtin_amdgcn_readlane(__double2loint(aw), src));
    cb = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(bw), src),
                          __builtin_amdgcn_readlane(__double2loint(bw), src));
  }
  if (!f) {
    ai += ca;
    bi += cb;
  }
  double pa = dpp_d<0x138, 0xf>(ai), pb = dpp_d<0x138, 0xf>(bi);
  if (lane == 0) {
    pa = ca;
    pb = cb;
  }
  ea = flag ? 0.0 : pa;
  eb = flag ? 0.0 : pb;
}

struct McParams {
  const MvItem* items;
  const int4* chunks;            // (first item, end item, instance, first context) per workgroup
  const McCtx* ctx;
  const uint4* q;
  const uint2* pos;
  const uint32_t* meta;
  const double* lam;
  const float* lamf;
  const int32_t* active;         // per-instance flag (NULL: all)
  void* part;                    // partial rows of rows cut into parts (IO elements)
  double scale;
  int32_t nchunk;
};
template <typename IO>
__device__ inline const IO* mc_lam(const McParams& P);
template <>
__device__ inline const float* mc_lam<float>(const McParams& P) { return P.lamf; }
template <>
__device__ inline const double* mc_lam<double>(const McParams& P) { return P.lam; }

// LDS value at a slot given as the byte offset of a 4-byte value.
template <typename IO>
__device__ inline IO& at_slot(IO* base, int off4) {
  return *(IO*)((char*)base + (sizeof(IO) == 4 ? off4 : 2 * off4));
}

template <typename IO>
struct Vec4;
template <>
struct Vec4<float> {
  static constexpr int N = 4;   // values per 16-byte LDS access
  __device__ static void ld(const float* p, float* v) {
    const float4 t = *(const float4*)p;
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  }
  __device__ static void st(float* p, const float* v) { *(float4*)p = make_float4(v[0], v[1], v[2], v[3]); }
};
template <>
struct Vec4<double> {
  static constexpr int N = 2;
  __device__ static void ld(const double* p, double* v) {
    const double2 t = *(const double2*)p;
    v[0] = t.x; v[1] = t.y;
  }
  __device__ static void st(double* p, const double* v) { *(double2*)p = make_double2(v[0], v[1]); }
};

// One workgroup per row chunk.  Per item: the weighted opponent inputs are
// written to their three slots (global, card 0, card 1), each thread sums its
// chunk of KE slots in FP64, a segmented block scan carries the sums across
// chunks of a segment, each thread writes its chunk's exclusive prefix sums
// (rounded once to IO) over the showdown channel and its segment totals, and
// every own hand reads the prefix sums at its query slots (Technique B) and
// the per-card fold totals (eq. cf).
// Wavefronts per SIMD each FP32 class is built for: the register budget of
// the workgroups per CU its LDS allows (4 of 256 threads for the small
// classes, 3 and 2 for the larger ones, 2 of 512).  The FP64 forms, used for
// the gap only, are left unconstrained.
template <int BLOCK, int KH, typename IO>
constexpr int mc_waves_per_simd() {
  return sizeof(IO) != 4 ? 1 : (BLOCK == 512 ? 4 : (KH <= 2 ? 4 : (KH <= 4 ? 3 : 2)));
}

template <int BLOCK, int KH, typename IO>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(mc_waves_per_simd<BLOCK, KH, IO>())))
void k_mvc(McParams P0, const IO* __restrict__ in0, IO* __restrict__ out0,
                                               McParams P1, const IO* __restrict__ in1, IO* __restrict__ out1,
                                               double* __restrict__ tick) {
  constexpr int KE = BLOCK == 512 ? 4 * KH : 4 * KH + 4;
  constexpr int SK = KE + (KE % 8 == 0 ? 4 : 0);
  constexpr int NW = BLOCK / 64;
  constexpr int NSLOT = BLOCK * SK;
  constexpr int VN = Vec4<IO>::N;
  static_assert(KE % 4 == 0, "chunks are read 16 bytes at a time");
  if (tick && blockIdx.x == 0 && threadIdx.x == 0) tick[0] += 1.0;
  const bool second = (int)blockIdx.x >= P0.nchunk;
  const McParams& P = second ? P1 : P0;
  const IO* __restrict__ in = second ? in1 : in0;
  IO* __restrict__ out = second ? out1 : out0;
  const IO* __restrict__ lam = mc_lam<IO>(P);
  const int4 cr = P.chunks[second ? (int)blockIdx.x - P0.nchunk : (int)blockIdx.x];
  if (P.active && !P.active[cr.z]) return;   // retired instance
  const int tid = threadIdx.x;
  extern __shared__ double smem[];
  double* segT = smem;                        // [2 * kMcSegMax] (showdown, fold) totals per segment
  double* scr = segT + 2 * kMcSegMax;         // [3 * NW] scan scratch
  IO* S = (IO*)(scr + 3 * NW);                // [NSLOT] showdown values, then exclusive prefix sums
  IO* F = S + NSLOT;                          // [NSLOT] fold values

  uint4 qr[KH];
  uint2 ps[KH];
  IO lo[KH], lp[KH];
  double acc[KH];
  IO nxs[KH], nxf[KH];
#pragma unroll
  for (int k = 0; k < KH; ++k) acc[k] = 0.0;
  uint32_t cm = 0;
  int n_own = 0, cph = 1, n_chunk = 0, cur = -2, fz = -2;

  const int it0 = cr.x, it1 = cr.y;
  // the records of the chunk's first context load beside its first item, so
  // that both the inputs and the context's per-hand records are one
  // dependent load away from the chunk record.  These loads and the input
  // fetches are written out at each use: lambdas capturing the per-hand
  // arrays by reference kept those arrays in scratch memory.
  if (cr.w >= 0) {
    const McCtx C = P.ctx[cr.w];
    n_own = C.n_own;
    cph = C.cph;
    n_chunk = C.n_chunk;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int h = tid + k * BLOCK;
      qr[k] = h < C.n_own ? P.q[C.q_off + h] : make_uint4(0xffffffffu, 0u, 0u, 0u);
      lo[k] = h < C.n_own ? lam[C.lam_own_off + h] : (IO)0;
      ps[k] = h < C.n_opp ? P.pos[C.pos_off + h] : make_uint2(0xffffffffu, 0xffffffffu);
      lp[k] = h < C.n_opp ? lam[C.lam_opp_off + h] : (IO)0;
    }
    cm = P.meta[C.meta_off + tid];
    cur = cr.w;
  }
  if (it0 < it1)
  {
    const MvItem nx = P.items[it0];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const int h = tid + k * BLOCK;
      nxs[k] = (h < nx.n_opp && nx.in_s >= 0) ? in[nx.in_s + h] : (IO)0;
      nxf[k] = (h < nx.n_opp && nx.in_f >= 0) ? in[nx.in_f + h] : (IO)0;
    }
  }
  for (int it = it0; it < it1; ++it) {
    const MvItem item = P.items[it];
    IO cs_in[KH], cf_in[KH];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      cs_in[k] = nxs[k];
      cf_in[k] = nxf[k];
    }
    if (it + 1 < it1)
    {
      const MvItem nx = P.items[it + 1];
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLOCK;
        nxs[k] = (h < nx.n_opp && nx.in_s >= 0) ? in[nx.in_s + h] : (IO)0;
        nxf[k] = (h < nx.n_opp && nx.in_f >= 0) ? in[nx.in_f + h] : (IO)0;
      }
    }
    if (item.ctx < 0) {
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLOCK;
        if (h < item.stride) out[item.out + h] = (IO)0;
      }
      continue;
    }
    __syncthreads();   // the previous item's readers of S, F and segT are done
    {
      // Slots past each segment's entries must read as 0 in the chunk sums.
      // Fold slots are written only by the scatter, so they are zeroed once
      // per context; showdown slots also receive the previous item's
      // prefixes, so each thread zeroes its own chunk before every scatter.
      // Both replace a mask per entry in the sums.
      const bool zf = item.ctx != fz, zs = item.in_s >= 0;
      if (zf || zs) {
        IO z[VN];
#pragma unroll
        for (int u = 0; u < VN; ++u) z[u] = (IO)0;
        if (zs)
#pragma unroll
          for (int j = 0; j < KE; j += VN) Vec4<IO>::st(&S[tid * SK + j], z);
        if (zf)
#pragma unroll
          for (int j = 0; j < SK; j += VN) Vec4<IO>::st(&F[tid * SK + j], z);
        fz = item.ctx;
        __syncthreads();
      }
    }
    if (item.ctx != cur) {
      const McCtx C = P.ctx[item.ctx];
      n_own = C.n_own;
      cph = C.cph;
      n_chunk = C.n_chunk;
  #pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLOCK;
        qr[k] = h < C.n_own ? P.q[C.q_off + h] : make_uint4(0xffffffffu, 0u, 0u, 0u);
        lo[k] = h < C.n_own ? lam[C.lam_own_off + h] : (IO)0;
        ps[k] = h < C.n_opp ? P.pos[C.pos_off + h] : make_uint2(0xffffffffu, 0xffffffffu);
        lp[k] = h < C.n_opp ? lam[C.lam_opp_off + h] : (IO)0;
      }
      cm = P.meta[C.meta_off + tid];
      cur = item.ctx;
    }
    const bool hs = item.in_s >= 0, hf = item.in_f >= 0;
    // weighted opponent inputs into their slots
    const IO ks = (IO)item.ks, kf = (IO)item.kf;
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const uint2 pp = ps[k];
      const int g = lo16(pp.x);
      if (g >= 0) {
        const int c0 = hi16(pp.x), c1 = lo16(pp.y);
        if (hs) {
          const IO v = ks * lp[k] * cs_in[k];
          at_slot(S, g) = v;
          at_slot(S, c0) = v;
          if (c1 >= 0) at_slot(S, c1) = v;
        }
        if (hf) {
          const IO v = kf * lp[k] * cf_in[k];
          at_slot(F, g) = v;
          at_slot(F, c0) = v;
          if (c1 >= 0) at_slot(F, c1) = v;
        }
      }
    }
    __syncthreads();
    // Chunk sums in the I/O type (at most KE terms; slots past a segment's
    // entries hold 0), carried across chunks in FP64; the chunk is read
    // again after the scan rather than held in registers.  Wavefronts past
    // the last chunk skip both passes.
    const bool wlive = (tid & ~63) < n_chunk;
    IO ls = (IO)0, lf = (IO)0;
    if (hs && wlive) {
#pragma unroll
      for (int j = 0; j < KE; j += VN) {
        IO v[VN];
        Vec4<IO>::ld(&S[tid * SK + j], v);
#pragma unroll
        for (int u = 0; u < VN; ++u) ls += v[u];
      }
    }
    if (hf && wlive) {
#pragma unroll
      for (int j = 0; j < KE; j += VN) {
        IO v[VN];
        Vec4<IO>::ld(&F[tid * SK + j], v);
#pragma unroll
        for (int u = 0; u < VN; ++u) lf += v[u];
      }
    }
    const double ts = (double)ls, tf = (double)lf;
    double es, ef;
    block_seg_scan_x<NW>((int)((cm >> 8) & 1u), ts, tf, scr, es, ef);
    if (hs && wlive) {
      // FP32: the FP64 carry as a rounded head plus its remainder, so each
      // prefix is head + (remainder + partial) in two FP32 adds.  The slot
      // after a segment's last entry receives the segment's total; the
      // zeroed slots after it add nothing, and no query reads past it.
      const IO eh = (IO)es;
      IO run = sizeof(IO) == 4 ? (IO)(es - (double)eh) : (IO)0;
#pragma unroll
      for (int j = 0; j < KE; j += VN) {
        IO v[VN], pc[VN];
        Vec4<IO>::ld(&S[tid * SK + j], v);
#pragma unroll
        for (int u = 0; u < VN; ++u) {
          pc[u] = eh + run;
          run += v[u];
        }
        Vec4<IO>::st(&S[tid * SK + j], pc);
      }
    }
    const int endseg = (int)((cm >> 16) & 255u);
    if (endseg) {
      segT[2 * (endseg - 1)] = es + ts;
      segT[2 * (endseg - 1) + 1] = ef + tf;
    }
    __syncthreads();
    // own hands: prefix sums at the query slots, fold totals per card
    const double2* T2 = (const double2*)segT;   // (showdown, fold) total of each segment
    const double2 T0 = T2[0];
#pragma unroll
    for (int k = 0; k < KH; ++k) {
      const uint4 r = qr[k];
      const int lt = lo16(r.x);
      if (lt >= 0) {
        const int c0 = r.w & 255, c1 = (r.w >> 8) & 255;
        const double2 Ta = T2[1 + c0];
        const double2 Tb = cph == 2 ? T2[1 + c1] : make_double2(0.0, 0.0);
        double v = 0.0;
        if (hs) {
          double sd = (double)at_slot(S, lt) + (double)at_slot(S, hi16(r.x)) - T0.x;
          sd -= (double)at_slot(S, lo16(r.y)) + (double)at_slot(S, hi16(r.y)) - Ta.x;
          if (cph == 2) sd -= (double)at_slot(S, lo16(r.z)) + (double)at_slot(S, hi16(r.z)) - Tb.x;
          v += sd;
        }
        if (hf) {
          double fo = T0.y - Ta.y - Tb.y;
          const int self = hi16(r.w);
          if (cph == 2 && self >= 0) fo += (double)at_slot(F, self);
          v += fo;
        }
        acc[k] += v;
      }
    }
    if (item.last) {
      IO* __restrict__ dst = item.last == 2 ? (IO*)P.part : out;
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLOCK;
        if (h < item.stride) dst[item.out + h] = (IO)(h < n_own ? P.scale * (double)lo[k] * acc[k] : 0.0);
        acc[k] = 0.0;
      }
    }
  }
}

// Rows cut into parts: each output row is the sum of its partial rows, taken
// in part order (FP64 sum, one rounding to IO).  One workgroup per row of
// either direction; rows of retired instances are skipped.
template <typename IO>
__global__ __launch_bounds__(256) void k_mv_reduce(const MvRed* __restrict__ r0, int n0, const IO* __restrict__ part0,
                                                   IO* __restrict__ out0, const MvRed* __restrict__ r1,
                                                   const IO* __restrict__ part1, IO* __restrict__ out1,
                                                   const int32_t* __restrict__ active) {
  const bool second = (int)blockIdx.x >= n0;
  const MvRed r = second ? r1[blockIdx.x - n0] : r0[blockIdx.x];
  if (active && !active[r.inst]) return;
  const IO* __restrict__ part = (second ? part1 : part0) + r.part;
  IO* __restrict__ out = (second ? out1 : out0) + r.out;
  for (int h = threadIdx.x; h < r.stride; h += 256) {
    double v = 0.0;
    for (int j = 0; j < r.n_parts; ++j) v += (double)part[(int64_t)j * r.stride + h];
    out[h] = (IO)v;
  }
}

// ---------------------------------------------------------------------------
// grouped matvec (kernel 4, FP32; layout in GCtx / GGroup)
// ---------------------------------------------------------------------------
struct GParams {
  const GGroup* groups;
  const int4* chunks;            // (first group, end group, instance, context of the first group)
  const GCtx* ctx;
  const uint4* q;
  const uint16_t* rk;
  const uint32_t* src;
  const uint32_t* meta;
  const float* lamf;
  const int32_t* active;         // per-instance flag (NULL: all)
  double scale;
  int32_t nchunk;
};

// One step of an inclusive segmented scan of (flag, a[0..3]): the values of
// the earlier lane are added unless this lane's run already holds a flag.
// With every row enabled, a lane without a source reads 0 through the DPP
// bound control, and no old value has to be set first.
template <int CTRL>
__device__ inline int dpp_iz(int v) {
  return __builtin_amdgcn_mov_dpp(v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ inline double dpp_dz(double v) {
  return __hiloint2double(dpp_iz<CTRL>(__double2hiint(v)), dpp_iz<CTRL>(__double2loint(v)));
}
template <int CTRL, int RM, int NC>
__device__ inline void seg_step4(int& f, double (&a)[NC]) {
  const int f2 = RM == 0xf ? dpp_iz<CTRL>(f) : dpp_i<CTRL, RM>(f);
  const double m = f ? 0.0 : 1.0;
#pragma unroll
  for (int j = 0; j < NC; ++j) a[j] = fma(RM == 0xf ? dpp_dz<CTRL>(a[j]) : dpp_d<CTRL, RM>(a[j]), m, a[j]);
  f |= f2;
}

// Exclusive segmented scan of NC values over the threads of a block (as
// block_seg_scan_x): the exclusive sum is the inclusive one minus the own
// value.  One barrier; `scr` holds 5 doubles per wavefront.
template <int NW, int NC>
__device__ inline void block_seg_scan4(int flag, const double (&a)[NC], double* scr, double (&e)[NC]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int f = flag;
  double ai[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) ai[j] = a[j];
  seg_step4<0x111, 0xf, NC>(f, ai);
  seg_step4<0x112, 0xf, NC>(f, ai);
  seg_step4<0x114, 0xf, NC>(f, ai);
  seg_step4<0x118, 0xf, NC>(f, ai);
  seg_step4<0x142, 0xa, NC>(f, ai);
  seg_step4<0x143, 0xc, NC>(f, ai);
  if (lane == 63) {
    scr[5 * wid] = (double)f;
#pragma unroll
    for (int j = 0; j < NC; ++j) scr[5 * wid + 1 + j] = ai[j];
  }
  __syncthreads();
  static_assert(NW <= 8, "wavefront totals are scanned within one DPP row");
  int fw = 0;
  double aw[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) aw[j] = 0.0;
  if (lane < NW) {
    fw = scr[5 * lane] != 0.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) aw[j] = scr[5 * lane + 1 + j];
  }
  seg_step4<0x111, 0xf, NC>(fw, aw);
  seg_step4<0x112, 0xf, NC>(fw, aw);
  seg_step4<0x114, 0xf, NC>(fw, aw);
  const double m = (wid > 0 && !f) ? 1.0 : 0.0;
  const int src = wid > 0 ? wid - 1 : 0;
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    const double c = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(aw[j]), src),
                                      __builtin_amdgcn_readlane(__double2loint(aw[j]), src));
    e[j] = fma(c, m, ai[j]) - a[j];
  }
}

// Records every lane reads at the same address (chunks, groups, contexts) are
// read through the constant address space: the plans do not change during a
// launch, so the loads go through the scalar cache into scalar registers.
template <typename T>
__device__ inline const __attribute__((address_space(4))) T* cst(const T* p) {
  return (const __attribute__((address_space(4))) T*)p;
}

// Loads issued whatever the condition (at index 0 when it fails) and
// selected afterwards, so that no branch waits on them.
template <typename T>
__device__ inline T ld_sel(const T* p, int64_t i, bool ok, T zero) {
  const T v = p[ok ? i : 0];
  return ok ? v : zero;
}

// A group record in scalar registers.
struct GGroupS {
  int32_t in[kGrpComps], out[kGrpComps];
  double ks[kGrpComps], kf[kGrpComps];
  int32_t ctx, fc, sc, acc, n_own, stride, n_in;
};
__device__ inline GGroupS load_group(const GGroup* p) {
  const auto gp = cst(p);
  GGroupS G;
#pragma unroll
  for (int j = 0; j < kGrpComps; ++j) {
    G.in[j] = gp->in[j];
    G.out[j] = gp->out[j];
    G.ks[j] = gp->ks[j];
    G.kf[j] = gp->kf[j];
  }
  G.ctx = gp->ctx;
  G.fc = gp->fc;
  G.sc = gp->sc;
  G.acc = gp->acc;
  G.n_own = gp->n_own;
  G.stride = gp->stride;
  G.n_in = gp->n_in;
  return G;
}

// Position of a workgroup in the chunk list: the hardware deals workgroups
// to the eight XCDs in turn, so consecutive chunks (one instance, its
// context records and input rows) are given to the workgroups of one XCD
// and share its L2.
__device__ inline int xcd_chunk(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// LDS slots of a group: NC FP32 values (16 bytes for four components, 8 for
// two).  The layout's byte offsets are built for 16-byte slots; a two-wide
// launch halves them.
template <int NC>
struct GSlot;
template <>
struct GSlot<4> {
  static constexpr int SB = 16, SH = 0;
  __device__ static void ld(const char* p, float (&v)[4]) {
    const float4 t = *(const float4*)p;
    v[0] = t.x, v[1] = t.y, v[2] = t.z, v[3] = t.w;
  }
  __device__ static void st(char* p, const float (&v)[4]) { *(float4*)p = make_float4(v[0], v[1], v[2], v[3]); }
};
template <>
struct GSlot<2> {
  static constexpr int SB = 8, SH = 1;
  __device__ static void ld(const char* p, float (&v)[2]) {
    const float2 t = *(const float2*)p;
    v[0] = t.x, v[1] = t.y;
  }
  __device__ static void st(char* p, const float (&v)[2]) { *(float2*)p = make_float2(v[0], v[1]); }
};
template <int NC>
__device__ inline void grp_slot(const char* R, uint32_t slot, float (&v)[NC]) {
  GSlot<NC>::ld(R + GSlot<NC>::SB * slot, v);
}

// Showdown values of the NS components held in prefix slots and fold values
// of all NC components for one own hand, from the prefix slots, the segment
// totals and the identical hand.  With NS == NC the identical hand's value
// is the difference of the prefix sums at its global entry and the next one;
// with NS < NC (the fold-only components have no slots) it is read from its
// staging row in St.
template <int KE, int NC, int NS>
__device__ inline void grp_query(const char* R, const char* St, const double* segT, uint4 r, int cph,
                                 double (&sd)[NS], double (&fo)[NC]) {
  constexpr int BLK = kGrpBlock;
  float g0[NS], g1[NS], a0[NS], a1[NS];
  grp_slot<NS>(R, r.x & 0xffffu, g0);
  grp_slot<NS>(R, r.x >> 16, g1);
  grp_slot<NS>(R, r.y & 0xffffu, a0);
  grp_slot<NS>(R, r.y >> 16, a1);
  const int c0 = r.w & 63, c1 = (r.w >> 6) & 63;
  const double* T = segT;   // NC doubles per segment
#pragma unroll
  for (int j = 0; j < NS; ++j) {
    const double t0 = T[j], ta = T[NC * (1 + c0) + j];
    sd[j] = ((double)(g0[j] + g1[j]) - t0) - ((double)(a0[j] + a1[j]) - ta);
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) fo[j] = T[j] - T[NC * (1 + c0) + j];
  if (cph == 2) {
    float b0[NS], b1[NS], u[NC];
    grp_slot<NS>(R, r.z & 0xffffu, b0);
    grp_slot<NS>(R, r.z >> 16, b1);
#pragma unroll
    for (int j = 0; j < NC; ++j) u[j] = 0.f;
    if (r.w & (1u << 12)) {
      const uint32_t s0 = r.w >> 14;
      if (NS == NC) {
        // the difference of the prefix sums at the identical hand's global
        // entry and the next one (the next chunk's first entry when it ends
        // its chunk)
        const uint32_t s1 = (r.w & (1u << 13)) ? s0 - (uint32_t)((KE - 1) * BLK) + 1u : s0 + (uint32_t)BLK;
        float p0[NS], p1[NS];
        grp_slot<NS>(R, s0, p0);
        grp_slot<NS>(R, s1, p1);
#pragma unroll
        for (int j = 0; j < NS; ++j) u[j] = p1[j] - p0[j];
      } else {
        // global entry i sits at slot (i % KE) * BLK + i / KE; its staging
        // row is the one of strength position i
        const int i = (int)(s0 % (uint32_t)BLK) * KE + (int)(s0 / (uint32_t)BLK);
        float uv[NC];
        GSlot<NC>::ld(St + GSlot<NC>::SB * (i + (i >> 4)), uv);   // rows padded one per 16
#pragma unroll
        for (int j = 0; j < NC; ++j) u[j] = uv[j];
      }
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) sd[j] -= (double)(b0[j] + b1[j]) - T[NC * (1 + c1) + j];
#pragma unroll
    for (int j = 0; j < NC; ++j) fo[j] += (double)u[j] - T[NC * (1 + c1) + j];
  }
}

// One workgroup per chunk of groups.  Per group: every opponent hand stages
// its weighted values of the group's components (one 16-byte row at its
// strength position), each thread gathers its chunk of the segmented entry
// list from those rows and sums it, a segmented block scan carries the sums
// across the chunks of a segment in FP64, every entry's exclusive prefix sum
// (rounded once to FP32) is stored at its slot over the staging rows, and
// every own hand reads six prefix sums, the segment totals and the identical
// hand (Technique B's solve and the inclusion-exclusion of eq. cf) for all
// four components at once, then weights them by each output's coefficients.
// Wavefronts per SIMD each class is built for: at most the workgroups per CU
// its LDS region allows (four for one hand per thread, three for two or three,
// two beyond), lowered where the registers of a class would otherwise spill
// (the carrying form serves only the few sequences of rows summed over boards).
// Groups of at most two components (about half of a batch's) take launches
// of their own with two-wide slots: half the LDS, so more workgroups per CU.
// Four-component groups whose showdown terms read only two of them (most of
// the rest) keep prefix slots for those two (NS = 2): the staging rows of all
// four sit in a region of their own, and the fold-only components need no
// slots, only their segment totals and the identical hand's staging row.
template <int KH, bool CARRY, int NC, int NS>
constexpr int mvg_waves_per_simd() {
  return NC == 2 ? (KH <= 2 ? 4 : 3)
       : NS == 2 ? (KH <= 2 ? 4 : KH <= 4 ? 3 : 2)
                 : KH == 1 ? 4 : (KH == 2 || (KH == 3 && !CARRY)) ? 3 : (KH == 5 && CARRY) ? 1 : 2;
}

// Bytes of the staging region of a launch whose prefix slots hold fewer
// components than it stages (NS < NC): 16-byte rows for KH * block hands,
// one padding row per 16, the zero row and the trash row.
template <int KH>
constexpr int grp_stage_bytes() {
  return 16 * (KH * kGrpBlock + KH * kGrpBlock / 16 + 2);
}

template <int KH, int KE, bool CARRY, int NC, int NS>
__global__ __launch_bounds__(kGrpBlock) __attribute__((amdgpu_waves_per_eu(mvg_waves_per_simd<KH, CARRY, NC, NS>())))
void k_mvg(GParams P0, const float* __restrict__ in0, float* __restrict__ out0, GParams P1,
           const float* __restrict__ in1, float* __restrict__ out1, double* __restrict__ tick) {
  constexpr int BLK = kGrpBlock, NW = BLK / 64, SH = GSlot<NC>::SH, SBS = GSlot<NS>::SB;
  static_assert(NC == 2 || NC == kGrpComps, "two or four components");
  static_assert(NS == NC || (NC == kGrpComps && NS == 2 && !CARRY), "prefix slots for all, or two of four");
  static_assert(KE % 2 == 0, "entry sources are stored in pairs");
  if (tick && blockIdx.x == 0 && threadIdx.x == 0) tick[0] += 1.0;
  const int b = xcd_chunk((int)blockIdx.x, P0.nchunk + P1.nchunk);
  const bool second = b >= P0.nchunk;
  const GParams& P = second ? P1 : P0;
  const float* __restrict__ in = second ? in1 : in0;
  float* __restrict__ out = second ? out1 : out0;
  const auto crp = cst((const int32_t*)(P.chunks + (second ? b - P0.nchunk : b)));
  const int4 cr = make_int4(crp[0], crp[1], crp[2], crp[3]);
  if (P.active && !*cst(P.active + cr.z)) return;   // retired instance
  const int tid = threadIdx.x;
  extern __shared__ double smem[];
  double* segT = smem;                         // [kMcSegMax][NC] segment totals
  double* scr = segT + NC * kMcSegMax;         // [5 * NW] scan scratch
  char* R = (char*)(scr + 5 * NW);             // prefix slots (SBS bytes each), over the staging rows
  char* St = NS < NC ? R + SBS * KE * BLK : R; //   or staging rows of their own (NS < NC)

  const int g0 = cr.x, g1 = cr.y;
  if (cr.w < 0) {
    // a chunk of rows without terms: zeros
    for (int gi = g0; gi < g1; ++gi) {
      const GGroupS G = load_group(P.groups + gi);
#pragma unroll
      for (int o = 0; o < kGrpComps; ++o) {
        if (G.out[o] < 0) continue;
#pragma unroll
        for (int k = 0; k < KH; ++k) {
          const int h = tid + k * BLK;
          if (h < G.stride) out[G.out[o] + h] = 0.f;
        }
      }
    }
    return;
  }

  double acc[CARRY ? kGrpComps : 1][CARRY ? KH : 1];   // sums of rows over several groups
  float v[NC][KH];                             // the inputs of the group in flight
#pragma unroll
  for (int o = 0; o < (CARRY ? kGrpComps : 1); ++o)
#pragma unroll
    for (int k = 0; k < (CARRY ? KH : 1); ++k) acc[o][k] = 0.0;
  {
    const GGroupS G = load_group(P.groups + g0);
#pragma unroll
    for (int j = 0; j < NC; ++j)
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLK;
        v[j][k] = ld_sel(in, G.in[j] + h, G.in[j] >= 0 && h < G.n_in, 0.f);
      }
  }
  int gi = g0;
  while (gi < g1) {
    // a run of groups on one board context: its records stay in registers
    const int ctx = cst(P.groups + gi)->ctx;
    const auto cp = cst(P.ctx + ctx);
    const int n_own = cp->n_own, n_opp = cp->n_opp, cph = cp->cph, n_chunk = cp->n_chunk;
    const int zrow = cp->zrow;
    const uint32_t trash = (uint32_t)cp->trash;
    uint32_t rko[KH], srcp[KE / 2];
    float lop[KH], low[KH];
    uint4 qr[KH];
    {
      const uint16_t* rk = P.rk + cp->rk_off;
      const float* lopp = P.lamf + cp->lam_opp_off;
      const float* lown = P.lamf + cp->lam_own_off;
      const uint4* qp = P.q + cp->q_off;
      const uint32_t* sp = P.src + cp->src_off;
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLK;
        rko[k] = h < n_opp ? (uint32_t)ld_sel(rk, h, h < n_opp, (uint16_t)0) : trash;
        lop[k] = ld_sel(lopp, h, h < n_opp, 0.f);
        qr[k] = ld_sel(qp, h, h < n_own, make_uint4(0xffffffffu, 0u, 0u, 0u));
        low[k] = ld_sel(lown, h, h < n_own, 0.f);
      }
#pragma unroll
      for (int j = 0; j < KE / 2; ++j) srcp[j] = sp[j * BLK + tid];
    }
    const uint32_t cm = P.meta[cp->meta_off + tid];
    const bool wlive = (tid & ~63) < n_chunk;
    for (; gi < g1; ++gi) {
      const GGroupS G = load_group(P.groups + gi);
      if (G.ctx != ctx) break;
      // the next group's input rows, read with this group's record so that
      // its inputs can be requested right after the staging
      int nin[NC], nn_in = 0;
      {
        const auto np = cst(P.groups + min(gi + 1, g1 - 1));
#pragma unroll
        for (int j = 0; j < NC; ++j) nin[j] = np->in[j];
        nn_in = np->n_in;
      }
      // the per-hand records are decoded again in every group: hoisting the
      // decoded LDS addresses out of the loop costs more registers than the
      // few integer operations it saves
#pragma unroll
      for (int k = 0; k < KH; ++k) asm volatile("" : "+v"(qr[k].x), "+v"(qr[k].y), "+v"(qr[k].z), "+v"(qr[k].w));
#pragma unroll
      for (int j = 0; j < KE / 2; ++j) asm volatile("" : "+v"(srcp[j]));
      // stage the weighted components at the hands' strength positions, then
      // fetch the next group's inputs into the same registers
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLK;
        if (h < n_opp) {
          float w[NC];
#pragma unroll
          for (int j = 0; j < NC; ++j) w[j] = lop[k] * v[j][k];
          GSlot<NC>::st(St + (rko[k] >> SH), w);
        }
      }
      if (tid == 0) {
        float z[NC];
#pragma unroll
        for (int j = 0; j < NC; ++j) z[j] = 0.f;
        GSlot<NC>::st(St + (zrow >> SH), z);
      }
      if (gi + 1 < g1) {
#pragma unroll
        for (int j = 0; j < NC; ++j)
#pragma unroll
          for (int k = 0; k < KH; ++k) {
            const int h = tid + k * BLK;
            v[j][k] = ld_sel(in, nin[j] + h, nin[j] >= 0 && h < nn_in, 0.f);
          }
      }
      __syncthreads();
      // gather the chunk and sum it (the entries of the components with
      // prefix slots stay in registers); carry the sums across the
      // segment's chunks
      float ev[KE][NS];
      float s4[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) s4[j] = 0.f;
      if (wlive) {
#pragma unroll
        for (int i = 0; i < KE; ++i) {
          const uint32_t off = (i & 1) ? srcp[i / 2] >> 16 : srcp[i / 2] & 0xffffu;
          float evf[NC];
          GSlot<NC>::ld(St + (off >> SH), evf);
#pragma unroll
          for (int j = 0; j < NC; ++j) s4[j] += evf[j];
#pragma unroll
          for (int j = 0; j < NS; ++j) ev[i][j] = evf[j];
        }
      }
      double a[NC], e[NC];
#pragma unroll
      for (int j = 0; j < NC; ++j) a[j] = (double)s4[j];
      block_seg_scan4<NW, NC>((int)((cm >> 8) & 1u), a, scr, e);
      // every gather is done (the scan's barrier): the exclusive prefix sums
      // of the slotted components overwrite the staging rows (or fill their
      // own region), each the FP64 carry's FP32 head plus (remainder +
      // partial)
      if (wlive) {
        float eh[NS], run[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
          eh[j] = (float)e[j];
          run[j] = (float)(e[j] - (double)eh[j]);
        }
#pragma unroll
        for (int i = 0; i < KE; ++i) {
          float w[NS];
#pragma unroll
          for (int j = 0; j < NS; ++j) {
            w[j] = eh[j] + run[j];
            run[j] += ev[i][j];
          }
          GSlot<NS>::st(R + SBS * (i * BLK + tid), w);
        }
      }
      const int endseg = (int)((cm >> 16) & 255u);
      if (endseg) {
        double* T = segT + NC * (endseg - 1);
#pragma unroll
        for (int j = 0; j < NC; ++j) T[j] = e[j] + a[j];
      }
      __syncthreads();
      // own hands: the outputs' values, stored (or carried to the next group
      // of the sequence)
#pragma unroll
      for (int k = 0; k < KH; ++k) {
        const int h = tid + k * BLK;
        // outputs: four in every kind; components: NC, NS of them with
        // prefix slots (with two, the outputs name their showdown component
        // as they name their fold component)
        double val[kGrpComps];
#pragma unroll
        for (int o = 0; o < kGrpComps; ++o) val[o] = 0.0;
        if (h < n_own && qr[k].x != 0xffffffffu) {
          double sd[NS], fo[NC];
          grp_query<KE, NC, NS>(R, St, segT, qr[k], cph, sd, fo);
#pragma unroll
          for (int o = 0; o < kGrpComps; ++o) {
            const int fj = (G.fc >> (2 * o)) & 3;
            double f = fo[0];
#pragma unroll
            for (int c = 1; c < NC; ++c) f = fj == c ? fo[c] : f;
            const double sv = NS == 2 ? (((G.sc >> (2 * o)) & 3) == 1 ? sd[1] : sd[0]) : sd[o % NS];
            val[o] = G.ks[o] * sv + G.kf[o] * f;
          }
        }
        const double sl = P.scale * (double)low[k];
#pragma unroll
        for (int o = 0; o < kGrpComps; ++o) {
          if (CARRY) {
            acc[o][k] = ((G.acc & (1 << o)) ? 0.0 : acc[o][k]) + val[o];
            if (G.out[o] >= 0 && (G.acc & (1 << (4 + o))) && h < G.stride)
              out[G.out[o] + h] = h < n_own ? (float)(sl * acc[o][k]) : 0.f;
          } else if (G.out[o] >= 0 && h < G.stride) {
            out[G.out[o] + h] = h < n_own ? (float)(sl * val[o]) : 0.f;
          }
        }
        // one hand's LDS reads in flight at a time: the next hand's are not
        // hoisted above this one's arithmetic (register pressure)
        __builtin_amdgcn_sched_barrier(0);
      }
      __syncthreads();   // the next group's staging overwrites the prefix slots
    }
  }
}

// ---------------------------------------------------------------------------
// treeplex kernels (one thread per hand of a task)
// ---------------------------------------------------------------------------
struct TpParams {
  const int32_t* inf_parent;
  const int32_t* inf_first;
  const int32_t* inf_nact;
  const int32_t* order;
  const TpTask* tasks;
  const TpPull* pulls;
  const int2* blocks;
  int32_t stage_stride;
  const int32_t* active;     // per-instance flag (NULL: all); inactive tasks are skipped
  int32_t dcfr;              // 0: regret matching+, 1: discounted CFR
  int32_t gamma;             // averaging weight t^gamma (1 for RM+)
  float alpha, beta;         // DCFR regret discounts
};

// Per-iteration constants of the regret update and the averaging weight.
struct RmStep {
  double w;                  // weight of this iteration's plan in the average
  float dp, dn;              // factors for positive / other regrets
  bool floor;                // RM+: clip regrets at 0
};
__device__ inline RmStep rm_step(int dcfr, int gamma, float alpha, float beta, double t) {
  RmStep r;
  r.w = gamma == 1 ? t : (gamma == 2 ? t * t : t * t * t);
  r.dp = 1.f;
  r.dn = 1.f;
  r.floor = !dcfr;
  if (dcfr) {
    const float tf = (float)t;
    const float ta = powf(tf, alpha), tb = powf(tf, beta);
    r.dp = ta / (ta + 1.f);
    r.dn = tb / (tb + 1.f);
  }
  return r;
}
__device__ inline RmStep rm_step(const TpParams& P, double t) {
  return rm_step(P.dcfr, P.gamma, P.alpha, P.beta, t);
}
// New regret from the old one and the instantaneous regret: RM+ clips at 0;
// discounted CFR scales positive and other regrets by their factors.
template <bool DC>
__device__ inline float rm_new(float r, float inst, const RmStep& k) {
  if (!DC) return fmaxf(r + inst, 0.f);
  return r * (r > 0.f ? k.dp : k.dn) + inst;
}

// 1 / (den * sc) for den > 0, with sc = 2^64 when den is so small that 1 / den
// would overflow FP32.  A quotient v / den is formed as (v * sc) * rcp, so
// it never passes through 1 / den: behaviour probabilities (v <= den) stay
// at most 1 and expected values stay in the range of v / den.
__device__ inline float rm_rcp(float den, float& sc) {
  sc = den < 0x1p-64f ? 0x1p64f : 1.f;
  return __builtin_amdgcn_rcpf(den * sc);
}

constexpr int TPB = 128;

constexpr int MAXA = 8;       // actions handled in registers by the walks

__global__ void k_set1(double* tdev, double v) { tdev[0] = v; }
__global__ void k_add1(double* tdev) { tdev[0] += 1.0; }

// ---------------------------------------------------------------------------
// regret update on treeplex pieces (RmTask): the piece's rows of g, R and x
// for 64 hands live in LDS; every wavefront of the block loads and stores an
// equal share of the rows (all loads in flight at once), each wavefront walks
// one subtree group of the piece and wavefront 0 the top part.  Row,
// infoset, pull, group and external-parent tables are held one entry per
// lane and read with readlane, so the walk touches LDS only for the slab
// itself.
// ---------------------------------------------------------------------------
// One workgroup of a regret-update launch: its piece and first hand.
struct RmBlock {
  RmTask t;
  int32_t h0, pad[3];
};

struct RmParams {
  const RmBlock* blocks;
  const int32_t* rows;
  const int32_t* infs;
  const int32_t* pulls;
  const int32_t* ext_seq;
  const int32_t* ext_slot;
  const int32_t* grp;           // group tables of split pieces
  const int32_t* active;        // per-instance flag (NULL: all)
  int32_t stage_stride;
  int32_t max_rows, max_ext;    // LDS layout of the launch
  int32_t dcfr, gamma;
  float alpha, beta;
};
constexpr int RMW = kRmGroups;              // wavefronts per block, one per subtree group
constexpr int RMR = kTaskRowsMax / RMW;     // rows loaded per wavefront

__device__ inline int rl(int v, int i) { return __builtin_amdgcn_readlane(v, i); }

// Bottom-up step of one infoset with n <= W actions for one hand (LDS rows,
// 64 lanes apart): V(I) from the current behaviour, the regret update from
// q = A (g plus the values below), and V added into the LDS row `pp` (the
// parent's row, a group-root slot, or the sink).  The W row reads and the
// parent's issue together; positions past the last action read and rewrite
// the last action's row (the same value to the same address) and are left
// out of the sums, so the step has no branch and one body serves every
// action count up to W.
template <int W, bool DC>
__device__ inline void rmp_up_w(float* __restrict__ Al, float* __restrict__ Rl, float* pp, int f, int n, int lane,
                                const RmStep& K) {
  float rr[W], gg[W];
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const int o = (f + min(a, n - 1)) * 64 + lane;
    rr[a] = Rl[o];
    gg[a] = Al[o];
  }
  const float pv = *pp;
  float rs = 0.f, dot = 0.f, gs = 0.f;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const float r = a < n ? fmaxf(rr[a], 0.f) : 0.f;
    rs += r;
    dot += r * gg[a];
    gs += a < n ? gg[a] : 0.f;
  }
  const bool pos = rs > 0.f;
  float sc;
  const float rc = rm_rcp(pos ? rs : (float)n, sc);
  const float V = ((pos ? dot : gs) * sc) * rc;
#pragma unroll
  for (int a = 0; a < W; ++a) Rl[(f + min(a, n - 1)) * 64 + lane] = rm_new<DC>(rr[a], gg[a] - V, K);
  *pp = pv + V;
}

// Top-down step: the new behaviour from the regrets times the parent's
// realization weight *xpp, into the rows of Al; positions past the last
// action as in the bottom-up step.
template <int W>
__device__ inline void rmp_down_w(float* __restrict__ Al, const float* __restrict__ Rl, const float* xpp, int f,
                                  int n, int lane) {
  float rr[W];
#pragma unroll
  for (int a = 0; a < W; ++a) rr[a] = fmaxf(Rl[(f + min(a, n - 1)) * 64 + lane], 0.f);
  const float xp = *xpp;
  float rs = 0.f;
#pragma unroll
  for (int a = 0; a < W; ++a) rs += a < n ? rr[a] : 0.f;
  const bool pos = rs > 0.f;
  float sc;
  const float rc = rm_rcp(pos ? rs : (float)n, sc);
#pragma unroll
  for (int a = 0; a < W; ++a) Al[(f + min(a, n - 1)) * 64 + lane] = xp * (((pos ? rr[a] : 1.f) * sc) * rc);
}

// Any action count (beyond MAXA).
template <bool DC>
__device__ inline void rmp_up_any(float* __restrict__ Al, float* __restrict__ Rl, float* pp, int f, int n,
                                  int lane, const RmStep& K) {
  float rs = 0.f, dot = 0.f, gs = 0.f;
  for (int a = 0; a < n; ++a) {
    const float r = fmaxf(Rl[(f + a) * 64 + lane], 0.f), gv = Al[(f + a) * 64 + lane];
    rs += r;
    dot += r * gv;
    gs += gv;
  }
  const bool pos = rs > 0.f;
  float sc;
  const float rc = rm_rcp(pos ? rs : (float)n, sc);
  const float V = ((pos ? dot : gs) * sc) * rc;
  for (int a = 0; a < n; ++a)
    Rl[(f + a) * 64 + lane] = rm_new<DC>(Rl[(f + a) * 64 + lane], Al[(f + a) * 64 + lane] - V, K);
  *pp += V;
}
__device__ inline void rmp_down_any(float* __restrict__ Al, const float* __restrict__ Rl, const float* xpp,
                                    int f, int n, int lane) {
  const float xp = *xpp;
  float rs = 0.f;
  for (int a = 0; a < n; ++a) rs += fmaxf(Rl[(f + a) * 64 + lane], 0.f);
  const bool pos = rs > 0.f;
  float sc;
  const float rc = rm_rcp(pos ? rs : (float)n, sc);
  for (int a = 0; a < n; ++a)
    Al[(f + a) * 64 + lane] = xp * (((pos ? fmaxf(Rl[(f + a) * 64 + lane], 0.f) : 1.f) * sc) * rc);
}

// Three widths (2: fold / call, 4, 8) keep the common small infosets cheap;
// one call site per direction in the kernel keeps its code small.
template <bool DC>
__device__ inline void rmp_up(float* Al, float* Rl, float* pp, int f, int n, int lane, const RmStep& K) {
  if (n <= 2) rmp_up_w<2, DC>(Al, Rl, pp, f, n, lane, K);
  else if (n <= 4) rmp_up_w<4, DC>(Al, Rl, pp, f, n, lane, K);
  else if (n <= MAXA) rmp_up_w<MAXA, DC>(Al, Rl, pp, f, n, lane, K);
  else rmp_up_any<DC>(Al, Rl, pp, f, n, lane, K);
}
__device__ inline void rmp_down(float* Al, const float* Rl, const float* xpp, int f, int n, int lane) {
  if (n <= 2) rmp_down_w<2>(Al, Rl, xpp, f, n, lane);
  else if (n <= 4) rmp_down_w<4>(Al, Rl, xpp, f, n, lane);
  else if (n <= MAXA) rmp_down_w<MAXA>(Al, Rl, xpp, f, n, lane);
  else rmp_down_any(Al, Rl, xpp, f, n, lane);
}

// Values of deeper pieces into the rows they hang from (pulls; the host lists
// them per wavefront, a row's pulls consecutive, behind a header of counts):
// each wavefront takes its own, eight stage loads in flight, and adds each
// row's sum once.  Rows of RW hands; `col` is the lane's hand column, `hs` an
// in-bounds hand for the loads, `wr` whether the lane writes.
template <int RW>
__device__ inline void rm_pulls(const RmParams& P, const RmTask& T, float* __restrict__ Al,
                                const float* __restrict__ stage, int lane, int wv, int col, int64_t hs, bool wr) {
  const int32_t* pl = P.pulls + T.pull_off;
  const int hdr = lane < RMW ? pl[lane] : 0;
  int beg = RMW;
  for (int w = 0; w < wv; ++w) beg += rl(hdr, w);
  const int cnt = rl(hdr, wv);
  float acc = 0.f;
  int row = -1;
  for (int c0 = 0; c0 < cnt; c0 += 64) {
    const int pv = c0 + lane < cnt ? pl[beg + c0 + lane] : 0;
    const int nn = min(64, cnt - c0);
    for (int j0 = 0; j0 < nn; j0 += 8) {
      float sv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        sv[u] = stage[(int64_t)((uint32_t)rl(pv, min(j0 + u, nn - 1)) >> 8) * P.stage_stride + hs];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (j0 + u < nn) {
          const int lr = rl(pv, j0 + u) & 255;
          if (lr != row) {
            if (row >= 0 && wr) Al[row * RW + col] += acc;
            acc = 0.f;
            row = lr;
          }
          acc += sv[u];
        }
      }
    }
  }
  if (row >= 0 && wr) Al[row * RW + col] += acc;
}

// Group-root values into their targets (wavefront 0, after the groups): every
// slot value and target value is read before the first wait; a run of
// entries with one target (entries are sorted by target) sums its slots in
// registers, and every entry writes the target's value plus the run so far,
// so the run's last write, which lands last, leaves the whole sum: no branch
// per entry.  Rows of RW hands, as in rm_pulls.
template <int RW>
__device__ inline void rm_merge(float* __restrict__ rsm, int grpv, int col, bool wr) {
  int mge[kRmMergeMax / 2];   // two entries per int, into SGPRs
#pragma unroll
  for (int e = 0; e < kRmMergeMax / 2; ++e) mge[e] = rl(grpv, kRmGMrg + e);
  float sv[kRmMergeMax], tv[kRmMergeMax];
#pragma unroll
  for (int e = 0; e < kRmMergeMax; ++e) {
    const int c = (mge[e / 2] >> (16 * (e & 1))) & 0xffff;
    sv[e] = rsm[(c & 255) * RW + col];
    tv[e] = rsm[(c >> 8) * RW + col];
  }
  float run = 0.f;
  int prev = -1;
#pragma unroll
  for (int e = 0; e < kRmMergeMax; ++e) {
    const int tg = ((mge[e / 2] >> (16 * (e & 1))) >> 8) & 255;
    run = (tg == prev ? run : 0.f) + sv[e];
    if (wr) rsm[tg * RW + col] = tv[e] + run;
    prev = tg;
  }
}

// MODE 0: bottom-up and top-down of a piece with no external parent (pulls
// from deeper pieces first); 1: bottom-up of a deep piece (root values to the
// stage buffer); 2: top-down of a deep piece (parent weights from x).  The
// running average takes the previous plan (weight K.w) in the pass that
// overwrites x.  DC: discounted CFR regrets (else RM+).
template <int MODE, bool DC>
__global__ __launch_bounds__(64 * RMW) void k_rmp(RmParams P, float* __restrict__ g, float* __restrict__ R,
                                                  float* __restrict__ x, double* __restrict__ xs,
                                                  float* __restrict__ stage, const double* __restrict__ tdev) {
  extern __shared__ float rsm[];
  const RmTask T = P.blocks[blockIdx.x].t;
  const int h0 = P.blocks[blockIdx.x].h0;
  if (P.active && !P.active[T.inst]) return;   // whole block: T is uniform
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int h = h0 + lane;
  const bool act = h < T.n_hands;
  const int SL = T.n_rows;
  float* Xw = rsm + kRmRowSlot * 64;        // group-root values
  float* Xl = rsm + kRmRowExt * 64;         // root values / parent weights of external parents
  float* Al = rsm + kRmRowLocal * 64;       // [max_rows][64]: g, then the new x
  float* Rl = Al + P.max_rows * 64;         // [max_rows][64]
  const int64_t base = T.vec_base + h, stride = T.stride;
  const RmStep K = rm_step(DC, P.gamma, P.alpha, P.beta, *tdev);
  // row ids, one per lane (a second for rows 64 + lane when pieces may
  // exceed 64 rows): computed for contiguous pieces, else from the table
  static_assert(kTaskRowsMax <= 128, "row ids are held in at most two registers");
  const int rowv = T.row0 >= 0 ? T.row0 + lane : (lane < SL ? P.rows[T.rows_off + lane] : 0);
  int rowv2 = 0;
  if (kTaskRowsMax > 64) rowv2 = T.row0 >= 0 ? T.row0 + 64 + lane : (64 + lane < SL ? P.rows[T.rows_off + 64 + lane] : 0);
  auto row_id = [rowv, rowv2](int r) { return kTaskRowsMax <= 64 || r < 64 ? rl(rowv, r) : rl(rowv2, r - 64); };
  const int infv = lane < T.n_inf ? P.infs[T.inf_off + lane] : 0;
  const bool grouped = T.grp_off >= 0;
  const int grpv = grouped ? P.grp[T.grp_off + lane] : 0;
  const int extv = (MODE != 0 && wv == 0 && lane < T.n_ext)
                       ? (MODE == 1 ? P.ext_slot[T.ext_off + lane] : P.ext_seq[T.ext_off + lane]) : 0;
  // loads at in-bounds hands (clamped) of the wavefront's rows, all issued
  // before the first is waited for (the rows past the piece's end are not
  // loaded: a uniform exit, no wait); the old plan and the running average
  // stay in registers until the stores at the end
  float c[RMR];
  double d[RMR];
  {
    float a[RMR], b[RMR];
    const int64_t cbase = T.vec_base + (act ? h : T.n_hands - 1);
#pragma unroll
    for (int k = 0; k < RMR; ++k) {
      if (wv + RMW * k >= SL) break;
      const int r = wv + RMW * k;
      const int64_t idx = cbase + (int64_t)row_id(r) * stride;
      if (MODE != 2) a[k] = g[idx];
      b[k] = R[idx];
      if (MODE != 1) {
        c[k] = x[idx];
        d[k] = xs[idx];
      }
    }
    if (MODE == 2 && wv == 0 && T.n_ext > 0) {
      // parent weights of the external parents, all loads in flight at once
      float xe[kTaskExtMax];
#pragma unroll
      for (int k = 0; k < kTaskExtMax; ++k)
        xe[k] = x[cbase + (int64_t)rl(extv, min(k, T.n_ext - 1)) * stride];
#pragma unroll
      for (int k = 0; k < kTaskExtMax; ++k)
        if (k < T.n_ext) Xl[k * 64 + lane] = xe[k];
    }
#pragma unroll
    for (int k = 0; k < RMR; ++k) {
      const int r = wv + RMW * k;
      if (r < SL) {
        if (MODE != 2) Al[r * 64 + lane] = a[k];
        Rl[r * 64 + lane] = b[k];
      }
    }
  }
  if (MODE != 2 && T.n_pull > 0)   // a wavefront's pulls go into rows it loaded: no barrier first
    rm_pulls<64>(P, T, Al, stage, lane, wv, lane, act ? h : T.n_hands - 1, true);
  if (MODE != 2 && wv == 0)
    for (int k = 0; k < T.n_ext; ++k) Xl[k * 64 + lane] = 0.f;
  // infoset ranges: wavefront wv's group, and the top part (all infosets when
  // the piece is not split)
  const int gb = grouped ? rl(grpv, kRmGBeg + wv) : 0, ge = grouped ? rl(grpv, kRmGEnd + wv) : 0;
  const int tb = grouped ? rl(grpv, kRmGTop) : 0, te = grouped ? rl(grpv, kRmGTop + 1) : T.n_inf;
  if (MODE != 2 && grouped)
    for (int j = 0; j < rl(grpv, kRmGCnt + wv); ++j) Xw[(wv * kRmGroupSlots + j) * 64 + lane] = 0.f;
  __syncthreads();
  if (MODE != 2) {
    // pass 0: the wavefront's group (groups concurrently, a group root's
    // value to its slot); pass 1: the top part on wavefront 0, after the
    // slots are added into their targets in a fixed order
#pragma unroll 1
    for (int ps = grouped ? 0 : 1; ps < 2; ++ps) {
      if (ps == 1 && grouped) {
        __syncthreads();
        if (wv == 0) rm_merge<64>(rsm, grpv, lane, true);
      }
      if (ps == 1 && wv != 0) break;
      const int i0 = ps ? tb : gb, i1 = ps ? te : ge;
      for (int i = i1 - 1; i >= i0; --i) {
        const int v = rl(infv, i);
        rmp_up<DC>(Al, Rl, &rsm[((v >> 16) & 255) * 64 + lane], v & 255, (v >> 8) & 255, lane, K);
      }
    }
    if (MODE == 1 && wv == 0 && act)
      for (int k = 0; k < T.n_ext; ++k) stage[(int64_t)rl(extv, k) * P.stage_stride + h] = Xl[k * 64 + lane];
  }
  if (MODE != 1) {
    // pass 0: the top part on wavefront 0 (root weight 1); pass 1: the
    // wavefront's group
#pragma unroll 1
    for (int ps = 0; ps < (grouped ? 2 : 1); ++ps) {
      if (ps == 1) __syncthreads();
      else if (wv != 0) continue;
      else rsm[kRmRowOne * 64 + lane] = 1.f;
      const int i0 = ps ? gb : tb, i1 = ps ? ge : te;
      for (int i = i0; i < i1; ++i) {
        const int v = rl(infv, i);
        rmp_down(Al, Rl, &rsm[((uint32_t)v >> 24) * 64 + lane], v & 255, (v >> 8) & 255, lane);
      }
    }
  }
  __syncthreads();
  if (act) {
    // all LDS reads first, then the stores
    float a[RMR], b[RMR];
#pragma unroll
    for (int k = 0; k < RMR; ++k) {
      const int r = min(wv + RMW * k, SL - 1);
      if (MODE != 2) b[k] = Rl[r * 64 + lane];
      if (MODE != 1) a[k] = Al[r * 64 + lane];
    }
#pragma unroll
    for (int k = 0; k < RMR; ++k) {
      const int r = wv + RMW * k;
      if (r < SL) {
        const int64_t idx = base + (int64_t)row_id(r) * stride;
        if (MODE != 2) R[idx] = b[k];
        if (MODE != 1) {
          x[idx] = a[k];
          xs[idx] = d[k] + K.w * (double)c[k];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Regret update with four lanes per hand (k_rmq), for launches of few
// workgroups, where the walk's latency is the cost: a workgroup holds 16
// hands, lane 4 h + q of a wavefront takes action q (and q + 4, ...) of each
// infoset for hand h, and the sums over an infoset's actions are two DPP
// steps across the quad.  A walk step so runs about a quarter of the
// per-lane instructions of k_rmp.  Same pieces, tables and LDS row numbering
// as k_rmp, with rows of 16 hands; a block record of 64 hands is taken by
// four workgroups.
// ---------------------------------------------------------------------------
constexpr int RQH = 16;   // hands per workgroup

__device__ inline float quad_sum(float v) {
  v += __int_as_float(dpp_i<0xB1, 0xf>(__float_as_int(v)));   // quad_perm [1,0,3,2]
  v += __int_as_float(dpp_i<0x4E, 0xf>(__float_as_int(v)));   // quad_perm [2,3,0,1]
  return v;
}

// Bottom-up step for one hand's quad: actions q, q + 4, ... of the infoset.
template <bool DC>
__device__ inline void rmq_up(float* __restrict__ Al, float* __restrict__ Rl, float* __restrict__ rsm, int f,
                              int n, int up, int q, int hl, const RmStep& K) {
  const int na = (n + 3) >> 2;   // actions per lane
  float rs = 0.f, dot = 0.f, gs = 0.f;
  float rr[2], gg[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const int a = q + 4 * c;
    const int o = (f + min(a, n - 1)) * RQH + hl;
    rr[c] = Rl[o];
    gg[c] = Al[o];
    const bool on = c < na && a < n;
    const float r = on ? fmaxf(rr[c], 0.f) : 0.f;
    rs += r;
    dot += r * gg[c];
    gs += on ? gg[c] : 0.f;
  }
  for (int c = 2; c < na; ++c) {   // infosets of more than 8 actions
    const int a = q + 4 * c;
    const int o = (f + min(a, n - 1)) * RQH + hl;
    const bool on = a < n;
    const float r = on ? fmaxf(Rl[o], 0.f) : 0.f, gv = Al[o];
    rs += r;
    dot += r * gv;
    gs += on ? gv : 0.f;
  }
  rs = quad_sum(rs);
  dot = quad_sum(dot);
  gs = quad_sum(gs);
  const bool pos = rs > 0.f;
  float sc;
  const float rc = rm_rcp(pos ? rs : (float)n, sc);
  const float V = ((pos ? dot : gs) * sc) * rc;
  // positions past the last action rewrite the last action's row with the
  // value its own lane writes
#pragma unroll
  for (int c = 0; c < 2; ++c)
    if (c < na) Rl[(f + min(q + 4 * c, n - 1)) * RQH + hl] = rm_new<DC>(rr[c], gg[c] - V, K);
  for (int c = 2; c < na; ++c) {
    const int o = (f + min(q + 4 * c, n - 1)) * RQH + hl;
    Rl[o] = rm_new<DC>(Rl[o], Al[o] - V, K);
  }
  if (q == 0) rsm[up * RQH + hl] += V;
}

// Top-down step for one hand's quad.
__device__ inline void rmq_down(float* __restrict__ Al, const float* __restrict__ Rl, const float* __restrict__ rsm,
                                int f, int n, int dn, int q, int hl) {
  const int na = (n + 3) >> 2;
  float rs = 0.f;
  for (int c = 0; c < na; ++c) {
    const int a = q + 4 * c;
    rs += a < n ? fmaxf(Rl[(f + min(a, n - 1)) * RQH + hl], 0.f) : 0.f;
  }
  rs = quad_sum(rs);
  const float xp = rsm[dn * RQH + hl];
  const bool pos = rs > 0.f;
  float sc;
  const float rc = rm_rcp(pos ? rs : (float)n, sc);
  for (int c = 0; c < na; ++c) {
    const int o = (f + min(q + 4 * c, n - 1)) * RQH + hl;
    Al[o] = xp * (((pos ? fmaxf(Rl[o], 0.f) : 1.f) * sc) * rc);
  }
}

template <int MODE, bool DC, int ROWS = kTaskRowsMax>
__global__ __launch_bounds__(64 * RMW) void k_rmq(RmParams P, float* __restrict__ g, float* __restrict__ R,
                                                  float* __restrict__ x, double* __restrict__ xs,
                                                  float* __restrict__ stage, const double* __restrict__ tdev) {
  extern __shared__ float rsm[];
  const RmTask T = P.blocks[blockIdx.x >> 2].t;
  const int h0 = P.blocks[blockIdx.x >> 2].h0 + RQH * (int)(blockIdx.x & 3);
  if (h0 >= T.n_hands) return;                 // whole block
  if (P.active && !P.active[T.inst]) return;   // whole block: T is uniform
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int q = lane & 3, hl = lane >> 2;
  const int h = h0 + hl;
  const bool act = h < T.n_hands;
  const int SL = T.n_rows;
  float* Xw = rsm + kRmRowSlot * RQH;
  float* Xl = rsm + kRmRowExt * RQH;
  float* Al = rsm + kRmRowLocal * RQH;
  float* Rl = Al + P.max_rows * RQH;
  const int64_t hc = act ? h : T.n_hands - 1;   // in-bounds hand for loads
  const int64_t stride = T.stride;
  const RmStep K = rm_step(DC, P.gamma, P.alpha, P.beta, *tdev);
  const int rowv = T.row0 >= 0 ? T.row0 + lane : (lane < SL ? P.rows[T.rows_off + lane] : 0);
  const int infv = lane < T.n_inf ? P.infs[T.inf_off + lane] : 0;
  const bool grouped = T.grp_off >= 0;
  const int grpv = grouped ? P.grp[T.grp_off + lane] : 0;
  const int extv = (MODE != 0 && lane < T.n_ext)
                       ? (MODE == 1 ? P.ext_slot[T.ext_off + lane] : P.ext_seq[T.ext_off + lane]) : 0;
  // rows 4 (wv + RMW k) + q for k < 4, 16 hands each: lane (hl, q) takes
  // row 4 (wv + RMW k) + q of hand hl
  constexpr int RQK = ROWS / (4 * RMW);
  static_assert(ROWS == kTaskRowsMax || MODE == 0, "whole-treeplex pieces have no external parents");
  float c[RQK];
  double d[RQK];
  int rid[RQK];
  {
    float a[RQK], b[RQK];
#pragma unroll
    for (int k = 0; k < RQK; ++k) {
      const int r = min(4 * (wv + RMW * k) + q, SL - 1);
      rid[k] = T.row0 >= 0 ? T.row0 + r : r < 64 ? __shfl(rowv, r, 64) : P.rows[T.rows_off + r];
      const int64_t idx = T.vec_base + hc + (int64_t)rid[k] * stride;
      if (MODE != 2) a[k] = g[idx];
      b[k] = R[idx];
      if (MODE != 1) {
        c[k] = x[idx];
        d[k] = xs[idx];
      }
    }
    if (MODE == 2 && wv == 0 && T.n_ext > 0) {
      float xe[kTaskExtMax];
#pragma unroll
      for (int k = 0; k < kTaskExtMax; ++k)
        xe[k] = x[T.vec_base + hc + (int64_t)rl(extv, min(k, T.n_ext - 1)) * stride];
#pragma unroll
      for (int k = 0; k < kTaskExtMax; ++k)
        if (k < T.n_ext && q == 0) Xl[k * RQH + hl] = xe[k];
    }
#pragma unroll
    for (int k = 0; k < RQK; ++k) {
      const int r = 4 * (wv + RMW * k) + q;
      if (r < SL) {
        if (MODE != 2) Al[r * RQH + hl] = a[k];
        Rl[r * RQH + hl] = b[k];
      }
    }
  }
  if (MODE != 2 && wv == 0 && q == 0)
    for (int k = 0; k < T.n_ext; ++k) Xl[k * RQH + hl] = 0.f;
  const int gb = grouped ? rl(grpv, kRmGBeg + wv) : 0, ge = grouped ? rl(grpv, kRmGEnd + wv) : 0;
  const int tb = grouped ? rl(grpv, kRmGTop) : 0, te = grouped ? rl(grpv, kRmGTop + 1) : T.n_inf;
  if (MODE != 2 && grouped && q == 0)
    for (int j = 0; j < rl(grpv, kRmGCnt + wv); ++j) Xw[(wv * kRmGroupSlots + j) * RQH + hl] = 0.f;
  __syncthreads();
  if (MODE != 2 && T.n_pull > 0) {
    // after the barrier: a wavefront's pulls target rows other wavefronts
    // loaded; one lane per hand writes
    rm_pulls<RQH>(P, T, Al, stage, lane, wv, hl, hc, q == 0);
    __syncthreads();
  }
  if (MODE != 2) {
#pragma unroll 1
    for (int ps = grouped ? 0 : 1; ps < 2; ++ps) {
      if (ps == 1 && grouped) {
        __syncthreads();
        if (wv == 0) rm_merge<RQH>(rsm, grpv, hl, q == 0);
      }
      if (ps == 1 && wv != 0) break;
      const int i0 = ps ? tb : gb, i1 = ps ? te : ge;
      for (int i = i1 - 1; i >= i0; --i) {
        const int v = rl(infv, i);
        rmq_up<DC>(Al, Rl, rsm, v & 255, (v >> 8) & 255, (v >> 16) & 255, q, hl, K);
      }
    }
    if (MODE == 1 && wv == 0 && act && q == 0)
      for (int k = 0; k < T.n_ext; ++k) stage[(int64_t)rl(extv, k) * P.stage_stride + h] = Xl[k * RQH + hl];
  }
  if (MODE != 1) {
#pragma unroll 1
    for (int ps = 0; ps < (grouped ? 2 : 1); ++ps) {
      if (ps == 1) __syncthreads();
      else if (wv != 0) continue;
      else if (q == 0) rsm[kRmRowOne * RQH + hl] = 1.f;
      const int i0 = ps ? gb : tb, i1 = ps ? ge : te;
      for (int i = i0; i < i1; ++i) {
        const int v = rl(infv, i);
        rmq_down(Al, Rl, rsm, v & 255, (v >> 8) & 255, (uint32_t)v >> 24, q, hl);
      }
    }
  }
  __syncthreads();
  if (act) {
    float a[RQK], b[RQK];
#pragma unroll
    for (int k = 0; k < RQK; ++k) {
      const int r = min(4 * (wv + RMW * k) + q, SL - 1);
      if (MODE != 2) b[k] = Rl[r * RQH + hl];
      if (MODE != 1) a[k] = Al[r * RQH + hl];
    }
#pragma unroll
    for (int k = 0; k < RQK; ++k) {
      const int r = 4 * (wv + RMW * k) + q;
      if (r < SL) {
        const int64_t idx = T.vec_base + h + (int64_t)rid[k] * stride;
        if (MODE != 2) R[idx] = b[k];
        if (MODE != 1) {
          x[idx] = a[k];
          xs[idx] = d[k] + K.w * (double)c[k];
        }
      }
    }
  }
}

// Best response: per hand, bottom-up max (Player 1) or min (Player 2) of g
// plus the values below; sums of root values go to hv[hand_base + h].
template <int MODE, bool MAXIMIZE>
__global__ __launch_bounds__(TPB) void k_br(TpParams P, double* __restrict__ g,
                                            double* __restrict__ stage, double* __restrict__ hv) {
  const int2 bt = P.blocks[blockIdx.x];
  const TpTask T = P.tasks[bt.x];
  if (P.active && !P.active[T.inst]) return;   // instance not asked for
  const int h = bt.y + threadIdx.x;
  if (h >= T.n_hands) return;
  const int64_t base = T.vec_base + h, stride = T.stride;
  if (MODE == 2) {
    for (int i = T.pull_begin; i < T.pull_end; ++i) {
      const TpPull pl = P.pulls[i];
      g[base + (int64_t)pl.seq * stride] += stage[(int64_t)pl.stage * P.stage_stride + h];
    }
  }
  double vroot = 0.0;
  for (int i = T.inf_end - 1; i >= T.inf_begin; --i) {
    const int I = P.order[i];
    const int par = P.inf_parent[I], f = P.inf_first[I], n = P.inf_nact[I];
    double V = g[base + (int64_t)f * stride];
    for (int a = 1; a < n; ++a) {
      const double q = g[base + (int64_t)(f + a) * stride];
      // a NaN propagates (fmax / fmin would drop it): a non-finite gradient
      // must reach the host check
      if (isnan(q) || (MAXIMIZE ? q > V : q < V)) V = q;
    }
    if (par == T.ext_parent) vroot += V;
    else g[base + (int64_t)par * stride] += V;
  }
  if (MODE == 1) stage[(int64_t)T.stage * P.stage_stride + h] = vroot;
  else hv[T.hand_base + h] = vroot;
}

// Per-instance sum of per-hand values, fixed order (deterministic).
__global__ __launch_bounds__(256) void k_sum_instances(const double* __restrict__ hv,
                                                       const int64_t* __restrict__ off,
                                                       double* __restrict__ out) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  const int64_t a = off[i], b = off[i + 1];
  double s = 0.0;
  for (int64_t j = a + threadIdx.x; j < b; j += 256) s += hv[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = red[0];
}

// Uniform realization plan (top-down with zero regrets), thread per hand.
__global__ __launch_bounds__(TPB) void k_uniform(TpParams P, float* __restrict__ x) {
  const int2 bt = P.blocks[blockIdx.x];
  const TpTask T = P.tasks[bt.x];
  const int h = bt.y + threadIdx.x;
  if (h >= T.n_hands) return;
  const int64_t base = T.vec_base + h, stride = T.stride;
  for (int i = T.inf_begin; i < T.inf_end; ++i) {
    const int I = P.order[i];
    const int par = P.inf_parent[I], f = P.inf_first[I], n = P.inf_nact[I];
    const float xp = par >= 0 ? x[base + (int64_t)par * stride] : 1.f;
    for (int a = 0; a < n; ++a) x[base + (int64_t)(f + a) * stride] = xp / (float)n;
  }
}

// Regrets from a behavioural strategy (warm start): R = scale * b, and the
// matching realization plan (thread per hand, top-down).
__global__ __launch_bounds__(TPB) void k_warm(TpParams P, const float* __restrict__ b,
                                              float scale, float* __restrict__ R,
                                              float* __restrict__ x) {
  const int2 bt = P.blocks[blockIdx.x];
  const TpTask T = P.tasks[bt.x];
  const int h = bt.y + threadIdx.x;
  if (h >= T.n_hands) return;
  const int64_t base = T.vec_base + h, stride = T.stride;
  for (int i = T.inf_begin; i < T.inf_end; ++i) {
    const int I = P.order[i];
    const int par = P.inf_parent[I], f = P.inf_first[I], n = P.inf_nact[I];
    const float xp = par >= 0 ? x[base + (int64_t)par * stride] : 1.f;
    float s = 0.f;
    for (int a = 0; a < n; ++a) {
      float v = b[base + (int64_t)(f + a) * stride];
      s += v > 0.f ? v : 0.f;
    }
    for (int a = 0; a < n; ++a) {
      int64_t j = base + (int64_t)(f + a) * stride;
      float v = b[j] > 0.f ? b[j] : 0.f;
      float ba = s > 0.f ? v / s : 1.f / (float)n;
      R[j] = scale * ba;
      x[j] = xp * ba;
    }
  }
}

__global__ void k_fill_f32(float* p, int64_t n, float v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_fill_f64(double* p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
__global__ void k_f32_to_f64(const float* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = (double)a[i];
}
__global__ void k_fill_i32(int* p, int n, int v) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// warm start: rows = (infoset, hand) pairs of one player, instance by instance
// ---------------------------------------------------------------------------
struct WarmSeg {
  int64_t row_base;        // first row of this infoset
  int64_t vec_base;        // instance's vector block
  int32_t stride, n_hands, hand_base, first;
  int32_t nact, parent, inst, pad1;
};

__device__ inline uint16_t dev_f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// X[row] = betting features of the infoset ++ range features of the hand (BF16)
__global__ __launch_bounds__(256) void k_warm_features(const WarmSeg* __restrict__ segs,
                                                       const int2* __restrict__ blocks,
                                                       const float* __restrict__ inf_feat,
                                                       const float* __restrict__ hand_feat,
                                                       uint16_t* __restrict__ X) {
  const int2 bt = blocks[blockIdx.x];
  const WarmSeg S = segs[bt.x];
  const int h = bt.y + threadIdx.x;
  if (h >= S.n_hands) return;
  uint16_t* xr = X + (S.row_base + h) * kWarmIn;
  const float* fi = inf_feat + (int64_t)bt.x * kInfFeat;
  const float* fh = hand_feat + (int64_t)(S.hand_base + h) * kHandFeat;
  for (int j = 0; j < kInfFeat; ++j) xr[j] = dev_f2bf(fi[j]);
  for (int j = 0; j < kHandFeat; ++j) xr[kInfFeat + j] = dev_f2bf(fh[j]);
}

// Targets from the solver's average: b*(a|I,h) = xbar[Ia] / xbar[parent]
// (uniform where the parent is unreached); invalid action slots get -1.
// Weight = belief weight relative to the mean x average reach of the infoset
// (the sums over the instance's own averaging weight total).
__global__ __launch_bounds__(256) void k_warm_targets(const WarmSeg* __restrict__ segs,
                                                      const int2* __restrict__ blocks,
                                                      const double* __restrict__ xs,
                                                      const double* __restrict__ wsum_inst,
                                                      const float* __restrict__ hand_feat,
                                                      float* __restrict__ T, float* __restrict__ W) {
  const int2 bt = blocks[blockIdx.x];
  const WarmSeg S = segs[bt.x];
  const int h = bt.y + threadIdx.x;
  if (h >= S.n_hands) return;
  const int64_t base = S.vec_base + h, row = S.row_base + h;
  double tot = 0.0;
  for (int a = 0; a < S.nact; ++a) tot += xs[base + (int64_t)(S.first + a) * S.stride];
  float* tr = T + row * kWarmActions;
  for (int a = 0; a < kWarmActions; ++a) {
    float v = -1.f;
    if (a < S.nact)
      v = tot > 0.0 ? (float)(xs[base + (int64_t)(S.first + a) * S.stride] / tot) : 1.f / (float)S.nact;
    tr[a] = v;
  }
  const double wsum = wsum_inst[S.inst];
  const double reach = wsum > 0.0 ? tot / wsum : 0.0;
  W[row] = (float)(8.0 * hand_feat[(int64_t)(S.hand_base + h) * kHandFeat] * reach);
}

// Prior from network logits: masked softmax per row, regrets = scale * prior,
// plan = its realization (top-down), averages seeded with weight avg_w.
__global__ __launch_bounds__(TPB) void k_warm_apply(TpParams P, const int64_t* __restrict__ row_base,
                                                    const float* __restrict__ Z, int ldz, float scale,
                                                    double avg_w, const double* __restrict__ lam,
                                                    const int64_t* __restrict__ lam_off,
                                                    const double* __restrict__ pot, float* __restrict__ R,
                                                    float* __restrict__ x, double* __restrict__ xs) {
  const int2 bt = P.blocks[blockIdx.x];
  const TpTask T = P.tasks[bt.x];
  const int h = bt.y + threadIdx.x;
  if (h >= T.n_hands) return;
  const int64_t base = T.vec_base + h, stride = T.stride;
  // regrets in the units of this hand's gradients: lambda(h) x pot
  const float rs = scale * (float)(lam[lam_off[T.inst] + h] * pot[T.inst]);
  for (int i = T.inf_begin; i < T.inf_end; ++i) {
    const int I = P.order[i];
    const int par = P.inf_parent[I], f = P.inf_first[I], n = P.inf_nact[I];
    const float* zr = Z + (row_base[I] + h) * ldz;
    float mx = -INFINITY;
    for (int a = 0; a < n; ++a) mx = fmaxf(mx, zr[a]);
    float se = 0.f;
    for (int a = 0; a < n; ++a) se += __expf(zr[a] - mx);
    const float xp = par >= 0 ? x[base + (int64_t)par * stride] : 1.f;
    for (int a = 0; a < n; ++a) {
      const int64_t j = base + (int64_t)(f + a) * stride;
      float pa = __expf(zr[a] - mx) / se;
      if (!(pa >= 0.f)) pa = 1.f / (float)n;   // NaN guard: uniform
      R[j] = rs * pa;
      x[j] = xp * pa;
      xs[j] = avg_w * (double)(xp * pa);
    }
  }
}

// ---------------------------------------------------------------------------
// Technique B's explicit factors: CSR products and the chain solve of M
// ---------------------------------------------------------------------------
// y[r] (+)= sum_j val[j] x[idx[j]] over row r's entries; one wavefront per
// row, lanes striding over the entries, a butterfly sum across the lanes.
__global__ __launch_bounds__(256) void k_csr_spmv(int64_t rows, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ idx, const double* __restrict__ val,
                                                  const double* __restrict__ x, double* __restrict__ y, int accumulate) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= rows) return;
  double s = 0.0;
  for (int64_t j = ptr[r] + lane; j < ptr[r + 1]; j += 64) s += val[j] * x[idx[j]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) y[r] = accumulate ? y[r] + s : s;
}

// One round of pointer jumping on M's chains: an unknown's value is its
// right-hand side plus coef times the value at ptr; each round folds in the
// target's own term and doubles the span (z = r + c z_p -> z = (r + c r_p) +
// c c_p z_pp).
__global__ __launch_bounds__(256) void k_chain_round(int64_t m, const double* __restrict__ va,
                                                     const double* __restrict__ ca, const int32_t* __restrict__ pa,
                                                     double* __restrict__ vb, double* __restrict__ cb,
                                                     int32_t* __restrict__ pb) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  const int32_t p = pa[k];
  if (p >= 0) {
    vb[k] = va[k] + ca[k] * va[p];
    cb[k] = ca[k] * ca[p];
    pb[k] = pa[p];
  } else {
    vb[k] = va[k];
    cb[k] = 0.0;
    pb[k] = -1;
  }
}

// ---------------------------------------------------------------------------
// the Game object
// ---------------------------------------------------------------------------
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  ~DBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t count) {
    if (p) {
      (void)hipFree(p);
      p = nullptr;
    }
    n = count;
    if (count == 0) return PMX_OK;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return fail(PMX_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    return PMX_OK;
  }
  int upload(const std::vector<T>& v) {
    int rc = alloc(v.size());
    if (rc) return rc;
    if (!v.empty()) HIP_TRY(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return PMX_OK;
  }
};

struct DevDir {                 // the row chunks of one direction (the layouts' shared item list)
  DBuf<MvItem> items;
  DBuf<MvRed> red;              // rows summed from partial rows
  DBuf<double> part;            // partial rows (FP32 products use the first half)
  int nblk = 0, nred = 0;
};

struct DevMc {                  // chunk-aligned matvec layout of one direction
  DBuf<McCtx> ctx;
  DBuf<uint32_t> q, pos, meta;
  DBuf<int32_t> chunks[kMcClasses];
  int count[kMcClasses] = {0, 0, 0, 0, 0};
  DBuf<int32_t> chunks_act[kMcClasses];   // the solver's lists: chunks of active instances only
  int count_act[kMcClasses] = {0, 0, 0, 0, 0};
  int block = 0;                // 0: not built
};

struct DevGrp {                 // grouped matvec layout of one direction (kernel 4)
  DBuf<GCtx> ctx;
  DBuf<GGroup> groups;
  DBuf<uint32_t> q, src, meta;
  DBuf<uint16_t> rk;
  DBuf<int32_t> chunks[GrpDir::kKinds][kGrpClasses];       // [plain, carrying, two-wide][class]
  int count[GrpDir::kKinds][kGrpClasses] = {};
  DBuf<int32_t> chunks_act[GrpDir::kKinds][kGrpClasses];   // the solver's lists: active instances only
  int count_act[GrpDir::kKinds][kGrpClasses] = {};
  bool built = false;
};

struct DevTp {
  DBuf<int32_t> inf_parent, inf_first, inf_nact, order;
  DBuf<TpTask> tasks;
  DBuf<TpPull> pulls;
  DBuf<int2> b_single, b_deep, b_top, b_all;
  int n_single = 0, n_deep = 0, n_top = 0, n_all = 0;
  DBuf<float> stage;
  DBuf<double> stage_d;
  DBuf<double> hv;
  int stage_stride = 0;
};

struct DevRm {                  // regret-update pieces of one player
  DBuf<int32_t> rows, infs, pulls, ext_seq, ext_slot, grp;
  DBuf<RmBlock> blocks;         // blocks of the active instances, depth d at [blk_off[d], blk_off[d + 1])
  std::vector<int> blk_off;
  int blk_pull0 = 0;            // depth 0: blocks [blk_off[0], blk_pull0) have no pulls
  std::vector<int> max_rows, max_ext;   // per depth
  DBuf<float> stage;
  int stage_stride = 1;
};

struct Game {
  HostGame hg;
  bool device = false;
  int device_id = 0;
  DevDir dd[2];
  DevMc dm[2];
  DevGrp dg[2];
  DevTp dt[2];
  DevRm drm[2];
  DBuf<double> lam;
  DBuf<float> lamf;
  int64_t lam_base[2] = {0, 0};
  std::vector<int64_t> lam_off[2];   // per player: offset of each instance's lambdas
  DBuf<int64_t> inst_hand_off[2];
  // solver state
  DBuf<float> R[2], x[2], grad[2];
  DBuf<double> xs[2], gd[2], sd[2], br_inst;
  int t = 0;
  double wsum = 0.0;                // averaging weight total of the iterations so far
  std::vector<double> wsum_i;       // per instance: the weights of the iterations it took part in
  std::vector<char> act_h;          // per instance: host copy of the active flags
  DBuf<double> wsum_dev;            // wsum_i on the device (warm-start targets)
  // last FP64 gap per instance; valid while the instance's state is unchanged
  std::vector<double> gap_c, br1_c, br2_c;
  std::vector<char> gap_ok;
  // divergence guard: each instance's last computed gap and how many
  // computations in a row found it grown
  int gap_guard = 16;
  std::vector<double> gap_prev;
  std::vector<int> gap_grow;
  DBuf<int32_t> gap_need;           // per instance: 1 = the gap call computes it
  int mv_block = 256;
  int max_lds = 64 * 1024;          // dynamic LDS bytes a workgroup may use on this device
  DBuf<double> tdev;                // iteration index of the next step (device)
  // Technique B's explicit factors (tb_build): CSR matrices and M's chains
  struct TbDev {
    DBuf<int64_t> ptr[6];
    DBuf<int32_t> idx[6];
    DBuf<double> val[6];
    int64_t rows[6] = {0, 0, 0, 0, 0, 0};
    DBuf<int32_t> par, chi, ptrbuf[2];
    DBuf<double> cpar, cchi, tvec, valbuf[2], coefbuf[2];
    int64_t m = 0;
    int rounds = 0;
    bool built = false;
  } tb;
  std::unique_ptr<TbHost> tb_host;   // the host factors of the last tb_build
  TbCsr tb_m;                        // M after postprocessing as CSR (diagonal included)
  DBuf<int32_t> active;             // per-instance: 1 = iterated by solver_step
  DBuf<float> snap_R[2], snap_x[2];   // solver_snapshot: regrets, plans
  DBuf<double> snap_xs[2];            //   and average sums
  std::vector<double> snap_wsum_i;    //   per-instance weight totals
  int snap_t = -1;                    //   iterations at the snapshot (-1: none)
  std::vector<char> listed;         // instances the solver's launch lists include
  int n_listed = 0;
  int dcfr = 0, gamma = 1;          // solver rule (see solver_set_params)
  double alpha = 1.5, beta = 0.0;
  // warm start: per player infoset segments, their blocks, features
  DBuf<WarmSeg> wseg[2];
  DBuf<int2> wblk[2];
  DBuf<int64_t> wrow_base[2];
  DBuf<float> winf[2], whand[2];
  DBuf<int64_t> lam_inst[2];
  DBuf<double> pot_inst;
  int64_t wrows[2] = {0, 0};
  int wn_blk[2] = {0, 0};
  bool warm_ok = true;
  // solver iterations captured as a graph
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int graph_iters = 0;
  bool use_graph = true;
  // the hands-per-thread classes of one grouped matvec run concurrently: the
  // caller's stream forks to side streams (default priority) and joins them
  static constexpr int kSide = 3;
  hipStream_t side[kSide] = {};
  hipEvent_t fork_ev = nullptr, join_ev[kSide] = {};
  bool fork_ok = false;
  ~Game() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (int i = 0; i < kSide; ++i) {
      if (side[i]) (void)hipStreamDestroy(side[i]);
      if (join_ev[i]) (void)hipEventDestroy(join_ev[i]);
    }
    if (fork_ev) (void)hipEventDestroy(fork_ev);
  }
};

// Streams a grouped matvec spreads its class launches over: the caller's
// and Game::kSide side streams; products of fewer workgroups in all than
// kForkMinWorkgroups are not spread.
constexpr int kForkStreams = 1 + Game::kSide;
constexpr int kForkMinWorkgroups = 512;

// Side streams and events of the concurrent class launches (created once,
// outside any capture).
static int ensure_fork(Game* g) {
  if (g->fork_ok) return PMX_OK;
  HIP_TRY(hipEventCreateWithFlags(&g->fork_ev, hipEventDisableTiming));
  for (int i = 0; i < Game::kSide; ++i) {
    HIP_TRY(hipStreamCreateWithFlags(&g->side[i], hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&g->join_ev[i], hipEventDisableTiming));
  }
  g->fork_ok = true;
  return PMX_OK;
}

// Every instance's gap is computed again at the next saddle_gap; a new start
// of the solver state (reset, a loaded state, a warm start) also restarts the
// divergence guard's history, new weight totals do not.
static void invalidate_gaps(Game* g, bool restart = true) {
  g->gap_ok.assign(g->gap_ok.size(), 0);
  if (!restart) return;
  g->gap_prev.assign(g->gap_prev.size(), std::nan(""));
  g->gap_grow.assign(g->gap_grow.size(), 0);
}

static int ensure_device(Game* g) {
  if (!g) return fail(PMX_EINVAL, "null game");
  if (!g->device) return fail(PMX_ESTATE, "game was created host-only");
  HIP_TRY(hipSetDevice(g->device_id));
  return PMX_OK;
}

static std::vector<int2> tp_blocks(const TpPlan& T, const std::vector<int32_t>& ids, int per = TPB) {
  std::vector<int2> b;
  for (int id : ids)
    for (int h0 = 0; h0 < T.tasks[id].n_hands; h0 += per) b.push_back(make_int2(id, h0));
  return b;
}

// The solver's row-chunk lists of one direction: the chunks of the instances
// its launch lists include (g->listed; every instance when unset).
static int upload_mc_active(Game* g, int d) {
  DevMc& E = g->dm[d];
  const McDir& M = g->hg.mc[d];
  const bool all = g->listed.size() != g->hg.inst.size();
  for (int c = 0; c < kMcClasses; ++c) {
    std::vector<int32_t> L;
    const std::vector<int32_t>& F = M.chunks[c];
    for (size_t i = 0; i + 3 < F.size(); i += 4)
      if (all || g->listed[F[i + 2]]) L.insert(L.end(), F.begin() + i, F.begin() + i + 4);
    int rc = E.chunks_act[c].upload(L);
    if (rc) return rc;
    E.count_act[c] = (int)L.size() / 4;
  }
  return PMX_OK;
}

static int upload_mc(Game* g, int d) {
  HostGame& hg = g->hg;
  DevMc& E = g->dm[d];
  const int block = hg.mc_block;
  std::string m;
  int rc = build_mc_layout(hg, d, block, m);
  if (rc) return fail(rc, m);
  McDir& M = hg.mc[d];
  const int p = d, q = 1 - d;
  size_t ci = 0;
  for (size_t ii = 0; ii < hg.inst.size(); ++ii)
    for (int c = 0; c < hg.inst[ii].n_ctx; ++c, ++ci) {
      M.ctx[ci].lam_own_off = g->lam_off[p][ii];
      M.ctx[ci].lam_opp_off = g->lam_off[q][ii];
    }
  std::vector<uint32_t> qv;
  qv.reserve(M.q.size() * 4);
  for (const QueryRec16& r : M.q) {
    qv.push_back(r.x);
    qv.push_back(r.y);
    qv.push_back(r.z);
    qv.push_back(r.w);
  }
  if ((rc = E.ctx.upload(M.ctx)) || (rc = E.q.upload(qv)) || (rc = E.pos.upload(M.pos)) ||
      (rc = E.meta.upload(M.meta)))
    return rc;
  for (int c = 0; c < kMcClasses; ++c) {
    if ((rc = E.chunks[c].upload(M.chunks[c]))) return rc;
    E.count[c] = (int)M.chunks[c].size() / 4;
  }
  E.block = block;
  return upload_mc_active(g, d);
}

// The solver's chunk lists of the grouped layout (as upload_mc_active).
static int upload_grp_active(Game* g, int d) {
  DevGrp& E = g->dg[d];
  const GrpDir& M = g->hg.grp[d];
  const bool all = g->listed.size() != g->hg.inst.size();
  for (int kind = 0; kind < GrpDir::kKinds; ++kind)
    for (int c = 0; c < kGrpClasses; ++c) {
      std::vector<int32_t> L;
      const std::vector<int32_t>& F = M.chunks[kind][c];
      for (size_t i = 0; i + 3 < F.size(); i += 4)
        if (all || g->listed[F[i + 2]]) L.insert(L.end(), F.begin() + i, F.begin() + i + 4);
      int rc = E.chunks_act[kind][c].upload(L);
      if (rc) return rc;
      E.count_act[kind][c] = (int)L.size() / 4;
    }
  return PMX_OK;
}

static int upload_grp(Game* g, int d) {
  HostGame& hg = g->hg;
  DevGrp& E = g->dg[d];
  E.built = false;
  std::string m;
  int rc = build_grp_layout(hg, d, hg.groups_per_chunk, m);
  if (rc) return fail(rc, m);
  GrpDir& M = hg.grp[d];
  const int p = d, q = 1 - d;
  size_t ci = 0;
  for (size_t ii = 0; ii < hg.inst.size(); ++ii)
    for (int c = 0; c < hg.inst[ii].n_ctx; ++c, ++ci) {
      M.ctx[ci].lam_own_off = g->lam_off[p][ii];
      M.ctx[ci].lam_opp_off = g->lam_off[q][ii];
    }
  if ((rc = E.ctx.upload(M.ctx)) || (rc = E.groups.upload(M.groups)) || (rc = E.q.upload(M.q)) ||
      (rc = E.src.upload(M.src)) || (rc = E.meta.upload(M.meta)) || (rc = E.rk.upload(M.rk)))
    return rc;
  for (int kind = 0; kind < GrpDir::kKinds; ++kind)
    for (int c = 0; c < kGrpClasses; ++c) {
      if ((rc = E.chunks[kind][c].upload(M.chunks[kind][c]))) return rc;
      E.count[kind][c] = (int)M.chunks[kind][c].size() / 4;
    }
  E.built = true;
  return upload_grp_active(g, d);
}

static int upload_dir(Game* g, int d) {
  int rc;
  HostGame& hg = g->hg;
  const MvDir& D = hg.dir[d];
  DevDir& E = g->dd[d];
  if ((rc = E.items.upload(D.items))) return rc;
  E.nblk = (int)D.blk.size() - 1;
  if ((rc = E.red.upload(D.red))) return rc;
  E.nred = (int)D.red.size();
  if ((rc = E.part.alloc((size_t)std::max<int64_t>(D.part_elems, 1)))) return rc;
  g->dg[d].built = false;
  if (hg.mv_kernel == 4 && (rc = upload_grp(g, d))) return rc;
  return upload_mc(g, d);
}

// Block records of one player's regret launches for the instances marked in
// `act` (every instance when empty); the LDS sizing per depth covers every
// piece either way.
static int upload_rm_blocks(Game* g, int p, const std::vector<char>& act) {
  const RmPlan& T = g->hg.rm[p];
  DevRm& E = g->drm[p];
  std::vector<RmBlock> blocks;
  const int D = (int)T.by_depth.size();
  E.blk_off.assign(D + 1, 0);
  for (int d = 0; d < D; ++d) {
    E.blk_off[d] = (int)blocks.size();
    // depth 0: the pieces without pulls (no deeper piece hangs from them)
    // first, so that they can run beside the deep passes
    for (int pass = 0; pass < (d == 0 ? 2 : 1); ++pass) {
      if (d == 0 && pass == 1) E.blk_pull0 = (int)blocks.size();
      for (int id : T.by_depth[d]) {
        const RmTask& t = T.tasks[id];
        if (!act.empty() && !act[t.inst]) continue;
        if (d == 0 && (t.n_pull > 0) != (pass == 1)) continue;
        for (int h0 = 0; h0 < t.n_hands; h0 += 64) {
          RmBlock bk{};
          bk.t = t;
          bk.h0 = h0;
          blocks.push_back(bk);
        }
      }
    }
  }
  if (D == 0) E.blk_pull0 = 0;
  E.blk_off[D] = (int)blocks.size();
  return E.blocks.upload(blocks);
}

static int upload_rm(Game* g, int p) {
  const RmPlan& T = g->hg.rm[p];
  DevRm& E = g->drm[p];
  int rc;
  if ((rc = E.rows.upload(T.rows)) || (rc = E.infs.upload(T.infs)) ||
      (rc = E.pulls.upload(T.pulls)) || (rc = E.ext_seq.upload(T.ext_seq)) || (rc = E.ext_slot.upload(T.ext_slot)) ||
      (rc = E.grp.upload(T.grp)))
    return rc;
  const int D = (int)T.by_depth.size();
  E.max_rows.assign(D, 0);
  E.max_ext.assign(D, 0);
  for (int d = 0; d < D; ++d)
    for (int id : T.by_depth[d]) {
      E.max_rows[d] = std::max(E.max_rows[d], (int)T.tasks[id].n_rows);
      E.max_ext[d] = std::max(E.max_ext[d], (int)T.tasks[id].n_ext);
    }
  if ((rc = upload_rm_blocks(g, p, g->listed.size() == g->hg.inst.size() ? g->listed : std::vector<char>())))
    return rc;
  E.stage_stride = std::max(T.stage_stride, 1);
  return E.stage.alloc((size_t)std::max(T.n_slot, 1) * E.stage_stride);
}

static int upload_game(Game* g) {
  HostGame& hg = g->hg;
  // lambda of both players, all instances
  std::vector<double> lam;
  std::vector<int64_t> lam_off[2];
  for (int p = 0; p < 2; ++p) {
    g->lam_base[p] = (int64_t)lam.size();
    for (auto& b : hg.inst) {
      lam_off[p].push_back((int64_t)lam.size());
      lam.insert(lam.end(), b.lam[p].begin(), b.lam[p].end());
    }
  }
  int rc = g->lam.upload(lam);
  if (rc) return rc;
  std::vector<float> lamf(lam.begin(), lam.end());
  if ((rc = g->lamf.upload(lamf))) return rc;
  g->lam_off[0] = lam_off[0];
  g->lam_off[1] = lam_off[1];
  for (int d = 0; d < 2; ++d)
    if ((rc = upload_dir(g, d)) || (rc = upload_rm(g, d))) return rc;
  for (int p = 0; p < 2; ++p) {
    TpPlan& T = hg.tp[p];
    DevTp& E = g->dt[p];
    if ((rc = E.inf_parent.upload(T.inf_parent)) || (rc = E.inf_first.upload(T.inf_first)) ||
        (rc = E.inf_nact.upload(T.inf_nact)) || (rc = E.order.upload(T.order)) ||
        (rc = E.tasks.upload(T.tasks)) || (rc = E.pulls.upload(T.pulls)))
      return rc;
    auto bs = tp_blocks(T, T.single), bd = tp_blocks(T, T.deep), bt = tp_blocks(T, T.top);
    std::vector<int32_t> all_ids = T.single;
    all_ids.insert(all_ids.end(), T.deep.begin(), T.deep.end());
    auto ba = tp_blocks(T, all_ids);
    if ((rc = E.b_single.upload(bs)) || (rc = E.b_deep.upload(bd)) || (rc = E.b_top.upload(bt)) ||
        (rc = E.b_all.upload(ba)))
      return rc;
    E.n_single = (int)bs.size();
    E.n_deep = (int)bd.size();
    E.n_top = (int)bt.size();
    E.n_all = (int)ba.size();
    E.stage_stride = std::max(T.stage_stride, 1);
    if ((rc = E.stage.alloc((size_t)std::max(T.n_stage, 1) * E.stage_stride)) ||
        (rc = E.stage_d.alloc((size_t)std::max(T.n_stage, 1) * E.stage_stride)) ||
        (rc = E.hv.alloc((size_t)std::max<int64_t>(T.hands_total, 1))))
      return rc;
    std::vector<int64_t> ho(1, 0);
    for (auto& b : hg.inst) ho.push_back(ho.back() + b.inst.n[p]);
    if ((rc = g->inst_hand_off[p].upload(ho))) return rc;
  }
  for (int p = 0; p < 2; ++p) {
    size_t n = (size_t)hg.elems[p];
    if ((rc = g->R[p].alloc(n)) || (rc = g->x[p].alloc(n)) || (rc = g->grad[p].alloc(n)) ||
        (rc = g->xs[p].alloc(n)) || (rc = g->gd[p].alloc(n)) || (rc = g->sd[p].alloc(n)))
      return rc;
  }
  if ((rc = g->br_inst.alloc(2 * hg.inst.size()))) return rc;
  if ((rc = g->tdev.alloc(1))) return rc;
  if ((rc = g->active.upload(std::vector<int32_t>(hg.inst.size(), 1)))) return rc;
  g->listed.assign(hg.inst.size(), 1);
  g->n_listed = (int)hg.inst.size();
  g->act_h.assign(hg.inst.size(), 1);
  g->wsum_i.assign(hg.inst.size(), 0.0);
  if ((rc = g->wsum_dev.alloc(hg.inst.size()))) return rc;
  g->gap_c.assign(hg.inst.size(), 0.0);
  g->br1_c.assign(hg.inst.size(), 0.0);
  g->br2_c.assign(hg.inst.size(), 0.0);
  g->gap_ok.assign(hg.inst.size(), 0);
  g->gap_prev.assign(hg.inst.size(), std::nan(""));
  g->gap_grow.assign(hg.inst.size(), 0);
  if ((rc = g->gap_need.alloc(hg.inst.size()))) return rc;
  for (int p = 0; p < 2; ++p) {
    std::vector<WarmSeg> segs;
    std::vector<int2> blks;
    std::vector<int64_t> rb;
    std::vector<float> fi, fh;
    int64_t row = 0;
    int32_t hand_base = 0;
    for (auto& b : hg.inst) {
      for (size_t k = 0; k < b.sf.inf[p].size(); ++k) {
        const Infoset& I = b.sf.inf[p][k];
        if (I.nact > kWarmActions) g->warm_ok = false;
        WarmSeg S{};
        S.row_base = row;
        S.vec_base = b.vec_off[p];
        S.stride = b.stride[p];
        S.n_hands = b.inst.n[p];
        S.hand_base = hand_base;
        S.first = I.first;
        S.nact = I.nact;
        S.parent = I.parent;
        S.inst = (int32_t)(&b - hg.inst.data());
        for (int h0 = 0; h0 < S.n_hands; h0 += 256) blks.push_back(make_int2((int)segs.size(), h0));
        segs.push_back(S);
        rb.push_back(row);
        row += b.inst.n[p];
      }
      fi.insert(fi.end(), b.sf.inf_feat[p].begin(), b.sf.inf_feat[p].end());
      fh.insert(fh.end(), b.hand_feat[p].begin(), b.hand_feat[p].end());
      hand_base += b.inst.n[p];
    }
    if ((rc = g->wseg[p].upload(segs)) || (rc = g->wblk[p].upload(blks)) || (rc = g->wrow_base[p].upload(rb)) ||
        (rc = g->winf[p].upload(fi)) || (rc = g->whand[p].upload(fh)))
      return rc;
    g->wrows[p] = row;
    g->wn_blk[p] = (int)blks.size();
    if ((rc = g->lam_inst[p].upload(g->lam_off[p]))) return rc;
  }
  std::vector<double> pots;
  for (auto& b : hg.inst) pots.push_back(2.0 * b.inst.contrib);
  if ((rc = g->pot_inst.upload(pots))) return rc;
  return PMX_OK;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static MvParams mv_params(Game* g, int d, double scale) {
  MvParams P;
  P.scale = scale;
  P.dir = d;
  P.active = nullptr;
  P.nblk = g->dd[d].nblk;
  return P;
}

static McParams mc_params(Game* g, int d, const MvParams& like, int c) {
  DevMc& E = g->dm[d];
  McParams P;
  P.items = g->dd[d].items.p;
  // the solver's launches (active flags set) take the lists without retired
  // instances; the FP64 gap takes the full lists
  const bool solver = like.active != nullptr;
  P.chunks = (const int4*)(solver ? E.chunks_act[c].p : E.chunks[c].p);
  P.ctx = E.ctx.p;
  P.q = (const uint4*)E.q.p;
  P.pos = (const uint2*)E.pos.p;
  P.meta = E.meta.p;
  P.lam = g->lam.p;
  P.lamf = g->lamf.p;
  P.active = like.active;
  P.part = g->dd[d].part.p;
  P.scale = like.scale;
  P.nchunk = like.nblk > 0 ? (solver ? E.count_act[c] : E.count[c]) : 0;
  return P;
}

template <int BLOCK, int KH, typename IO>
static constexpr size_t mc_lds() {
  constexpr int KE = BLOCK == 512 ? 4 * KH : 4 * KH + 4;
  constexpr int SK = KE + (KE % 8 == 0 ? 4 : 0);
  return sizeof(double) * (2 * kMcSegMax + 3 * (BLOCK / 64)) + 2 * sizeof(IO) * (size_t)BLOCK * SK;
}

// LDS bytes of the largest class a launch of the chunk-aligned kernel needs.
template <typename IO>
static size_t mc_lds_max(Game* g) {
  size_t m = 0;
  for (int c = 0; c < kMcClasses; ++c) {
    if (!g->dm[0].count[c] && !g->dm[1].count[c]) continue;
    size_t b = 0;
    if (g->dm[0].block == 512)
      b = c == 0 ? mc_lds<512, 1, IO>() : c == 1 ? mc_lds<512, 2, IO>() : mc_lds<512, 3, IO>();
    else
      b = c == 0 ? mc_lds<256, 1, IO>() : c == 1 ? mc_lds<256, 2, IO>() : c == 2 ? mc_lds<256, 3, IO>()
        : c == 3 ? mc_lds<256, 4, IO>() : mc_lds<256, 5, IO>();
    m = std::max(m, b);
  }
  return m;
}

template <int BLOCK, int KH, typename IO>
static void launch_mc_class(const McParams& A, const IO* in0, IO* out0, const McParams& B, const IO* in1,
                            IO* out1, hipStream_t s, double* tick) {
  const size_t lds = mc_lds<BLOCK, KH, IO>();
  hipLaunchKernelGGL((k_mvc<BLOCK, KH, IO>), dim3(A.nchunk + B.nchunk), dim3(BLOCK), lds, s, A, in0, out0, B,
                     in1, out1, tick);
}

// Kernels 2 and 3: one launch per hands-per-thread class present.
// Independent launches (the hands-per-thread classes of one product: they
// write disjoint output rows) run concurrently: largest first, each onto the
// stream with the least work so far, among the caller's stream and up to
// Game::kSide side streams forked from it (an event recorded on s, waited
// for by each side stream) and joined back into s before the call returns.
// Under stream capture the fork and join become graph edges.  A class's
// tail then overlaps the others' work, and workgroups of different classes
// share a CU's LDS.  `launch(i, stream, first)` enqueues launch i; `first`
// marks the one launch that carries the iteration tick.
template <typename F>
static int fork_launches(Game* g, hipStream_t s, int n, const int64_t* work_in, int64_t workgroups, F&& launch) {
  int order[32];
  int64_t work[32];
  if (n > 32) return fail(PMX_EINVAL, "too many concurrent launches");
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    work[i] = work_in[i];
  }
  for (int i = 1; i < n; ++i)
    for (int j = i; j > 0 && work[j] > work[j - 1]; --j) {
      std::swap(work[j], work[j - 1]);
      std::swap(order[j], order[j - 1]);
    }
  // a fork and join cost about ten microseconds: small products (a single
  // river endgame's) stay on the caller's stream
  const int ns = (g->fork_ok && workgroups >= kForkMinWorkgroups) ? std::min(n, kForkStreams) : 1;
  int on[32];
  int64_t load[kForkStreams] = {};
  for (int i = 0; i < n; ++i) {
    int best = 0;
    for (int k = 1; k < ns; ++k)
      if (load[k] < load[best]) best = k;
    on[i] = best;
    load[best] += work[i];
  }
  if (ns > 1) {
    HIP_TRY(hipEventRecord(g->fork_ev, s));
    for (int k = 1; k < ns; ++k) HIP_TRY(hipStreamWaitEvent(g->side[k - 1], g->fork_ev, 0));
  }
  for (int i = 0; i < n; ++i) {
    const int rc = launch(order[i], on[i] > 0 ? g->side[on[i] - 1] : s, i == 0);
    if (rc) return rc;
  }
  for (int k = 1; k < ns; ++k) {
    HIP_TRY(hipEventRecord(g->join_ev[k - 1], g->side[k - 1]));
    HIP_TRY(hipStreamWaitEvent(s, g->join_ev[k - 1], 0));
  }
  return PMX_OK;
}

template <typename IO>
static int launch_mc(Game* g, const MvParams& P0, const IO* in0, IO* out0, const MvParams& P1, const IO* in1,
                     IO* out1, hipStream_t s, double* tick) {
  const int block = g->dm[0].block;
  if (block == 0 || g->dm[1].block != block) return fail(PMX_ESTATE, "matvec layout not built");
  int cls[kMcClasses], n = 0;
  int64_t work[kMcClasses], wgs = 0;
  for (int c = 0; c < kMcClasses; ++c) {
    const McParams A = mc_params(g, P0.dir, P0, c), B = mc_params(g, P1.dir, P1, c);
    if (A.nchunk + B.nchunk == 0) continue;
    if (block == 512 && c > 2) return fail(PMX_EINVAL, "no 512-thread matvec class for this hand count");
    work[n] = (int64_t)(A.nchunk + B.nchunk) * (c + 1);
    wgs += A.nchunk + B.nchunk;
    cls[n++] = c;
  }
  int rc = fork_launches(g, s, n, work, wgs, [&](int i, hipStream_t st, bool first) {
    const int c = cls[i];
    const McParams A = mc_params(g, P0.dir, P0, c), B = mc_params(g, P1.dir, P1, c);
    double* tk = first ? tick : nullptr;
    if (block == 512) {
      switch (c) {
        case 0: launch_mc_class<512, 1, IO>(A, in0, out0, B, in1, out1, st, tk); break;
        case 1: launch_mc_class<512, 2, IO>(A, in0, out0, B, in1, out1, st, tk); break;
        default: launch_mc_class<512, 3, IO>(A, in0, out0, B, in1, out1, st, tk); break;
      }
    } else {
      switch (c) {
        case 0: launch_mc_class<256, 1, IO>(A, in0, out0, B, in1, out1, st, tk); break;
        case 1: launch_mc_class<256, 2, IO>(A, in0, out0, B, in1, out1, st, tk); break;
        case 2: launch_mc_class<256, 3, IO>(A, in0, out0, B, in1, out1, st, tk); break;
        case 3: launch_mc_class<256, 4, IO>(A, in0, out0, B, in1, out1, st, tk); break;
        default: launch_mc_class<256, 5, IO>(A, in0, out0, B, in1, out1, st, tk); break;
      }
    }
    return PMX_OK;
  });
  if (rc) return rc;
  // every instance retired from the lists: the iteration still counts
  if (n == 0 && tick) hipLaunchKernelGGL(k_add1, dim3(1), dim3(1), 0, s, tick);
  // rows cut into parts: sum the partial rows (after the join into s)
  const int nr0 = P0.nblk > 0 ? g->dd[P0.dir].nred : 0, nr1 = P1.nblk > 0 ? g->dd[P1.dir].nred : 0;
  if (n > 0 && nr0 + nr1 > 0)
    hipLaunchKernelGGL((k_mv_reduce<IO>), dim3(nr0 + nr1), dim3(256), 0, s, g->dd[P0.dir].red.p, nr0,
                       (const IO*)g->dd[P0.dir].part.p, out0, g->dd[P1.dir].red.p,
                       (const IO*)g->dd[P1.dir].part.p, out1, P0.active);
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

static GParams grp_params(Game* g, int d, const MvParams& like, int kind, int c) {
  DevGrp& E = g->dg[d];
  GParams P;
  const bool solver = like.active != nullptr;
  P.groups = E.groups.p;
  P.chunks = (const int4*)(solver ? E.chunks_act[kind][c].p : E.chunks[kind][c].p);
  P.ctx = E.ctx.p;
  P.q = (const uint4*)E.q.p;
  P.rk = E.rk.p;
  P.src = E.src.p;
  P.meta = E.meta.p;
  P.lamf = g->lamf.p;
  P.active = like.active;
  P.scale = like.scale;
  P.nchunk = like.nblk > 0 ? (solver ? E.count_act[kind][c] : E.count[kind][c]) : 0;
  return P;
}

template <int KH, bool CARRY, int NC, int NS = NC>
static void launch_grp_class(const GParams& A, const float* in0, float* out0, const GParams& B, const float* in1,
                             float* out1, hipStream_t s, double* tick) {
  constexpr int KE = kGrpKE[KH - 1];
  const size_t lds = sizeof(double) * (NC * kMcSegMax + 5 * (kGrpBlock / 64)) +
                     (size_t)GSlot<NS>::SB * kGrpBlock * KE + (NS < NC ? (size_t)grp_stage_bytes<KH>() : 0);
  hipLaunchKernelGGL((k_mvg<KH, KE, CARRY, NC, NS>), dim3(A.nchunk + B.nchunk), dim3(kGrpBlock), lds, s, A, in0,
                     out0, B, in1, out1, tick);
}

// Weights for spreading a product's class launches over the streams (longest
// first, each to the least loaded stream).  A single-direction product (the
// solver's) weighs a class by per-workgroup durations measured on a batch of
// river endgames, by kind and class, plus a floor for the latency of a launch
// whose workgroups fit one round (the smallest and the largest hand classes);
// a pair launch, whose classes cover both directions, balances by scan
// entries, which measured better there.
static constexpr int64_t kGrpWgNs[GrpDir::kKinds][kGrpClasses] = {
    {300, 35, 57, 51, 127}, {300, 35, 57, 51, 127}, {200, 22, 31, 25, 59}, {300, 27, 44, 39, 98}};

static int64_t grp_launch_weight(int kind, int c, int nchunk, bool pair) {
  if (pair) return (int64_t)nchunk * kGrpKE[c] * (kind == 2 ? 2 : kind == 3 ? 3 : 4);
  return (int64_t)nchunk * kGrpWgNs[kind][c] + (kind == 2 ? 5000 : 7000) * (c == kGrpClasses - 1 ? 4 : 1);
}

// Kernel 4 (FP32 only): one launch per hands-per-thread class present, the
// classes concurrently (fork_launches).
static int launch_grp(Game* g, const MvParams& P0, const float* in0, float* out0, const MvParams& P1,
                      const float* in1, float* out1, hipStream_t s, double* tick) {
  if (!g->dg[0].built || !g->dg[1].built) return fail(PMX_ESTATE, "grouped matvec layout not built");
  int cls[GrpDir::kKinds * kGrpClasses], n = 0;
  int64_t work[GrpDir::kKinds * kGrpClasses], wgs = 0;
  for (int kind = 0; kind < GrpDir::kKinds; ++kind)
    for (int c = 0; c < kGrpClasses; ++c) {
      const GParams A = grp_params(g, P0.dir, P0, kind, c), B = grp_params(g, P1.dir, P1, kind, c);
      if (A.nchunk + B.nchunk == 0) continue;
      work[n] = grp_launch_weight(kind, c, A.nchunk + B.nchunk, A.nchunk > 0 && B.nchunk > 0);
      wgs += A.nchunk + B.nchunk;
      cls[n++] = kind * kGrpClasses + c;
    }
  int rc = fork_launches(g, s, n, work, wgs, [&](int i, hipStream_t st, bool first) {
    const int kind = cls[i] / kGrpClasses, c = cls[i] % kGrpClasses;
    const GParams A = grp_params(g, P0.dir, P0, kind, c), B = grp_params(g, P1.dir, P1, kind, c);
    double* tk = first ? tick : nullptr;
    if (kind == 0) {
      switch (c) {
        case 0: launch_grp_class<1, false, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        case 1: launch_grp_class<2, false, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        case 2: launch_grp_class<3, false, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        case 3: launch_grp_class<4, false, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        default: launch_grp_class<5, false, 4>(A, in0, out0, B, in1, out1, st, tk); break;
      }
    } else if (kind == 1) {
      switch (c) {
        case 0: launch_grp_class<1, true, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        case 1: launch_grp_class<2, true, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        case 2: launch_grp_class<3, true, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        case 3: launch_grp_class<4, true, 4>(A, in0, out0, B, in1, out1, st, tk); break;
        default: launch_grp_class<5, true, 4>(A, in0, out0, B, in1, out1, st, tk); break;
      }
    } else if (kind == 2) {
      switch (c) {
        case 0: launch_grp_class<1, false, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        case 1: launch_grp_class<2, false, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        case 2: launch_grp_class<3, false, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        case 3: launch_grp_class<4, false, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        default: launch_grp_class<5, false, 2>(A, in0, out0, B, in1, out1, st, tk); break;
      }
    } else {
      switch (c) {
        case 0: launch_grp_class<1, false, 4, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        case 1: launch_grp_class<2, false, 4, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        case 2: launch_grp_class<3, false, 4, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        case 3: launch_grp_class<4, false, 4, 2>(A, in0, out0, B, in1, out1, st, tk); break;
        default: launch_grp_class<5, false, 4, 2>(A, in0, out0, B, in1, out1, st, tk); break;
      }
    }
    return PMX_OK;
  });
  if (rc) return rc;
  // every instance retired from the lists: the iteration still counts
  if (n == 0 && tick) hipLaunchKernelGGL(k_add1, dim3(1), dim3(1), 0, s, tick);
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

template <typename IO>
static int launch_mv(Game* g, MvParams P0, const IO* in0, IO* out0, MvParams P1, const IO* in1,
                     IO* out1, hipStream_t s, double* tick = nullptr) {
  const int nb = P0.nblk + P1.nblk;
  if (nb == 0) return PMX_OK;
  if constexpr (sizeof(IO) == 4) {
    if (g->hg.mv_kernel == 4) return launch_grp(g, P0, in0, out0, P1, in1, out1, s, tick);
  }
  if (g->hg.mv_kernel < 2 || g->hg.mv_kernel > 4) return fail(PMX_ESTATE, "no matvec schedule set");
  if (mc_lds_max<IO>(g) > (size_t)g->max_lds)
    return fail(PMX_EINVAL, "matvec workgroup needs more LDS than this device gives a workgroup");
  return launch_mc<IO>(g, P0, in0, out0, P1, in1, out1, s, tick);
}

static MvParams empty_params(const MvParams& like) {
  MvParams P = like;
  P.nblk = 0;
  return P;
}

static TpParams tp_params(Game* g, int p, const int2* blocks) {
  DevTp& E = g->dt[p];
  TpParams P;
  P.inf_parent = E.inf_parent.p;
  P.inf_first = E.inf_first.p;
  P.inf_nact = E.inf_nact.p;
  P.order = E.order.p;
  P.tasks = E.tasks.p;
  P.pulls = E.pulls.p;
  P.blocks = blocks;
  P.stage_stride = E.stage_stride;
  P.active = nullptr;
  P.dcfr = 0;
  P.gamma = 1;
  P.alpha = 1.f;
  P.beta = 1.f;
  return P;
}


static RmParams rm_params(Game* g, int p, int depth, int first_block) {
  DevRm& E = g->drm[p];
  RmParams P;
  P.blocks = E.blocks.p + first_block;
  P.rows = E.rows.p;
  P.infs = E.infs.p;
  P.pulls = E.pulls.p;
  P.ext_seq = E.ext_seq.p;
  P.ext_slot = E.ext_slot.p;
  P.grp = E.grp.p;
  P.active = g->active.p;
  P.stage_stride = E.stage_stride;
  P.max_rows = E.max_rows[depth];
  P.max_ext = E.max_ext[depth];
  P.dcfr = g->dcfr;
  P.gamma = g->gamma;
  P.alpha = (float)g->alpha;
  P.beta = (float)g->beta;
  return P;
}

// One player's regret update: bottom-up passes of the deep pieces (deepest
// first), the pieces without external parents, then the top-down passes of
// the deep pieces (shallowest first).
static int rm_update(Game* g, int p, hipStream_t s) {
  DevRm& E = g->drm[p];
  float* gr = g->grad[p].p;
  const double* td = g->tdev.p;
  const int D = (int)E.max_rows.size();
  auto launch_range = [&](int mode, int d, int b0, int b1, hipStream_t s) {
    const int nb = b1 - b0;
    if (nb <= 0) return;
    const RmParams P = rm_params(g, p, d, b0);
    // few workgroups: the walk's latency is the cost, four lanes per hand
    // (k_rmq); many: the bytes are, one lane per hand (k_rmp)
    // pieces beyond a wavefront's rows (whole treeplexes) only fit the
    // four-lane form
    const bool whole = P.max_rows > kTaskRowsMax;
    const bool quad = whole || nb <= g->hg.rm_quad_max;
    const size_t lds = sizeof(float) * (quad ? RQH : 64) * (size_t)(kRmRowLocal + 2 * P.max_rows);
    auto go = [&](auto kern) {
      hipLaunchKernelGGL(kern, dim3(quad ? 4 * nb : nb), dim3(64 * RMW), lds, s, P, gr, g->R[p].p, g->x[p].p,
                         g->xs[p].p, E.stage.p, td);
    };
    if (whole) {
      // one piece per treeplex: the fused pass only
      if (P.dcfr) go(k_rmq<0, true, kTaskRowsWhole>);
      else go(k_rmq<0, false, kTaskRowsWhole>);
    } else if (quad) {
      if (P.dcfr) {
        if (mode == 0) go(k_rmq<0, true>);
        else if (mode == 1) go(k_rmq<1, true>);
        else go(k_rmq<2, true>);
      } else {
        if (mode == 0) go(k_rmq<0, false>);
        else if (mode == 1) go(k_rmq<1, false>);
        else go(k_rmq<2, false>);
      }
    } else if (P.dcfr) {
      if (mode == 0) go(k_rmp<0, true>);
      else if (mode == 1) go(k_rmp<1, true>);
      else go(k_rmp<2, true>);
    } else {
      if (mode == 0) go(k_rmp<0, false>);
      else if (mode == 1) go(k_rmp<1, false>);
      else go(k_rmp<2, false>);
    }
  };
  auto launch = [&](int mode, int d) { launch_range(mode, d, E.blk_off[d], E.blk_off[d + 1], s); };
  if (D == 0) return PMX_OK;
  // the pieces of depth 0 without pulls run on a side stream beside the
  // chain deep bottom-up -> depth 0 with pulls -> deep top-down (the
  // pieces of one pass are independent; only the chain is ordered)
  const bool side = g->fork_ok && D > 1 && E.blk_pull0 > E.blk_off[0] && E.blk_off[1] > E.blk_pull0 &&
                    E.blk_off[D] - E.blk_off[0] >= kForkMinWorkgroups;
  if (side) {
    HIP_TRY(hipEventRecord(g->fork_ev, s));
    HIP_TRY(hipStreamWaitEvent(g->side[0], g->fork_ev, 0));
    launch_range(0, 0, E.blk_off[0], E.blk_pull0, g->side[0]);
  }
  for (int d = D - 1; d >= 1; --d) launch(1, d);
  if (side) launch_range(0, 0, E.blk_pull0, E.blk_off[1], s);
  else launch(0, 0);
  for (int d = 1; d < D; ++d) launch(2, d);
  if (side) {
    HIP_TRY(hipEventRecord(g->join_ev[0], g->side[0]));
    HIP_TRY(hipStreamWaitEvent(s, g->join_ev[0], 0));
  }
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

static TpParams tp_params_for(Game* g, int p, const int2* blocks, const int32_t* need) {
  TpParams P = tp_params(g, p, blocks);
  P.active = need;
  return P;
}

// Best-response values per hand and their per-instance sums; need (device,
// NULL: all) limits the work to the instances flagged.
// Best-response values of player p from the FP64 gradient gvec; stage_d
// (the deep pieces' root values) and hv (per-hand values) are scratch, and
// the per-instance sums go to br_out[0 .. instances).
static int br_values(Game* g, int p, double* gvec, double* stage_d, double* hv, double* br_out, hipStream_t s,
                     const int32_t* need) {
  DevTp& E = g->dt[p];
  if (p == 0) {
    if (E.n_single)
      hipLaunchKernelGGL((k_br<0, true>), dim3(E.n_single), dim3(TPB), 0, s,
                         tp_params_for(g, p, E.b_single.p, need), gvec, stage_d, hv);
    if (E.n_deep)
      hipLaunchKernelGGL((k_br<1, true>), dim3(E.n_deep), dim3(TPB), 0, s,
                         tp_params_for(g, p, E.b_deep.p, need), gvec, stage_d, hv);
    if (E.n_top)
      hipLaunchKernelGGL((k_br<2, true>), dim3(E.n_top), dim3(TPB), 0, s,
                         tp_params_for(g, p, E.b_top.p, need), gvec, stage_d, hv);
  } else {
    if (E.n_single)
      hipLaunchKernelGGL((k_br<0, false>), dim3(E.n_single), dim3(TPB), 0, s,
                         tp_params_for(g, p, E.b_single.p, need), gvec, stage_d, hv);
    if (E.n_deep)
      hipLaunchKernelGGL((k_br<1, false>), dim3(E.n_deep), dim3(TPB), 0, s,
                         tp_params_for(g, p, E.b_deep.p, need), gvec, stage_d, hv);
    if (E.n_top)
      hipLaunchKernelGGL((k_br<2, false>), dim3(E.n_top), dim3(TPB), 0, s,
                         tp_params_for(g, p, E.b_top.p, need), gvec, stage_d, hv);
  }
  const int ni = (int)g->hg.inst.size();
  hipLaunchKernelGGL(k_sum_instances, dim3(ni), dim3(256), 0, s, hv, g->inst_hand_off[p].p, br_out);
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

static void fill_f32(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_f32, dim3(blocks), dim3(256), 0, s, p, n, v);
}
static void fill_f64(double* p, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return;
  int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(256), 0, s, p, n, v);
}

static int uniform_plan(Game* g, int p, hipStream_t s) {
  DevTp& E = g->dt[p];
  // the top task must run before the deep tasks (parents first)
  if (E.n_single)
    hipLaunchKernelGGL(k_uniform, dim3(E.n_single), dim3(TPB), 0, s, tp_params(g, p, E.b_single.p),
                       g->x[p].p);
  if (E.n_top)
    hipLaunchKernelGGL(k_uniform, dim3(E.n_top), dim3(TPB), 0, s, tp_params(g, p, E.b_top.p),
                       g->x[p].p);
  if (E.n_deep)
    hipLaunchKernelGGL(k_uniform, dim3(E.n_deep), dim3(TPB), 0, s, tp_params(g, p, E.b_deep.p),
                       g->x[p].p);
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* pmx_last_error(void) { return g_err.c_str(); }

static int static_scratch(int dev, double** out);

static int create_common(const GameDesc* descs, int32_t n, bool device, Game** out) {
  if (!out) return fail(PMX_EINVAL, "out is NULL");
  if (!descs || n < 1) return fail(PMX_EINVAL, "need at least one descriptor");
  std::unique_ptr<Game> g;
  try {
    g.reset(new Game());
    std::string msg;
    int rc = build_game(descs, n, g->hg, msg);
    if (rc) return fail(rc, msg);
  } catch (const std::bad_alloc&) {
    return fail(PMX_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(PMX_EINVAL, e.what());
  }
  if (device) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    g->device_id = dev;
    g->device = true;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
      g->max_lds = lds;
    int rc = upload_game(g.get());
    if (rc) return rc;
    if ((rc = ensure_fork(g.get()))) return rc;
    // set-up of the allocation-free gap on this device (once per device)
    double* scr = nullptr;
    if ((rc = static_scratch(dev, &scr))) return rc;
    hipStream_t s = nullptr;
    if ((rc = solver_reset(g.get(), s))) return rc;
    HIP_TRY(hipStreamSynchronize(s));
  }
  *out = g.release();
  g_err.clear();
  return PMX_OK;
}

int game_create(const GameDesc* desc, Game** out) { return create_common(desc, 1, true, out); }

int game_create_batch(const GameDesc* descs, int32_t n, Game** out) {
  return create_common(descs, n, true, out);
}

int game_create_host(const GameDesc* descs, int32_t n, Game** out) {
  return create_common(descs, n, false, out);
}

void game_destroy(Game* g) {
  if (!g) return;
  if (g->device) {
    (void)hipSetDevice(g->device_id);
    (void)hipDeviceSynchronize();
  }
  delete g;
}

int game_num_instances(const Game* g, int32_t* n) {
  if (!g || !n) return fail(PMX_EINVAL, "null argument");
  *n = (int32_t)g->hg.inst.size();
  return PMX_OK;
}

int game_layout(const Game* g, int32_t instance, int32_t player, Layout* out) {
  if (!g || !out) return fail(PMX_EINVAL, "null argument");
  if (instance < 0 || instance >= (int)g->hg.inst.size()) return fail(PMX_EINVAL, "bad instance");
  if (player < 0 || player > 1) return fail(PMX_EINVAL, "bad player");
  const Built& b = g->hg.inst[instance];
  Layout L;
  L.n_seq = b.sf.n_seq[player];
  L.n_hands = b.inst.n[player];
  L.stride = b.stride[player];
  L.vec_offset = b.vec_off[player];
  L.vec_elems = g->hg.elems[player];
  L.n_infosets = (int32_t)b.inf_parent[player].size();
  L.infoset_parent = b.inf_parent[player].data();
  L.infoset_first = b.inf_first[player].data();
  L.infoset_nact = b.inf_nact[player].data();
  L.infoset_board = b.inf_board[player].data();
  *out = L;
  return PMX_OK;
}

int game_terminals(const Game* g, int32_t instance, Terminals* out) {
  if (!g || !out) return fail(PMX_EINVAL, "null argument");
  if (instance < 0 || instance >= (int)g->hg.inst.size()) return fail(PMX_EINVAL, "bad instance");
  const Built& b = g->hg.inst[instance];
  Terminals T;
  T.n_terminals = (int32_t)b.t_seq1.size();
  T.seq1 = b.t_seq1.data();
  T.seq2 = b.t_seq2.data();
  T.kind = b.t_kind.data();
  T.board = b.t_board.data();
  T.runout = b.t_runout.data();
  T.c1 = b.t_c1.data();
  T.c2 = b.t_c2.data();
  *out = T;
  return PMX_OK;
}

int game_hand_meta(const Game* g, int32_t instance, int32_t ctx, int32_t player, HandMeta* out) {
  if (!g || !out) return fail(PMX_EINVAL, "null argument");
  if (instance < 0 || instance >= (int)g->hg.inst.size()) return fail(PMX_EINVAL, "bad instance");
  if (player < 0 || player > 1) return fail(PMX_EINVAL, "bad player");
  const Built& b = g->hg.inst[instance];
  if (ctx < 0 || ctx >= b.n_ctx) return fail(PMX_EINVAL, "bad board context");
  // exported views are rebuilt lazily into per-context vectors owned by the game
  static_assert(sizeof(QueryRec) == 8 * sizeof(int32_t), "QueryRec layout");
  const CtxMeta& m = b.ctx[player][ctx];
  HandMeta H;
  H.n_hands = b.inst.n[player];
  H.n_live = m.n_live;
  H.rank = m.rank.data();
  H.lt = &m.q.data()->lt;
  H.le = &m.q.data()->le;
  H.self_ = &m.q.data()->self;
  H.beta = b.beta;
  *out = H;
  return PMX_OK;
}

int game_tune(Game* g, int32_t kernel, int32_t rows_per_chunk) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (kernel < 2 || kernel > 4) return fail(PMX_EINVAL, "kernel must be in [2, 4]");
  if (rows_per_chunk < 1 || rows_per_chunk > 64) return fail(PMX_EINVAL, "rows_per_chunk must be in [1, 64]");
  HIP_TRY(hipDeviceSynchronize());
  if (g->graph_exec) {
    (void)hipGraphExecDestroy(g->graph_exec);
    g->graph_exec = nullptr;
  }
  if (g->graph) {
    (void)hipGraphDestroy(g->graph);
    g->graph = nullptr;
  }
  g->hg.mv_kernel = kernel;
  if (kernel == 4) {
    g->hg.groups_per_chunk = rows_per_chunk;   // the FP64 products keep their chunk-aligned layout
  } else {
    g->hg.rows_per_block = rows_per_chunk;
    g->hg.mc_block = kernel == 3 ? 512 : 256;
  }
  for (int d = 0; d < 2; ++d) {
    build_matvec_plan(g->hg, d, g->hg.rows_per_block);
    if ((rc = upload_dir(g, d))) return rc;
  }
  return PMX_OK;
}

int solver_set_gap_guard(Game* g, int32_t k) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (k < 0) return fail(PMX_EINVAL, "k must be >= 0 (0 disables the guard)");
  g->gap_guard = k;
  g->gap_grow.assign(g->gap_grow.size(), 0);
  return PMX_OK;
}

int solver_set_rm_quad(Game* g, int32_t max_records) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (max_records < 0) return fail(PMX_EINVAL, "max_records must be >= 0");
  HIP_TRY(hipDeviceSynchronize());
  if (g->graph_exec) {
    (void)hipGraphExecDestroy(g->graph_exec);
    g->graph_exec = nullptr;
  }
  if (g->graph) {
    (void)hipGraphDestroy(g->graph);
    g->graph = nullptr;
  }
  g->hg.rm_quad_max = max_records;
  return PMX_OK;
}

int solver_set_task_rows(Game* g, int32_t rows) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (rows < 1 || rows > kTaskRowsMax)
    return fail(PMX_EINVAL, "rows must be in [1, " + std::to_string(kTaskRowsMax) + "]");
  const bool was_whole = g->hg.rm_whole;
  HIP_TRY(hipDeviceSynchronize());
  if (g->graph_exec) {
    (void)hipGraphExecDestroy(g->graph_exec);
    g->graph_exec = nullptr;
  }
  if (g->graph) {
    (void)hipGraphDestroy(g->graph);
    g->graph = nullptr;
  }
  // an explicit cut replaces a whole-treeplex plan
  g->hg.rm_whole = false;
  for (int p = 0; p < 2; ++p) {
    std::string m;
    if ((rc = build_rm_plan(g->hg, p, rows, m))) {
      // keep a consistent plan: rebuild the previous one
      std::string m2;
      g->hg.rm_whole = was_whole;
      for (int q = 0; q < 2; ++q) (void)build_rm_plan(g->hg, q, was_whole ? kTaskRowsWhole : g->hg.task_rows, m2);
      for (int q = 0; q < 2; ++q) (void)upload_rm(g, q);
      return fail(rc, m);
    }
  }
  g->hg.task_rows = rows;
  for (int p = 0; p < 2; ++p)
    if ((rc = upload_rm(g, p))) return rc;
  return PMX_OK;
}

int game_get_tuning(const Game* g, int32_t* kernel, int32_t* rows_per_chunk) {
  if (!g || !kernel || !rows_per_chunk) return fail(PMX_EINVAL, "null argument");
  *kernel = g->hg.mv_kernel;
  *rows_per_chunk = g->hg.mv_kernel == 4 ? g->hg.groups_per_chunk : g->hg.rows_per_block;
  return PMX_OK;
}

int matvec_A(Game* g, const float* y, float* out, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!y || !out) return fail(PMX_EINVAL, "null vector");
  MvParams P = mv_params(g, 0, 1.0);
  return launch_mv<float>(g, P, y, out, empty_params(P), nullptr, nullptr, (hipStream_t)stream);
}

int matvec_AT(Game* g, const float* x, float* out, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!x || !out) return fail(PMX_EINVAL, "null vector");
  MvParams P = mv_params(g, 1, 1.0);
  return launch_mv<float>(g, P, x, out, empty_params(P), nullptr, nullptr, (hipStream_t)stream);
}

int matvec_A_f64(Game* g, const double* y, double* out, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!y || !out) return fail(PMX_EINVAL, "null vector");
  MvParams P = mv_params(g, 0, 1.0);
  return launch_mv<double>(g, P, y, out, empty_params(P), nullptr, nullptr, (hipStream_t)stream);
}

int matvec_AT_f64(Game* g, const double* x, double* out, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!x || !out) return fail(PMX_EINVAL, "null vector");
  MvParams P = mv_params(g, 1, 1.0);
  return launch_mv<double>(g, P, x, out, empty_params(P), nullptr, nullptr, (hipStream_t)stream);
}

int matvec_pair(Game* g, const float* y, const float* x, float* Ay, float* ATx, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!y || !x || !Ay || !ATx) return fail(PMX_EINVAL, "null vector");
  return launch_mv<float>(g, mv_params(g, 0, 1.0), y, Ay, mv_params(g, 1, 1.0), x, ATx,
                          (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Technique B's explicit factors (a cross-check of the structured operator)
// ---------------------------------------------------------------------------
int tb_build(Game* g, TbSizes* sizes) {
  if (!g) return fail(PMX_EINVAL, "null game");
  TbHost T;
  std::string msg;
  int rc = build_tb_factors(g->hg, T, msg);
  if (rc) return fail(rc, msg);
  if (g->device) {
    HIP_TRY(hipSetDevice(g->device_id));
    auto& D = g->tb;
    const TbCsr* m[6] = {&T.ahat, &T.ahat_t, &T.u, &T.u_t, &T.v, &T.v_t};
    for (int i = 0; i < 6; ++i) {
      if ((rc = D.ptr[i].upload(m[i]->ptr)) || (rc = D.idx[i].upload(m[i]->idx)) ||
          (rc = D.val[i].upload(m[i]->val)))
        return rc;
      D.rows[i] = m[i]->rows;
    }
    D.m = T.m_dim_pp;
    if ((rc = D.par.upload(T.par)) || (rc = D.chi.upload(T.chi)) || (rc = D.cpar.upload(T.cpar)) ||
        (rc = D.cchi.upload(T.cchi)) || (rc = D.tvec.alloc(std::max<int64_t>(D.m, 1))))
      return rc;
    for (int i = 0; i < 2; ++i)
      if ((rc = D.valbuf[i].alloc(std::max<int64_t>(D.m, 1))) || (rc = D.coefbuf[i].alloc(std::max<int64_t>(D.m, 1))) ||
          (rc = D.ptrbuf[i].alloc(std::max<int64_t>(D.m, 1))))
        return rc;
    int r = 0;
    while ((1 << r) < T.depth) ++r;
    D.rounds = r;
    D.built = true;
  }
  // M as CSR from its chains: the unit diagonal and each row's parent entry
  {
    TbCsr& Mc = g->tb_m;
    Mc.rows = Mc.cols = T.m_dim_pp;
    Mc.ptr.assign(T.m_dim_pp + 1, 0);
    Mc.idx.clear();
    Mc.val.clear();
    for (int64_t k = 0; k < T.m_dim_pp; ++k) {
      if (T.par[k] >= 0) {
        Mc.idx.push_back(T.par[k]);
        Mc.val.push_back(-T.cpar[k]);
      }
      Mc.idx.push_back((int32_t)k);
      Mc.val.push_back(1.0);
      Mc.ptr[k + 1] = (int64_t)Mc.idx.size();
    }
  }
  if (sizes) {
    TbSizes z;
    z.nnz_A = T.nnz_A;
    z.nnz_ahat = T.nnz[0];
    z.nnz_u = T.nnz[1];
    z.nnz_m = T.nnz[2];
    z.nnz_v = T.nnz[3];
    z.nnz_u_pp = T.nnz_pp[1];
    z.nnz_m_pp = T.nnz_pp[2];
    z.nnz_v_pp = T.nnz_pp[3];
    z.m_dim = T.m_dim;
    z.m_dim_pp = T.m_dim_pp;
    z.chain_depth = T.depth;
    *sizes = z;
  }
  g->tb_host.reset(new TbHost(std::move(T)));
  return PMX_OK;
}

int tb_matrix(const Game* g, int32_t which, TbMatrix* out) {
  if (!g || !out) return fail(PMX_EINVAL, "null argument");
  if (!g->tb_host) return fail(PMX_ESTATE, "tb_build has not been called on this game");
  const TbCsr* m = which == 0 ? &g->tb_host->ahat : which == 1 ? &g->tb_host->u : which == 2 ? &g->tb_m
                 : which == 3 ? &g->tb_host->v : nullptr;
  if (!m) return fail(PMX_EINVAL, "which must be 0 (Ahat), 1 (U), 2 (M) or 3 (V)");
  TbMatrix M;
  M.rows = m->rows;
  M.cols = m->cols;
  M.nnz = (int64_t)m->idx.size();
  M.ptr = m->ptr.data();
  M.idx = m->idx.data();
  M.val = m->val.data();
  *out = M;
  return PMX_OK;
}

// out = Ahat in + U (M^-1 (V^T in)) for dir 0 (A y); Ahat^T in + V (M^-T (U^T in))
// for dir 1 (A^T x).
static int tb_apply(Game* g, int dir, const double* in, double* out, hipStream_t s) {
  auto& D = g->tb;
  if (!D.built) return fail(PMX_ESTATE, "tb_build has not been called on this game");
  // CSR indices: 0 Ahat, 1 Ahat^T, 2 U, 3 U^T, 4 V, 5 V^T
  const int first = dir == 0 ? 5 : 3;    // V^T in  /  U^T in
  const int direct = dir == 0 ? 0 : 1;   // Ahat in /  Ahat^T in
  const int last = dir == 0 ? 2 : 4;     // U z     /  V w
  auto spmv = [&](int i, const double* x, double* y, int acc) {
    const int64_t rows = D.rows[i];
    if (rows == 0) return;
    hipLaunchKernelGGL(k_csr_spmv, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, s, rows, D.ptr[i].p, D.idx[i].p,
                       D.val[i].p, x, y, acc);
  };
  spmv(first, in, D.valbuf[0].p, 0);
  // the chains: parents for M z = r, children for M^T w = r
  const int32_t* p0 = dir == 0 ? D.par.p : D.chi.p;
  const double* c0 = dir == 0 ? D.cpar.p : D.cchi.p;
  HIP_TRY(hipMemcpyAsync(D.coefbuf[0].p, c0, D.m * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipMemcpyAsync(D.ptrbuf[0].p, p0, D.m * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  int a = 0;
  const unsigned nb = (unsigned)((D.m + 255) / 256);
  for (int r = 0; r < D.rounds && D.m > 0; ++r) {
    hipLaunchKernelGGL(k_chain_round, dim3(nb), dim3(256), 0, s, D.m, D.valbuf[a].p, D.coefbuf[a].p,
                       D.ptrbuf[a].p, D.valbuf[1 - a].p, D.coefbuf[1 - a].p, D.ptrbuf[1 - a].p);
    a = 1 - a;
  }
  spmv(direct, in, out, 0);
  spmv(last, D.valbuf[a].p, out, 1);
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

int matvec_A_tb(Game* g, const double* y, double* out, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!y || !out) return fail(PMX_EINVAL, "null vector");
  return tb_apply(g, 0, y, out, (hipStream_t)stream);
}

int matvec_AT_tb(Game* g, const double* x, double* out, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!x || !out) return fail(PMX_EINVAL, "null vector");
  return tb_apply(g, 1, x, out, (hipStream_t)stream);
}

// The solver's launch lists restricted to the instances marked in `act`: the
// matvec row chunks and regret blocks of the others are left out, so their
// workgroups are not dispatched at all (they would return at once on the
// active flags); the FP64 gap keeps the full lists.  Drops the captured
// solver graph, whose grid sizes change.
static int set_solver_lists(Game* g, const std::vector<char>& act) {
  HIP_TRY(hipDeviceSynchronize());
  if (g->graph_exec) {
    (void)hipGraphExecDestroy(g->graph_exec);
    g->graph_exec = nullptr;
  }
  if (g->graph) {
    (void)hipGraphDestroy(g->graph);
    g->graph = nullptr;
  }
  g->listed = act;
  g->n_listed = 0;
  for (char v : act) g->n_listed += v ? 1 : 0;
  int rc;
  for (int d = 0; d < 2; ++d) {
    if (g->dm[d].block && (rc = upload_mc_active(g, d))) return rc;
    if (g->dg[d].built && (rc = upload_grp_active(g, d))) return rc;
  }
  for (int p = 0; p < 2; ++p)
    if ((rc = upload_rm_blocks(g, p, g->listed))) return rc;
  return PMX_OK;
}

int solver_reset(Game* g, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int p = 0; p < 2; ++p) {
    const int64_t n = g->hg.elems[p];
    fill_f32(g->R[p].p, n, 0.f, s);
    fill_f32(g->x[p].p, n, 0.f, s);
    fill_f64(g->xs[p].p, n, 0.0, s);
    if ((rc = uniform_plan(g, p, s))) return rc;
  }
  hipLaunchKernelGGL(k_set1, dim3(1), dim3(1), 0, s, g->tdev.p, 0.0);
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(256), 0, s, g->active.p, (int)g->hg.inst.size(), 1);
  HIP_TRY(hipGetLastError());
  g->t = 0;
  g->wsum = 0.0;
  g->wsum_i.assign(g->wsum_i.size(), 0.0);
  g->act_h.assign(g->act_h.size(), 1);
  invalidate_gaps(g);
  // every instance is active again: the launch lists must include them all
  if (g->n_listed < (int)g->hg.inst.size()) {
    if ((rc = set_solver_lists(g, std::vector<char>(g->hg.inst.size(), 1)))) return rc;
  }
  return PMX_OK;
}

int solver_set_active(Game* g, const int32_t* active_host, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!active_host) return fail(PMX_EINVAL, "null argument");
  const size_t n = g->hg.inst.size();
  std::vector<int32_t> a(active_host, active_host + n);
  for (auto& v : a) v = v ? 1 : 0;
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(g->active.p, a.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (size_t i = 0; i < n; ++i) g->act_h[i] = (char)a[i];
  // rebuild the launch lists when an active instance is missing from them
  // (required) or the active set has halved since they were built
  int n_act = 0;
  bool missing = false;
  for (size_t i = 0; i < n; ++i) {
    n_act += a[i];
    if (a[i] && !g->listed[i]) missing = true;
  }
  if (missing || 2 * n_act <= g->n_listed) {
    std::vector<char> act(n);
    for (size_t i = 0; i < n; ++i) act[i] = (char)a[i];
    if ((rc = set_solver_lists(g, act))) return rc;
  }
  return PMX_OK;
}

// One alternating RM+ iteration, enqueued on s: g1 = A y_t (its launch also
// advances the device iteration index t, read by the updates as the
// averaging weight, so a captured sequence of iterations replays correctly)
// and Player 1's update, then g2 = -A^T x_{t+1} and Player 2's update.
static int enqueue_iteration(Game* g, hipStream_t s) {
  int rc;
  MvParams PA = mv_params(g, 0, 1.0), PT = mv_params(g, 1, -1.0);
  PA.active = PT.active = g->active.p;
  if ((rc = launch_mv<float>(g, PA, g->x[1].p, g->grad[0].p, empty_params(PA), nullptr, nullptr, s,
                             g->tdev.p)))
    return rc;
  if ((rc = rm_update(g, 0, s))) return rc;
  if ((rc = launch_mv<float>(g, PT, g->x[0].p, g->grad[1].p, empty_params(PT), nullptr, nullptr, s)))
    return rc;
  if ((rc = rm_update(g, 1, s))) return rc;
  return PMX_OK;
}

static constexpr int kGraphIters = 32;

static int capture_graph(Game* g) {
  if (g->graph_exec) return PMX_OK;
  if (!g->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
  HIP_TRY(hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeRelaxed));
  int rc = PMX_OK;
  for (int i = 0; i < kGraphIters && rc == PMX_OK; ++i) rc = enqueue_iteration(g, g->cap_stream);
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(g->cap_stream, &graph);
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  if (e != hipSuccess) return fail(PMX_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&g->graph_exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    g->graph_exec = nullptr;
    return fail(PMX_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  g->graph = graph;
  g->graph_iters = kGraphIters;
  return PMX_OK;
}

int solver_step(Game* g, int32_t n_iters, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (n_iters < 0) return fail(PMX_EINVAL, "n_iters must be >= 0");
  hipStream_t s = (hipStream_t)stream;
  int left = n_iters;
  if (g->use_graph && left >= kGraphIters) {
    if ((rc = capture_graph(g))) return rc;
    while (left >= g->graph_iters) {
      HIP_TRY(hipGraphLaunch(g->graph_exec, s));
      left -= g->graph_iters;
    }
  }
  for (int i = 0; i < left; ++i)
    if ((rc = enqueue_iteration(g, s))) return rc;
  double w = 0.0;
  for (int i = 0; i < n_iters; ++i) {
    g->t += 1;
    const double t = (double)g->t;
    w += g->gamma == 1 ? t : (g->gamma == 2 ? t * t : t * t * t);
  }
  g->wsum += w;
  // a retired instance's averages take no weight: its total stays with them,
  // and so does its last gap
  for (size_t i = 0; i < g->wsum_i.size(); ++i)
    if (g->act_h[i] && n_iters > 0) {
      g->wsum_i[i] += w;
      g->gap_ok[i] = 0;
    }
  return PMX_OK;
}

int solver_set_params(Game* g, int32_t kind, double alpha, double beta, int32_t gamma) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (kind != 0 && kind != 1) return fail(PMX_EINVAL, "kind must be 0 (RM+) or 1 (DCFR)");
  if (kind == 1 && (gamma < 1 || gamma > 3 || !std::isfinite(alpha) || !std::isfinite(beta)))
    return fail(PMX_EINVAL, "DCFR needs finite alpha, beta and gamma in {1, 2, 3}");
  HIP_TRY(hipDeviceSynchronize());
  g->dcfr = kind;
  g->gamma = kind == 1 ? gamma : 1;
  g->alpha = alpha;
  g->beta = beta;
  if (g->graph_exec) {
    (void)hipGraphExecDestroy(g->graph_exec);
    g->graph_exec = nullptr;
  }
  if (g->graph) {
    (void)hipGraphDestroy(g->graph);
    g->graph = nullptr;
  }
  return PMX_OK;
}

// Elements [b, e) of instance i in player p's vectors (instances are stored
// one after another).
static void inst_range(const Game* g, int p, size_t i, int64_t* b, int64_t* e) {
  *b = g->hg.inst[i].vec_off[p];
  *e = i + 1 < g->hg.inst.size() ? g->hg.inst[i + 1].vec_off[p] : g->hg.elems[p];
}

// Best responses to the given sequence-form sums; the values of instance i
// are multiplied by scale[i] (NULL: 1), which normalizes unnormalized sums
// since a best-response value is positively homogeneous in the opponent's
// strategy and the instances do not interact.
//
// need_dev (device flags, NULL: every instance) limits the work to the
// instances flagged, whose row chunks must all be in the solver's launch
// lists (the matvec then takes those lists); need_host is the same set on
// the host, and only its instances are written.
// Device scratch of an FP64 gap: both players' gradients, deep-piece stage
// rows and per-hand values, and the per-instance sums (2 x instances).
struct GapBufs {
  double* gd[2];
  double* stage[2];
  double* hv[2];
  double* br;
};
static GapBufs game_gap_bufs(Game* g) {
  GapBufs B;
  for (int p = 0; p < 2; ++p) {
    B.gd[p] = g->gd[p].p;
    B.stage[p] = g->dt[p].stage_d.p;
    B.hv[p] = g->dt[p].hv.p;
  }
  B.br = g->br_inst.p;
  return B;
}

static int gap_from_sums(Game* g, const double* xsum, const double* ysum, const double* scale,
                         const int32_t* need_dev, const int32_t* need_host, double* gap, double* br1,
                         double* br2, hipStream_t s, const GapBufs& B) {
  int rc;
  MvParams PA = mv_params(g, 0, 1.0), PT = mv_params(g, 1, 1.0);
  PA.active = PT.active = need_dev;
  const int ni = (int)g->hg.inst.size();
  if ((rc = launch_mv<double>(g, PA, ysum, B.gd[0], empty_params(PA), nullptr, nullptr, s))) return rc;
  if ((rc = launch_mv<double>(g, PT, xsum, B.gd[1], empty_params(PT), nullptr, nullptr, s))) return rc;
  if ((rc = br_values(g, 0, B.gd[0], B.stage[0], B.hv[0], B.br, s, need_dev))) return rc;
  if ((rc = br_values(g, 1, B.gd[1], B.stage[1], B.hv[1], B.br + ni, s, need_dev))) return rc;
  std::vector<double> h(2 * (size_t)ni);
  HIP_TRY(hipMemcpyAsync(h.data(), B.br, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < ni; ++i) {
    if (need_host && !need_host[i]) continue;
    const double c = scale ? scale[i] : 1.0;
    double a = h[i] * c, b = h[ni + i] * c;
    if (!std::isfinite(a) || !std::isfinite(b)) return fail(PMX_ENUMERIC, "non-finite best response");
    if (br1) br1[i] = a;
    if (br2) br2[i] = b;
    if (gap) gap[i] = a - b;
  }
  return PMX_OK;
}

// Each instance's average is its weighted sum over its own weight total (the
// weights of the iterations it took part in); an instance with none yet
// stands at its current plan.  An instance whose state has not changed since
// the last call (a retired one) reuses that call's values; the others are
// computed, on the solver's launch lists when those hold them all.
int saddle_gap(Game* g, double* gap, double* br1, double* br2, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const size_t ni = g->hg.inst.size();
  std::vector<int32_t> need(ni);
  size_t n_need = 0;
  bool unlisted = false;
  for (size_t i = 0; i < ni; ++i) {
    need[i] = g->gap_ok[i] ? 0 : 1;
    n_need += need[i];
    if (need[i] && !g->listed[i]) unlisted = true;
  }
  if (n_need) {
    const bool part = n_need < ni && !unlisted;
    if (part)
      HIP_TRY(hipMemcpyAsync(g->gap_need.p, need.data(), ni * sizeof(int32_t), hipMemcpyHostToDevice, s));
    const int32_t* need_dev = part ? g->gap_need.p : nullptr;
    std::vector<double> scale(ni);
    bool any_sum = false, any_plan = false;
    for (size_t i = 0; i < ni; ++i) {
      const bool has = g->wsum_i[i] > 0;
      scale[i] = has ? 1.0 / g->wsum_i[i] : 1.0;
      any_sum |= has;
      any_plan |= !has;
    }
    const double *xa = g->xs[0].p, *ya = g->xs[1].p;
    if (any_plan) {
      for (int p = 0; p < 2; ++p) {
        const int64_t n = g->hg.elems[p];
        if (!any_sum) {
          if (n > 0) {
            const int blocks = (int)std::min<int64_t>((n + 255) / 256, 4096);
            hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks), dim3(256), 0, s, g->x[p].p, g->sd[p].p, n);
          }
          continue;
        }
        HIP_TRY(hipMemcpyAsync(g->sd[p].p, g->xs[p].p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
        // runs of instances without a weight total take their current plan
        for (size_t i = 0; i < ni;) {
          if (g->wsum_i[i] > 0) {
            ++i;
            continue;
          }
          size_t j = i;
          while (j < ni && !(g->wsum_i[j] > 0)) ++j;
          int64_t b, e, b2, e2;
          inst_range(g, p, i, &b, &e);
          inst_range(g, p, j - 1, &b2, &e2);
          if (e2 > b) {
            const int blocks = (int)std::min<int64_t>((e2 - b + 255) / 256, 4096);
            hipLaunchKernelGGL(k_f32_to_f64, dim3(blocks), dim3(256), 0, s, g->x[p].p + b,
                               g->sd[p].p + b, e2 - b);
          }
          i = j;
        }
      }
      HIP_TRY(hipGetLastError());
      xa = g->sd[0].p;
      ya = g->sd[1].p;
    }
    if ((rc = gap_from_sums(g, xa, ya, scale.data(), need_dev, need.data(), g->gap_c.data(),
                            g->br1_c.data(), g->br2_c.data(), s, game_gap_bufs(g))))
      return rc;
    for (size_t i = 0; i < ni; ++i) g->gap_ok[i] = 1;
    // divergence guard: a gap that grows over gap_guard computations in a row
    int bad = -1;
    for (size_t i = 0; i < ni; ++i) {
      if (!need[i]) continue;
      const double pot = 2.0 * g->hg.inst[i].inst.contrib, prev = g->gap_prev[i];
      g->gap_grow[i] = (!std::isnan(prev) && g->gap_c[i] > prev + 1e-12 * pot) ? g->gap_grow[i] + 1 : 0;
      g->gap_prev[i] = g->gap_c[i];
      if (g->gap_guard > 0 && g->gap_grow[i] >= g->gap_guard && bad < 0) bad = (int)i;
    }
    if (bad >= 0)
      return fail(PMX_ENUMERIC, "instance " + std::to_string(bad) + ": the FP64 gap grew over " +
                                    std::to_string(g->gap_guard) + " computations in a row (the solve diverges)");
  }
  for (size_t i = 0; i < ni; ++i) {
    if (gap) gap[i] = g->gap_c[i];
    if (br1) br1[i] = g->br1_c[i];
    if (br2) br2[i] = g->br2_c[i];
  }
  return PMX_OK;
}

// ---------------------------------------------------------------------------
// the gap of given strategies with no allocation (for callers that cannot
// allocate device memory)
// ---------------------------------------------------------------------------
// Scratch of saddle_gap_of_static: one array per GPU the library runs on,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in; the device address comes from hipGetSymbolAddress, once per
// device with that device current, and only that address is used.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];
static std::mutex g_scratch_mu;
static std::vector<double*> g_scratch_dev;   // per device id; nullptr until resolved

static int static_scratch(int dev, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    HIP_TRY(hipSetDevice(dev));
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(PMX_EDEVICE, "hipGetSymbolAddress gave no address for the static scratch");
    g_scratch_dev[dev] = (double*)ptr;
  }
  *out = g_scratch_dev[dev];
  return PMX_OK;
}

int saddle_gap_of_static(Game* g, const double* x, const double* y, double* gap, double* br1, double* br2,
                         void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!x || !y) return fail(PMX_EINVAL, "null vector");
  if (!br1 || !br2) return fail(PMX_EINVAL, "br1 and br2 are required (they receive the per-instance sums)");
  double* base = nullptr;
  if ((rc = static_scratch(g->device_id, &base))) return rc;
  // carve the FP64 gradients, stage rows, per-hand values and the
  // per-instance sums out of the static array, each on 256-byte boundaries
  const int ni = (int)g->hg.inst.size();
  size_t need[7] = {(size_t)g->hg.elems[0], (size_t)g->hg.elems[1], g->dt[0].stage_d.n, g->dt[1].stage_d.n,
                    g->dt[0].hv.n, g->dt[1].hv.n, 2 * (size_t)ni};
  double* part[7];
  size_t off = 0;
  for (int k = 0; k < 7; ++k) {
    part[k] = base + off;
    off += (need[k] + 31) / 32 * 32;
  }
  if (off * sizeof(double) > kStaticScratchBytes)
    return fail(PMX_EINVAL, "saddle_gap_of_static: the game needs " + std::to_string(off * sizeof(double)) +
                                " bytes of scratch; the static buffer holds " +
                                std::to_string(kStaticScratchBytes) + " (use saddle_gap_of)");
  GapBufs B;
  B.gd[0] = part[0];
  B.gd[1] = part[1];
  B.stage[0] = part[2];
  B.stage[1] = part[3];
  B.hv[0] = part[4];
  B.hv[1] = part[5];
  B.br = part[6];
  hipStream_t s = (hipStream_t)stream;
  MvParams PA = mv_params(g, 0, 1.0), PT = mv_params(g, 1, 1.0);
  if ((rc = launch_mv<double>(g, PA, y, B.gd[0], empty_params(PA), nullptr, nullptr, s))) return rc;
  if ((rc = launch_mv<double>(g, PT, x, B.gd[1], empty_params(PT), nullptr, nullptr, s))) return rc;
  if ((rc = br_values(g, 0, B.gd[0], B.stage[0], B.hv[0], B.br, s, nullptr))) return rc;
  if ((rc = br_values(g, 1, B.gd[1], B.stage[1], B.hv[1], B.br + ni, s, nullptr))) return rc;
  // the sums straight into the caller's arrays (no host buffer either)
  HIP_TRY(hipMemcpyAsync(br1, B.br, (size_t)ni * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(br2, B.br + ni, (size_t)ni * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int i = 0; i < ni; ++i) {
    if (!std::isfinite(br1[i]) || !std::isfinite(br2[i])) return fail(PMX_ENUMERIC, "non-finite best response");
    if (gap) gap[i] = br1[i] - br2[i];
  }
  return PMX_OK;
}

int saddle_gap_of(Game* g, const double* x, const double* y, double* gap, double* br1, double* br2,
                  void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!x || !y) return fail(PMX_EINVAL, "null vector");
  return gap_from_sums(g, x, y, nullptr, nullptr, nullptr, gap, br1, br2, (hipStream_t)stream, game_gap_bufs(g));
}

int solver_get_state(Game* g, int32_t player, float* regret, float* plan, double* avg_sum, int32_t* t,
                     double* wsum) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (player < 0 || player > 1) return fail(PMX_EINVAL, "bad player");
  HIP_TRY(hipDeviceSynchronize());
  const size_t n = (size_t)g->hg.elems[player];
  if (regret) HIP_TRY(hipMemcpy(regret, g->R[player].p, n * sizeof(float), hipMemcpyDeviceToHost));
  if (plan) HIP_TRY(hipMemcpy(plan, g->x[player].p, n * sizeof(float), hipMemcpyDeviceToHost));
  if (avg_sum) HIP_TRY(hipMemcpy(avg_sum, g->xs[player].p, n * sizeof(double), hipMemcpyDeviceToHost));
  if (t) *t = g->t;
  if (wsum) *wsum = g->wsum;
  return PMX_OK;
}

int solver_set_state(Game* g, int32_t player, const float* regret, const float* plan,
                     const double* avg_sum, int32_t t, double wsum) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (player < 0 || player > 1) return fail(PMX_EINVAL, "bad player");
  if (t < 0 || !std::isfinite(wsum) || wsum < 0) return fail(PMX_EINVAL, "bad iteration state");
  HIP_TRY(hipDeviceSynchronize());
  const size_t n = (size_t)g->hg.elems[player];
  if (regret) HIP_TRY(hipMemcpy(g->R[player].p, regret, n * sizeof(float), hipMemcpyHostToDevice));
  if (plan) HIP_TRY(hipMemcpy(g->x[player].p, plan, n * sizeof(float), hipMemcpyHostToDevice));
  if (avg_sum) HIP_TRY(hipMemcpy(g->xs[player].p, avg_sum, n * sizeof(double), hipMemcpyHostToDevice));
  g->t = t;
  g->wsum = wsum;
  g->wsum_i.assign(g->wsum_i.size(), wsum);
  invalidate_gaps(g);
  const double cur = (double)t;   // the next iteration's first launch makes it t + 1
  HIP_TRY(hipMemcpy(g->tdev.p, &cur, sizeof(double), hipMemcpyHostToDevice));
  return PMX_OK;
}

int solver_get_weights(Game* g, double* wsum_host) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!wsum_host) return fail(PMX_EINVAL, "null argument");
  std::copy(g->wsum_i.begin(), g->wsum_i.end(), wsum_host);
  return PMX_OK;
}

int solver_snapshot(Game* g, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  for (int p = 0; p < 2; ++p) {
    const size_t n = (size_t)g->hg.elems[p];
    if (g->snap_R[p].n != n) {
      if ((rc = g->snap_R[p].alloc(n)) || (rc = g->snap_x[p].alloc(n)) || (rc = g->snap_xs[p].alloc(n))) return rc;
    }
    if (n) {
      HIP_TRY(hipMemcpyAsync(g->snap_R[p].p, g->R[p].p, n * sizeof(float), hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemcpyAsync(g->snap_x[p].p, g->x[p].p, n * sizeof(float), hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemcpyAsync(g->snap_xs[p].p, g->xs[p].p, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    }
  }
  g->snap_wsum_i = g->wsum_i;
  g->snap_t = g->t;
  return PMX_OK;
}

int solver_restore_instances(Game* g, const int32_t* restore, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!restore) return fail(PMX_EINVAL, "null argument");
  if (g->snap_t < 0) return fail(PMX_ESTATE, "no snapshot");
  if (g->snap_t != g->t) return fail(PMX_ESTATE, "the snapshot was taken at another iteration count");
  hipStream_t s = (hipStream_t)stream;
  bool any = false;
  for (size_t i = 0; i < g->hg.inst.size(); ++i) {
    if (!restore[i]) continue;
    any = true;
    const Built& b = g->hg.inst[i];
    for (int p = 0; p < 2; ++p) {
      const size_t off = (size_t)b.vec_off[p], n = (size_t)b.sf.n_seq[p] * (size_t)b.stride[p];
      if (!n) continue;
      HIP_TRY(hipMemcpyAsync(g->R[p].p + off, g->snap_R[p].p + off, n * sizeof(float), hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemcpyAsync(g->x[p].p + off, g->snap_x[p].p + off, n * sizeof(float), hipMemcpyDeviceToDevice, s));
      HIP_TRY(hipMemcpyAsync(g->xs[p].p + off, g->snap_xs[p].p + off, n * sizeof(double), hipMemcpyDeviceToDevice,
                             s));
    }
    g->wsum_i[i] = g->snap_wsum_i[i];
  }
  if (any) invalidate_gaps(g);
  return PMX_OK;
}

int solver_set_weights(Game* g, const double* wsum_host) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!wsum_host) return fail(PMX_EINVAL, "null argument");
  const size_t n = g->wsum_i.size();
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(wsum_host[i]) || wsum_host[i] < 0) return fail(PMX_EINVAL, "bad weight total");
  std::copy(wsum_host, wsum_host + n, g->wsum_i.begin());
  invalidate_gaps(g, false);
  return PMX_OK;
}

int get_average_strategy(Game* g, int32_t player, double* x_host) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (player < 0 || player > 1 || !x_host) return fail(PMX_EINVAL, "bad argument");
  const size_t n = (size_t)g->hg.elems[player];
  HIP_TRY(hipDeviceSynchronize());
  HIP_TRY(hipMemcpy(x_host, g->xs[player].p, n * sizeof(double), hipMemcpyDeviceToHost));
  std::vector<float> xf;
  for (size_t i = 0; i < g->hg.inst.size(); ++i) {
    int64_t b, e;
    inst_range(g, player, i, &b, &e);
    const double w = g->wsum_i[i];
    if (w > 0) {
      for (int64_t k = b; k < e; ++k) x_host[k] /= w;
      continue;
    }
    // no iteration of this instance yet: its average is the current plan
    if (xf.empty()) {
      xf.resize(n);
      HIP_TRY(hipMemcpy(xf.data(), g->x[player].p, n * sizeof(float), hipMemcpyDeviceToHost));
    }
    for (int64_t k = b; k < e; ++k) x_host[k] = xf[k];
  }
  return PMX_OK;
}

int set_initial_strategy(Game* g, int32_t player, const float* behav, float scale, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (player < 0 || player > 1 || !behav) return fail(PMX_EINVAL, "bad argument");
  if (!(scale >= 0) || !std::isfinite(scale)) return fail(PMX_EINVAL, "scale must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  invalidate_gaps(g);
  DevTp& E = g->dt[player];
  if (E.n_single)
    hipLaunchKernelGGL(k_warm, dim3(E.n_single), dim3(TPB), 0, s, tp_params(g, player, E.b_single.p),
                       behav, scale, g->R[player].p, g->x[player].p);
  if (E.n_top)
    hipLaunchKernelGGL(k_warm, dim3(E.n_top), dim3(TPB), 0, s, tp_params(g, player, E.b_top.p), behav,
                       scale, g->R[player].p, g->x[player].p);
  if (E.n_deep)
    hipLaunchKernelGGL(k_warm, dim3(E.n_deep), dim3(TPB), 0, s, tp_params(g, player, E.b_deep.p),
                       behav, scale, g->R[player].p, g->x[player].p);
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

int warm_num_rows(const Game* g, int32_t player, int64_t* rows) {
  if (!g || !rows || player < 0 || player > 1) return fail(PMX_EINVAL, "bad argument");
  if (!g->device) return fail(PMX_ESTATE, "game was created host-only");
  *rows = g->wrows[player];
  return PMX_OK;
}

int warm_features(Game* g, int32_t player, uint16_t* x_dev, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (player < 0 || player > 1 || !x_dev) return fail(PMX_EINVAL, "bad argument");
  if (g->wn_blk[player])
    hipLaunchKernelGGL(k_warm_features, dim3(g->wn_blk[player]), dim3(256), 0, (hipStream_t)stream,
                       g->wseg[player].p, g->wblk[player].p, g->winf[player].p, g->whand[player].p, x_dev);
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

int warm_targets(Game* g, int32_t player, float* target_dev, float* weight_dev, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (player < 0 || player > 1 || !target_dev || !weight_dev) return fail(PMX_EINVAL, "bad argument");
  if (!g->warm_ok) return fail(PMX_EINVAL, "an infoset has more actions than the network's slots");
  if (!(g->wsum > 0)) return fail(PMX_ESTATE, "no solver iterations to take targets from");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(g->wsum_dev.p, g->wsum_i.data(), g->wsum_i.size() * sizeof(double),
                         hipMemcpyHostToDevice, s));
  if (g->wn_blk[player])
    hipLaunchKernelGGL(k_warm_targets, dim3(g->wn_blk[player]), dim3(256), 0, s, g->wseg[player].p,
                       g->wblk[player].p, g->xs[player].p, g->wsum_dev.p, g->whand[player].p, target_dev,
                       weight_dev);
  // the weight totals are host memory that later solver steps change
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipGetLastError());
  return PMX_OK;
}

int warm_apply(Game* g, const float* logits0_dev, const float* logits1_dev, int32_t ldz, float regret_scale,
               double avg_weight, void* stream) {
  int rc = ensure_device(g);
  if (rc) return rc;
  if (!logits0_dev || !logits1_dev || ldz < kWarmActions) return fail(PMX_EINVAL, "bad argument");
  if (!g->warm_ok) return fail(PMX_EINVAL, "an infoset has more actions than the network's slots");
  if (!(regret_scale >= 0) || !std::isfinite(regret_scale) || !(avg_weight >= 0) || !std::isfinite(avg_weight))
    return fail(PMX_EINVAL, "scale and weight must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = solver_reset(g, s))) return rc;
  for (int p = 0; p < 2; ++p) {
    DevTp& E = g->dt[p];
    const float* Z = p == 0 ? logits0_dev : logits1_dev;
    // parents before children: single, then top, then deep tasks
    if (E.n_single)
      hipLaunchKernelGGL(k_warm_apply, dim3(E.n_single), dim3(TPB), 0, s, tp_params(g, p, E.b_single.p),
                         g->wrow_base[p].p, Z, ldz, regret_scale, avg_weight, g->lam.p, g->lam_inst[p].p,
                         g->pot_inst.p, g->R[p].p, g->x[p].p, g->xs[p].p);
    if (E.n_top)
      hipLaunchKernelGGL(k_warm_apply, dim3(E.n_top), dim3(TPB), 0, s, tp_params(g, p, E.b_top.p),
                         g->wrow_base[p].p, Z, ldz, regret_scale, avg_weight, g->lam.p, g->lam_inst[p].p,
                         g->pot_inst.p, g->R[p].p, g->x[p].p, g->xs[p].p);
    if (E.n_deep)
      hipLaunchKernelGGL(k_warm_apply, dim3(E.n_deep), dim3(TPB), 0, s, tp_params(g, p, E.b_deep.p),
                         g->wrow_base[p].p, Z, ldz, regret_scale, avg_weight, g->lam.p, g->lam_inst[p].p,
                         g->pot_inst.p, g->R[p].p, g->x[p].p, g->xs[p].p);
  }
  HIP_TRY(hipGetLastError());
  g->t = 0;
  g->wsum = avg_weight;
  g->wsum_i.assign(g->wsum_i.size(), avg_weight);
  invalidate_gaps(g);
  return PMX_OK;
}

}  // extern "C"
