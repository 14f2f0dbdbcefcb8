// Token-parallel GEMMs of the velocity network on gfx950 matrix cores.
//
// C[M, N] = epi(pro(A)[M, K] W[K, N] + b) where pro is an optional LayerNorm over the K
// features of each row (FP32 statistics computed once per row by k_row_stats, applied while
// the A tile is staged into LDS) and epi stores, applies the exact
// GELU, or accumulates into the FP32 residual stream. Rows are tokens of the packed CSR
// batch: every row is independent and its K-reduction order does not depend on where
// the row sits in a tile, so a token's result is the same whatever batch it is part of.
//
// Tiling: block tile 128 x BN (BN = 128 or 64) x 32, four waves in a 2 x 2 grid, each wave
// 64 x BN/2 made of 32 x 32 MFMA tiles.
//   FP32: v_mfma_f32_32x32x2_f32   (lane l: A row l%32, one k; B col l%32, one k)
//   BF16: v_mfma_f32_32x32x16_bf16 (lane l: A row l%32, 8 consecutive k; same for B)
// Accumulator layout (both): lane l, register r holds row 8(r/4) + 4(l/32) + r%4 and column
// l%32 of the 32 x 32 tile.
// A and W^T slices are staged through double-buffered LDS (one barrier per 32-wide K
// step, global loads of step k+1 in flight during the MFMAs of step k). The k order inside
// a step is permuted consistently for A and B so that each lane reads contiguous 16-byte
// LDS vectors.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace fmd {

constexpr int BM = 128, BK = 32, NT = 256;

template <typename T> struct LdsPad { static constexpr int v = 4; };   // 144 B rows (fp32)
template <> struct LdsPad<bf16> { static constexpr int v = 8; };       // 80 B rows (bf16)

// 16-byte global chunk -> LDS row segment, converting FP32 to T on the way.
template <typename T>
__device__ __forceinline__ void store4(T* dst, float4 v);
template <>
__device__ __forceinline__ void store4<float>(float* dst, float4 v) { *(float4*)dst = v; }
template <>
__device__ __forceinline__ void store4<bf16>(bf16* dst, float4 v) {
  bf16x4 o;
  o[0] = (bf16)v.x; o[1] = (bf16)v.y; o[2] = (bf16)v.z; o[3] = (bf16)v.w;
  *(bf16x4*)dst = o;
}

template <typename T, bool LN, int EPI, int BN>
__device__ __forceinline__ void gemm_body(const void* __restrict__ A_, int lda,
                                          const T* __restrict__ Wt, int K,
                                          const float* __restrict__ bias,
                                          const float2* __restrict__ stats,
                                          const float* __restrict__ ln_g,
                                          const float* __restrict__ ln_s,
                                          void* __restrict__ C_, int ldc, int n_tiles,
                                          const OdeArgs& ode) {
  using AT = typename std::conditional<LN, float, T>::type;
  constexpr int LDK = BK + LdsPad<T>::v;
  constexpr int TN = BN / 64;                        // 32-wide tiles per wave along N
  constexpr int A_ELEMS = 16 / sizeof(AT);           // elements per 16-byte chunk of A
  constexpr int A_CPR = BK / A_ELEMS;                // chunks per A row slice
  constexpr int A_PER_T = BM * A_CPR / NT;
  constexpr int B_ELEMS = 16 / sizeof(T);
  constexpr int B_CPR = BK / B_ELEMS;
  constexpr int B_PER_T = BN * B_CPR / NT;

  __shared__ __attribute__((aligned(16))) T As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN][LDK];
  __shared__ float sMean[LN ? BM : 1], sRstd[LN ? BM : 1];

  const AT* A = (const AT*)A_;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int mt = logical / n_tiles, nt = logical % n_tiles;
  const int64_t m0 = (int64_t)mt * BM;
  const int n0 = nt * BN;

  if constexpr (LN) {
    if (tid < BM) {
      const float2 st = stats[m0 + tid];
      sMean[tid] = st.x;
      sRstd[tid] = st.y;
    }
    __syncthreads();
  }

  u32x4 ra[A_PER_T], rb[B_PER_T];

#define FMD_LOAD_TILES(k0)                                                                  \
  _Pragma("unroll") for (int i = 0; i < A_PER_T; ++i) {                                    \
    const int idx = tid + i * NT;                                                           \
    ra[i] = *(const u32x4*)(A + (m0 + idx / A_CPR) * lda + (k0) + (idx % A_CPR) * A_ELEMS); \
  }                                                                                         \
  _Pragma("unroll") for (int i = 0; i < B_PER_T; ++i) {                                    \
    const int idx = tid + i * NT;                                                           \
    rb[i] = *(const u32x4*)(Wt + (int64_t)(n0 + idx / B_CPR) * K + (k0) +                   \
                            (idx % B_CPR) * B_ELEMS);                                       \
  }

#define FMD_STORE_TILES(buf, k0)                                                            \
  _Pragma("unroll") for (int i = 0; i < A_PER_T; ++i) {                                    \
    const int idx = tid + i * NT;                                                           \
    const int row = idx / A_CPR, ch = idx % A_CPR;                                          \
    if constexpr (std::is_same<AT, float>::value) {                                         \
      float4 v = make_float4(__uint_as_float(ra[i][0]), __uint_as_float(ra[i][1]),         \
                             __uint_as_float(ra[i][2]), __uint_as_float(ra[i][3]));         \
      if constexpr (LN) {                                                                   \
        const int k = (k0) + ch * 4;                                                        \
        const float mu = sMean[row], rs = sRstd[row];                                       \
        v.x = (v.x - mu) * rs * ln_g[k + 0] + ln_s[k + 0];                                  \
        v.y = (v.y - mu) * rs * ln_g[k + 1] + ln_s[k + 1];                                  \
        v.z = (v.z - mu) * rs * ln_g[k + 2] + ln_s[k + 2];                                  \
        v.w = (v.w - mu) * rs * ln_g[k + 3] + ln_s[k + 3];                                  \
      }                                                                                     \
      store4<T>(&As[buf][row][ch * 4], v);                                                  \
    } else {                                                                                \
      *(u32x4*)&As[buf][row][ch * A_ELEMS] = ra[i];                                         \
    }                                                                                       \
  }                                                                                         \
  _Pragma("unroll") for (int i = 0; i < B_PER_T; ++i) {                                    \
    const int idx = tid + i * NT;                                                           \
    *(u32x4*)&Bs[buf][idx / B_CPR][(idx % B_CPR) * B_ELEMS] = rb[i];                        \
  }

  f32x16 acc[2][TN];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int nj = 0; nj < TN; ++nj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mi][nj][r] = 0.f;

  const int nk = K / BK;
  FMD_LOAD_TILES(0);
  FMD_STORE_TILES(0, 0);
  __syncthreads();

  const int arow = wm * 64 + (lane & 31);
  const int brow = wn * (BN / 2) + (lane & 31);
  const int half = lane >> 5;

  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) { FMD_LOAD_TILES((kt + 1) * BK); }
    if constexpr (std::is_same<T, bf16>::value) {
#pragma unroll
      for (int ks = 0; ks < BK / 16; ++ks) {
        bf16x8 a[2], b[TN];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
          a[mi] = *(const bf16x8*)&As[buf][arow + mi * 32][ks * 16 + half * 8];
#pragma unroll
        for (int nj = 0; nj < TN; ++nj)
          b[nj] = *(const bf16x8*)&Bs[buf][brow + nj * 32][ks * 16 + half * 8];
#pragma unroll
        for (int mi = 0; mi < 2; ++mi)
#pragma unroll
          for (int nj = 0; nj < TN; ++nj)
            acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[nj], acc[mi][nj], 0, 0, 0);
      }
    } else {
      // lane half h supplies k = h*16 + m to MFMA m (m < 16), for A and B alike
      float4 a[2][4], b[TN][4];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          a[mi][q] = *(const float4*)&As[buf][arow + mi * 32][half * 16 + q * 4];
#pragma unroll
      for (int nj = 0; nj < TN; ++nj)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          b[nj][q] = *(const float4*)&Bs[buf][brow + nj * 32][half * 16 + q * 4];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
#pragma unroll
        for (int mi = 0; mi < 2; ++mi) {
          const float av = a[mi][m >> 2][m & 3];
#pragma unroll
          for (int nj = 0; nj < TN; ++nj)
            acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[nj][m >> 2][m & 3],
                                                               acc[mi][nj], 0, 0, 0);
        }
      }
    }
    if (more) { FMD_STORE_TILES(buf ^ 1, (kt + 1) * BK); }
    __syncthreads();
  }

#undef FMD_LOAD_TILES
#undef FMD_STORE_TILES

  // epilogue
  if constexpr (EPI == EPI_RESID) {
    // per 32-row tile, read the residual values first: the stores may alias later loads
    float* C = (float*)C_;
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      float old[TN][16];
#pragma unroll
      for (int nj = 0; nj < TN; ++nj) {
        const int col = n0 + wn * (BN / 2) + nj * 32 + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * 64 + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          old[nj][r] = C[row * ldc + col];
        }
      }
#pragma unroll
      for (int nj = 0; nj < TN; ++nj) {
        const int col = n0 + wn * (BN / 2) + nj * 32 + (lane & 31);
        const float bv = bias ? bias[col] : 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * 64 + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          C[row * ldc + col] = old[nj][r] + (acc[mi][nj][r] + bv);
        }
      }
    }
  } else {
#pragma unroll
    for (int nj = 0; nj < TN; ++nj) {
      const int col = n0 + wn * (BN / 2) + nj * 32 + (lane & 31);
      const float bv = bias ? bias[col] : 0.f;
#pragma unroll
      for (int mi = 0; mi < 2; ++mi) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * 64 + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          const float v = acc[mi][nj][r] + bv;
          if constexpr (EPI == EPI_ODE) {
            if (col < ode.nf && row < ode.m_valid) {
              const int64_t o = row * ode.ldx + col;
              ode_update(ode.mode, ode.h, v, ode.x + o, ode.acc + o, ode.xs + o,
                         ode.out ? ode.out + row * ode.ldo + col : nullptr);
            }
          } else if constexpr (EPI == EPI_GELU) {
            ((T*)C_)[row * ldc + col] = from_f32<T>(gelu_erf(v));
          } else {
            ((T*)C_)[row * ldc + col] = from_f32<T>(v);
          }
        }
      }
    }
  }
}

// One kernel name per class of GEMM in the network, so that profiles separate them.
#define FMD_GEMM_KERNEL(NAME)                                                                 \
  template <typename T, bool LN, int EPI, int BN>                                             \
  __global__ __launch_bounds__(NT) void NAME(const void* __restrict__ A, int lda,             \
                                             const T* __restrict__ Wt, int K,                 \
                                             const float* __restrict__ bias,                  \
                                             const float2* __restrict__ stats,                \
                                             const float* __restrict__ g,                     \
                                             const float* __restrict__ s,                     \
                                             void* __restrict__ C, int ldc, int n_tiles,      \
                                             OdeArgs ode) {                                   \
    gemm_body<T, LN, EPI, BN>(A, lda, Wt, K, bias, stats, g, s, C, ldc, n_tiles, ode);        \
  }
FMD_GEMM_KERNEL(k_gemm_qkv)     // LN1 -> [Q|K|V]
FMD_GEMM_KERNEL(k_gemm_proj)    // attention output projections (+ residual), LN2 -> cross Q
FMD_GEMM_KERNEL(k_gemm_up)      // LN3 -> MLP up + GELU
FMD_GEMM_KERNEL(k_gemm_down)    // MLP down (+ residual)
FMD_GEMM_KERNEL(k_gemm_head)    // LN_f -> output head + fused Euler/RK4 state update
FMD_GEMM_KERNEL(k_gemm_any)     // truth K/V cache and test hooks
#undef FMD_GEMM_KERNEL

template <typename T>
using GemmKernel = void (*)(const void*, int, const T*, int, const float*, const float2*,
                            const float*, const float*, void*, int, int, OdeArgs);

template <typename T, int BN>
static hipError_t go(GemmKernel<T> k, hipStream_t st, int64_t Mp, int N, int K, const void* A,
                     int lda, const T* Wt, const float* bias, const float2* stats,
                     const float* g, const float* s, void* C, int ldc, const OdeArgs& ode) {
  const int n_tiles = N / BN;
  const int64_t grid = (Mp / BM) * n_tiles;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(NT), 0, st, A, lda, Wt, K, bias, stats, g, s,
                     C, ldc, n_tiles, ode);
  return hipGetLastError();
}

template <typename T, int BN>
static hipError_t dispatch(hipStream_t st, int cls, bool ln, int epi, int64_t Mp, int N, int K,
                           const void* A, int lda, const T* Wt, const float* bias,
                           const float2* stats, const float* g, const float* s, void* C,
                           int ldc, const OdeArgs& ode) {
#define FMD_GO(KER, L, E) \
  return go<T, BN>(KER<T, L, E, BN>, st, Mp, N, K, A, lda, Wt, bias, stats, g, s, C, ldc, ode)
  switch (cls) {
    case FMD_K_GEMM_QKV:
      if (ln && epi == EPI_STORE) FMD_GO(k_gemm_qkv, true, EPI_STORE);
      break;
    case FMD_K_GEMM_PROJ:
      if (ln && epi == EPI_STORE) FMD_GO(k_gemm_proj, true, EPI_STORE);
      if (!ln && epi == EPI_RESID) FMD_GO(k_gemm_proj, false, EPI_RESID);
      break;
    case FMD_K_GEMM_UP:
      if (ln && epi == EPI_GELU) FMD_GO(k_gemm_up, true, EPI_GELU);
      break;
    case FMD_K_GEMM_DOWN:
      if (!ln && epi == EPI_RESID) FMD_GO(k_gemm_down, false, EPI_RESID);
      break;
    default:
      if (epi == EPI_ODE) {
        if (ln) FMD_GO(k_gemm_head, true, EPI_ODE);
        break;
      }
      if (ln) {
        if (epi == EPI_STORE) FMD_GO(k_gemm_any, true, EPI_STORE);
        if (epi == EPI_GELU) FMD_GO(k_gemm_any, true, EPI_GELU);
        FMD_GO(k_gemm_any, true, EPI_RESID);
      }
      if (epi == EPI_STORE) FMD_GO(k_gemm_any, false, EPI_STORE);
      if (epi == EPI_GELU) FMD_GO(k_gemm_any, false, EPI_GELU);
      FMD_GO(k_gemm_any, false, EPI_RESID);
  }
#undef FMD_GO
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_gemm(hipStream_t st, int cls, bool ln, int epi, int64_t Mp, int N, int K,
                       const void* A, int lda, const T* Wt, const float* bias,
                       const float2* stats, const float* g, const float* s, void* C, int ldc,
                       const OdeArgs* ode) {
  if (Mp % BM || K % BK || N % 64) return hipErrorInvalidValue;
  if (ln && !stats) return hipErrorInvalidValue;
  if ((epi == EPI_ODE) != (ode != nullptr)) return hipErrorInvalidValue;
  const OdeArgs none{};
  const OdeArgs& oa = ode ? *ode : none;
  if (N % 128 == 0)
    return dispatch<T, 128>(st, cls, ln, epi, Mp, N, K, A, lda, Wt, bias, stats, g, s, C, ldc, oa);
  return dispatch<T, 64>(st, cls, ln, epi, Mp, N, K, A, lda, Wt, bias, stats, g, s, C, ldc, oa);
}

// LayerNorm row statistics: one wave per row, the row held in registers for two passes.
// VEC: each lane reads 4 consecutive floats per step (rows whose length is a multiple of 256).
template <bool VEC>
__global__ __launch_bounds__(256) void k_row_stats(const float* __restrict__ A, int ld, int K,
                                                   int64_t M, float2* __restrict__ stats) {
  constexpr int kMax = 16;   // K <= 1024
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= M) return;
  const float* rowp = A + r * ld;
  float v[kMax];
  float s = 0.f;
  if constexpr (VEC) {
    const int n = K >> 8;
#pragma unroll
    for (int i = 0; i < kMax / 4; ++i)
      if (i < n) {
        const float4 q = *(const float4*)(rowp + lane * 4 + 256 * i);
        v[4 * i] = q.x; v[4 * i + 1] = q.y; v[4 * i + 2] = q.z; v[4 * i + 3] = q.w;
        s += (q.x + q.y) + (q.z + q.w);
      }
    const float mean = wave_sum(s) / K;
    float q = 0.f;
#pragma unroll
    for (int i = 0; i < kMax; ++i)
      if (i < 4 * n) { const float dv = v[i] - mean; q = fmaf(dv, dv, q); }
    const float var = wave_sum(q) / K;
    if (lane == 0) stats[r] = make_float2(mean, rsqrtf(var + kLnEps));
  } else {
    const int n = K >> 6;
#pragma unroll
    for (int i = 0; i < kMax; ++i)
      if (i < n) { v[i] = rowp[lane + 64 * i]; s += v[i]; }
    const float mean = wave_sum(s) / K;
    float q = 0.f;
#pragma unroll
    for (int i = 0; i < kMax; ++i)
      if (i < n) { const float dv = v[i] - mean; q = fmaf(dv, dv, q); }
    const float var = wave_sum(q) / K;
    if (lane == 0) stats[r] = make_float2(mean, rsqrtf(var + kLnEps));
  }
}

hipError_t launch_row_stats(hipStream_t st, const float* A, int ld, int K, int64_t M,
                            float2* stats) {
  if (M <= 0) return hipSuccess;
  if (K % 64 || K > 1024) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((M + 3) / 4));
  if (K % 256 == 0 && ld % 4 == 0)
    hipLaunchKernelGGL(k_row_stats<true>, grid, dim3(256), 0, st, A, ld, K, M, stats);
  else
    hipLaunchKernelGGL(k_row_stats<false>, grid, dim3(256), 0, st, A, ld, K, M, stats);
  return hipGetLastError();
}

template hipError_t launch_gemm<float>(hipStream_t, int, bool, int, int64_t, int, int,
                                       const void*, int, const float*, const float*,
                                       const float2*, const float*, const float*, void*, int,
                                       const OdeArgs*);
template hipError_t launch_gemm<bf16>(hipStream_t, int, bool, int, int64_t, int, int,
                                      const void*, int, const bf16*, const float*, const float2*,
                                      const float*, const float*, void*, int, const OdeArgs*);

}  // namespace fmd
