// Instantiation of the GEMM kernels for one element type FMD_GEMM_T; included by
// gemm_f32.hip and gemm_bf16.hip so that the two compile in parallel.
#pragma once

#include "gemm_body.h"

namespace fmd {

// One kernel name per class of GEMM in the network, so that profiles separate them.
#define FMD_GEMM_KERNEL(NAME)                                                                \
  template <typename T, bool LN, int EPI, typename TL>                                       \
  __global__ __launch_bounds__(TL::NT) void NAME(                                            \
      const void* __restrict__ A, int lda, const T* __restrict__ Wt, int K,                  \
      const float* __restrict__ bias, const float2* __restrict__ stats,                      \
      const float* __restrict__ g, const float* __restrict__ s, void* __restrict__ C,        \
      int ldc, int n_tiles, OdeArgs ode) {                                                   \
    gemm_body<T, LN, EPI, TL>(A, lda, Wt, K, bias, stats, g, s, C, ldc, n_tiles, ode);       \
  }
FMD_GEMM_KERNEL(k_gemm_qkv)     // LN1 -> [Q|K|V]
FMD_GEMM_KERNEL(k_gemm_proj)    // attention output projections (+ residual)
FMD_GEMM_KERNEL(k_gemm_qc)      // LN2 -> cross-attention query
FMD_GEMM_KERNEL(k_gemm_up)      // LN3 -> MLP up + GELU
FMD_GEMM_KERNEL(k_gemm_down)    // MLP down (+ residual)
FMD_GEMM_KERNEL(k_gemm_head)    // LN_f -> output head + fused Euler/RK4 state update
FMD_GEMM_KERNEL(k_gemm_any)     // truth K/V cache and test hooks
#undef FMD_GEMM_KERNEL

template <typename T>
using GemmKernel = void (*)(const void*, int, const T*, int, const float*, const float2*,
                            const float*, const float*, void*, int, int, OdeArgs);

template <typename T, typename TL>
static hipError_t go(GemmKernel<T> k, hipStream_t st, int64_t Mp, int N, int K, const void* A,
                     int lda, const T* Wt, const float* bias, const float2* stats,
                     const float* g, const float* s, void* C, int ldc, const OdeArgs& ode) {
  const int n_tiles = N / TL::BN;
  const int64_t grid = (Mp / TL::BM) * n_tiles;
  if (grid <= 0) return hipSuccess;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k, dim3((unsigned)grid), dim3(TL::NT), 0, st, A, lda, Wt, K, bias, stats, g,
                     s, C, ldc, n_tiles, ode);
  return hipGetLastError();
}

// The hot classes get every tiling; the K/V cache, test hooks and head only tiles 0 and 4.
template <typename T, int ID, typename TL>
static hipError_t dispatch_cls(hipStream_t st, int cls, bool ln, int epi, int64_t Mp, int N,
                               int K, const void* A, int lda, const T* Wt, const float* bias,
                               const float2* stats, const float* g, const float* s, void* C,
                               int ldc, const OdeArgs& ode) {
#define FMD_GO(KER, L, E) \
  return go<T, TL>(KER<T, L, E, TL>, st, Mp, N, K, A, lda, Wt, bias, stats, g, s, C, ldc, ode)
  switch (cls) {
    case FMD_K_GEMM_QKV:
      if (ln && epi == EPI_STORE) FMD_GO(k_gemm_qkv, true, EPI_STORE);
      break;
    case FMD_K_GEMM_PROJ:
      if (!ln && epi == EPI_RESID) FMD_GO(k_gemm_proj, false, EPI_RESID);
      if constexpr (TL::TM % 2 == 0)
        if (!ln && epi == EPI_RESID_LN) FMD_GO(k_gemm_proj, false, EPI_RESID_LN);
      break;
    case FMD_K_GEMM_QC:
      if (ln && epi == EPI_STORE) FMD_GO(k_gemm_qc, true, EPI_STORE);
      break;
    case FMD_K_GEMM_UP:
      if (ln && epi == EPI_GELU) FMD_GO(k_gemm_up, true, EPI_GELU);
      break;
    case FMD_K_GEMM_DOWN:
      if (!ln && epi == EPI_RESID) FMD_GO(k_gemm_down, false, EPI_RESID);
      if constexpr (TL::TM % 2 == 0)
        if (!ln && epi == EPI_RESID_LN) FMD_GO(k_gemm_down, false, EPI_RESID_LN);
      break;
    default:
      if constexpr (ID == 0 || ID == 4) {
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
      break;
  }
#undef FMD_GO
  return hipErrorInvalidValue;
}

template <>
hipError_t launch_gemm_tile<FMD_GEMM_T>(hipStream_t st, int tile, int cls, bool ln, int epi,
                                        int64_t Mp, int N, int K, const void* A, int lda,
                                        const FMD_GEMM_T* Wt, const float* bias,
                                        const float2* stats, const float* g, const float* s,
                                        void* C, int ldc, const OdeArgs& ode) {
  switch (tile) {
#define FMD_TILE_CASE(ID, BM_, BN_, BK_, WM_, WN_)                                             \
  case ID:                                                                                   \
    if (Mp % BM_ || N % BN_ || K % BK_) return hipErrorInvalidValue;                         \
    if (epi == EPI_RESID_LN && N != BN_) return hipErrorInvalidValue;                        \
    return dispatch_cls<FMD_GEMM_T, ID, Tile<BM_, BN_, BK_, WM_, WN_>>(                      \
        st, cls, ln, epi, Mp, N, K, A, lda, Wt, bias, stats, g, s, C, ldc, ode);
    FMD_GEMM_TILES(FMD_TILE_CASE)
#undef FMD_TILE_CASE
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace fmd
