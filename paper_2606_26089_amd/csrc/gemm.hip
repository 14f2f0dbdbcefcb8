// GEMM launcher and LayerNorm row statistics. The kernels themselves are instantiated
// per element type in gemm_f32.hip and gemm_bf16.hip from gemm_body.h.
#include "gemm_body.h"

namespace fmd {

int default_tile(int N) { return N % 128 == 0 ? 0 : 4; }

template <typename T>
hipError_t launch_gemm(hipStream_t st, int cls, bool ln, int epi, int64_t Mp, int N, int K,
                       const void* A, int lda, const T* Wt, const float* bias,
                       const float2* stats, const float* g, const float* s, void* C, int ldc,
                       const OdeArgs* ode, int tile) {
  if (Mp % kGemmBM || K % 32 || N % 64) return hipErrorInvalidValue;
  if (ln && !stats) return hipErrorInvalidValue;
  if ((epi == EPI_ODE || epi == EPI_RESID_LN) != (ode != nullptr)) return hipErrorInvalidValue;
  if (epi == EPI_RESID_LN && !ode->stats_out) return hipErrorInvalidValue;
  const OdeArgs none{};
  const OdeArgs& oa = ode ? *ode : none;
  if (tile < 0) tile = default_tile(N);
  return launch_gemm_tile<T>(st, tile, cls, ln, epi, Mp, N, K, A, lda, Wt, bias, stats, g, s, C,
                             ldc, oa);
}

bool tile_fits(int tile, int64_t Mp, int N, int K, bool full_rows) {
  if (tile < 0 || tile >= kNumTiles) return false;
  const TileDims t = tile_dims(tile);
  if (full_rows && (N != t.BN || t.TM % 2)) return false;
  return Mp % t.BM == 0 && N % t.BN == 0 && K % t.BK == 0;
}

int default_tile_rows(int N) {
  for (int t = 0; t < kNumTiles; ++t)
    if (tile_dims(t).BN == N && tile_dims(t).TM % 2 == 0) return t;
  return -1;
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
                                       const OdeArgs*, int);
template hipError_t launch_gemm<bf16>(hipStream_t, int, bool, int, int64_t, int, int,
                                      const void*, int, const bf16*, const float*, const float2*,
                                      const float*, const float*, void*, int, const OdeArgs*,
                                      int);

}  // namespace fmd
