// Token-parallel GEMM body of the velocity network on gfx950 matrix cores.
//
// C[M, N] = epi(pro(A)[M, K] W[K, N] + b). pro is an optional LayerNorm over the K
// features of each row: FP32 statistics come precomputed per row, and the normalisation
// is applied while the A tile is staged into LDS. epi stores, applies the exact GELU,
// accumulates into the FP32 residual stream, or performs the Euler/RK4 state update.
// Rows are tokens of the packed CSR batch. Every row is independent, and its K-reduction
// order does not depend on where the row sits in a tile, so a token's result is the same
// whatever batch it is part of.
//
// Tiling (template Tile): block tile BM x BN x BK, WM x WN waves, each wave owning a
// (BM/WM) x (BN/WN) tile of 32 x 32 MFMA blocks.
//   FP32: v_mfma_f32_32x32x2_f32   (lane l: A row l%32, one k; B col l%32, one k)
//   BF16: v_mfma_f32_32x32x16_bf16 (lane l: A row l%32, 8 consecutive k; same for B)
// Accumulator layout (both): lane l, register r holds row 8(r/4) + 4(l/32) + r%4 and column
// l%32 of the 32 x 32 block.
// A and W^T slices are staged through double-buffered LDS, with one barrier per K step and
// the global loads of step k+1 in flight during the MFMAs of step k. The k order inside a
// step is permuted the same way for A and B, so each lane reads contiguous 16-byte LDS
// vectors.
#pragma once

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace fmd {

template <int BM_, int BN_, int BK_, int WM_, int WN_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int WTM = BM / WM, WTN = BN / WN;    // wave tile
  static constexpr int TM = WTM / 32, TN = WTN / 32;    // 32 x 32 MFMA blocks per wave
  static_assert(TM * 32 * WM == BM && TN * 32 * WN == BN, "tile does not split into waves");
};

template <typename T> struct LdsPad { static constexpr int v = 4; };   // fp32 rows: 16 B pad
template <> struct LdsPad<bf16> { static constexpr int v = 8; };       // bf16 rows: 16 B pad

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

template <typename T, bool LN, int EPI, typename TL>
__device__ __forceinline__ void gemm_body(const void* __restrict__ A_, int lda,
                                          const T* __restrict__ Wt, int K,
                                          const float* __restrict__ bias,
                                          const float2* __restrict__ stats,
                                          const float* __restrict__ ln_g,
                                          const float* __restrict__ ln_s,
                                          void* __restrict__ C_, int ldc, int n_tiles,
                                          const OdeArgs& ode) {
  constexpr int BM = TL::BM, BN = TL::BN, BK = TL::BK, NT = TL::NT;
  constexpr int TM = TL::TM, TN = TL::TN;
  using AT = typename std::conditional<LN, float, T>::type;
  constexpr int LDK = BK + LdsPad<T>::v;
  constexpr int A_ELEMS = 16 / sizeof(AT);           // elements per 16-byte chunk of A
  constexpr int A_CPR = BK / A_ELEMS;                // chunks per A row slice
  constexpr int A_PER_T = BM * A_CPR / NT;
  constexpr int B_ELEMS = 16 / sizeof(T);
  constexpr int B_CPR = BK / B_ELEMS;
  constexpr int B_PER_T = BN * B_CPR / NT;
  static_assert(A_PER_T * NT == BM * A_CPR && B_PER_T * NT == BN * B_CPR, "staging split");

  __shared__ __attribute__((aligned(16))) T As[2][BM][LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][BN][LDK];
  __shared__ float sMean[LN ? BM : 1], sRstd[LN ? BM : 1];

  const AT* A = (const AT*)A_;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / TL::WN, wn = wave % TL::WN;
  const int logical = xcd_remap(blockIdx.x, gridDim.x);
  const int mt = logical / n_tiles, nt = logical % n_tiles;
  const int64_t m0 = (int64_t)mt * BM;
  const int n0 = nt * BN;

  if constexpr (LN) {
    for (int i = tid; i < BM; i += NT) {
      const float2 st = stats[m0 + i];
      sMean[i] = st.x;
      sRstd[i] = st.y;
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

  f32x16 acc[TM][TN];
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int nj = 0; nj < TN; ++nj)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mi][nj][r] = 0.f;

  const int nk = K / BK;
  FMD_LOAD_TILES(0);
  FMD_STORE_TILES(0, 0);
  __syncthreads();

  const int arow = wm * TL::WTM + (lane & 31);
  const int brow = wn * TL::WTN + (lane & 31);
  const int half = lane >> 5;

  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    const bool more = kt + 1 < nk;
    if (more) { FMD_LOAD_TILES((kt + 1) * BK); }
    if constexpr (std::is_same<T, bf16>::value) {
#pragma unroll
      for (int ks = 0; ks < BK / 16; ++ks) {
        bf16x8 a[TM], b[TN];
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
          a[mi] = *(const bf16x8*)&As[buf][arow + mi * 32][ks * 16 + half * 8];
#pragma unroll
        for (int nj = 0; nj < TN; ++nj)
          b[nj] = *(const bf16x8*)&Bs[buf][brow + nj * 32][ks * 16 + half * 8];
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int nj = 0; nj < TN; ++nj)
            acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b[nj], acc[mi][nj], 0, 0, 0);
      }
    } else {
      // lane half h supplies k = h*16 + m to MFMA m (m < 16) of each 32-wide slice
#pragma unroll
      for (int ks = 0; ks < BK / 32; ++ks) {
        float4 a[TM][4], b[TN][4];
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            a[mi][q] = *(const float4*)&As[buf][arow + mi * 32][ks * 32 + half * 16 + q * 4];
#pragma unroll
        for (int nj = 0; nj < TN; ++nj)
#pragma unroll
          for (int q = 0; q < 4; ++q)
            b[nj][q] = *(const float4*)&Bs[buf][brow + nj * 32][ks * 32 + half * 16 + q * 4];
#pragma unroll
        for (int m = 0; m < 16; ++m) {
#pragma unroll
          for (int mi = 0; mi < TM; ++mi) {
            const float av = a[mi][m >> 2][m & 3];
#pragma unroll
            for (int nj = 0; nj < TN; ++nj)
              acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x2f32(av, b[nj][m >> 2][m & 3],
                                                                 acc[mi][nj], 0, 0, 0);
          }
        }
      }
    }
    if (more) { FMD_STORE_TILES(buf ^ 1, (kt + 1) * BK); }
    __syncthreads();
  }

#undef FMD_LOAD_TILES
#undef FMD_STORE_TILES

  // epilogue
  if constexpr (EPI == EPI_RESID || EPI == EPI_RESID_LN) {
    // per 32-row block, read the residual values first: the stores may alias later loads;
    // the new values stay in acc for the statistics below
    float* C = (float*)C_;
#pragma unroll
    for (int mi = 0; mi < TM; ++mi) {
      float old[TN][16];
#pragma unroll
      for (int nj = 0; nj < TN; ++nj) {
        const int col = n0 + wn * TL::WTN + nj * 32 + (lane & 31);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * TL::WTM + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          old[nj][r] = C[row * ldc + col];
        }
      }
#pragma unroll
      for (int nj = 0; nj < TN; ++nj) {
        const int col = n0 + wn * TL::WTN + nj * 32 + (lane & 31);
        const float bv = bias ? bias[col] : 0.f;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * TL::WTM + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          const float nv = old[nj][r] + (acc[mi][nj][r] + bv);
          acc[mi][nj][r] = nv;
          C[row * ldc + col] = nv;
        }
      }
    }
    if constexpr (EPI == EPI_RESID_LN) {
      // LayerNorm statistics of the block's full rows (BN == N): per-wave partial sums by a
      // transpose-reduction over the lanes, then across the WN column waves through LDS;
      // two passes (mean, then squared deviations).
      static_assert(TM % 2 == 0, "row statistics take 32-row groups per lane half");
      __shared__ float red[TL::WN][BM];
      __shared__ float srow[BM];
      const int nn = n_tiles * BN;   // = N: the launcher checks n_tiles == 1
      // row (within the block) of transposed slot j of group g for this lane
      auto row_of = [&](int g, int j) {
        const int mi = 2 * g + (j >> 4), r = j & 15;
        return wm * TL::WTM + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
      };
#pragma unroll
      for (int pass = 0; pass < 2; ++pass) {
#pragma unroll
        for (int g = 0; g < TM / 2; ++g) {
          float v[32];
#pragma unroll
          for (int j = 0; j < 32; ++j) {
            const int mi = 2 * g + (j >> 4), r = j & 15;
            float s = 0.f;
            if (pass == 0) {
#pragma unroll
              for (int nj = 0; nj < TN; ++nj) s += acc[mi][nj][r];
            } else {
              const float mu = srow[row_of(g, j)];
#pragma unroll
              for (int nj = 0; nj < TN; ++nj) {
                const float dv = acc[mi][nj][r] - mu;
                s = fmaf(dv, dv, s);
              }
            }
            v[j] = s;
          }
          transpose_reduce32(v, lane);
          red[wn][row_of(g, lane & 31)] = v[0];
        }
        __syncthreads();
        for (int i = tid; i < BM; i += NT) {
          float t = 0.f;
#pragma unroll
          for (int q = 0; q < TL::WN; ++q) t += red[q][i];
          if (pass == 0) {
            srow[i] = t / nn;
          } else {
            ode.stats_out[m0 + i] = make_float2(srow[i], rsqrtf(t / nn + kLnEps));
          }
        }
        __syncthreads();
      }
    }
  } else {
    int mode = ode.mode;
    float h = ode.h;
    float* out = ode.out;
    if constexpr (EPI == EPI_ODE) {
      if (ode.desc && !ode.tok_event) {
        const StageDesc sd = ode.desc[*ode.ctr];
        mode = sd.mode;
        h = sd.h;
        if (!sd.write_out) out = nullptr;
      }
    }
#pragma unroll
    for (int nj = 0; nj < TN; ++nj) {
      const int col = n0 + wn * TL::WTN + nj * 32 + (lane & 31);
      const float bv = bias ? bias[col] : 0.f;
#pragma unroll
      for (int mi = 0; mi < TM; ++mi) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t row = m0 + wm * TL::WTM + mi * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
          const float v = acc[mi][nj][r] + bv;
          if constexpr (EPI == EPI_ODE) {
            if (col < ode.nf && row < ode.m_valid) {
              const int64_t o = row * ode.ldx + col;
              if (ode.tok_event) {
                const StageDesc sd = ode.desc[ode.tok_event[row]];
                ode_update(sd.mode, sd.h, v, ode.x + o, ode.acc + o, ode.xs + o,
                           out && sd.write_out ? out + row * ode.ldo + col : nullptr);
              } else {
                ode_update(mode, h, v, ode.x + o, ode.acc + o, ode.xs + o,
                           out ? out + row * ode.ldo + col : nullptr);
              }
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

// Candidate tilings (index = tile id in the tuning table).
#define FMD_GEMM_TILES(X)   \
  X(0, 128, 128, 32, 2, 2)  \
  X(1, 128, 128, 64, 2, 2)  \
  X(2, 256, 128, 32, 4, 2)  \
  X(3, 128, 256, 32, 2, 4)  \
  X(4, 128, 64, 32, 2, 2)   \
  X(5, 128, 128, 32, 1, 2)  \
  X(6, 256, 256, 32, 2, 2)
constexpr int kNumTiles = 7;

struct TileDims { int BM, BN, BK, threads, TM; };   // TM: 32-row blocks per wave
__host__ __device__ constexpr TileDims tile_dims(int id) {
  return id == 0 ? TileDims{128, 128, 32, 256, 2} : id == 1 ? TileDims{128, 128, 64, 256, 2}
       : id == 2 ? TileDims{256, 128, 32, 512, 2} : id == 3 ? TileDims{128, 256, 32, 512, 2}
       : id == 4 ? TileDims{128, 64, 32, 256, 2}  : id == 5 ? TileDims{128, 128, 32, 128, 4}
       : TileDims{256, 256, 32, 256, 4};
}

// Per-T launcher over (class, LN, epilogue, tile); defined in gemm_f32.hip / gemm_bf16.hip.
template <typename T>
hipError_t launch_gemm_tile(hipStream_t st, int tile, int cls, bool ln, int epi, int64_t Mp,
                            int N, int K, const void* A, int lda, const T* Wt,
                            const float* bias, const float2* stats, const float* g,
                            const float* s, void* C, int ldc, const OdeArgs& ode);

}  // namespace fmd
