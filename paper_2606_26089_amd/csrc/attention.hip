// Masked multi-head attention over ragged CSR events on gfx950 matrix cores.
//
// Each workgroup takes one (event, 64-query tile) work item for one head. Each of its four
// waves owns 16 queries. Keys and values of the event stream through LDS in chunks of 64
// keys, with an online (running max / running sum) softmax. Keys of other events are
// never touched. Slots past the end of the event are excluded by a select before the
// exponential, and their K and V rows are zero-filled in LDS, so garbage cannot reach
// the result.
//
// The scores are formed transposed, S^T = K Q^T, on 16 x 16 MFMA tiles. Lane l then
// holds query l%16 and keys 4(l/16) + r, so a query's statistics need only two
// cross-lane exchanges (xor 16, xor 32). Those registers are already the B operand of
// O^T = V^T P^T. The MFMA contracts over slot positions, and V^T is read from LDS with
// the same key-to-slot assignment.
//   FP32: v_mfma_f32_16x16x4_f32 (one k per lane; lane group g = l/16 holds k = g)
//   BF16: v_mfma_f32_16x16x32_bf16 (8 consecutive k per lane group), or 16x16x16 for dh 16
// Accumulator layout: lane l, register r holds row 4(l/16) + r, column l%16.
#include "common.h"
#include "kernels.h"

namespace fmd {

constexpr int KC = 64;   // keys per LDS chunk
constexpr int QT = 64;   // queries per workgroup (4 waves x 16)

template <typename T> struct AttnPad { static constexpr int v = 4; };
template <> struct AttnPad<bf16> { static constexpr int v = 8; };

template <typename T, int DH>
__device__ __forceinline__ void attention_body(
    const T* __restrict__ Q, int ldq, const T* __restrict__ Kp, const T* __restrict__ Vp,
    int ldkv, T* __restrict__ O, int ldo, const int64_t* __restrict__ q_off,
    const int64_t* __restrict__ kv_off, const int2* __restrict__ work, float scale_log2e) {
  constexpr bool BF = sizeof(T) == 2;
  constexpr int PAD = AttnPad<T>::v;
  constexpr int DB = DH / 16;                 // 16-wide output blocks along dh
  constexpr int CH = 16 / sizeof(T);          // elements per 16-byte chunk
  constexpr int CPR = DH / CH;                // chunks per K/V row
  __shared__ __attribute__((aligned(16))) T Ks[KC][DH + PAD];
  __shared__ __attribute__((aligned(16))) T Vt[DH][KC + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, j = lane & 15;
  const int2 wk = work[blockIdx.x];
  const int e = wk.x, h = blockIdx.y;
  const int64_t qs = q_off[e], ks = kv_off[e];
  const int nq = (int)(q_off[e + 1] - qs), nk = (int)(kv_off[e + 1] - ks);
  const int qbase = wk.y * QT + wave * 16;
  const bool wave_active = qbase < nq;
  const int qi = qbase + j;
  const bool qvalid = qi < nq;
  const T* qrow = Q + (qs + (qvalid ? qi : 0)) * ldq + h * DH;

  // Q fragment (B operand of S^T = K Q^T).
  constexpr int QN = BF ? (DH == 16 ? 4 : 8 * (DH / 32)) : DH / 4;
  float qf32[BF ? 1 : QN];
  bf16x8 qb[BF && DH >= 32 ? DH / 32 : 1];
  bf16x4 qb4;
  if constexpr (BF) {
    if constexpr (DH == 16) {
      qb4 = *(const bf16x4*)(qrow + 4 * g);
      if (!qvalid) for (int i = 0; i < 4; ++i) qb4[i] = (bf16)0.f;
    } else {
#pragma unroll
      for (int m = 0; m < DH / 32; ++m) {
        qb[m] = *(const bf16x8*)(qrow + 32 * m + 8 * g);
        if (!qvalid) for (int i = 0; i < 8; ++i) qb[m][i] = (bf16)0.f;
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < QN; ++m) qf32[m] = qvalid ? to_f32(qrow[g * QN + m]) : 0.f;
  }

  float m_run = -INFINITY, l_run = 0.f;
  f32x4 o[DB];
#pragma unroll
  for (int b = 0; b < DB; ++b) o[b] = f32x4{0.f, 0.f, 0.f, 0.f};

  for (int c0 = 0; c0 < nk; c0 += KC) {
    // stage K rows and V^T columns of keys c0 .. c0 + 63
    for (int idx = tid; idx < KC * CPR; idx += 256) {
      const int row = idx / CPR, ch = idx % CPR;
      u32x4 kv = {0u, 0u, 0u, 0u}, vv = {0u, 0u, 0u, 0u};
      if (c0 + row < nk) {
        const int64_t gr = (ks + c0 + row) * ldkv + h * DH + ch * CH;
        kv = *(const u32x4*)(Kp + gr);
        vv = *(const u32x4*)(Vp + gr);
      }
      *(u32x4*)&Ks[row][ch * CH] = kv;
      const T* vp = (const T*)&vv;
#pragma unroll
      for (int i = 0; i < CH; ++i) Vt[ch * CH + i][row] = vp[i];
    }
    __syncthreads();
    if (wave_active) {
      f32x4 s[4];
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        s[kb] = f32x4{0.f, 0.f, 0.f, 0.f};
        const T* krow = &Ks[kb * 16 + j][0];
        if constexpr (BF) {
          if constexpr (DH == 16) {
            const bf16x4 ka = *(const bf16x4*)(krow + 4 * g);
            s[kb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ka, qb4, s[kb], 0, 0, 0);
          } else {
#pragma unroll
            for (int m = 0; m < DH / 32; ++m) {
              const bf16x8 ka = *(const bf16x8*)(krow + 32 * m + 8 * g);
              s[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ka, qb[m], s[kb], 0, 0, 0);
            }
          }
        } else {
#pragma unroll
          for (int m = 0; m < QN; ++m)
            s[kb] = __builtin_amdgcn_mfma_f32_16x16x4f32(to_f32(krow[g * QN + m]), qf32[m],
                                                         s[kb], 0, 0, 0);
        }
      }
      float cmax = -INFINITY;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int key = c0 + kb * 16 + 4 * g + r;
          const float v = key < nk ? s[kb][r] * scale_log2e : -INFINITY;
          s[kb][r] = v;
          cmax = fmaxf(cmax, v);
        }
      cmax = fmaxf(cmax, __shfl_xor(cmax, 16, kWave));
      cmax = fmaxf(cmax, __shfl_xor(cmax, 32, kWave));
      const float m_new = fmaxf(m_run, cmax);      // finite: key c0 < nk is in this chunk
      const float alpha = exp2f(m_run - m_new);
      l_run *= alpha;
#pragma unroll
      for (int b = 0; b < DB; ++b) o[b] *= alpha;
#pragma unroll
      for (int kb = 0; kb < 4; ++kb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float p = exp2f(s[kb][r] - m_new);
          s[kb][r] = p;
          l_run += p;
        }
      m_run = m_new;
      // O^T += V^T P^T
      if constexpr (BF) {
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          bf16x8 pb;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            pb[r] = (bf16)s[2 * c][r];
            pb[4 + r] = (bf16)s[2 * c + 1][r];
          }
#pragma unroll
          for (int b = 0; b < DB; ++b) {
            const T* vrow = &Vt[b * 16 + j][0];
            const bf16x4 lo = *(const bf16x4*)(vrow + 32 * c + 4 * g);
            const bf16x4 hi = *(const bf16x4*)(vrow + 32 * c + 16 + 4 * g);
            bf16x8 va;
#pragma unroll
            for (int r = 0; r < 4; ++r) { va[r] = lo[r]; va[4 + r] = hi[r]; }
            o[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, pb, o[b], 0, 0, 0);
          }
        }
      } else {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
#pragma unroll
          for (int b = 0; b < DB; ++b) {
            const float4 va = *(const float4*)&Vt[b * 16 + j][kb * 16 + 4 * g];
            o[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.x, s[kb][0], o[b], 0, 0, 0);
            o[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.y, s[kb][1], o[b], 0, 0, 0);
            o[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.z, s[kb][2], o[b], 0, 0, 0);
            o[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(va.w, s[kb][3], o[b], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  if (wave_active) {
    float l = l_run + __shfl_xor(l_run, 16, kWave);
    l += __shfl_xor(l, 32, kWave);
    const float inv = 1.0f / l;
    if (qvalid) {
      T* orow = O + (qs + qi) * ldo + h * DH;
#pragma unroll
      for (int b = 0; b < DB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) orow[b * 16 + 4 * g + r] = from_f32<T>(o[b][r] * inv);
    }
  }
}

// Separate kernel names for self- and cross-attention so that profiles separate them.
#define FMD_ATTN_KERNEL(NAME)                                                                 \
  template <typename T, int DH>                                                               \
  __global__ __launch_bounds__(256) void NAME(                                                \
      const T* __restrict__ Q, int ldq, const T* __restrict__ K, const T* __restrict__ V,     \
      int ldkv, T* __restrict__ O, int ldo, const int64_t* __restrict__ q_off,                \
      const int64_t* __restrict__ kv_off, const int2* __restrict__ work, float sl2e) {        \
    attention_body<T, DH>(Q, ldq, K, V, ldkv, O, ldo, q_off, kv_off, work, sl2e);             \
  }
FMD_ATTN_KERNEL(k_attn_self)
FMD_ATTN_KERNEL(k_attn_cross)
#undef FMD_ATTN_KERNEL

template <typename T, int DH>
static hipError_t go_attn(bool cross, dim3 grid, hipStream_t st, const T* Q, int ldq,
                          const T* K, const T* V, int ldkv, T* O, int ldo, const int64_t* q_off,
                          const int64_t* kv_off, const int2* work, float sl2e) {
  if (cross)
    hipLaunchKernelGGL((k_attn_cross<T, DH>), grid, dim3(256), 0, st, Q, ldq, K, V, ldkv, O, ldo,
                       q_off, kv_off, work, sl2e);
  else
    hipLaunchKernelGGL((k_attn_self<T, DH>), grid, dim3(256), 0, st, Q, ldq, K, V, ldkv, O, ldo,
                       q_off, kv_off, work, sl2e);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_attention(hipStream_t st, bool cross, int dh, int n_heads, int64_t n_items,
                            const int2* work, const T* Q, int ldq, const T* K, const T* V,
                            int ldkv, T* O, int ldo, const int64_t* q_off,
                            const int64_t* kv_off) {
  if (n_items <= 0) return hipSuccess;
  if (n_items > 0x7fffffff) return hipErrorInvalidValue;
  const float sl2e = 1.4426950408889634f / sqrtf((float)dh);
  const dim3 grid((unsigned)n_items, n_heads);
  switch (dh) {
    case 16: return go_attn<T, 16>(cross, grid, st, Q, ldq, K, V, ldkv, O, ldo, q_off, kv_off, work, sl2e);
    case 32: return go_attn<T, 32>(cross, grid, st, Q, ldq, K, V, ldkv, O, ldo, q_off, kv_off, work, sl2e);
    case 64: return go_attn<T, 64>(cross, grid, st, Q, ldq, K, V, ldkv, O, ldo, q_off, kv_off, work, sl2e);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_attention<float>(hipStream_t, bool, int, int, int64_t, const int2*,
                                            const float*, int, const float*, const float*, int,
                                            float*, int, const int64_t*, const int64_t*);
template hipError_t launch_attention<bf16>(hipStream_t, bool, int, int, int64_t, const int2*,
                                           const bf16*, int, const bf16*, const bf16*, int,
                                           bf16*, int, const int64_t*, const int64_t*);

}  // namespace fmd
