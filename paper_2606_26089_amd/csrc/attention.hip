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
#include <algorithm>
#include <vector>

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
    int ldkv, T* __restrict__ O, int ldo, const AttnItem* __restrict__ work,
    float scale_log2e) {
  constexpr bool BF = sizeof(T) == 2;
  constexpr int PAD = AttnPad<T>::v;
  constexpr int DB = DH / 16;                 // 16-wide output blocks along dh
  constexpr int CH = 16 / sizeof(T);          // elements per 16-byte chunk
  constexpr int CPR = DH / CH;                // chunks per K/V row
  __shared__ __attribute__((aligned(16))) T Ks[KC][DH + PAD];
  __shared__ __attribute__((aligned(16))) T Vt[DH][KC + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, j = lane & 15;
  const AttnItem wk = work[blockIdx.x];     // rows are those of the item's query tile
  const int h = blockIdx.y;
  const int64_t qs = wk.q0, ks = wk.k0;
  const int nq = wk.nq, nk = wk.nk;
  const int qbase = wave * 16;
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
      int ldkv, T* __restrict__ O, int ldo, const AttnItem* __restrict__ work, float sl2e) {  \
    attention_body<T, DH>(Q, ldq, K, V, ldkv, O, ldo, work, sl2e);                            \
  }
FMD_ATTN_KERNEL(k_attn_self)
FMD_ATTN_KERNEL(k_attn_cross)
#undef FMD_ATTN_KERNEL

// ---------------------------------------------------------------------------------------
// BF16 with heads of 32: the same work split as above (one head of one 64-query tile per
// workgroup, four waves of 16 queries), tuned for gfx950.
//  - Chunks of 128 keys: most events fit in one, so the load -> barrier -> compute round
//    trip is paid once. K rows are staged by waves 2-3 and V by waves 0-1, 4 loads each.
//    A last chunk of at most 96 keys is staged and computed for its first 32, 64 or 96 keys
//    only (a straight-line form for each, after the loop over full chunks).
//  - One-dimensional grid over (work item, head), heads fastest: the workgroups that read
//    the two halves of a K/V cache line run together, so the line is fetched once. (The
//    work list is sorted longest event first; dealing contiguous ranges of it to the XCDs
//    would load one XCD with all the long events.)
//  - V is staged transposed with packed 8-byte LDS stores (no two lanes write the same
//    dword) and with a key permutation inside each 32-key group (key 16 hi + 4 g + r at
//    position 8 g + 4 hi + r): the eight keys lane group g feeds to one MFMA are adjacent,
//    so each V^T operand is one 16-byte LDS read.
//  - The softmax runs on unscaled scores: one multiply-add forms the exp2 argument
//    (s - max) * scale, and the hardware exp2 is used (arguments <= 0). The row sums of P
//    come from the P V product itself, through a third 16-row block of V^T whose first row
//    is the key validity. Keys past the event end repeat its last key (clamped reads) and
//    have zero V and validity, so there is no per-score masking.
namespace {
constexpr int kH32 = 32;
constexpr int kKc2 = 128;           // keys per chunk
constexpr int kSchedMfma = 0x008;   // sched_group_barrier instruction classes: MFMA
constexpr int kSchedDsRead = 0x100; // LDS read
constexpr int kLdK32 = kH32 + 8;    // Ks pitch (bf16)
constexpr int kLdV32 = kKc2 + 8;    // Vt pitch (bf16)

__device__ __forceinline__ int vt_pos(int k) {
  const int grp = k >> 5, hi = (k >> 4) & 1, g = (k >> 2) & 3, r = k & 3;
  return grp * 32 + 8 * g + 4 * hi + r;
}
}  // namespace

// One staged chunk of KB key blocks of 16 for this wave's query tiles: the scores
// S^T = K Q^T, the online-softmax update of the running max and the output, and
// O^T += V^T P^T with the row sums of P from the validity row of V^T.
template <int TPW, int KB>
__device__ __forceinline__ void attn32_chunk(const bf16* __restrict__ Ks,
                                             const bf16* __restrict__ Vt,
                                             const bf16x8 (&qf)[TPW], float (&m_run)[TPW],
                                             f32x4 (&o)[TPW][3], int nq, int wave, int g, int j,
                                             float sl2e) {
  auto qbase = [&](int t) { return (t * 4 + wave) * 16; };
  // compiler-only barrier: the LDS reads (and so the products) of the forms of this
  // function are not merged and hoisted above the branches between them
  asm volatile("" ::: "memory");
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    if (qbase(t) >= nq) continue;   // wave-uniform
    // all KB key blocks, also past the event end: no branches, and the zero accumulator
    // is an inline constant
    f32x4 s[KB];
    {
      bf16x8 kf[KB];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) kf[kb] = *(const bf16x8*)&Ks[(kb * 16 + j) * kLdK32 + 8 * g];
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
        s[kb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kf[kb], qf[t], f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      // the K operand reads kept two ahead of their products (left alone, the compiler reads
      // each one right before its product into the same registers and waits for it)
      __builtin_amdgcn_sched_group_barrier(kSchedDsRead, 2, 0);
#pragma unroll
      for (int i = 0; i < KB - 2; ++i) {
        __builtin_amdgcn_sched_group_barrier(kSchedMfma, 1, 0);
        __builtin_amdgcn_sched_group_barrier(kSchedDsRead, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(kSchedMfma, 2, 0);
    }
    float cmax = -INFINITY;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int r = 0; r < 4; ++r) cmax = fmaxf(cmax, s[kb][r]);
    {   // max over lanes l, l ^ 16, then l, l ^ 32: a row swap and a half swap of the
        // register with itself, no LDS round trip (max is exact)
      const auto r16 = __builtin_amdgcn_permlane16_swap(__float_as_uint(cmax),
                                                        __float_as_uint(cmax), false, false);
      cmax = fmaxf(__uint_as_float(r16[0]), __uint_as_float(r16[1]));
      const auto r32 = __builtin_amdgcn_permlane32_swap(__float_as_uint(cmax),
                                                        __float_as_uint(cmax), false, false);
      cmax = fmaxf(__uint_as_float(r32[0]), __uint_as_float(r32[1]));
    }
    const float m_new = fmaxf(m_run[t], cmax);    // finite: key c0 < nk is in this chunk
    const float alpha = __builtin_amdgcn_exp2f((m_run[t] - m_new) * sl2e);
#pragma unroll
    for (int db = 0; db < 3; ++db) o[t][db] *= alpha;
    const float mb = -m_new * sl2e;
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
      for (int r = 0; r < 4; ++r) s[kb][r] = __builtin_amdgcn_exp2f(fmaf(s[kb][r], sl2e, mb));
    m_run[t] = m_new;
#pragma unroll
    for (int c = 0; c < KB / 2; ++c) {
      bf16x8 pb;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        pb[r] = (bf16)s[2 * c][r];
        pb[4 + r] = (bf16)s[2 * c + 1][r];
      }
#pragma unroll
      for (int db = 0; db < 2; ++db) {
        const bf16x8 vf = *(const bf16x8*)&Vt[(db * 16 + j) * kLdV32 + 32 * c + 8 * g];
        o[t][db] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vf, pb, o[t][db], 0, 0, 0);
      }
      const bf16x8 vld = *(const bf16x8*)&Vt[(kH32 + j) * kLdV32 + 32 * c + 8 * g];
      o[t][2] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(vld, pb, o[t][2], 0, 0, 0);
    }
  }
}

// Stages keys c0 .. c0 + 16 KB - 1 of the event into Ks and V^T.
template <int KB>
__device__ __forceinline__ void attn32_stage(bf16* __restrict__ Ks, bf16* __restrict__ Vt,
                                             const bf16* __restrict__ Kp,
                                             const bf16* __restrict__ Vp, int ldkv, int64_t hskv,
                                             int64_t ks0, int c0, int nk, int h, int tid,
                                             int wave) {
  // Keys past the event end are read clamped to its last key: their scores repeat a real
  // score (the running max is unchanged), and their V rows and validity are zero, so they
  // add nothing to P V or to the row sums. No per-score masking is needed.
  const int lim = nk - 1 - c0;
  if (wave >= 2) {   // K: 16 KB keys x 4 chunks of 16 bytes
    const char* kc = (const char*)(Kp + (ks0 + c0) * ldkv + h * hskv);
    const int t2 = tid - 128;
    u32x4 v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = t2 + i * 128, row = idx >> 2, ch = idx & 3;
      if (i < KB / 2) v[i] = *(const u32x4*)(kc + (uint32_t)((min(row, lim) * ldkv + ch * 8) * 2));
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int idx = t2 + i * 128, row = idx >> 2, ch = idx & 3;
      if (i < KB / 2) *(u32x4*)&Ks[row * kLdK32 + ch * 8] = v[i];
    }
  } else if ((tid & 31) < 4 * KB) {   // V^T: thread = (4 consecutive keys, 8 dims)
    const char* vc = (const char*)(Vp + (ks0 + c0) * ldkv + h * hskv);
    const int kg = tid & 31, dg = tid >> 5;
    u32x4 v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int key = kg * 4 + r;
      v[r] = *(const u32x4*)(vc + (uint32_t)((min(key, lim) * ldkv + dg * 8) * 2));
      if (key > lim) v[r] = u32x4{0u, 0u, 0u, 0u};
    }
    const int pos = vt_pos(kg * 4);
    if (dg == 0) {
      bf16x4 valid;
#pragma unroll
      for (int r = 0; r < 4; ++r) valid[r] = (bf16)(kg * 4 + r <= lim ? 1.f : 0.f);
      *(bf16x4*)&Vt[kH32 * kLdV32 + pos] = valid;
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      bf16x4 w4;
#pragma unroll
      for (int r = 0; r < 4; ++r) w4[r] = __builtin_bit_cast(bf16x8, v[r])[i];
      *(bf16x4*)&Vt[(dg * 8 + i) * kLdV32 + pos] = w4;
    }
  }
}

template <int TPW>
__device__ __forceinline__ void attention32_body(
    const bf16* __restrict__ Q, int ldq, int64_t hsq, const bf16* __restrict__ Kp,
    const bf16* __restrict__ Vp, int ldkv, int64_t hskv, bf16* __restrict__ O, int ldo,
    int64_t hso, const AttnItem* __restrict__ work, const AttnBins& bins, int n_heads, float sl2e) {
  __shared__ __attribute__((aligned(16))) bf16 Ks[kKc2 * kLdK32];
  // V^T rows 0-31; row 32 = key validity (1 for a key of the event, 0 past its end), rows
  // 33-47 = 0: the A operand of the row-sum block of P V
  __shared__ __attribute__((aligned(16))) bf16 Vt[(kH32 + 16) * kLdV32];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int g = lane >> 4, j = lane & 15;
  for (int i = tid; i < 15 * kLdV32; i += 256) Vt[(kH32 + 1) * kLdV32 + i] = (bf16)0.f;
  // workgroup b: bin b % kAttnBins (so one XCD), unit k = b / kAttnBins of that bin
  const int bin = blockIdx.x % kAttnBins, k = blockIdx.x / kAttnBins;
  const int item = k / n_heads;
  if (item >= bins.len[bin]) return;     // the bin is shorter than the longest one
  // the item carries its rows: no dependent loads of event offsets before the data loads
  const AttnItem wk = work[bins.start[bin] + item];
  const int h = k % n_heads;
  const int64_t qs0 = wk.q0, ks0 = wk.k0;
  const int nq = wk.nq, nk = wk.nk;
  // query tile t of this wave (16 queries): tiles are dealt to the waves round-robin
  auto qbase = [&](int t) { return (t * 4 + wave) * 16; };

  bf16x8 qf[TPW];
  float m_run[TPW];
  // o[t][0], o[t][1]: output dims 0-15, 16-31; o[t][2] row 0 (lanes 0-15, register 0): sum of P
  f32x4 o[TPW][3];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int qi = qbase(t) + j;
    const char* qc = (const char*)(Q + qs0 * ldq + h * hsq);
    u32x4 v = *(const u32x4*)(qc + (uint32_t)((min(qi, nq - 1) * ldq + 8 * g) * 2));
    if (qi >= nq) v = u32x4{0u, 0u, 0u, 0u};
    qf[t] = __builtin_bit_cast(bf16x8, v);
    m_run[t] = -INFINITY;
#pragma unroll
    for (int db = 0; db < 3; ++db) o[t][db] = f32x4{0.f, 0.f, 0.f, 0.f};
  }

  // A last chunk of at most 96 keys is staged and computed for its first 32, 64 or 96 keys
  // only: the rest are all past the event end (their scores repeat a real score, their
  // P V and row-sum terms are exact zeros), so the results are the same.
  const int last = (nk - 1) & (kKc2 - 1);           // last key's position in its chunk
  const int nfull = last < 96 ? nk - 1 - last : nk;  // keys before the shortened last chunk
  for (int c0 = 0; c0 < nfull; c0 += kKc2) {
    attn32_stage<8>(Ks, Vt, Kp, Vp, ldkv, hskv, ks0, c0, nk, h, tid, wave);
    __syncthreads();
    attn32_chunk<TPW, 8>(Ks, Vt, qf, m_run, o, nq, wave, g, j, sl2e);
    __syncthreads();
  }
  const int rest = nk - nfull;   // 0 .. 96, wave-uniform
  if (rest > 64) {
    attn32_stage<6>(Ks, Vt, Kp, Vp, ldkv, hskv, ks0, nfull, nk, h, tid, wave);
    __syncthreads();
    attn32_chunk<TPW, 6>(Ks, Vt, qf, m_run, o, nq, wave, g, j, sl2e);
  } else if (rest > 32) {
    attn32_stage<4>(Ks, Vt, Kp, Vp, ldkv, hskv, ks0, nfull, nk, h, tid, wave);
    __syncthreads();
    attn32_chunk<TPW, 4>(Ks, Vt, qf, m_run, o, nq, wave, g, j, sl2e);
  } else if (rest > 0) {
    attn32_stage<2>(Ks, Vt, Kp, Vp, ldkv, hskv, ks0, nfull, nk, h, tid, wave);
    __syncthreads();
    attn32_chunk<TPW, 2>(Ks, Vt, qf, m_run, o, nq, wave, g, j, sl2e);
  }

#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    const int qi = qbase(t) + j;
    if (qbase(t) >= nq) continue;
    // row 0 of the row-sum block sits in register 0 of lanes 0-15 (query j)
    const float l = __shfl(o[t][2][0], j, kWave);
    const float inv = 1.0f / l;
    if (qi < nq) {
      bf16* orow = O + (qs0 + qi) * ldo + h * hso;
#pragma unroll
      for (int db = 0; db < 2; ++db) {
        bf16x4 w4;
#pragma unroll
        for (int r = 0; r < 4; ++r) w4[r] = (bf16)(o[t][db][r] * inv);
        *(bf16x4*)(orow + db * 16 + 4 * g) = w4;
      }
    }
  }
}

template <int TPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_attn32_self(
    const bf16* __restrict__ Q, int ldq, int64_t hsq, const bf16* __restrict__ K,
    const bf16* __restrict__ V, int ldkv, int64_t hskv, bf16* __restrict__ O, int ldo,
    int64_t hso, const AttnItem* __restrict__ work, AttnBins bins, int n_heads, float sl2e) {
  attention32_body<TPW>(Q, ldq, hsq, K, V, ldkv, hskv, O, ldo, hso, work, bins, n_heads, sl2e);
}
template <int TPW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_attn32_cross(
    const bf16* __restrict__ Q, int ldq, int64_t hsq, const bf16* __restrict__ K,
    const bf16* __restrict__ V, int ldkv, int64_t hskv, bf16* __restrict__ O, int ldo,
    int64_t hso, const AttnItem* __restrict__ work, AttnBins bins, int n_heads, float sl2e) {
  attention32_body<TPW>(Q, ldq, hsq, K, V, ldkv, hskv, O, ldo, hso, work, bins, n_heads, sl2e);
}


template <typename T, int DH>
static hipError_t go_attn(bool cross, dim3 grid, hipStream_t st, const T* Q, int ldq,
                          const T* K, const T* V, int ldkv, T* O, int ldo,
                          const AttnItem* work, float sl2e) {
  if (cross)
    hipLaunchKernelGGL((k_attn_cross<T, DH>), grid, dim3(256), 0, st, Q, ldq, K, V, ldkv, O, ldo,
                       work, sl2e);
  else
    hipLaunchKernelGGL((k_attn_self<T, DH>), grid, dim3(256), 0, st, Q, ldq, K, V, ldkv, O, ldo,
                       work, sl2e);
  return hipGetLastError();
}

namespace {
// The builder over accessors: queries of event k at q_off[ids[k]], nq(k) rows; its keys at
// k0(k), nk(k) rows.
template <typename Nq, typename K0, typename Nk>
int64_t build_work(const int64_t* q_off, const int64_t* ids, int64_t n, int qt, Nq nq, K0 k0,
                   Nk nk, AttnItem* items, AttnBins* bins) {
  // longest-processing-time assignment of whole events to bins; cost = query tiles x keys
  std::vector<int64_t> order;
  order.reserve((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    if (nq(k) <= 0) continue;
    if (q_off[ids[k]] + nq(k) > INT32_MAX || k0(k) + nk(k) > INT32_MAX) return -1;
    order.push_back(k);
  }
  auto tiles = [&](int64_t k) { return (nq(k) + qt - 1) / qt; };
  auto cost = [&](int64_t k) { return tiles(k) * nk(k); };
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return cost(a) > cost(b); });
  std::vector<int> bin_of(order.size());
  int64_t load[kAttnBins] = {0};
  int64_t cnt[kAttnBins] = {0};
  for (size_t i = 0; i < order.size(); ++i) {
    int best = 0;
    for (int b = 1; b < kAttnBins; ++b)
      if (load[b] < load[best]) best = b;
    bin_of[i] = best;
    load[best] += cost(order[i]);
    cnt[best] += tiles(order[i]);
  }
  int64_t pos = 0;
  bins->max_len = 0;
  for (int b = 0; b < kAttnBins; ++b) {
    bins->start[b] = (int32_t)pos;
    bins->len[b] = (int32_t)cnt[b];
    bins->max_len = std::max<int32_t>(bins->max_len, (int32_t)cnt[b]);
    for (size_t i = 0; i < order.size(); ++i) {
      if (bin_of[i] != b) continue;
      const int64_t k = order[i], e = ids[k];
      for (int64_t q = 0; q < tiles(k); ++q)
        items[pos++] = AttnItem{(int32_t)(q_off[e] + q * qt),
                                (int32_t)std::min<int64_t>(qt, nq(k) - q * qt),
                                (int32_t)k0(k), (int32_t)nk(k)};
    }
  }
  return pos;
}
}  // namespace

int64_t build_attention_work(const int64_t* q_off, const int64_t* kv_off, const int64_t* ids,
                             int64_t n, int qt, AttnItem* items, AttnBins* bins) {
  return build_work(
      q_off, ids, n, qt, [&](int64_t k) { return q_off[ids[k] + 1] - q_off[ids[k]]; },
      [&](int64_t k) { return kv_off[ids[k]]; },
      [&](int64_t k) { return kv_off[ids[k] + 1] - kv_off[ids[k]]; }, items, bins);
}

int64_t build_attention_work_kv(const int64_t* q_off, const int64_t* kv_start,
                                const int64_t* kv_len, const int64_t* ids, int64_t n, int qt,
                                AttnItem* items, AttnBins* bins) {
  return build_work(
      q_off, ids, n, qt, [&](int64_t k) { return q_off[ids[k] + 1] - q_off[ids[k]]; },
      [&](int64_t k) { return kv_start[ids[k]]; }, [&](int64_t k) { return kv_len[ids[k]]; },
      items, bins);
}

int attention_query_tile(bool bf16, int dh, int n_heads) {
  (void)n_heads;
  return bf16 && dh == kH32 ? 128 : QT;
}

int attention_query_tiles(bool bf16, int dh, int* tiles) {
  if (bf16 && dh == kH32) {
    tiles[0] = 64;    // one 16-query tile per wave
    tiles[1] = 128;   // two
    tiles[2] = 192;   // three: events of up to 192 slots in one item (one workgroup per head)
    return 3;
  }
  tiles[0] = QT;
  return 1;
}

template <typename T>
hipError_t launch_attention(hipStream_t st, bool cross, int dh, int n_heads, int qt,
                            int64_t n_items, const AttnBins& bins, const AttnItem* work, const T* Q, int ldq,
                            int64_t hsq, const T* K, const T* V, int ldkv, int64_t hskv, T* O,
                            int ldo, int64_t hso) {
  if (n_items <= 0) return hipSuccess;
  if (n_items > 0x7fffffff) return hipErrorInvalidValue;
  const float sl2e = 1.4426950408889634f / sqrtf((float)dh);
  if constexpr (std::is_same<T, bf16>::value) {
    if (dh == kH32) {
      // 16-byte row chunks: row pitches and head offsets are multiples of 8 elements
      if (ldq % 8 || ldkv % 8 || ldo % 4 || hsq % 8 || hskv % 8 || hso % 4 || hsq < dh ||
          hskv < dh || hso < dh)
        return hipErrorInvalidValue;
      const int64_t blocks = (int64_t)kAttnBins * bins.max_len * n_heads;
      if (blocks > 0x7fffffff) return hipErrorInvalidValue;
      if (blocks == 0) return hipSuccess;
#define FMD_ATTN32_GO(TPW)                                                                     \
  do {                                                                                          \
    if (cross)                                                                                  \
      hipLaunchKernelGGL((k_attn32_cross<TPW>), dim3((unsigned)blocks), dim3(256), 0, st, Q,     \
                         ldq, hsq, K, V, ldkv, hskv, O, ldo, hso, work, bins, n_heads, sl2e);   \
    else                                                                                        \
      hipLaunchKernelGGL((k_attn32_self<TPW>), dim3((unsigned)blocks), dim3(256), 0, st, Q,      \
                         ldq, hsq, K, V, ldkv, hskv, O, ldo, hso, work, bins, n_heads, sl2e);   \
  } while (0)
      if (qt == 64)
        FMD_ATTN32_GO(1);
      else if (qt == 128)
        FMD_ATTN32_GO(2);
      else if (qt == 192)
        FMD_ATTN32_GO(3);
      else
        return hipErrorInvalidValue;
#undef FMD_ATTN32_GO
      return hipGetLastError();
    }
  }
  // the general kernel takes row-major operands only, in work items of QT queries
  if (hsq != dh || hskv != dh || hso != dh || qt != QT) return hipErrorInvalidValue;
  const dim3 grid((unsigned)n_items, n_heads);
  switch (dh) {
    case 16: return go_attn<T, 16>(cross, grid, st, Q, ldq, K, V, ldkv, O, ldo, work, sl2e);
    case 32: return go_attn<T, 32>(cross, grid, st, Q, ldq, K, V, ldkv, O, ldo, work, sl2e);
    case 64: return go_attn<T, 64>(cross, grid, st, Q, ldq, K, V, ldkv, O, ldo, work, sl2e);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_attention<float>(hipStream_t, bool, int, int, int, int64_t,
                                            const AttnBins&, const AttnItem*, const float*, int,
                                            int64_t, const float*, const float*, int, int64_t,
                                            float*, int, int64_t);
template hipError_t launch_attention<bf16>(hipStream_t, bool, int, int, int, int64_t,
                                           const AttnBins&, const AttnItem*, const bf16*, int,
                                           int64_t, const bf16*, const bf16*, int, int64_t,
                                           bf16*, int, int64_t);

}  // namespace fmd
