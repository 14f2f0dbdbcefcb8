// Fused BF16 kernels of one transformer block of the velocity network, written for model
// width d = 256 with 8 heads of 32 on gfx950. The paper's flow-matching model (Sec. 2.2) is
// conditioned on the event's truth particles and leaves its architecture to the works it
// cites; the block here is the stand-in read from that: a pre-LayerNorm block of
// self-attention over the reco slots, cross-attention to the truth encoding and a 4x GELU MLP.
//
// The rows' FP32 residual values live in registers for the whole kernel, as a full-width
// accumulator in the 32x32 MFMA output layout (lane l, register r of fragment mi: row
// 32 mi + 8 (r/4) + 4 (l/32) + r%4, column l%32). k_fused_qkv and k_fused_oqc take 64 rows
// with 8 waves, wave w holding columns [32w, 32w + 32); k_fused_mlp takes 64 rows with 4
// waves, wave w holding columns [64w, 64w + 64), so that two of its workgroups share a CU
// and overlap each other's barriers and memory phases. The A operands of the products (an
// attention output tile, the LayerNorm of the residual rows, an MLP hidden chunk) sit in
// LDS; the weights stream from L2 as pre-packed MFMA B fragments, 8 in flight per wave, with
// no LDS staging. LayerNorm statistics are computed inside the kernel from the full rows
// (two passes: mean, then squared deviations).
//
//   k_fused_qkv  LN1(H) -> [Q|K|V]
//   k_fused_oqc  H += att W_o + b_o;  qc = LN2(H) W_qc + b_qc
//   k_fused_mlp  H += att_c W_oc + b_oc;  H += GELU(LN3(H) W_up + b_up) W_dn + b_dn,
//                with the LayerNorm statistics of the final rows written for the next LN
//
// Weight fragment layout (k_pack_frag): for a K x N matrix W, fragment (nb, ks) of lane l
// holds W[16 ks + 8 (l/32) + j][32 nb + l%32], j = 0..7, as 8 consecutive bf16; fragments
// are stored [N/32][K/16][64 lanes], so one wave reads one contiguous kilobyte per fragment.

#include "common.h"
#include "kernels.h"

namespace fmd {
namespace {

constexpr int kD = 256;              // model width
constexpr int kDh = 32;              // head width: wave w of a 256-wide slab = head w
constexpr int kBM = 128;             // token rows per workgroup
constexpr int kWaves = 8;            // wave w owns columns [32w, 32w + 32) of a 256-wide slab
constexpr int kThreads = 64 * kWaves;
constexpr int kRing = 8;             // weight fragments in flight per wave
constexpr int kLdA = kD + 8;         // LDS pitch (bf16) of the 128 x 256 activation tile
constexpr int kBH = 128;             // MLP hidden units per chunk
constexpr int kLdH = kBH + 8;        // LDS pitch (bf16) of a hidden chunk
constexpr int kKs = kD / 16;         // fragments along K = 256

__device__ __forceinline__ int acc_row(int mi, int r, int lane) {
  return mi * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
}

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// acc[mi] += A[row0 + 32 mi + .., k] x B over `nks` fragments along K, A in LDS (pitch ld,
// first K column 0). B fragments stream through a ring of kRing registers: on entry the
// ring holds this phase's fragments 0 .. kRing-1; each consumed slot is refilled with the
// fragment kRing positions ahead, taken from `cur` (this phase's fragment 0, wave-uniform)
// or, in the last kRing steps, from the start of the next phase (`next`; with
// kPrefetchNext false the ring is left empty instead). nks is a multiple of kRing.
__device__ __forceinline__ void ring_fill(u32x4 (&ring)[kRing], const u32x4* __restrict__ src,
                                          int lane) {
#pragma unroll
  for (int j = 0; j < kRing; ++j) ring[j] = src[j * 64 + lane];
}

template <int TM, bool kPrefetchNext = true>
__device__ __forceinline__ void mfma_phase(f32x16 (&acc)[TM], const bf16* __restrict__ lds,
                                           int ld, int row0, int nks, u32x4 (&ring)[kRing],
                                           const u32x4* __restrict__ cur,
                                           const u32x4* __restrict__ next, int lane) {
  // compiler-only barrier: keeps the LDS reads of a tile that several phases read (the
  // same LayerNorm tile for Q, K and V, or for every MLP chunk) inside their phase instead
  // of hoisted out of the enclosing loop into hundreds of live registers
  asm volatile("" ::: "memory");
  const bf16* arow = lds + (row0 + (lane & 31)) * ld + (lane >> 5) * 8;
  for (int g = 0; g < nks; g += kRing) {
    const bool more = g + kRing < nks;
    const u32x4* src = more ? cur + (g + kRing) * 64 : next;
#pragma unroll
    for (int j = 0; j < kRing; ++j) {
      const int k = (g + j) * 16;
      bf16x8 a[TM];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi) a[mi] = *(const bf16x8*)(arow + mi * 32 * ld + k);
      const bf16x8 b = as_bf16x8(ring[j]);
      if (kPrefetchNext || more) ring[j] = src[j * 64 + lane];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
        acc[mi] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b, acc[mi], 0, 0, 0);
    }
  }
}

// Global row access in the accumulator layout. Element (mi, r) of a lane sits at byte
// (32 mi + 8 (r/4) + r%4) * pitch + lane_off from the tile's first row, where
// lane_off = (4 (lane/32) * ld + col) * sizeof(elem). The row-group part is added to a
// wave-uniform base and r%4 becomes an immediate offset, so only one 32-bit per-lane
// offset stays live instead of one 64-bit address per element.
template <typename E, int LD>
struct RowIo {
  const char* base;     // wave-uniform: first row of the tile
  uint32_t lane_off;
  __device__ RowIo(const E* X, int64_t m0, int col, int lane)
      : base((const char*)(X + m0 * LD)),
        lane_off((uint32_t)((4 * (lane >> 5) * LD + col) * sizeof(E))) {
    // opaque to the compiler: the addresses are formed here, where they are used, and not
    // computed early and held live across the phases in between
    asm volatile("" : "+v"(lane_off));
  }
  __device__ __forceinline__ E* at(int mi, int r) const {
    const char* gb = base + (size_t)(mi * 32 + 8 * (r >> 2)) * LD * sizeof(E);
    return (E*)(gb + lane_off + (r & 3) * LD * sizeof(E));
  }
};

// Every row and tile transfer of these kernels is a non-temporal load or store: the rows
// stream through once, and kept in L2 they would evict the weight fragments that every
// workgroup re-reads.
//
// acc = rows m0.. of X (FP32, pitch kD) at the wave's columns, plus bias (may be null).
template <int TM>
__device__ __forceinline__ void load_rows(f32x16 (&acc)[TM], const float* __restrict__ X,
                                          int64_t m0, int col,
                                          const float* __restrict__ bias, int lane) {
  const float bv = bias ? bias[col] : 0.f;
  const RowIo<float, kD> io(X, m0, col, lane);
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[mi][r] = __builtin_nontemporal_load(io.at(mi, r)) + bv;
}

template <int TM>
__device__ __forceinline__ void fill(f32x16 (&acc)[TM], float bv) {
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[mi][r] = bv;
}

// ROWS x 256 BF16 tile at rows m0.. of a head-major attention output [8 heads][Mp][32]
// (plane = Mp x 32 elements) into LDS (pitch kLdA, row-major): consecutive threads read
// consecutive 16-byte chunks of one head's rows.
template <int ROWS, int NT = kThreads>
__device__ __forceinline__ void tile_hm_to_lds(bf16* __restrict__ A, const bf16* __restrict__ S,
                                               int64_t plane, int64_t m0, int tid) {
  constexpr int kChunks = ROWS * kD / 8;                // 16-byte chunks
  constexpr int kPer = kChunks / NT;
  constexpr int kHeadChunks = ROWS * kDh / 8;           // chunks of one head's rows
  u32x4 v[kPer];
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int idx = tid + i * NT, hd = idx / kHeadChunks, rem = idx % kHeadChunks;
    const u32x4* src = (const u32x4*)((const char*)(S + hd * plane + m0 * kDh) + (uint32_t)rem * 16);
    v[i] = __builtin_nontemporal_load(src);
  }
#pragma unroll
  for (int i = 0; i < kPer; ++i) {
    const int idx = tid + i * NT, hd = idx / kHeadChunks, rem = idx % kHeadChunks;
    *(u32x4*)(A + (rem / (kDh / 8)) * kLdA + hd * kDh + (rem % (kDh / 8)) * 8) = v[i];
  }
}

// Cross-lane data movement inside 16-lane rows (DPP controls).
constexpr int kDppXor1 = 0xB1;        // quad_perm [1,0,3,2]: lane i <- lane i ^ 1
constexpr int kDppXor2 = 0x4E;        // quad_perm [2,3,0,1]: lane i <- lane i ^ 2
constexpr int kDppHalfMirror = 0x141; // lane i <- lane 7 - i within each group of 8
constexpr int kDppRor8 = 0x128;       // lane i <- lane (i + 8) mod 16, i.e. i ^ 8

// One halving step of the transpose-reduction: lanes pair up across lane bit `bit` (the DPP
// partner differs from the lane in that bit and agrees in every bit already reduced); of the
// value pairs (v[i], v[i + N/2]) both lanes sum the pair with the partner's copy and keep the
// half their bit selects.
template <int CTRL, int N>
__device__ __forceinline__ void reduce_step(float (&v)[32], bool up) {
#pragma unroll
  for (int i = 0; i < N / 2; ++i) {
    const float ra = v[i] + __builtin_amdgcn_update_dpp(0.f, v[i], CTRL, 0xF, 0xF, false);
    const float rb = v[i + N / 2] + __builtin_amdgcn_update_dpp(0.f, v[i + N / 2], CTRL, 0xF, 0xF, false);
    v[i] = up ? rb : ra;
  }
}

// Transpose-reduction over the 32 lanes of a half wave, in vector instructions only: lane
// bit 4 by a row swap (v_permlane16_swap exchanges the upper row of one register with the
// lower row of the other, so a single add leaves v[i] summed over lanes l, l ^ 16 in the
// lower row and v[i + 16] in the upper row), bits 3..0 by DPP. Afterwards v[0] of lane l
// holds the sum over the half wave of value (l & 31). Every value is summed in the same
// tree of column groups, so the result does not depend on which value slot a row uses.
__device__ __forceinline__ void transpose_reduce32(float (&v)[32], int lane) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 16]),
                                                    false, false);
    v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  }
  reduce_step<kDppRor8, 16>(v, (lane & 8) != 0);
  reduce_step<kDppHalfMirror, 8>(v, (lane & 4) != 0);
  reduce_step<kDppXor2, 4>(v, (lane & 2) != 0);
  reduce_step<kDppXor1, 2>(v, (lane & 1) != 0);
}

// Row-statistics scratch: per-pass partial sums [row][wave] and each wave's own copy of
// the row means and inverse deviations (a wave writes and reads only its copy, so no
// barrier is needed after they are formed).
struct SharedLn {
  float red[2][kBM * kWaves];
  float mu[kWaves][kBM];
  float rs[kWaves][kBM];
};

// Partial sums over the wave's 32 columns of the 32 TM rows in acc, one 32-value group of
// two fragments at a time; lane l ends with the row own(g, l) of group g.
__device__ __forceinline__ int own_row(int g, int lane) {
  const int j = lane & 31;
  return acc_row(2 * g + (j >> 4), j & 15, lane);
}

// LayerNorm statistics of the 32 TM full rows held in acc: mean and 1/sqrt(biased variance +
// eps) into this wave's sl.mu[w] / sl.rs[w], optionally also to stats_out[m0 + row]. Per
// pass: a transpose-reduction over the wave's columns, partials to LDS, one barrier, then
// every lane adds the 8 wave partials of its own rows in wave order. Contains two barriers.
template <int TM>
__device__ __forceinline__ void row_stats(const f32x16 (&acc)[TM], SharedLn& sl,
                                          float2* __restrict__ stats_out, int64_t m0, int lane,
                                          int w) {
  // No multiply-add contraction here: a square fused into the lane exchange's add would be
  // exact on one lane of a pair and rounded on the other, so the statistics would depend on
  // the row's position in the tile.
#pragma clang fp contract(off)
  static_assert(TM % 2 == 0, "row statistics take 32-value groups of two fragments");
  constexpr int G = TM / 2;
  float* mu = sl.mu[w];
  float* rs = sl.rs[w];
  // pass 1: row sums
#pragma unroll
  for (int g = 0; g < G; ++g) {
    float v[32];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) v[h * 16 + r] = acc[2 * g + h][r];
    transpose_reduce32(v, lane);
    sl.red[0][own_row(g, lane) * kWaves + w] = v[0];
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const float* p = &sl.red[0][own_row(g, lane) * kWaves];
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) t += p[q];
    mu[own_row(g, lane)] = t * (1.0f / kD);
  }
  // pass 2: sums of squared deviations (mu read back from this wave's own copy)
#pragma unroll
  for (int g = 0; g < G; ++g) {
    float v[32];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc[2 * g + h][r] - mu[acc_row(2 * g + h, r, lane)];
        v[h * 16 + r] = dv * dv;
      }
    transpose_reduce32(v, lane);
    sl.red[1][own_row(g, lane) * kWaves + w] = v[0];
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = own_row(g, lane);
    const float* p = &sl.red[1][row * kWaves];
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) t += p[q];
    const float r = rsqrtf(t * (1.0f / kD) + kLnEps);
    rs[row] = r;
    if (stats_out && w == 0) stats_out[m0 + row] = make_float2(mu[row], r);
  }
}

// LDS tile A (pitch kLdA) = LayerNorm(acc rows) with gain gv and shift sv of column col, in
// BF16.
template <int TM>
__device__ __forceinline__ void ln_to_lds(const f32x16 (&acc)[TM], const float* __restrict__ mu,
                                          const float* __restrict__ rs, float gv, float sv,
                                          bf16* __restrict__ A, int col, int lane) {
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = acc_row(mi, r, lane);
      A[row * kLdA + col] = (bf16)((acc[mi][r] - mu[row]) * rs[row] * gv + sv);
    }
}

template <int TM>
__device__ __forceinline__ void store_rows_f32(const f32x16 (&acc)[TM], float* __restrict__ X,
                                               int64_t m0, int col, int lane) {
  const RowIo<float, kD> io(X, m0, col, lane);
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int r = 0; r < 16; ++r) __builtin_nontemporal_store(acc[mi][r], io.at(mi, r));
}

template <int LD, int TM>
__device__ __forceinline__ void store_rows_bf16(const f32x16 (&acc)[TM], bf16* __restrict__ X,
                                                int64_t m0, int col, int lane) {
  const RowIo<bf16, LD> io(X, m0, col, lane);
#pragma unroll
  for (int mi = 0; mi < TM; ++mi)
#pragma unroll
    for (int r = 0; r < 16; ++r) __builtin_nontemporal_store((bf16)acc[mi][r], io.at(mi, r));
}

// GELU(z) = z/2 (1 + erf(z / sqrt 2)) with erf by Abramowitz & Stegun 7.1.27:
// erf(x) = 1 - (1 + a1 x + a2 x^2 + a3 x^3 + a4 x^4)^-4 for x >= 0, absolute error at most
// 5e-4, far below the BF16 rounding of the result (relative step 2^-8). Branch-free (a
// library erf branches on |x|), one hardware reciprocal and no exponential. The variable is
// u = z / sqrt(2 ln 2) (the callers fold the bias into it as bu = bias / sqrt(2 ln 2)), so
// x = |u| sqrt(ln 2), whose powers are folded into the coefficients b_k = a_k (ln 2)^(k/2);
// with h = sqrt(ln 2 / 2), GELU = h (u + |u| erf(x)). 10 vector instructions per value.
constexpr float kGeluU = 0.84932180028801904f;   // 1 / sqrt(2 ln 2)
__device__ __forceinline__ float gelu_as(float a, float bu) {
  constexpr float s = 0.83255461115769775f;   // sqrt(ln 2)
  constexpr float b1 = 0.278393f * s, b2 = 0.230389f * s * s, b3 = 0.000972f * s * s * s,
                  b4 = 0.078108f * s * s * s * s;
  constexpr float h = 0.5f / kGeluU;
  const float u = fmaf(a, kGeluU, bu);
  const float x = fabsf(u);
  float q = fmaf(b4, x, b3);
  q = fmaf(q, x, b2);
  q = fmaf(q, x, b1);
  q = fmaf(q, x, 1.0f);
  q = q * q;
  const float r = __builtin_amdgcn_rcpf(q * q);
  const float he = fmaf(-h, r, h);                  // h erf(|x|)
  return fmaf(x, he, u * h);
}

// ---- helpers of the 64-row MLP kernel: four waves, wave w owning output column blocks
// 2w and 2w + 1 (64 columns) of all rows and hidden column block w of every chunk.
constexpr int kWaves4 = 4;
constexpr int kThreads4 = 64 * kWaves4;
// sched_barrier mask: instructions of these kinds may be scheduled across it (VALU 0x2,
// SALU 0x4, LDS reads 0x100); vector-memory loads and MFMAs may not
constexpr int kKeepLoadsAndMfma = 0x2 | 0x4 | 0x100;

// Fragment t of a weight stream over NC column blocks taken together: K step t / NC of
// column block t % NC (blocks cstride fragments-of-64-lanes apart).
template <int NC>
__device__ __forceinline__ const u32x4* frag_at(const u32x4* p, int cstride, int t) {
  return p + (t % NC) * cstride + (t / NC) * 64;
}

template <int NC>
__device__ __forceinline__ void ring_fill_nc(u32x4 (&ring)[kRing], const u32x4* __restrict__ p,
                                             int cstride, int lane) {
#pragma unroll
  for (int t = 0; t < kRing; ++t) ring[t] = frag_at<NC>(p, cstride, t)[lane];
}

// acc[mi][nj] += A[row0 + 32 mi + .., K] x B[K, column block nj] over NK K steps (A in LDS,
// pitch ld). Fragment t = NC k + nj sits in ring slot t % kRing; on use the slot is refilled
// with fragment t + kRing of this stream or, past its end, of the next phase's stream
// (NCN column blocks, stride nstride), unless kNext is false.
template <int TM, int NC, int NK, int NCN, bool kNext>
__device__ __forceinline__ void mfma_phase_nc(f32x16 (&acc)[TM][NC], const bf16* __restrict__ lds,
                                              int ld, int row0, u32x4 (&ring)[kRing],
                                              const u32x4* __restrict__ cur, int cstride,
                                              const u32x4* __restrict__ next, int nstride,
                                              int lane) {
  asm volatile("" ::: "memory");
  constexpr int F = NC * NK;
  const bf16* arow = lds + (row0 + (lane & 31)) * ld + (lane >> 5) * 8;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    bf16x8 a[TM];
#pragma unroll
    for (int mi = 0; mi < TM; ++mi) a[mi] = *(const bf16x8*)(arow + mi * 32 * ld + k * 16);
#pragma unroll
    for (int nj = 0; nj < NC; ++nj) {
      const int t = k * NC + nj;
      const bf16x8 b = as_bf16x8(ring[t % kRing]);
      if (t + kRing < F)
        ring[t % kRing] = frag_at<NC>(cur, cstride, t + kRing)[lane];
      else if (kNext)
        ring[t % kRing] = frag_at<NCN>(next, nstride, t + kRing - F)[lane];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
        acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b, acc[mi][nj], 0, 0, 0);
    }
    // keeps the weight loads and the MFMAs of this K step in it (LDS reads and plain
    // arithmetic may still move): the refill above stays kRing fragments ahead of its use
    // instead of being sunk next to it, which exposed the L2 latency at every K step
    __builtin_amdgcn_sched_barrier(kKeepLoadsAndMfma);
  }
}

// Up-projection of one hidden chunk for all rows (if UP: h2n += LN tile x W_up chunk, one
// column block, 16 K steps) software-pipelined with the GELU of the previous chunk's
// products h2 (two values per K step, bias term bv = bias x kGeluU, BF16 into the hidden
// tile hb at column hcol); the prefetch past the end reads the next phase's stream (NCN blocks).
// GELU of P values of h2 starting at value v0 (value v: row block v / 16, register v % 16),
// bias term bv = bias x kGeluU, written as BF16 into the hidden tile hb at column hcol
template <int TA, int P>
__device__ __forceinline__ void gelu_vals(const f32x16 (&h2)[TA][1], int v0, float bv,
                                          bf16* __restrict__ hb, int hcol, int lane) {
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const int v = v0 + q, mi = v >> 4, r = v & 15;
    hb[acc_row(mi, r, lane) * kLdH + hcol] = (bf16)gelu_as(h2[mi][0][r], bv);
  }
}

template <bool UP, int TA, int NCN, int V0 = 0, int NV = 16 * TA>
__device__ __forceinline__ void up_gelu_nc(f32x16 (&h2n)[TA][1], const f32x16 (&h2)[TA][1],
                                           const bf16* __restrict__ A, u32x4 (&ring)[kRing],
                                           const u32x4* __restrict__ cur,
                                           const u32x4* __restrict__ next, int nstride, float bv,
                                           bf16* __restrict__ hb, int hcol, int lane) {
  static_assert(NV % kKs == 0, "GELU values spread evenly over the K steps");
  asm volatile("" ::: "memory");
  const bf16* arow = A + (lane & 31) * kLdA + (lane >> 5) * 8;
#pragma unroll
  for (int ks = 0; ks < kKs; ++ks) {
    if constexpr (UP) {
      bf16x8 a[TA];
#pragma unroll
      for (int mi = 0; mi < TA; ++mi) a[mi] = *(const bf16x8*)(arow + mi * 32 * kLdA + ks * 16);
      const bf16x8 b = as_bf16x8(ring[ks % kRing]);
      ring[ks % kRing] = ks + kRing < kKs ? cur[(ks + kRing) * 64 + lane]
                                          : frag_at<NCN>(next, nstride, ks + kRing - kKs)[lane];
#pragma unroll
      for (int mi = 0; mi < TA; ++mi)
        h2n[mi][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b, h2n[mi][0], 0, 0, 0);
    }
    gelu_vals<TA, NV / kKs>(h2, V0 + (NV / kKs) * ks, bv, hb, hcol, lane);
  }
}

// mfma_phase_nc with the GELU of NV values of h2g (from value V0 on) spread over its K steps
template <int TM, int NC, int NK, int NCN, bool kNext, int TA, int V0, int NV>
__device__ __forceinline__ void mfma_gelu_nc(f32x16 (&acc)[TM][NC], const bf16* __restrict__ lds,
                                             int ld, u32x4 (&ring)[kRing],
                                             const u32x4* __restrict__ cur, int cstride,
                                             const u32x4* __restrict__ next, int nstride,
                                             const f32x16 (&h2g)[TA][1], float bv,
                                             bf16* __restrict__ hb, int hcol, int lane) {
  static_assert(NV % NK == 0, "GELU values spread evenly over the K steps");
  asm volatile("" ::: "memory");
  constexpr int F = NC * NK;
  const bf16* arow = lds + (lane & 31) * ld + (lane >> 5) * 8;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    bf16x8 a[TM];
#pragma unroll
    for (int mi = 0; mi < TM; ++mi) a[mi] = *(const bf16x8*)(arow + mi * 32 * ld + k * 16);
#pragma unroll
    for (int nj = 0; nj < NC; ++nj) {
      const int t = k * NC + nj;
      const bf16x8 b = as_bf16x8(ring[t % kRing]);
      if (t + kRing < F)
        ring[t % kRing] = frag_at<NC>(cur, cstride, t + kRing)[lane];
      else if (kNext)
        ring[t % kRing] = frag_at<NCN>(next, nstride, t + kRing - F)[lane];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
        acc[mi][nj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[mi], b, acc[mi][nj], 0, 0, 0);
    }
    gelu_vals<TA, NV / NK>(h2g, V0 + (NV / NK) * k, bv, hb, hcol, lane);
    __builtin_amdgcn_sched_barrier(kKeepLoadsAndMfma);
  }
}

struct SharedLn4 {
  float red[2][64 * kWaves4];
  float mu[kWaves4][64];
  float rs[kWaves4][64];
};

// LayerNorm statistics of the 32 TM rows held as acc[TM][2] (this wave: column blocks
// nj = 0, 1): the two columns a lane holds of a row are added first, then the
// transpose-reduction over the 32 lanes, then the kWaves4 wave partials in wave order.
// Means / inverse deviations land in this wave's sl.mu[w] / sl.rs[w]. Two barriers.
template <int TM>
__device__ __forceinline__ void row_stats_nc(const f32x16 (&acc)[TM][2], SharedLn4& sl,
                                             float2* __restrict__ stats_out, int64_t m0,
                                             int lane, int w) {
#pragma clang fp contract(off)
  static_assert(TM % 2 == 0, "row statistics take 32-value groups of two fragments");
  constexpr int G = TM / 2;
  float* mu = sl.mu[w];
  float* rs = sl.rs[w];
#pragma unroll
  for (int g = 0; g < G; ++g) {
    float v[32];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) v[h * 16 + r] = acc[2 * g + h][0][r] + acc[2 * g + h][1][r];
    transpose_reduce32(v, lane);
    sl.red[0][own_row(g, lane) * kWaves4 + w] = v[0];
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const float* p = &sl.red[0][own_row(g, lane) * kWaves4];
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kWaves4; ++q) t += p[q];
    mu[own_row(g, lane)] = t * (1.0f / kD);
  }
#pragma unroll
  for (int g = 0; g < G; ++g) {
    float v[32];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float m = mu[acc_row(2 * g + h, r, lane)];
        const float d0 = acc[2 * g + h][0][r] - m, d1 = acc[2 * g + h][1][r] - m;
        v[h * 16 + r] = d0 * d0 + d1 * d1;
      }
    transpose_reduce32(v, lane);
    sl.red[1][own_row(g, lane) * kWaves4 + w] = v[0];
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int row = own_row(g, lane);
    const float* p = &sl.red[1][row * kWaves4];
    float t = 0.f;
#pragma unroll
    for (int q = 0; q < kWaves4; ++q) t += p[q];
    const float r = rsqrtf(t * (1.0f / kD) + kLnEps);
    rs[row] = r;
    if (stats_out && w == 0) stats_out[m0 + row] = make_float2(mu[row], r);
  }
}

// Head partials of the 32 TM rows: lane l ends with the sum over this wave's 64 columns of
// y * w for its own row own_row(0, l) (the lane's two columns by one fused multiply-add,
// then the transpose-reduction).
__device__ __forceinline__ float head_partial(const f32x16 (&y)[2][2], float w0, float w1,
                                              int lane) {
  float v[32];
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int r = 0; r < 16; ++r) v[h * 16 + r] = fmaf(y[h][1][r], w1, y[h][0][r] * w0);
  transpose_reduce32(v, lane);
  return v[0];
}

}  // namespace

// ---------------------------------------------------------------------------------------

// Input embedding of block 0, formed in the QKV kernel instead of read from H, for a stage
// whose time is the same for every row: row r is temb + sum_k xs[r][k] W_xin[k] over the 9
// state features, in that order (the order of the embedding kernel, so the rows are the
// same), and is stored to H. Rows at or past T (padding) are zero. (Per-event times would
// need a time-embedding row per tile row; those calls keep the embedding kernel.)
struct EmbedRows {
  const float* xs;             // state rows, pitch kEmbLd floats, first 9 used
  int64_t T;
  const float* temb;           // [256] time embedding of the stage, b_xin included
  const float* W;              // W_xin [9][256]
  float* H;                    // [Mp][256] output
};
constexpr int kEmbLd = 16;     // pitch of the ODE state rows
constexpr int kEmbF9 = 9;

// Which row tiles a launch covers: tile b of the grid is rows [ROWS t, ROWS t + ROWS) with
// t = tiles[b] when a map is given (the serving loop skips the tiles of gaps between
// requests), t = b otherwise. Mp is the padded row count of the call: the head-major planes
// hold Mp rows each, whatever tiles run.
struct RowMap {
  const int32_t* tiles;
  int64_t Mp;
  __device__ __forceinline__ int64_t first_row(int rows) const {
    return (int64_t)(tiles ? tiles[blockIdx.x] : (int32_t)blockIdx.x) * rows;
  }
};

template <int TM, bool EMBED>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(TM == 2 ? 4 : 2))) void k_fused_qkv(const float* __restrict__ H,
                                                        const float* __restrict__ g,
                                                        const float* __restrict__ s,
                                                        const u32x4* __restrict__ Wf,
                                                        const float* __restrict__ bias,
                                                        bf16* __restrict__ qkv, EmbedRows em,
                                                        RowMap rm) {
  constexpr int ROWS = 32 * TM;
  __shared__ __attribute__((aligned(16))) bf16 A[ROWS * kLdA];
  __shared__ SharedLn sl;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t m0 = rm.first_row(ROWS);
  const int64_t plane = rm.Mp * kDh;   // Mp rows x 32 per head
  const int col = w * 32 + (lane & 31);
  const u32x4* wf = Wf + w * kKs * 64;            // slab s: + s * kWaves * kKs * 64
  // column parameters first: waiting for them later then does not drain the weight ring
  const float gv = g[col], sv = s[col];
  float bcur = bias[col];
  u32x4 ring[kRing];
  if constexpr (!EMBED) ring_fill(ring, wf, lane);
  f32x16 acc[TM];
  if constexpr (EMBED) {
    // the tile's state rows (ROWS x 16 floats), staged in the A buffer
    static_assert(ROWS * kEmbLd * 4 <= ROWS * kLdA * 2, "staging fits the A tile");
    float* xt = reinterpret_cast<float*>(A);
    for (int i = tid; i < ROWS * kEmbLd / 4; i += kThreads)
      *(float4*)&xt[4 * i] = *(const float4*)&em.xs[m0 * kEmbLd + 4 * i];
    __syncthreads();
    float wv[kEmbF9];
#pragma unroll
    for (int k = 0; k < kEmbF9; ++k) wv[k] = em.W[k * kD + col];
    const float t0 = em.temb[col];
#pragma unroll
    for (int mi = 0; mi < TM; ++mi)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = acc_row(mi, r, lane);
        const float* x = &xt[row * kEmbLd];
        float v = t0;
#pragma unroll
        for (int k = 0; k < kEmbF9; ++k) v = fmaf(x[k], wv[k], v);
        acc[mi][r] = m0 + row < em.T ? v : 0.f;
        asm volatile("" ::: "memory");   // a row at a time: the LDS reads are not all hoisted
      }
    ring_fill(ring, wf, lane);             // after the rows: fewer registers live at once
    store_rows_f32(acc, em.H, m0, col, lane);
  } else {
    load_rows(acc, H, m0, col, nullptr, lane);
  }
  row_stats(acc, sl, nullptr, m0, lane, w);   // barriers: the staged rows are consumed
  ln_to_lds(acc, sl.mu[w], sl.rs[w], gv, sv, A, col, lane);
  __syncthreads();
#pragma unroll 1
  for (int slab = 0; slab < 3; ++slab) {
    fill(acc, bcur);
    bcur = bias[(slab < 2 ? slab + 1 : slab) * kD + col];   // the next slab's, ahead of its ring
    const u32x4* cur = wf + slab * kWaves * kKs * 64;
    mfma_phase<TM>(acc, A, kLdA, 0, kKs, ring, cur, slab < 2 ? cur + kWaves * kKs * 64 : cur,
                  lane);
    // head-major: wave w of slab s (Q, K, V) writes head w's plane (8 s + w), rows contiguous
    store_rows_bf16<kDh>(acc, qkv + (int64_t)(slab * kWaves + w) * plane, m0, lane & 31, lane);
  }
}

template <int TM>
__global__ __launch_bounds__(kThreads) void k_fused_oqc(
    const bf16* __restrict__ att, const u32x4* __restrict__ Wf_o, const float* __restrict__ b_o,
    float* __restrict__ H, const float* __restrict__ g, const float* __restrict__ s,
    const u32x4* __restrict__ Wf_qc, const float* __restrict__ b_qc, bf16* __restrict__ qc,
    RowMap rm) {
  constexpr int ROWS = 32 * TM;
  __shared__ __attribute__((aligned(16))) bf16 A[ROWS * kLdA];
  __shared__ SharedLn sl;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t m0 = rm.first_row(ROWS);
  const int64_t plane = rm.Mp * kDh;   // Mp rows x 32 per head
  const int col = w * 32 + (lane & 31);
  const u32x4* wo = Wf_o + w * kKs * 64;
  const u32x4* wq = Wf_qc + w * kKs * 64;
  u32x4 ring[kRing];
  ring_fill(ring, wo, lane);
  tile_hm_to_lds<ROWS>(A, att, plane, m0, tid);   // head-major attention output
  f32x16 acc[TM];
  load_rows(acc, H, m0, col, b_o, lane);
  // column parameters before the weight stream: waiting for them then drains no ring
  const float gv = g[col], sv = s[col], bq = b_qc[col];
  __syncthreads();
  // the W_o phase prefetches the first W_qc fragments
  mfma_phase<TM>(acc, A, kLdA, 0, kKs, ring, wo, wq, lane);
  store_rows_f32(acc, H, m0, col, lane);
  row_stats(acc, sl, nullptr, m0, lane, w);   // barrier: A reads done
  ln_to_lds(acc, sl.mu[w], sl.rs[w], gv, sv, A, col, lane);
  __syncthreads();
  fill(acc, bq);
  mfma_phase<TM>(acc, A, kLdA, 0, kKs, ring, wq, wq, lane);
  store_rows_bf16<kDh>(acc, qc + (int64_t)w * plane, m0, lane & 31, lane);   // head-major
}

// ---- FP8 (OCP e4m3) operands of the MLP's two projections (the FP8 precision form).
// The LayerNorm tile and the hidden chunks are FP8 bytes in LDS; W_up and W_dn are FP8
// fragments of the weights times a power of two per output column (so that the column's
// largest magnitude lies in (224, 448]) for the 32 x 32 x 64 matrix instruction: fragment
// (nb, ks) of lane l holds W[64 ks + 32 (l/32) + j][32 nb + l%32] s_col, j < 32, as 32 bytes,
// stored [N/32][K/64][64 lanes]. A operands from LDS take the same k order (row l%32, bytes
// 64 ks + 32 (l/32) ..), so products pair the same k on both sides. The up-projection output
// is scaled back by 1/s per hidden column before the GELU; the down-projection accumulates
// onto the residual rows multiplied by s per output column and divides by it afterwards,
// exact for powers of two. Accumulation, statistics, GELU and residual stay FP32.
typedef int i32x8 __attribute__((ext_vector_type(8)));

struct Mlp8 {
  const i32x8* up;      // W_up s_up fragments [1024/32][256/64][64]
  const i32x8* dn;      // W_dn s_dn fragments [256/32][1024/64][64]
  const float* up_inv;  // 1 / s_up per hidden column [1024]
  const float* dn_scale;   // s_dn per output column [256]
  const float* dn_inv;  // 1 / s_dn [256]
};

constexpr int kLdA8 = kD + 16;        // bytes per row of the FP8 LayerNorm tile
constexpr int kLdH8 = kBH + 16;       // bytes per row of an FP8 hidden chunk
constexpr int kKs8 = kD / 64;         // 64-deep K steps over d

__device__ __forceinline__ f32x16 mfma_f8(i32x8 a, i32x8 b, f32x16 c) {
  // block scales 2^(127 - 127) = 1: plain FP8 x FP8 products
  return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
}

// x rounded to the nearest e4m3 value (ties to even), as one byte
__device__ __forceinline__ uint32_t to_fp8(float x) {
  return (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(x, x, 0, false) & 0xFFu;
}

// A operand of one 32-row block: row `row` of an FP8 tile (pitch ld bytes), K step ks
__device__ __forceinline__ i32x8 lds_frag8(const uint8_t* __restrict__ t, int ld, int row, int ks,
                                           int lane) {
  const uint8_t* p = t + row * ld + ks * 64 + (lane >> 5) * 32;
  const u32x4 lo = *(const u32x4*)p, hi = *(const u32x4*)(p + 16);
  i32x8 r;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    r[i] = (int)lo[i];
    r[4 + i] = (int)hi[i];
  }
  return r;
}

// MLP block on 64-row tiles with four waves: two workgroups share a CU, one wave of each per
// SIMD, so one workgroup's barriers, LDS traffic and loads overlap the other's matrix work.
// With QKV, the kernel goes on to the next block's LN1 + [Q|K|V] projection from the final
// rows still in registers (as k_fused_qkv does from H), writing head-major planes.
struct NextQkv {
  const float* g;        // LN1 gain and shift of the next block
  const float* s;
  const u32x4* Wf;       // its W_qkv fragments
  const float* bias;
  bf16* qkv;             // [3][8 heads][Mp][32]
};

// With HEAD (the last block), the kernel applies the output head to the final rows instead:
// LN_f, the 9-wide projection (FP32, per-wave partial sums over the wave's 64 columns by the
// transpose-reduction, then the 4 wave partials in wave order) and the ODE update of the
// state, as the separate head kernel does; the residual rows are then not stored.
struct NextHead {
  const float* g;        // LN_f gain and shift
  const float* s;
  const float* Wt;       // W_out transposed: row c = weights of output c (c < 9), 256 wide
  const float* b;
  OdeArgs ode;
};

enum MlpTail { kTailStats = 0, kTailQkv = 1, kTailHead = 2 };

template <int TM, int TAIL, bool F8>
__global__ __launch_bounds__(kThreads4) __attribute__((amdgpu_waves_per_eu(2))) void k_fused_mlp(
    const bf16* __restrict__ att, const u32x4* __restrict__ Wf_oc, const float* __restrict__ b_oc,
    float* __restrict__ H, const float* __restrict__ g, const float* __restrict__ s,
    const u32x4* __restrict__ Wf_up, const float* __restrict__ b_up,
    const u32x4* __restrict__ Wf_dn, const float* __restrict__ b_dn,
    float2* __restrict__ stats_out, NextQkv nq, NextHead nh, Mlp8 f8, RowMap rm) {
  constexpr bool QKV = TAIL == kTailQkv;
  constexpr int ROWS = 32 * TM;
  static_assert(ROWS == 64, "statistics scratch sized for 64 rows");
  __shared__ __attribute__((aligned(16))) bf16 A[ROWS * kLdA];
  __shared__ __attribute__((aligned(16))) bf16 Hc[2][ROWS * kLdH];
  __shared__ SharedLn4 sl;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t m0 = rm.first_row(ROWS);
  const int col0 = 64 * w + (lane & 31);     // column of block nj: col0 + 32 nj
  constexpr int kChunks = 4 * kD / kBH;      // 8
  constexpr int kDnKs = kBH / 16;            // 8 K steps per down-projection chunk
  constexpr int kOcStride = kKs * 64;        // column-block stride, K = d
  constexpr int kDnStride = (4 * kD / 16) * 64;   // column-block stride, K = 4d
  const u32x4* woc = Wf_oc + 2 * w * kOcStride;
  auto up_c = [&](int c) { return Wf_up + (4 * c + w) * kKs * 64; };
  auto dn_c = [&](int c) { return Wf_dn + 2 * w * kDnStride + c * kDnKs * 64; };
  // slab sl of the next block's W_qkv: column blocks 8 sl + 2w, 8 sl + 2w + 1
  auto qkv_c = [&](int slab) { return nq.Wf + (8 * slab + 2 * w) * kOcStride; };
  float gq[2], sq[2], bq[2];   // next block's LN1 gain / shift and Q bias (chained form)
  u32x4 ring[kRing];
  ring_fill_nc<2>(ring, woc, kOcStride, lane);
  // head-major attention output [8 heads][Mp][32]
  tile_hm_to_lds<ROWS, kThreads4>(A, att, rm.Mp * kDh, m0, tid);
  f32x16 acc[TM][2];
#pragma unroll
  for (int nj = 0; nj < 2; ++nj) {
    const float bv = b_oc[col0 + 32 * nj];
    const RowIo<float, kD> io(H, m0, col0 + 32 * nj, lane);
#pragma unroll
    for (int mi = 0; mi < TM; ++mi)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[mi][nj][r] = __builtin_nontemporal_load(io.at(mi, r)) + bv;
  }
  __syncthreads();
  float g3[2], s3[2], bd[2];
#pragma unroll
  for (int nj = 0; nj < 2; ++nj) {
    g3[nj] = g[col0 + 32 * nj];
    s3[nj] = s[col0 + 32 * nj];
    if constexpr (QKV && !F8) bd[nj] = b_dn[col0 + 32 * nj];
  }
  mfma_phase_nc<TM, 2, kKs, 1, !F8>(acc, A, kLdA, 0, ring, woc, kOcStride, up_c(0), 0, lane);
  row_stats_nc(acc, sl, nullptr, m0, lane, w);   // barriers: A reads done
  if constexpr (!F8) {
    {
      const float* mu = sl.mu[w];
      const float* rs = sl.rs[w];
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        const int col = col0 + 32 * nj;
        const float gv = g3[nj], sv = s3[nj];
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = acc_row(mi, r, lane);
            A[row * kLdA + col] = (bf16)((acc[mi][nj][r] - mu[row]) * rs[row] * gv + sv);
          }
      }
    }
    __syncthreads();
    const int hcol = 32 * w + (lane & 31);
    f32x16 h2[2][TM][1];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
#pragma unroll
        for (int r = 0; r < 16; ++r) h2[u][mi][0][r] = 0.f;
    float bu = b_up[hcol];   // chunk biases one chunk ahead: issued before the chunk's
                             // weight loads, so their wait does not drain the ring
    mfma_phase_nc<TM, 1, kKs, 1, true>(h2[0], A, kLdA, 0, ring, up_c(0), 0, up_c(1), 0, lane);
    // The GELU of chunk c is done in two halves (values 0-15 and 16-31 of each lane), each
    // beside matrix work: the first during the down-projection of chunk c-1, the second
    // during the up-projection of chunk c+1. Chunk 0's first half runs alone.
    gelu_vals<TM, 16>(h2[0], 0, kGeluU * bu, Hc[0], hcol, lane);
    // chunk cc: [up-projection cc+1 | GELU cc, second half] -> barrier ->
    // [down-projection cc | GELU cc+1, first half]. Weight stream order: up 0, up 1, down 0,
    // up 2, down 1, ..., up 7, down 6, down 7.
#pragma unroll 1
    for (int c = 0; c < kChunks - 2; c += 2) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int cc = c + u;
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int r = 0; r < 16; ++r) h2[u ^ 1][mi][0][r] = 0.f;
        const float bun = b_up[(cc + 1) * kBH + hcol];
        up_gelu_nc<true, TM, 2, 16, 16>(h2[u ^ 1], h2[u], A, ring, up_c(cc + 1), dn_c(cc),
                                        kDnStride, kGeluU * bu, Hc[u], hcol, lane);
        __syncthreads();
        mfma_gelu_nc<TM, 2, kDnKs, 1, true, TM, 0, 16>(acc, Hc[u], kLdH, ring, dn_c(cc),
                                                       kDnStride, up_c(cc + 2), 0, h2[u ^ 1],
                                                       kGeluU * bun, Hc[u ^ 1], hcol, lane);
        bu = bun;
      }
    }
    // chunks 6 and 7: chunk 7's whole GELU beside the down-projection of chunk 6
#pragma unroll
    for (int mi = 0; mi < TM; ++mi)
#pragma unroll
      for (int r = 0; r < 16; ++r) h2[1][mi][0][r] = 0.f;
    const float bu7 = b_up[7 * kBH + hcol];
    up_gelu_nc<true, TM, 2, 16, 16>(h2[1], h2[0], A, ring, up_c(7), dn_c(6), kDnStride,
                                    kGeluU * bu, Hc[0], hcol, lane);
    __syncthreads();
    mfma_gelu_nc<TM, 2, kDnKs, 2, true, TM, 0, 32>(acc, Hc[0], kLdH, ring, dn_c(6), kDnStride,
                                                   dn_c(7), kDnStride, h2[1], kGeluU * bu7,
                                                   Hc[1], hcol, lane);
    __syncthreads();
    if constexpr (QKV) {
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        gq[nj] = nq.g[col0 + 32 * nj];
        sq[nj] = nq.s[col0 + 32 * nj];
        bq[nj] = nq.bias[col0 + 32 * nj];
      }
    }
    mfma_phase_nc<TM, 2, kDnKs, 2, QKV>(acc, Hc[1], kLdH, 0, ring, dn_c(7), kDnStride,
                                        QKV ? qkv_c(0) : dn_c(7), QKV ? kOcStride : kDnStride, lane);
  } else {
    // FP8 operands for W_up and W_dn: the LayerNorm tile and the hidden chunks as e4m3 bytes
    // (aliasing the BF16 tile and chunk buffers), the residual rows in W_dn's scaled domain
    uint8_t* A8 = reinterpret_cast<uint8_t*>(A);
    uint8_t* H8 = reinterpret_cast<uint8_t*>(&Hc[0][0]);
    {
      const float* mu = sl.mu[w];
      const float* rs = sl.rs[w];
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        const int col = col0 + 32 * nj;
        const float gv = g3[nj], sv = s3[nj], sd = f8.dn_scale[col];
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = acc_row(mi, r, lane);
            A8[row * kLdA8 + col] = (uint8_t)to_fp8((acc[mi][nj][r] - mu[row]) * rs[row] * gv + sv);
            acc[mi][nj][r] *= sd;
          }
      }
    }
    const int hcol = 32 * w + (lane & 31);
    // up-projection fragments of the current chunk (column block 4 c + w, 4 K steps) and
    // down-projection fragments (column blocks 2 w + nj, K steps 2 c + ks)
    i32x8 fu[kKs8], fd[4];
#pragma unroll
    for (int ks = 0; ks < kKs8; ++ks) fu[ks] = f8.up[(w * kKs8 + ks) * 64 + lane];
    __syncthreads();
#pragma unroll 1
    for (int c = 0; c < kChunks; ++c) {
      // the chunk's GELU scale and bias first: waiting for them then drains no fragment loads
      const float ui = f8.up_inv[c * kBH + hcol], bu = kGeluU * b_up[c * kBH + hcol];
#pragma unroll
      for (int nj = 0; nj < 2; ++nj)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
          fd[2 * nj + ks] = f8.dn[((2 * w + nj) * 16 + 2 * c + ks) * 64 + lane];
      asm volatile("" ::: "memory");
      f32x16 h[TM];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
#pragma unroll
        for (int r = 0; r < 16; ++r) h[mi][r] = 0.f;
#pragma unroll
      for (int ks = 0; ks < kKs8; ++ks)
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
          h[mi] = mfma_f8(lds_frag8(A8, kLdA8, 32 * mi + (lane & 31), ks, lane), fu[ks], h[mi]);
      if (c + 1 < kChunks) {
#pragma unroll
        for (int ks = 0; ks < kKs8; ++ks)
          fu[ks] = f8.up[((4 * (c + 1) + w) * kKs8 + ks) * 64 + lane];
      }
      uint8_t* hb = H8 + (c & 1) * (ROWS * kLdH8);
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
#pragma unroll
        for (int r = 0; r < 16; ++r)
          hb[acc_row(mi, r, lane) * kLdH8 + hcol] = (uint8_t)to_fp8(gelu_as(h[mi][r] * ui, bu));
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < 2; ++ks) {
        i32x8 a[TM];
#pragma unroll
        for (int mi = 0; mi < TM; ++mi) a[mi] = lds_frag8(hb, kLdH8, 32 * mi + (lane & 31), ks, lane);
#pragma unroll
        for (int nj = 0; nj < 2; ++nj)
#pragma unroll
          for (int mi = 0; mi < TM; ++mi) acc[mi][nj] = mfma_f8(a[mi], fd[2 * nj + ks], acc[mi][nj]);
      }
    }
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) {
      const float sdi = f8.dn_inv[col0 + 32 * nj];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[mi][nj][r] *= sdi;
    }
  }
#pragma unroll
  for (int nj = 0; nj < 2; ++nj) {
    const float bv = QKV && !F8 ? bd[nj] : b_dn[col0 + 32 * nj];
    const RowIo<float, kD> io(H, m0, col0 + 32 * nj, lane);
#pragma unroll
    for (int mi = 0; mi < TM; ++mi)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        acc[mi][nj][r] += bv;
        if constexpr (TAIL != kTailHead) __builtin_nontemporal_store(acc[mi][nj][r], io.at(mi, r));
      }
  }
  if constexpr (TAIL == kTailStats) {
    row_stats_nc(acc, sl, stats_out, m0, lane, w);
  } else if constexpr (TAIL == kTailHead) {
    static_assert(TM == 2, "one 32-value group per lane");
    constexpr int kF = 9;
    row_stats_nc(acc, sl, nullptr, m0, lane, w);   // barriers: the hidden buffers are free
    const float* mu = sl.mu[w];
    const float* rs = sl.rs[w];
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) {
      const int col = col0 + 32 * nj;
      const float gv = nh.g[col], sv = nh.s[col];
#pragma unroll
      for (int mi = 0; mi < TM; ++mi)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = acc_row(mi, r, lane);
          acc[mi][nj][r] = fmaf((acc[mi][nj][r] - mu[row]) * rs[row], gv, sv);
        }
    }
    float* part = reinterpret_cast<float*>(Hc[0]);    // [ROWS][kF][kWaves4]
#pragma unroll 1
    for (int c = 0; c < kF; ++c) {
      part[(own_row(0, lane) * kF + c) * kWaves4 + w] =
          head_partial(acc, nh.Wt[c * kD + col0], nh.Wt[c * kD + col0 + 32], lane);
    }
    __syncthreads();
    const OdeArgs& od = nh.ode;
    int mode = od.mode;
    float hs = od.h;
    float* out = od.out;
    if (od.desc && !od.tok_event) {
      const StageDesc sd = od.desc[*od.ctr];
      mode = sd.mode;
      hs = sd.h;
      if (!sd.write_out) out = nullptr;
    }
    for (int t = tid; t < ROWS * kF; t += kThreads4) {
      const int row = t / kF, f = t % kF;
      const int64_t r = m0 + row;
      if (r >= od.m_valid) continue;
      const float* p = &part[t * kWaves4];
      const float v = ((p[0] + p[1]) + p[2]) + p[3] + nh.b[f];
      const int64_t o = r * od.ldx + f;
      if (od.tok_event) {
        const StageDesc sd = od.desc[od.tok_event[r]];
        ode_update(sd.mode, sd.h, v, od.x + o, od.acc + o, od.xs + o,
                   out && sd.write_out ? out + r * od.ldo + f : nullptr);
      } else {
        ode_update(mode, hs, v, od.x + o, od.acc + o, od.xs + o, out ? out + r * od.ldo + f : nullptr);
      }
    }
  } else {
    if constexpr (F8) {   // (the BF16 form loaded these before its last down-projection)
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        gq[nj] = nq.g[col0 + 32 * nj];
        sq[nj] = nq.s[col0 + 32 * nj];
        bq[nj] = nq.bias[col0 + 32 * nj];
      }
      ring_fill_nc<2>(ring, qkv_c(0), kOcStride, lane);
    }
    row_stats_nc(acc, sl, stats_out, m0, lane, w);   // barriers: every wave is past its
    {                                                // last read of the LN3 tile A
      const float* mu = sl.mu[w];
      const float* rs = sl.rs[w];
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        const int col = col0 + 32 * nj;
        const float gv = gq[nj], sv = sq[nj];
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int row = acc_row(mi, r, lane);
            A[row * kLdA + col] = (bf16)((acc[mi][nj][r] - mu[row]) * rs[row] * gv + sv);
          }
      }
    }
    __syncthreads();
    const int64_t plane = rm.Mp * kDh;
    float bcur[2];
#pragma unroll
    for (int nj = 0; nj < 2; ++nj) bcur[nj] = bq[nj];
#pragma unroll 1
    for (int slab = 0; slab < 3; ++slab) {
      float bnext[2];
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int r = 0; r < 16; ++r) acc[mi][nj][r] = bcur[nj];
        bnext[nj] = nq.bias[(slab < 2 ? slab + 1 : slab) * kD + col0 + 32 * nj];
      }
      mfma_phase_nc<TM, 2, kKs, 2, true>(acc, A, kLdA, 0, ring, qkv_c(slab), kOcStride,
                                         qkv_c(slab < 2 ? slab + 1 : slab), kOcStride, lane);
      // head-major: column block nj of this wave is head 2w + nj
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) {
        const RowIo<bf16, kDh> io(nq.qkv + (int64_t)(slab * (kD / kDh) + 2 * w + nj) * plane, m0,
                                  lane & 31, lane);
#pragma unroll
        for (int mi = 0; mi < TM; ++mi)
#pragma unroll
          for (int r = 0; r < 16; ++r) __builtin_nontemporal_store((bf16)acc[mi][nj][r], io.at(mi, r));
      }
#pragma unroll
      for (int nj = 0; nj < 2; ++nj) bcur[nj] = bnext[nj];
    }
  }
}

__global__ void k_pack_frag(const float* __restrict__ W, int K, int N, u32x4* __restrict__ Wf) {
  const int nks = K / 16;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)(N / 32) * nks * 64) return;
  const int lane = (int)(e % 64);
  const int ks = (int)((e / 64) % nks);
  const int nb = (int)(e / (64 * nks));
  const int n = nb * 32 + (lane & 31);
  bf16x8 v;
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = (bf16)W[(int64_t)(ks * 16 + (lane >> 5) * 8 + j) * N + n];
  Wf[e] = __builtin_bit_cast(u32x4, v);
}

// ---------------------------------------------------------------------------------------

bool fused_supported(int d_model, int n_heads, int mlp_ratio) {
  return d_model == kD && n_heads * kDh == kD && mlp_ratio == 4;
}

hipError_t launch_pack_frag(hipStream_t st, const float* W, int K, int N, void* Wf) {
  if (K % 16 || N % 32) return hipErrorInvalidValue;
  const int64_t n = (int64_t)(N / 32) * (K / 16) * 64;
  hipLaunchKernelGGL(k_pack_frag, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, K, N,
                     (u32x4*)Wf);
  return hipGetLastError();
}

// The QKV and OQC kernels come in 64-row tiles (half the accumulator: two workgroups share a
// CU and one's loads overlap the other's products) and 128-row tiles (twice the reuse of
// each weight fragment); the autotuner picks one per token-count bucket.

// Grid of a fused launch: the mapped tiles (64-row tiles only) or all of Mp.
static bool fused_grid(int64_t Mp, int rows, const int32_t* tiles, int64_t n_tiles, unsigned* grid) {
  if ((rows != 64 && rows != 128) || Mp % rows || (tiles && (rows != 64 || n_tiles > Mp / 64)))
    return false;
  *grid = (unsigned)(tiles ? n_tiles : Mp / rows);
  return true;
}

hipError_t launch_fused_qkv(hipStream_t st, int64_t Mp, const float* H, const float* g,
                            const float* s, const void* Wf, const float* bias, void* qkv,
                            int rows, const int32_t* tiles, int64_t n_tiles) {
  unsigned grid = 0;
  if (!fused_grid(Mp, rows, tiles, n_tiles, &grid)) return hipErrorInvalidValue;
  if (grid == 0) return hipSuccess;
  const RowMap rm{tiles, Mp};
  if (rows == 64)
    hipLaunchKernelGGL((k_fused_qkv<2, false>), dim3(grid), dim3(kThreads), 0, st,
                       H, g, s, (const u32x4*)Wf, bias, (bf16*)qkv, EmbedRows{}, rm);
  else
    hipLaunchKernelGGL((k_fused_qkv<4, false>), dim3(grid), dim3(kThreads), 0, st,
                       H, g, s, (const u32x4*)Wf, bias, (bf16*)qkv, EmbedRows{}, rm);
  return hipGetLastError();
}

hipError_t launch_fused_embed_qkv(hipStream_t st, int64_t Mp, const float* xs, int ldx, int f,
                                  int64_t T, const float* temb, const float* W_xin, float* H,
                                  const float* g, const float* s, const void* Wf,
                                  const float* bias, void* qkv, int rows) {
  if ((rows != 64 && rows != 128) || Mp % rows || ldx != kEmbLd || f != kEmbF9 || T > Mp)
    return hipErrorInvalidValue;
  if (Mp == 0) return hipSuccess;
  const EmbedRows em{xs, T, temb, W_xin, H};
  const RowMap rm{nullptr, Mp};
  if (rows == 64)
    hipLaunchKernelGGL((k_fused_qkv<2, true>), dim3((unsigned)(Mp / 64)), dim3(kThreads), 0, st,
                       nullptr, g, s, (const u32x4*)Wf, bias, (bf16*)qkv, em, rm);
  else
    hipLaunchKernelGGL((k_fused_qkv<4, true>), dim3((unsigned)(Mp / 128)), dim3(kThreads), 0, st,
                       nullptr, g, s, (const u32x4*)Wf, bias, (bf16*)qkv, em, rm);
  return hipGetLastError();
}

hipError_t launch_fused_oqc(hipStream_t st, int64_t Mp, const void* att, const void* Wf_o,
                            const float* b_o, float* H, const float* g, const float* s,
                            const void* Wf_qc, const float* b_qc, void* qc, int rows,
                            const int32_t* tiles, int64_t n_tiles) {
  unsigned grid = 0;
  if (!fused_grid(Mp, rows, tiles, n_tiles, &grid)) return hipErrorInvalidValue;
  if (grid == 0) return hipSuccess;
  const RowMap rm{tiles, Mp};
  if (rows == 64)
    hipLaunchKernelGGL(k_fused_oqc<2>, dim3(grid), dim3(kThreads), 0, st,
                       (const bf16*)att, (const u32x4*)Wf_o, b_o, H, g, s, (const u32x4*)Wf_qc,
                       b_qc, (bf16*)qc, rm);
  else
    hipLaunchKernelGGL(k_fused_oqc<4>, dim3(grid), dim3(kThreads), 0, st,
                       (const bf16*)att, (const u32x4*)Wf_o, b_o, H, g, s, (const u32x4*)Wf_qc,
                       b_qc, (bf16*)qc, rm);
  return hipGetLastError();
}

hipError_t launch_fused_mlp(hipStream_t st, int64_t Mp, const void* att, const void* Wf_oc,
                            const float* b_oc, float* H, const float* g, const float* s,
                            const void* Wf_up, const float* b_up, const void* Wf_dn,
                            const float* b_dn, float2* stats_out, const float* g1n,
                            const float* s1n, const void* Wf_qkv_n, const float* b_qkv_n,
                            void* qkv, const float* gf, const float* sf, const float* Wt_out,
                            const float* b_out, const OdeArgs* head, const Fp8Mlp* fp8,
                            const int32_t* tiles, int64_t n_tiles) {
  unsigned gsz = 0;
  if (!fused_grid(Mp, 64, tiles, n_tiles, &gsz)) return hipErrorInvalidValue;
  if (gsz == 0) return hipSuccess;
  const RowMap rm{tiles, Mp};
  if (qkv && head) return hipErrorInvalidValue;
  if (fp8 && (!fp8->up || !fp8->dn || !fp8->up_inv || !fp8->dn_scale || !fp8->dn_inv))
    return hipErrorInvalidValue;
  const Mlp8 f8 = fp8 ? Mlp8{(const i32x8*)fp8->up, (const i32x8*)fp8->dn, fp8->up_inv,
                             fp8->dn_scale, fp8->dn_inv}
                      : Mlp8{};
  const dim3 grid(gsz);
#define FMD_MLP_GO(TAIL, NQ, NH)                                                              \
  do {                                                                                        \
    if (fp8)                                                                                  \
      hipLaunchKernelGGL((k_fused_mlp<2, TAIL, true>), grid, dim3(kThreads4), 0, st,          \
                         (const bf16*)att, (const u32x4*)Wf_oc, b_oc, H, g, s,                \
                         (const u32x4*)Wf_up, b_up, (const u32x4*)Wf_dn, b_dn, stats_out, NQ, \
                         NH, f8, rm);                                                         \
    else                                                                                      \
      hipLaunchKernelGGL((k_fused_mlp<2, TAIL, false>), grid, dim3(kThreads4), 0, st,         \
                         (const bf16*)att, (const u32x4*)Wf_oc, b_oc, H, g, s,                \
                         (const u32x4*)Wf_up, b_up, (const u32x4*)Wf_dn, b_dn, stats_out, NQ, \
                         NH, f8, rm);                                                         \
  } while (0)
  if (qkv) {
    if (!g1n || !s1n || !Wf_qkv_n || !b_qkv_n) return hipErrorInvalidValue;
    const NextQkv nq{g1n, s1n, (const u32x4*)Wf_qkv_n, b_qkv_n, (bf16*)qkv};
    FMD_MLP_GO(kTailQkv, nq, NextHead{});
  } else if (head) {
    if (!gf || !sf || !Wt_out || !b_out || head->nf != 9) return hipErrorInvalidValue;
    const NextHead nh{gf, sf, Wt_out, b_out, *head};
    FMD_MLP_GO(kTailHead, NextQkv{}, nh);
  } else {
    FMD_MLP_GO(kTailStats, NextQkv{}, NextHead{});
  }
#undef FMD_MLP_GO
  return hipGetLastError();
}

// Per-column power-of-two scale of a K x N FP32 matrix for FP8 e4m3: s_n = 2^e with e the
// largest integer such that max_k |W[k][n]| s_n <= 448 (s_n = 1 for a zero column); inv = 1/s.
__global__ void k_fp8_col_scale(const float* __restrict__ W, int K, int N, float* __restrict__ scale,
                                float* __restrict__ inv) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= N) return;
  float mx = 0.f;
  for (int k = 0; k < K; ++k) mx = fmaxf(mx, fabsf(W[(int64_t)k * N + n]));
  int e = 0;
  if (mx > 0.f) {
    e = (int)floorf(log2f(448.0f / mx));
    while (ldexpf(mx, e) > 448.0f) --e;        // log2f may round up across a power of two
    while (ldexpf(mx, e + 1) <= 448.0f) ++e;
  }
  scale[n] = ldexpf(1.0f, e);
  inv[n] = ldexpf(1.0f, -e);
}

// FP8 fragments (layout of the Mlp8 comment) of W s_n.
__global__ void k_pack_frag8(const float* __restrict__ W, int K, int N, const float* __restrict__ scale,
                             i32x8* __restrict__ Wf) {
  const int nks = K / 64;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)(N / 32) * nks * 64) return;
  const int lane = (int)(e % 64);
  const int ks = (int)((e / 64) % nks);
  const int nb = (int)(e / (64 * nks));
  const int n = nb * 32 + (lane & 31);
  const float sc = scale[n];
  i32x8 v;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    uint32_t word = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int k = ks * 64 + (lane >> 5) * 32 + 4 * q + b;
      word |= to_fp8(W[(int64_t)k * N + n] * sc) << (8 * b);
    }
    v[q] = (int)word;
  }
  Wf[e] = v;
}

hipError_t launch_pack_frag8(hipStream_t st, const float* W, int K, int N, void* Wf, float* scale,
                             float* inv) {
  if (K % 64 || N % 32) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_fp8_col_scale, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, W, K, N,
                     scale, inv);
  const int64_t n = (int64_t)(N / 32) * (K / 64) * 64;
  hipLaunchKernelGGL(k_pack_frag8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, K, N,
                     (const float*)scale, (i32x8*)Wf);
  return hipGetLastError();
}

}  // namespace fmd
