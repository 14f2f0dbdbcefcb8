// Host-side launchers of the fmdet HIP kernels. All pointers are device pointers unless
// stated; every launcher enqueues on `st` and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fmd.h"

namespace fmd {

// EPI_RESID_LN: EPI_RESID plus the LayerNorm statistics of every updated row, written to
// OdeArgs::stats_out (needs one block per full row: tile BN == N).
enum Epi { EPI_STORE = 0, EPI_GELU = 1, EPI_RESID = 2, EPI_ODE = 3, EPI_RESID_LN = 4 };

// ODE update modes of the fused head kernel.
enum UpdMode {
  UPD_EULER = 0,      // x <- x + h v ; xs <- x
  UPD_RK4_0 = 1,      // acc <- v ;        xs <- x + h/2 v
  UPD_RK4_1 = 2,      // acc <- acc + 2v ; xs <- x + h/2 v
  UPD_RK4_2 = 3,      // acc <- acc + 2v ; xs <- x + h v
  UPD_RK4_3 = 4,      // x <- x + h/6 (acc + v) ; xs <- x
  UPD_VELOCITY = 5,   // v only, written to `out`
  UPD_NONE = 6,       // no update (rows that belong to no event)
  UPD_MID_0 = 7,      // xs <- x + h/2 v  (explicit midpoint, first stage)
  UPD_MID_1 = 8       // x <- x + h v ; xs <- x
};

constexpr int kStateLd = 16;       // row stride (floats) of the device ODE state arrays

// One ODE stage of a schedule: evaluation time, step, update mode (UpdMode) and whether
// this stage writes the caller's output. A call uploads its stages once; a device
// counter selects the current one, so one captured graph replays every stage.
struct StageDesc {
  float t, h;
  int32_t mode, write_out;
};

// Fused ODE update in a GEMM epilogue (EPI_ODE): the GEMM result v[r, c] for c < nf and
// r < m_valid updates state element (r, c). With desc and tok_event set, mode, h and the
// output write of row r come from desc[tok_event[r]] (one entry per event: the serving
// loop); with desc alone from desc[*ctr] (one entry per stage); otherwise from the fields.
struct OdeArgs {
  float* x;
  float* acc;
  float* xs;
  float* out;       // optional [m_valid, ldo] copy of the new state (or of v)
  int64_t m_valid;
  int ldx, ldo, nf, mode;
  float h;
  const StageDesc* desc;
  const int32_t* ctr;
  const int32_t* tok_event;
  float2* stats_out;   // EPI_RESID_LN only
};
constexpr int kGemmBM = 256;       // largest GEMM row tile; token buffers are padded to this

// C = epi(pro(A) W + b). A: float [Mp, lda] if ln, else T [Mp, lda]. Wt: T [N, K]
// (the transpose of the [K, N] weight). C: T [Mp, ldc] for STORE/GELU, float for RESID.
// With ln, stats holds (mean, 1/sqrt(var + eps)) of every row of A (launch_row_stats)
// and pro(A) = (A - mean) * rstd * g + s.
// Requires Mp % 256 == 0, K % 32 == 0, N % 64 == 0 and a tiling that divides the shape.
// `cls` (an FMD_K_* class) selects the kernel name the launch appears under in profiles;
// `tile` picks one of the candidate tilings (gemm_body.h), -1 the default for N.
template <typename T>
hipError_t launch_gemm(hipStream_t st, int cls, bool ln, int epi, int64_t Mp, int N, int K,
                       const void* A, int lda, const T* Wt, const float* bias,
                       const float2* stats, const float* g, const float* s, void* C, int ldc,
                       const OdeArgs* ode = nullptr, int tile = -1);

// Candidate GEMM tilings the autotuner chooses from, and whether one divides a shape.
constexpr int kGemmTiles = 7;
// full_rows: the tiling must give one block the whole row (BN == N), as EPI_RESID_LN needs.
bool tile_fits(int tile, int64_t Mp, int N, int K, bool full_rows = false);
int default_tile(int N);
int default_tile_rows(int N);   // a full-row tiling for N, or -1

// LayerNorm statistics of the rows of a float [M, ld] matrix over its first K columns:
// stats[r] = (mean, 1/sqrt(biased var + eps)), two passes in registers, one wave per row.
hipError_t launch_row_stats(hipStream_t st, const float* A, int ld, int K, int64_t M,
                            float2* stats);

// Queries per attention work item (event, query tile) for a precision and head shape, by
// default; BF16 with heads of 32 also accepts the tiles of attention_query_tiles (64, 128, 192),
// among which the autotuner chooses. The work lists passed to launch_attention are built
// with the tile it is given.
int attention_query_tile(bool bf16, int dh, int n_heads);
int attention_query_tiles(bool bf16, int dh, int* tiles);   // candidates; returns their count

// Attention work list split into kAttnBins bins of whole events with about equal work, each
// bin's items stored contiguously (bin i: items [start[i], start[i] + len[i])). Workgroup b
// of the BF16 kernel takes bin b % kAttnBins, so that all workgroups of an event land on one
// XCD (workgroups are dealt to the 8 XCDs round-robin) and share its L2.
constexpr int kAttnBins = 8;
struct AttnBins {
  int32_t start[kAttnBins], len[kAttnBins];
  int32_t max_len;
};
// One attention work item: a query tile of one event, with its rows: queries
// [q0, q0 + nq) (nq <= the query tile) against the event's keys [k0, k0 + nk).
struct AttnItem {
  int32_t q0, nq, k0, nk;
};
// Fills `items` (capacity >= sum over the events of ceil(n_q / qt)) for the events ids[0..n)
// of the CSR offsets q_off / kv_off (host arrays): events with the most work first within
// each bin, bins balanced by attention work (longest-processing-time assignment); events
// without queries get no item. Returns the item count, or -1 if a row index exceeds 2^31-1.
int64_t build_attention_work(const int64_t* q_off, const int64_t* kv_off, const int64_t* ids,
                             int64_t n, int qt, AttnItem* items, AttnBins* bins);
// As build_attention_work, with the keys of event e at rows kv_start[e] .. + kv_len[e] (for
// key sets that are not one CSR sequence, e.g. truth rows of pooled requests).
int64_t build_attention_work_kv(const int64_t* q_off, const int64_t* kv_start,
                                const int64_t* kv_len, const int64_t* ids, int64_t n, int qt,
                                AttnItem* items, AttnBins* bins);

// Masked multi-head attention over ragged events, one work item per (event, query tile).
// Element (row, head, dim) of Q sits at Q[row * ldq + head * hsq + dim], of K / V at
// [row * ldkv + head * hskv + dim], of O at [row * ldo + head * hso + dim]: hs = dh for
// row-major [rows, heads x dh] operands, ld = dh and hs = plane size for head-major ones
// (BF16 with dh 32 only).
template <typename T>
hipError_t launch_attention(hipStream_t st, bool cross, int dh, int n_heads, int qt,
                            int64_t n_items, const AttnBins& bins,
                            const AttnItem* work, const T* Q, int ldq, int64_t hsq, const T* K,
                            const T* V, int ldkv, int64_t hskv, T* O, int ldo, int64_t hso);

hipError_t launch_token_map(hipStream_t st, const int64_t* off, int64_t E, int64_t T,
                            int32_t* tok_event);

// x0 noise into x [T, ldx] (features >= n_feat and < ldx zeroed); also into xs if non-null.
hipError_t launch_noise(hipStream_t st, uint64_t seed, const int64_t* off,
                        const int32_t* tok_event, int64_t T, int n_feat, float* x, float* xs,
                        int ldx);

// Copies a [T, f] state into the padded [T, ldx] arrays x and xs (xs may be null).
hipError_t launch_load_state(hipStream_t st, const float* src, int f, int64_t T, float* x,
                             float* xs, int ldx);

template <typename T>
hipError_t launch_truth_encode(hipStream_t st, const float* u, int ldu, int f, int64_t T_,
                               const float* W, const float* b, const float* g,
                               const float* s, int d, T* c, int ldc);

// temb[e, :] = b_xin + b_time + phi(t_e) W_time for e < n; t_e = t_ev[e] if t_ev is set,
// else desc[*ctr].t if desc is set, else t_uniform.
hipError_t launch_time_embed(hipStream_t st, const float* t_ev, const StageDesc* desc,
                             const int32_t* ctr, float t_uniform, int n, const float* W_time,
                             const float* b_time, const float* b_xin, int E_dim, int d,
                             float* temb);

// Stage counter control: *ctr = v, and *ctr += 1 (one thread; the last kernel of a stage).
hipError_t launch_set_counter(hipStream_t st, int32_t* ctr, int32_t v);
hipError_t launch_stage_advance(hipStream_t st, int32_t* ctr);

// H[r, :] = temb[tok_event[r] or 0, :] + xs[r, :f] W_xin, with the LayerNorm
// statistics of every new row written to stats[r].
hipError_t launch_embed(hipStream_t st, const float* xs, int ldx, int f, int64_t T,
                        const int32_t* tok_event, const float* temb, const float* W_xin,
                        int d, float* H, int ldh, float2* stats);

// v = (alpha + beta t) xs, then the same ODE update, with t, h, mode and the output write
// taken from desc[*ctr].
// Output head for d_model 256 and 9 features: ode-update(LN(H; stats, g, s) Wt^T + b) over
// the ode.m_valid valid rows, Wt float [>= 9, 256] (row c: weights of output c).
// One block's BF16 cross K/V rows [rows][2d] into the head-major cache planes (plane rows
// each; this block's first plane at dst): rows land at [row0, row0 + rows).
hipError_t launch_kv_headmajor(hipStream_t st, const void* src, int64_t rows, int d, int dh,
                               int n_heads, void* dst, int64_t plane, int64_t row0);
// Event observables (H_T, MET per event; lepton isolation per particle, NaN otherwise) of
// reconstructed particles feat [rows, ldf] FP32 with device CSR offsets.
hipError_t launch_event_observables(hipStream_t st, const float* feat, int ldf,
                                    const int64_t* off_device, int64_t n_events, float* ht,
                                    float* met, float* iso);
// Truth preprocessing: per-event keep flags and counts (pass 1), then the kept rows in input
// order at off_out (pass 2); see fmd_truth_select.
// Reco multiplicity per event under the stand-in law (cnt [E] int32; off device [E + 1]).
hipError_t launch_reco_counts(hipStream_t st, const int64_t* off, int64_t n_events, uint64_t seed,
                              uint64_t thr_q, uint64_t thr_p, int fake_trials, int n_max,
                              int32_t* cnt);
hipError_t launch_select_count(hipStream_t st, const float* feat, int ldf, const int64_t* off,
                               int64_t n_events, float c0, int limit, uint8_t* keep,
                               int32_t* cnt);
hipError_t launch_select_write(hipStream_t st, const float* feat, int ldf, const int64_t* off,
                               const int64_t* off_out, int64_t n_events, const uint8_t* keep,
                               float* out);
bool head256_supported(int d, int nf);
hipError_t launch_head256(hipStream_t st, const float* H, const float2* stats, const float* g,
                          const float* s, const float* Wt, const float* b, const OdeArgs& ode);

hipError_t launch_linear_update(hipStream_t st, float alpha, float beta, const StageDesc* desc,
                                const int32_t* ctr, int64_t T, int f, float* x, float* acc,
                                float* xs, int ldx, float* out, int ldo);

// Wt[n, k] = T(W[k, n]) for a [K, N] row-major FP32 matrix.
template <typename T>
hipError_t launch_pack_weight(hipStream_t st, const float* W, int K, int N, T* Wt);

// Fused BF16 block kernels for d = 256 with 8 heads of 32 and a 4x MLP (block_bf16.hip):
// their Q/K/V and cross-query stores are 8 head-major planes of width 32. Row counts Mp are
// multiples of 128; weights are in the fragment layout of launch_pack_frag.
bool fused_supported(int d_model, int n_heads, int mlp_ratio);
// W: FP32 K x N (y = x W) -> BF16 MFMA B fragments [N/32][K/16][64 lanes][8].
hipError_t launch_pack_frag(hipStream_t st, const float* W, int K, int N, void* Wf);
// [Q | K | V] = LN(H; g, s) Wqkv + b, head-major: qkv [3][8 heads][Mp][32] (plane = Mp x 32).
// rows: the workgroup's row tile, 64 or 128 (the autotuner's candidates; same results).
// tiles (optional, device int32 [n_tiles]): run only these 64-row tiles (rows must be 64).
hipError_t launch_fused_qkv(hipStream_t st, int64_t Mp, const float* H, const float* g,
                            const float* s, const void* Wf, const float* bias, void* qkv,
                            int rows = 64, const int32_t* tiles = nullptr, int64_t n_tiles = 0);
// As launch_fused_qkv for block 0, with the input embedding formed in the kernel for a
// stage time shared by every row: H rows [0, T) = temb[0..255] + xs[r][0..8] W_xin (the
// order of launch_embed's d = 256 kernel, so H is the same; rows [T, Mp) are zero) are
// written to H and feed LN1 + QKV. xs has pitch 16 and at least Mp rows; f must be 9.
hipError_t launch_fused_embed_qkv(hipStream_t st, int64_t Mp, const float* xs, int ldx, int f,
                                  int64_t T, const float* temb, const float* W_xin, float* H,
                                  const float* g, const float* s, const void* Wf,
                                  const float* bias, void* qkv, int rows = 64);
// H += att Wo + b_o;  qc = LN(H; g, s) Wqc + b_qc, head-major: qc [8 heads][Mp][32]. The
// attention output att is head-major [8 heads][Mp][32] as well. rows: 64 or 128.
hipError_t launch_fused_oqc(hipStream_t st, int64_t Mp, const void* att, const void* Wf_o,
                            const float* b_o, float* H, const float* g, const float* s,
                            const void* Wf_qc, const float* b_qc, void* qc, int rows = 64,
                            const int32_t* tiles = nullptr, int64_t n_tiles = 0);
// att (head-major [8 heads][Mp][32]): H += att Woc + b_oc;  H += GELU(LN(H; g, s) Wup + b_up) Wdn + b_dn;  stats_out = LN stats of
// H. With qkv set, also the next block's [Q | K | V] = LN(H; g1n, s1n) Wqkv_n + b_qkv_n into
// qkv, head-major like launch_fused_qkv (the next block then skips its QKV kernel). With head
// set instead (the last block, 9 features), the output head LN_f(H; gf, sf) Wt_out^T + b_out
// and the ODE update of *head, as launch_head256 does; H is then not written.
// FP8 operands of the MLP's two projections (the FP8 precision form): FP8 e4m3 fragments of
// W_up s_up and W_dn s_dn (launch_pack_frag8) with the power-of-two column scales.
struct Fp8Mlp {
  const void* up;          // [1024/32][256/64][64 lanes][32 bytes]
  const void* dn;          // [256/32][1024/64][64 lanes][32 bytes]
  const float* up_inv;     // 1 / s_up [1024]
  const float* dn_scale;   // s_dn [256]
  const float* dn_inv;     // 1 / s_dn [256]
};
// W: FP32 K x N -> FP8 e4m3 fragments of W diag(scale) [N/32][K/64][64 lanes][32 bytes], with
// scale[n] the power of two that brings the column's largest magnitude into (224, 448] and
// inv[n] = 1 / scale[n] (both written, device [N]). K % 64 == 0, N % 32 == 0.
hipError_t launch_pack_frag8(hipStream_t st, const float* W, int K, int N, void* Wf, float* scale,
                             float* inv);
hipError_t launch_fused_mlp(hipStream_t st, int64_t Mp, const void* att, const void* Wf_oc,
                            const float* b_oc, float* H, const float* g, const float* s,
                            const void* Wf_up, const float* b_up, const void* Wf_dn,
                            const float* b_dn, float2* stats_out, const float* g1n = nullptr,
                            const float* s1n = nullptr, const void* Wf_qkv_n = nullptr,
                            const float* b_qkv_n = nullptr, void* qkv = nullptr,
                            const float* gf = nullptr, const float* sf = nullptr,
                            const float* Wt_out = nullptr, const float* b_out = nullptr,
                            const OdeArgs* head = nullptr, const Fp8Mlp* fp8 = nullptr,
                            const int32_t* tiles = nullptr, int64_t n_tiles = 0);

// dst[i] = T(src[i]).
template <typename T>
hipError_t launch_convert(hipStream_t st, const float* src, int64_t n, T* dst);
template <typename T>
hipError_t launch_to_f32(hipStream_t st, const T* src, int64_t n, float* dst);

hipError_t launch_philox(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t* ctr,
                         int64_t n, uint64_t* out);

hipError_t launch_pack_padded(hipStream_t st, const float* padded, const int32_t* lengths,
                              int64_t E, int n_max, int f, int64_t* off_out, float* feat_out);

}  // namespace fmd
