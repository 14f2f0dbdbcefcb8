/*
 * fmd.h — C ABI of fmdet, conditional flow-matching detector simulation on MI355X.
 *
 * The library computes  simulate(truth particle sets, seed, step schedule) -> reco sets.
 * This is the problem the paper states for its detector backends (arXiv 2606.26089,
 * program summary and Sec. 1): truth-level particles go in, detector-level
 * reconstructed particles come out. The method is the neural backend (Sec. 2.2): a
 * continuous-time model trained by conditional flow matching and conditioned on the
 * event's truth particles. It is sampled by integrating its vector field from Gaussian
 * noise with a run-time number of steps (App. C, generator block: num_steps,
 * batch_size). The velocity network is a stand-in with caller-supplied weights.
 *
 * Conventions for every call:
 *  - Every function returns an fmd_status. On a non-OK status, fmd_last_error() gives a
 *    message for the calling thread, and no output buffer has been written.
 *  - Nothing aborts, and no C++ exception crosses this interface.
 *  - hip_stream is a hipStream_t, or NULL for the null stream. Work is enqueued
 *    asynchronously on that stream. Device inputs are borrowed until that work
 *    completes, and device outputs are valid only after it completes.
 *  - Host arrays passed in are consumed before the call returns. For calls whose results
 *    go to host memory, the call synchronises the stream before returning.
 *  - A model is bound to the HIP device that was current at fmd_model_create(). Calls on
 *    one model share its workspace, so they must be issued on one stream or serialised
 *    by the caller.
 *  - Particle sets are CSR. `offsets` is int64[n_events + 1], offsets[0] = 0,
 *    non-decreasing, always in HOST memory. `feat` is float32
 *    [offsets[n_events], n_feat], row-major, in host or device memory as `on_device`
 *    says. Event e owns rows [offsets[e], offsets[e+1]). Empty events are legal and
 *    produce no rows.
 *  - There is one reco particle slot per truth particle, so reco sets use the truth
 *    offsets.
 */
#ifndef FMD_H
#define FMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FMD_OK = 0,
  FMD_PENDING = 1,          /* server: request not finished yet */
  FMD_E_INVALID = -1,       /* bad argument (null pointer, bad offsets, bad config) */
  FMD_E_NOMEM = -2,         /* device or host allocation failed */
  FMD_E_BUDGET = -3,        /* server: request can never fit the HBM budget */
  FMD_E_UNSUPPORTED = -4,   /* valid but unsupported (event larger than n_max, head dim) */
  FMD_E_DEVICE = -5,        /* HIP runtime error */
  FMD_E_STATE = -6          /* wrong object state (destroyed server, unknown request) */
} fmd_status;

typedef struct fmd_model fmd_model;     /* opaque */

/* Precision of GEMM / attention operands. FMD_FP8: the BF16 form with the two MLP projections
 * on FP8 (OCP e4m3) operands: the LayerNorm output and the GELU output rounded to e4m3, W_up
 * and W_dn times a power of two per output column rounded to e4m3, FP32 accumulation; the
 * paper lets the user trade generation speed for quality (Sec. 2.2), and this is one more
 * such step. It exists for the fused kernels' shape only (d_model 256, 8 heads of 32, MLP
 * ratio 4; FMD_E_UNSUPPORTED otherwise). */
enum { FMD_FP32 = 0, FMD_BF16 = 1, FMD_FP8 = 2 };
/* integration scheme: Euler (one evaluation per step, the paper's), classic RK4 (four),
 * explicit midpoint (two: x <- x + h v(x + h/2 v(x, t), t + h/2)) */
enum { FMD_EULER = 0, FMD_RK4 = 1, FMD_MIDPOINT = 2 };

/* Network shape. Supported: d_model = n_heads * dh with dh in {16, 32, 64}; d_model a
 * multiple of 64; mlp_ratio = 4; t_embed_dim = 32; f_truth = f_reco = 9; 1 <= n_max <= 4096.
 * precision FMD_FP32 runs every GEMM and attention product as FP32 MFMA. FMD_BF16 feeds
 * BF16 operands to the MFMA with FP32 accumulation. In both, the residual stream,
 * LayerNorm and softmax statistics, the output head and the ODE state stay FP32. */
typedef struct {
  int32_t d_model, n_blocks, n_heads, mlp_ratio, t_embed_dim, f_truth, f_reco, n_max, precision;
} fmd_model_config;

typedef struct {
  int64_t n_events;
  const int64_t* offsets;   /* host, [n_events + 1] */
  const float* feat;        /* [offsets[n_events], f_truth] FP32 */
  int32_t on_device;        /* 1: feat is device memory, 0: host memory */
} fmd_events_in;

typedef struct {
  float* feat;              /* [offsets[n_events], f_reco] FP32, caller-allocated */
  int32_t on_device;
} fmd_events_out;

/* Uniform grid t_k = t0 + k h, h = (t1 - t0) / n_steps. Noise sits at t0, data at t1.
 * The paper uses Euler with n_steps = 50 by default (Sec. 2.2, App. C). Classic RK4
 * evaluates the field at t_k, t_k + h/2 (twice) and t_k + h. */
typedef struct {
  int32_t scheme, n_steps;
  double t0, t1;
} fmd_schedule;

/* ---- model ------------------------------------------------------------------------ */

/* Number of FP32 parameters of a config, in the flat order below. Returns 0 for an
 * invalid config.
 * Flat order (every matrix is [in, out] row-major, applied as y = x W + b; d = d_model,
 * F = 9, E = t_embed_dim, R = mlp_ratio):
 *   W_tin[F,d] b_tin[d] g_t[d] s_t[d]  W_xin[F,d] b_xin[d]  W_time[E,d] b_time[d]
 *   per block: g1 s1 W_qkv[d,3d] b_qkv[3d] W_o[d,d] b_o  g2 s2 W_qc[d,d] b_qc W_kc[d,d] b_kc
 *              W_vc[d,d] b_vc W_oc[d,d] b_oc  g3 s3 W_up[d,Rd] b_up[Rd] W_dn[Rd,d] b_dn
 *   g_f s_f W_out[d,F] b_out[F]
 * The columns of W_qkv are [Q | K | V]; head h owns columns [h dh, (h+1) dh) of each.
 * The network:
 *   c  = LN_t(u W_tin + b_tin)                                   (truth encoding)
 *   H  = x W_xin + b_xin + phi(t) W_time + b_time,   phi(t) = [sin(w_k t) | cos(w_k t)],
 *        w_k = 10000^(-k/(E/2))
 *   per block: H += MHA(LN1 H, LN1 H) W_o + b_o; H += MHA(LN2 H, c) W_oc + b_oc;
 *              H += GELU(LN3(H) W_up + b_up) W_dn + b_dn
 *   v  = LN_f(H) W_out + b_out
 * Attention is restricted to the event's own particles. LayerNorm uses eps 1e-5 and the
 * biased variance. GELU is the exact erf form. */
size_t fmd_param_count(const fmd_model_config* cfg);

/* Copies `params` (host, n_params FP32 values in the flat order above) to the current
 * device, repacked for the kernels (BF16 with round-to-nearest-even for FMD_BF16). The
 * caller keeps ownership of `params`. *out receives a new handle. */
int fmd_model_create(const fmd_model_config* cfg, const float* params, size_t n_params,
                     fmd_model** out);
int fmd_model_destroy(fmd_model* m);

/* Analytic test field v(x, t) = (alpha + beta t) x. The handle runs the same integrator
 * and state-update kernels as a network model. Its closed-form solution pins them:
 * Euler gives prod_k (1 + h (alpha + beta t_k)) x0. Creating it touches no device, so
 * argument validation can be exercised without a GPU. */
int fmd_linear_field_create(double alpha, double beta, fmd_model** out);

/* ---- sampling ----------------------------------------------------------------------- */

/* Draws x0 ~ N(0, 1) for every reco slot from the seed, integrates the flow over the
 * schedule, and writes the state at t1 (raw 9-feature rows, same layout as the truth
 * features) to reco->feat.
 * The noise of slot i of event e is Philox4x64-10 (Salmon et al., SC'11) of counter
 * (b, i, e, 0) with key (seed, 0), b = 0, 1, 2 for features 0-3, 4-7, 8. Each 64-bit
 * word w gives u = ((w >> 41) + 1/2) 2^-23. Box-Muller on word pairs (0,1), (2,3) gives
 * r = sqrt(-2 ln u_a): z_a = r cos(2 pi u_b), z_b = r sin(2 pi u_b).
 * e is the event's index within this call, so an event's result does not depend on the
 * other events of the call.
 * With device input and output the call only enqueues work: it does not wait for earlier
 * work on the stream (its host-built arrays go through two pinned staging sets used by
 * alternate calls, so it waits at most for the uploads of the call two calls back). The
 * first call whose padded size falls in a new power-of-two bucket also times the
 * autotuner's candidates, and waits for them.
 * Errors: FMD_E_INVALID (null pointers, bad offsets, n_steps < 1, unknown scheme,
 * t1 == t0); FMD_E_UNSUPPORTED (an event with more than n_max particles). */
int fmd_simulate(fmd_model* m, const fmd_events_in* truth, uint64_t seed,
                 const fmd_schedule* schedule, fmd_events_out* reco, void* hip_stream);

/* As fmd_simulate, with a reco multiplicity per event given by the caller (the model can
 * emit more or fewer reco particles than truth particles, Sec. 2.2; how the count is chosen
 * the paper does not describe, so it is an input here). The reco slots of event e are rows
 * reco_offsets[e] .. reco_offsets[e + 1] - 1 of reco->feat ([reco_offsets[n], f_reco] FP32,
 * where reco->on_device says); they self-attend and cross-attend to the event's truth
 * particles. reco_offsets is a host array [n_events + 1], read during the call only; slot i
 * of event e draws the noise fmd_simulate describes for (e, i), whatever the truth count.
 * With reco_offsets equal to truth->offsets the result equals fmd_simulate's.
 * Errors: as fmd_simulate; FMD_E_INVALID also for null or decreasing reco offsets and for
 * reco slots in an event without truth particles; FMD_E_UNSUPPORTED for more than n_max
 * reco slots in an event. */
int fmd_simulate_reco(fmd_model* m, const fmd_events_in* truth, const int64_t* reco_offsets,
                      uint64_t seed, const fmd_schedule* schedule, fmd_events_out* reco,
                      void* hip_stream);

/* Reco multiplicities drawn on the device before sampling, for fmd_simulate_reco. The paper's
 * model can emit particles that correspond to no truth particle (pile-up-like "fake"
 * particles it generates implicitly, Sec. 2.2 and the configuration appendix on pile-up) but
 * does not say how their number is drawn; this is a stand-in law. For event e (index within
 * the call) with N truth particles: N_reco = min(n_max, N - lost + fakes) if N > 0, else 0,
 * where lost counts the truth particles missed (each with probability loss_prob) and fakes
 * the successes of fake_trials Bernoulli trials of probability fake_prob. Every trial
 * compares one 64-bit word of Philox4x64-10 (key (seed, 1), counters (c, e, 0, 0), four words
 * per counter: the N loss words first, then the fake words) with floor(prob 2^64), so the
 * counts are exact integers, independent of the other events of the call and of the slot
 * noise (key (seed, 0)).
 * truth_offsets: HOST int64 [n_events + 1], offsets[0] = 0, nondecreasing. reco_offsets_out:
 * HOST int64 [n_events + 1], written (reco_offsets_out[0] = 0). Returns after the results are
 * complete. Errors: FMD_E_INVALID (null pointers, bad offsets, probabilities outside [0, 1),
 * fake_trials outside [0, 4096], n_max < 0), FMD_E_NOMEM, FMD_E_DEVICE. */
typedef struct {
  double loss_prob;      /* probability that a truth particle gets no reco slot, [0, 1) */
  double fake_prob;      /* success probability of each fake trial, [0, 1) */
  int32_t fake_trials;   /* Bernoulli trials for extra slots, [0, 4096] */
} fmd_multiplicity_law;

int fmd_reco_multiplicity(const int64_t* truth_offsets, int64_t n_events, uint64_t seed,
                          const fmd_multiplicity_law* law, int32_t n_max, int64_t* reco_offsets_out,
                          void* hip_stream);

/* As fmd_simulate, but starts from a given state x0 [offsets[n], f_reco] FP32. x0 lives
 * where truth->feat lives (on_device). Passage: Sec. 2.2 (the sampler integrates the learned
 * vector field from a starting sample; here the caller supplies that sample instead of the
 * seeded noise, which lets tests pin the integrator against closed forms). */
int fmd_simulate_from_state(fmd_model* m, const fmd_events_in* truth, const float* x0,
                            const fmd_schedule* schedule, fmd_events_out* reco,
                            void* hip_stream);

/* One evaluation of the velocity field: v = v(x, t_e | truth). x and v are
 * [offsets[n], f_reco] FP32. t_per_event is [n_events] FP32. All three live where
 * truth->feat lives. Passage: Sec. 2.2 (the learned vector field over the reco set,
 * conditioned on the event's truth particles, at continuous time t). */
int fmd_velocity(fmd_model* m, const fmd_events_in* truth, const float* x,
                 const float* t_per_event, float* v, void* hip_stream);

/* The initial noise alone: x0 [offsets[n_events], n_feat] FP32 in DEVICE memory, with
 * n_feat <= 12 and the law of fmd_simulate. Passage: Sec. 2.2 (flow-matching samples start
 * from Gaussian noise); the counter-based law is this library's reading. The call ends with
 * the stream synchronized. Errors: FMD_E_INVALID (bad offsets, n_feat), FMD_E_NOMEM,
 * FMD_E_DEVICE. */
int fmd_noise(uint64_t seed, const int64_t* offsets, int64_t n_events, int32_t n_feat,
              float* x0_device, void* hip_stream);

/* Event observables of reconstructed events (Sec. 2.4, event post-processing, and its
 * isolation equation): per event the scalar sum H_T of the particles' pT and MET, the
 * magnitude of their vector pT sum; per particle the isolation of an electron or muon,
 * R_iso = (sum of the pT of the event's other particles with Delta R = sqrt(Delta eta^2 +
 * Delta phi^2) < 0.4) / its own pT, and NaN for the other classes.
 * reco: n_events, offsets (HOST array [n_events + 1], offsets[0] = 0, nondecreasing) and feat
 * [offsets[n_events], 9] FP32 in the particle state layout of fmd_simulate's output; the
 * kinematics are pT = 10 GeV exp(x0), eta = x1, phi = x2 and the class is the first
 * maximum of x3..x7 (charged hadron, electron, muon, neutral hadron, photon).
 * ht, met [n_events] and iso [offsets[n_events]] FP32 are written in the memory reco->feat
 * lives in (reco->on_device). Delta phi is wrapped by multiples of 2 pi; the cone test and
 * the class maximum are taken in FP32, pT and all sums in FP64. The final-state-radiation
 * photon exclusion is not applied (the paper does not define it). The call returns after
 * the results are complete. Errors: FMD_E_INVALID (bad offsets, null pointers),
 * FMD_E_NOMEM, FMD_E_DEVICE. */
int fmd_event_observables(const fmd_events_in* reco, float* ht, float* met, float* iso,
                          void* hip_stream);

/* Truth preprocessing before sampling: the model's selection of truth particles (the neural
 * backend's pT cut and particle limit come with the released model: 0.25 GeV and 400
 * particles for the CMS model, 0.5 GeV and 128 for the ALEPH one; Sec. 2.2 and the
 * configuration reference appendix). A particle survives when pT > pt_cut_gev, decided as
 * x0 > (float)ln(pt_cut_gev / 10) on the state value x0 = ln(pT / 10 GeV); an event with
 * more than max_particles survivors keeps the max_particles of largest x0 (equal x0: the
 * earlier one). Kept particles stay in input order; the event count is unchanged (events may
 * become empty).
 * truth: offsets on the HOST, feat [offsets[n], 9] FP32 in device or host memory
 * (on_device). offsets_out: HOST int64 [n_events + 1], written. feat_out: same memory kind
 * as truth->feat, capacity offsets[n_events] rows; rows [0, offsets_out[n_events]) written.
 * Returns after the results are complete. Errors: FMD_E_INVALID (bad offsets, null
 * pointers, pt_cut_gev <= 0, max_particles < 0), FMD_E_NOMEM, FMD_E_DEVICE. */
int fmd_truth_select(const fmd_events_in* truth, double pt_cut_gev, int32_t max_particles,
                     int64_t* offsets_out, float* feat_out, void* hip_stream);

/* As fmd_truth_select, for callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): no device or pinned memory
 * is allocated. Every intermediate buffer (device offsets, per-event counts, keep flags) lives
 * in one fixed device array of the library, 9.5 MiB per GPU, held from the first call on a
 * device until the process ends. Limits: n_events <= 65536 and offsets[n_events] <= 8388608
 * (2^23) particles, else FMD_E_UNSUPPORTED; truth->feat and feat_out must be DEVICE memory
 * (truth->on_device = 1), else FMD_E_INVALID. Results are those of fmd_truth_select bit for
 * bit; offsets_out is a HOST array [n_events + 1], written; the call returns after the
 * results are complete. All calls on one GPU share its array: calls from different host
 * threads are serialized by the library, but work of one call that overlaps another's on the
 * same GPU (for instance replays of captured work on several streams) races on it. */
int fmd_truth_select_noalloc(const fmd_events_in* truth, double pt_cut_gev, int32_t max_particles,
                             int64_t* offsets_out, float* feat_out, void* hip_stream);

/* Ragged packing. `padded` is [n_events, n_max, f] FP32 (device), lengths is int32
 * [n_events] (device); lengths are clamped to [0, n_max]. The call writes offsets_out
 * int64[n_events + 1] (device, exclusive prefix sum of the lengths) and feat_out
 * [sum(lengths), f] (device, rows of each event in order). Pad rows are never read.
 * The capacity of feat_out is n_events * n_max rows. Passage: none in the paper's method
 * (a data-layout helper: the paper batches a fixed number of events padded to the model's
 * particle limit, App. C batch_size; this library works on packed CSR sets instead). */
int fmd_pack_padded(const float* padded, const int32_t* lengths, int64_t n_events,
                    int32_t n_max, int32_t f, int64_t* offsets_out, float* feat_out,
                    void* hip_stream);

/* Raw Philox4x64-10 blocks, for bit-exact checks of the noise generator: for i < n,
 * out[i] = Philox4x64-10(counters[i], key = (key0, key1)). counters and out are uint64
 * [n, 4] in DEVICE memory. */
int fmd_debug_philox(uint64_t key0, uint64_t key1, const uint64_t* counters, int64_t n,
                     uint64_t* out, void* hip_stream);

/* ---- instrumentation ----------------------------------------------------------------- */

/* Kernel classes timed by HIP events on the launch stream when timing is on. */
/* QKV: LN1 + [Q|K|V] projection (a GEMM, or the fused kernel); PROJ: self- and
 * cross-attention output projections with the residual update; QC: LN2 + cross-attention
 * query projection; UP: LN3 + MLP up + GELU; DOWN: MLP down with the residual update;
 * FUSED_OQC: the fused kernel for PROJ (self) + QC; FUSED_MLP: the fused kernel for
 * PROJ (cross) + UP + DOWN; OTHER: everything else (embedding, head with the state update,
 * statistics, noise, truth encoding, bookkeeping). */
enum { FMD_K_GEMM_QKV = 0, FMD_K_GEMM_PROJ = 1, FMD_K_GEMM_QC = 2, FMD_K_GEMM_UP = 3,
       FMD_K_GEMM_DOWN = 4, FMD_K_FUSED_OQC = 5, FMD_K_FUSED_MLP = 6, FMD_K_ATTN_SELF = 7,
       FMD_K_ATTN_CROSS = 8, FMD_K_OTHER = 9, FMD_K_COUNT = 10 };

/* Turns on (1) or off (0) per-launch timing of the kernel classes above and clears the
 * counters. Timing brackets each launch with events and adds a little host overhead. */
int fmd_timing_enable(fmd_model* m, int32_t enable);

/* Reads the counters of one class: total device milliseconds, number of launches, and the
 * algorithmic work summed over those launches: `flops` counts the method's floating-point
 * operations (no padding rows, no recomputation), `bytes` the HBM traffic of reading every
 * operand and writing every result exactly once. Any output pointer may be NULL.
 * Synchronises the device. */
int fmd_timing_read(fmd_model* m, int32_t kernel_class, double* total_ms, int64_t* launches,
                    double* flops, double* bytes);

/* Name of the HIP kernel behind a class, as rocprofv3 reports it (static string). */
const char* fmd_kernel_name(fmd_model* m, int32_t kernel_class);

/* ---- launch mode --------------------------------------------------------------------- */

/* While enabled (the default), the kernels of one ODE stage are captured once per call
 * shape into a HIP graph on the model's private stream. The graph is replayed once per
 * stage: time, step and update mode come from a per-call stage table in device memory. A
 * later call with the same token count, event count, output buffer and workspace reuses
 * the graph without re-capturing it. With timing on, or with graphs disabled, the same
 * kernels are launched one by one. Results are identical either way. */
int fmd_graphs_enable(fmd_model* m, int32_t enable);

/* Fused block kernels (BF16 models with d_model 256 and MLP ratio 4; on by default there).
 * Each transformer block then runs as three matrix-core kernels around the two attention
 * kernels: LN1 + QKV; the self-attention output projection with the residual update, LN2
 * and the cross-attention query; the cross-attention output projection with the residual
 * update, LN3 and the whole MLP with its residual update. Every 128-row tile keeps its FP32
 * residual rows in registers and its LayerNorm / hidden activations in LDS, so the MLP
 * hidden layer never reaches device memory. Results agree with the unfused kernels to BF16
 * rounding, not bitwise (different summation order and LayerNorm statistics computed in
 * the kernel). `mask` selects the segments that use their fused kernel (FMD_FUSED_*; the
 * others run the GEMM kernels); 0 selects the GEMM kernels throughout. FMD_FUSED_EMBED
 * (with FMD_FUSED_QKV) forms the input embedding inside block 0's QKV kernel instead of a
 * kernel of its own; the embedded rows are the same either way. A mask outside
 * [0, FMD_FUSED_ALL] is FMD_E_INVALID; a nonzero mask on a model without the fused kernels
 * is FMD_E_UNSUPPORTED. */
enum { FMD_FUSED_QKV = 1, FMD_FUSED_OQC = 2, FMD_FUSED_MLP = 4, FMD_FUSED_EMBED = 8,
       FMD_FUSED_ALL = 15 };
int fmd_fused_enable(fmd_model* m, int32_t mask);

/* ---- tile autotuner ------------------------------------------------------------------- */

/* The GEMM sites of the network (QKV, attention projections with the residual, cross-query,
 * MLP up, MLP down) each choose among candidate tilings of the matrix-core kernel.
 * While enabled (the default), the first call whose padded token count falls in a new
 * power-of-two bucket times every candidate on that call's real shapes and buffers and
 * keeps the fastest. Tilings differ only in speed: every tiling produces bitwise-identical
 * results. */
int fmd_autotune_enable(fmd_model* m, int32_t enable);

/* On the BF16 path with heads of 32 the autotuner also chooses, per token bucket, the
 * attention query tile (candidate 0: work items of 64 queries of one event, 1: of 128, 2: of
 * 192), and
 * on the fused path (d = 256) the row tile of block 0's fused QKV kernel and of the OQC kernel
 * (candidate 0: 64 rows, 1: 128 rows). These too change only the speed: every candidate gives
 * bitwise-identical results.
 * fmd_tuning_set fixes the choice of one of these sites for the padded token counts in
 * [2^tokens_log2, 2^(tokens_log2 + 1)) (rows padded to a multiple of 256), e.g. to reuse a
 * table measured earlier or to compare candidates.
 * Errors: FMD_E_INVALID for a null model, another site, a bucket outside [0, 40) or a
 * candidate the model's kernels do not offer. */
enum { FMD_TUNE_ATTN_QUERY_TILE = 5, FMD_TUNE_FUSED_QKV = 6, FMD_TUNE_FUSED_OQC = 7 };
int fmd_tuning_set(fmd_model* m, int32_t site, int32_t tokens_log2, int32_t candidate);

/* The chosen tilings as a JSON object (site, log2 token bucket, tile id and shape, measured
 * microseconds). Writes at most cap bytes including the terminator; *needed receives
 * the full size. */
int fmd_tuning_table(fmd_model* m, char* buf, size_t cap, size_t* needed);

/* ---- kernel test hooks (used by the parity tests) --------------------------------------- */

/* C[M,N] = epi(pro(A) W + b) with the model's GEMM kernel, all operands DEVICE FP32.
 * W is [K,N] row-major. With ln != 0, pro(A) = LN(A; g, s) over K features, otherwise
 * pro(A) = A. epi: 0 = store, 1 = exact GELU, 2 = accumulate (C += ...). For FMD_BF16,
 * A (after LN), W and the GELU output are rounded to BF16 as in the model.
 * Requires K % 32 == 0 and N % 64 == 0; with ln also K % 64 == 0 and K <= 1024.
 * tile selects a candidate tiling of the autotuner (-1: default); (ln, store), (ln, GELU)
 * and (no ln, accumulate) accept every tiling that divides the shape, other combinations
 * tilings 0 and 4. FMD_E_UNSUPPORTED if the tiling does not divide the shape. */
int fmd_debug_gemm(int32_t precision, int64_t M, int32_t N, int32_t K, const float* A,
                   const float* W, const float* bias, int32_t ln, const float* g,
                   const float* s, int32_t epi, float* C, int32_t tile, void* hip_stream);

/* Masked multi-head attention per event with the model's kernel, all operands DEVICE FP32.
 * Q is [Tq, H*dh] and K, V are [Tk, H*dh] in CSR events (q_offsets, kv_offsets: host
 * int64 [n_events+1]). O is [Tq, H*dh]. Each query attends to the keys of its own event
 * only. For FMD_BF16, Q, K, V and the probabilities are rounded to BF16. */
int fmd_debug_attention(int32_t precision, int64_t n_events, const int64_t* q_offsets,
                        const int64_t* kv_offsets, int32_t n_heads, int32_t dh,
                        const float* Q, const float* K, const float* V, float* O,
                        void* hip_stream);

/* ---- serving ----------------------------------------------------------------------------- */

/* A continuous-batching server over one model. Requests are admitted FIFO when a
 * contiguous range of their particle count, rounded up to whole 64-row tiles, is free in a
 * device token pool. The pool is sized as hbm_budget_bytes divided by the per-token
 * footprint (ODE state, activations, truth encoding, cross K/V cache and output), rounded
 * down to whole tiles. An admitted request's state stays on the device until it completes.
 * Each server iteration advances every resident event by one stage of its own schedule; the
 * block kernels run only the tiles of resident requests. The worker enqueues the next
 * iteration before it waits for the current one to end, so the device does not idle while
 * the host prepares work.
 * Euler and RK4 requests and requests at different points of their integration share
 * one launch. A request's result is bitwise the same alone and in any mix: noise is
 * keyed by (seed, event index in the request, slot). The batch-of-the-paper knob
 * (App. C, batch_size) becomes the budget and the limits below.
 * While a server exists, the model's own sampling calls return FMD_E_STATE, and the
 * server must be destroyed before the model. */
typedef struct fmd_server fmd_server;   /* opaque */

typedef struct {
  size_t hbm_budget_bytes;      /* device bytes the resident requests may hold */
  int64_t max_tokens_per_iter;  /* cap on the resident particles (0: only the budget) */
  int32_t max_requests;         /* cap on resident requests (0: no cap) */
} fmd_server_config;

typedef struct {
  uint64_t t_submit_ns, t_admit_ns, t_done_ns;   /* CLOCK_MONOTONIC */
} fmd_request_stats;

/* Server counters: pool size (rows) and bytes per row; requests queued and resident and the
 * rows they hold; iterations run; rows processed by them (the span from the first pool row
 * to the last resident one, gaps between requests included) and the live rows among them;
 * device time of the iterations (admission included), in nanoseconds. */
typedef struct {
  int64_t pool_tokens, bytes_per_token, queued_requests, resident_requests, resident_tokens;
  int64_t iterations, rows_processed, busy_ns, rows_live;
} fmd_server_info;

/* Starts the worker thread. FMD_E_BUDGET if the budget holds less than one particle. */
int fmd_server_create(fmd_model* m, const fmd_server_config* cfg, fmd_server** out);

/* Queues a request. truth->feat must be host memory; it is copied before the call
 * returns. *req_id identifies the request. FMD_E_BUDGET if it can never fit the pool,
 * FMD_E_UNSUPPORTED if an event exceeds n_max, FMD_E_STATE if the server has failed. */
int fmd_server_submit(fmd_server* s, const fmd_events_in* truth, uint64_t seed,
                      const fmd_schedule* schedule, uint64_t* req_id);

/* As fmd_server_submit, with per-event reco counts (host reco_offsets [n_events + 1], copied
 * before the call returns), as fmd_simulate_reco takes them (Sec. 2.2). The request takes
 * max(truth particles, reco slots) pool rows; its result has reco_offsets[n] rows and is
 * bitwise the result of fmd_simulate_reco for the same request. Errors as
 * fmd_server_submit, plus those fmd_simulate_reco gives for the reco offsets. */
int fmd_server_submit_reco(fmd_server* s, const fmd_events_in* truth,
                           const int64_t* reco_offsets, uint64_t seed,
                           const fmd_schedule* schedule, uint64_t* req_id);

/* FMD_PENDING while the request runs. Once it has finished, copies the result
 * ([reco slots, 9] FP32, host) and the timestamps, forgets the request and returns its
 * status. A request is collected once. */
int fmd_server_poll(fmd_server* s, uint64_t req_id, float* reco_host, fmd_request_stats* st);
int fmd_server_wait(fmd_server* s, uint64_t req_id, float* reco_host, fmd_request_stats* st);

int fmd_server_get_info(fmd_server* s, fmd_server_info* info);

/* Stops the worker after its current iteration. Requests not yet finished end with
 * FMD_E_STATE, and uncollected results are dropped. */
int fmd_server_destroy(fmd_server* s);

/* Message for the last non-OK status of the calling thread ("" if none). */
const char* fmd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FMD_H */
