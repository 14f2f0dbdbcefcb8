// fmdet engine: model handles, validation, workspace, the ODE stage loop and the C ABI.
//
// One velocity evaluation over the packed tokens of all events of a call runs as:
//   time embedding -> input embedding -> L x [LN1+QKV GEMM -> self attention -> W_o
//   GEMM (+residual) -> LN2+Q_c GEMM -> cross attention (cached truth K/V) -> W_oc GEMM
//   (+residual) -> LN3+W_up GEMM+GELU -> W_dn GEMM (+residual)] -> LN_f + head + fused
//   Euler/RK4 state update.
// The truth encoding and the per-block cross-attention K/V are constant over the whole
// integration, so they are computed once per call into a cache.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "engine_impl.h"
#include "gemm_body.h"

using namespace fmd;

namespace fmd {
namespace eng {

thread_local std::string g_err;

int fail(int status, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return status;
}

// ---------------------------------------------------------------------------------------
// configuration and parameter layout

int check_cfg(const fmd_model_config* c) {
  if (!c) return fail(FMD_E_INVALID, "null model config");
  if (c->d_model <= 0 || c->n_blocks <= 0 || c->n_heads <= 0)
    return fail(FMD_E_INVALID, "d_model, n_blocks and n_heads must be positive");
  if (c->d_model % c->n_heads)
    return fail(FMD_E_INVALID, "d_model %d is not a multiple of n_heads %d", c->d_model, c->n_heads);
  if (c->d_model % 64 || c->d_model > 1024)
    return fail(FMD_E_UNSUPPORTED, "d_model must be a multiple of 64 and at most 1024");
  const int dh = c->d_model / c->n_heads;
  if (dh != 16 && dh != 32 && dh != 64)
    return fail(FMD_E_UNSUPPORTED, "head dimension %d not in {16, 32, 64}", dh);
  if (c->mlp_ratio != 4) return fail(FMD_E_UNSUPPORTED, "mlp_ratio must be 4");
  if (c->t_embed_dim != 32) return fail(FMD_E_UNSUPPORTED, "t_embed_dim must be 32");
  if (c->f_truth != 9 || c->f_reco != 9) return fail(FMD_E_UNSUPPORTED, "f_truth and f_reco must be 9");
  if (c->n_max < 1 || c->n_max > 4096) return fail(FMD_E_UNSUPPORTED, "n_max must be in [1, 4096]");
  if (c->precision != FMD_FP32 && c->precision != FMD_BF16 && c->precision != FMD_FP8)
    return fail(FMD_E_INVALID, "unknown precision %d", c->precision);
  if (c->precision == FMD_FP8 && !fused_supported(c->d_model, c->n_heads, c->mlp_ratio))
    return fail(FMD_E_UNSUPPORTED, "FP8 operands exist in the fused kernels only (d_model 256, 8 heads of 32)");
  return FMD_OK;
}

// Walks the flat parameter order, calling f(name_id, offset, rows, cols) per tensor
// (cols = 0 for vectors). Returns the total count.
enum PId {
  P_W_TIN, P_B_TIN, P_G_T, P_S_T, P_W_XIN, P_B_XIN, P_W_TIME, P_B_TIME,
  P_G1, P_S1, P_W_QKV, P_B_QKV, P_W_O, P_B_O, P_G2, P_S2, P_W_QC, P_B_QC, P_W_KC, P_B_KC,
  P_W_VC, P_B_VC, P_W_OC, P_B_OC, P_G3, P_S3, P_W_UP, P_B_UP, P_W_DN, P_B_DN,
  P_G_F, P_S_F, P_W_OUT, P_B_OUT
};

template <typename F>
size_t walk_params(const fmd_model_config& c, F&& f) {
  const int64_t d = c.d_model, F_ = c.f_truth, Fo = c.f_reco, E = c.t_embed_dim, R = c.mlp_ratio;
  size_t o = 0;
  auto put = [&](int id, int blk, int64_t rows, int64_t cols) {
    f(id, blk, o, rows, cols);
    o += (size_t)(rows * (cols ? cols : 1));
  };
  put(P_W_TIN, -1, F_, d); put(P_B_TIN, -1, d, 0); put(P_G_T, -1, d, 0); put(P_S_T, -1, d, 0);
  put(P_W_XIN, -1, Fo, d); put(P_B_XIN, -1, d, 0); put(P_W_TIME, -1, E, d); put(P_B_TIME, -1, d, 0);
  for (int l = 0; l < c.n_blocks; ++l) {
    put(P_G1, l, d, 0); put(P_S1, l, d, 0); put(P_W_QKV, l, d, 3 * d); put(P_B_QKV, l, 3 * d, 0);
    put(P_W_O, l, d, d); put(P_B_O, l, d, 0);
    put(P_G2, l, d, 0); put(P_S2, l, d, 0); put(P_W_QC, l, d, d); put(P_B_QC, l, d, 0);
    put(P_W_KC, l, d, d); put(P_B_KC, l, d, 0); put(P_W_VC, l, d, d); put(P_B_VC, l, d, 0);
    put(P_W_OC, l, d, d); put(P_B_OC, l, d, 0);
    put(P_G3, l, d, 0); put(P_S3, l, d, 0); put(P_W_UP, l, d, R * d); put(P_B_UP, l, R * d, 0);
    put(P_W_DN, l, R * d, d); put(P_B_DN, l, d, 0);
  }
  put(P_G_F, -1, d, 0); put(P_S_F, -1, d, 0); put(P_W_OUT, -1, d, Fo); put(P_B_OUT, -1, Fo, 0);
  return o;
}

size_t elem_size(const fmd_model_config& c) { return c.precision == FMD_FP32 ? 4 : 2; }

// ---------------------------------------------------------------------------------------
// workspace

void free_ws(Workspace& w) {
  void* dev[] = {w.x, w.acc, w.xs, w.H, w.qkv, w.att, w.qc, w.hid, w.c, w.kv, w.u, w.io,
                 w.temb, w.tev, w.stats, w.tok_event, w.off, w.work, w.desc, w.ctr};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  for (auto& h : w.hs) {
    if (h.live) (void)hipEventSynchronize(h.ev);
    if (h.ev) (void)hipEventDestroy(h.ev);
    if (h.desc) (void)hipHostFree(h.desc);
    if (h.off) (void)hipHostFree(h.off);
    if (h.work) (void)hipHostFree(h.work);
  }
  w = Workspace();
}

int ensure_ws_alloc(fmd_model* m, int64_t T, int64_t E, int64_t items, bool* grew);

// Grows the workspace; new buffers are zero-filled and the device is synchronised so that
// no stream can observe them before the fill.
int ensure_ws(fmd_model* m, int64_t T, int64_t E, int64_t items) {
  bool grew = false;
  FMD_TRY(ensure_ws_alloc(m, T, E, items, &grew));
  if (grew) {
    HIP_TRY(hipDeviceSynchronize());
    m->ws.generation++;
  }
  return FMD_OK;
}

int ensure_ws_alloc(fmd_model* m, int64_t T, int64_t E, int64_t items, bool* grew) {
  Workspace& w = m->ws;
  const fmd_model_config& c = m->cfg;
  const size_t es = m->kind == 0 ? elem_size(c) : 4;
  const int64_t d = m->kind == 0 ? c.d_model : 64, L = m->kind == 0 ? c.n_blocks : 1;
  const int64_t Tp = round_up(std::max<int64_t>(T, 1), kGemmBM);
  if (Tp > w.cap_tok) {
    const int64_t cap = std::max(Tp, round_up(w.cap_tok + w.cap_tok / 4, kGemmBM));
    const size_t st = (size_t)cap * kStateLd * 4;
    FMD_TRY(grow(w.x, st));
    FMD_TRY(grow(w.acc, st));
    FMD_TRY(grow(w.xs, st));
    FMD_TRY(grow(w.u, (size_t)cap * 9 * 4));
    FMD_TRY(grow(w.io, (size_t)cap * 9 * 4));
    FMD_TRY(grow(w.tok_event, (size_t)cap * 4));
    if (!w.ctr) FMD_TRY(grow(w.ctr, 64));
    if (m->kind == 0) {
      FMD_TRY(grow(w.H, (size_t)cap * d * 4));
      FMD_TRY(grow(w.stats, (size_t)cap * sizeof(float2)));
      FMD_TRY(grow(w.qkv, (size_t)cap * 3 * d * es));
      FMD_TRY(grow(w.att, (size_t)cap * d * es));
      FMD_TRY(grow(w.qc, (size_t)cap * d * es));
      FMD_TRY(grow(w.hid, (size_t)cap * 4 * d * es));
      FMD_TRY(grow(w.c, (size_t)cap * d * es));
      FMD_TRY(grow(w.kv, (size_t)cap * 2 * d * L * es));
    }
    w.cap_tok = cap;
    w.elem = es;
    *grew = true;
  }
  if (E + 1 > w.cap_ev) {
    const int64_t cap = std::max(E + 1, w.cap_ev + w.cap_ev / 4);
    FMD_TRY(grow(w.off, (size_t)cap * 8));
    FMD_TRY(grow(w.tev, (size_t)cap * 4));
    FMD_TRY(grow(w.temb, (size_t)cap * d * 4));
    w.cap_ev = cap;
    *grew = true;
  }
  if (items > w.cap_items) {
    const int64_t cap = std::max(items, w.cap_items + w.cap_items / 4);
    FMD_TRY(grow(w.work, (size_t)cap * sizeof(AttnItem)));
    w.cap_items = cap;
    *grew = true;
  }
  return FMD_OK;
}

// Switches to the other pinned staging set and makes it writable (waits for the uploads of
// the call that used it last) with room for E events and `items` work items.
int next_host_stage(Workspace& w, int64_t E, int64_t items) {
  w.cur ^= 1;
  Workspace::HostStage& h = w.hs[w.cur];
  if (!h.ev) HIP_TRY(hipEventCreateWithFlags(&h.ev, hipEventDisableTiming));
  if (h.live) {
    HIP_TRY(hipEventSynchronize(h.ev));
    h.live = false;
  }
  if (E + 1 > h.cap_ev) {
    FMD_TRY(grow_host(h.off, (size_t)(E + 1) * 8));
    h.cap_ev = E + 1;
  }
  if (items > h.cap_items) {
    FMD_TRY(grow_host(h.work, (size_t)std::max<int64_t>(items, 1) * sizeof(AttnItem)));
    h.cap_items = std::max<int64_t>(items, 1);
  }
  return FMD_OK;
}

// The uploads from the current set are enqueued on st: record its event after them.
int mark_host_stage(Workspace& w, hipStream_t st) {
  Workspace::HostStage& h = w.hs[w.cur];
  HIP_TRY(hipEventRecord(h.ev, st));
  h.live = true;
  return FMD_OK;
}

// ---------------------------------------------------------------------------------------
// validation

int check_events(const fmd_model* m, const fmd_events_in* ev, int64_t* T_out, int64_t* max_n) {
  if (!ev) return fail(FMD_E_INVALID, "null event set");
  if (ev->n_events < 0) return fail(FMD_E_INVALID, "negative n_events");
  if (!ev->offsets) return fail(FMD_E_INVALID, "null offsets");
  if (ev->offsets[0] != 0) return fail(FMD_E_INVALID, "offsets[0] must be 0");
  int64_t mx = 0;
  for (int64_t e = 0; e < ev->n_events; ++e) {
    const int64_t n = ev->offsets[e + 1] - ev->offsets[e];
    if (n < 0) return fail(FMD_E_INVALID, "offsets decrease at event %lld", (long long)e);
    mx = std::max(mx, n);
  }
  if (m && m->kind == 0 && mx > m->cfg.n_max)
    return fail(FMD_E_UNSUPPORTED, "an event has %lld particles, above n_max %d", (long long)mx,
                m->cfg.n_max);
  const int64_t T = ev->offsets[ev->n_events];
  if (T > ((int64_t)1 << 31) - 4096) return fail(FMD_E_UNSUPPORTED, "too many particles in one call");
  if (T > 0 && !ev->feat) return fail(FMD_E_INVALID, "null feature array");
  *T_out = T;
  if (max_n) *max_n = mx;
  return FMD_OK;
}

int check_schedule(const fmd_schedule* s) {
  if (!s) return fail(FMD_E_INVALID, "null schedule");
  if (s->scheme != FMD_EULER && s->scheme != FMD_RK4 && s->scheme != FMD_MIDPOINT)
    return fail(FMD_E_INVALID, "unknown scheme %d", s->scheme);
  if (s->n_steps < 1) return fail(FMD_E_INVALID, "n_steps must be >= 1");
  if (!std::isfinite(s->t0) || !std::isfinite(s->t1) || s->t0 == s->t1)
    return fail(FMD_E_INVALID, "t0 and t1 must be finite and different");
  return FMD_OK;
}

// ---------------------------------------------------------------------------------------
// timing

hipEvent_t take_event(fmd_model* m) {
  if (!m->ev_pool.empty()) {
    hipEvent_t e = m->ev_pool.back();
    m->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void flush_timing(fmd_model* m) {
  for (auto& r : m->trec) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      m->t_ms[r.cls] += ms;
      m->t_n[r.cls] += 1;
      m->t_work[r.cls] += r.work;
      m->t_bytes[r.cls] += r.bytes;
    }
    m->ev_pool.push_back(r.a);
    m->ev_pool.push_back(r.b);
  }
  m->trec.clear();
}

// ---------------------------------------------------------------------------------------
// one call's device state

int bucket_of(int64_t Tp);
int attn_tiles(const fmd_model* m, int* tiles);
int attn_tile_for(const fmd_model* m, int64_t Tp);
template <typename F>
float time_best_us(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F&& launch);
template <typename T>
hipError_t launch_self_attention(fmd_model* m, const Call& c, int qt, int64_t items,
                                 const AttnBins& bins, const AttnItem* work);

// Uploads offsets and the attention work lists; runs the token map. With reco_off (host,
// [E + 1], already checked) the reco slots of event e are reco_off[e] .. reco_off[e + 1]
// and their cross-attention keys the event's truth particles; otherwise reco = truth.
int stage_events(fmd_model* m, const fmd_events_in* ev, Call& c, const int64_t* reco_off = nullptr) {
  Workspace& w = m->ws;
  const int64_t E = ev->n_events;
  const int64_t* roff = reco_off ? reco_off : ev->offsets;
  const int64_t Tt = ev->offsets[E];
  // work items: (event, query tile), in bins of whole events balanced by attention work
  int tiles[4];
  const int n_tiles = attn_tiles(m, tiles);
  std::vector<int64_t> ids((size_t)E);
  auto count_items = [&](int qt) {
    int64_t k = 0;
    for (int64_t e = 0; e < E; ++e) k += (roff[e + 1] - roff[e] + qt - 1) / qt;
    return k;
  };
  double s2 = 0, sx = 0;
  for (int64_t e = 0; e < E; ++e) {
    const int64_t n = roff[e + 1] - roff[e], nt = ev->offsets[e + 1] - ev->offsets[e];
    ids[e] = e;
    s2 += (double)n * (double)n;
    sx += (double)n * (double)nt;
  }
  c.sum_n2 = s2;
  // capacity for the smallest candidate tile (the most items)
  const int64_t cap_items = count_items(tiles[0]) * (reco_off ? 2 : 1);
  FMD_TRY(ensure_ws(m, std::max(c.T, Tt), E, cap_items));
  // the pinned staging set of this call (the other set may still feed the last call's copies)
  FMD_TRY(next_host_stage(w, E, cap_items));
  Workspace::HostStage& hs = w.hs[w.cur];
  const int b = bucket_of(c.Tp);
  if (n_tiles > 1 && m->autotune && m->kind == 0 && m->tune[TS_ATTN][b] < 0) {
    // the attention query tile: time the self-attention with each candidate's work list on
    // the call's shapes (the buffers hold nothing used later)
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    int best = -1;
    float best_us = 0.f;
    int status = FMD_OK;
    for (int k = 0; k < n_tiles && status == FMD_OK; ++k) {
      const int64_t nk = count_items(tiles[k]);
      AttnBins bk{};
      if (build_attention_work(roff, roff, ids.data(), E, tiles[k], hs.work, &bk) != nk) {
        status = fail(FMD_E_INVALID, "token rows beyond 2^31");
        break;
      }
      if (hipMemcpyAsync(w.work, hs.work, (size_t)nk * sizeof(AttnItem), hipMemcpyHostToDevice, c.st) !=
              hipSuccess ||
          hipStreamSynchronize(c.st) != hipSuccess) {
        status = fail(FMD_E_DEVICE, "autotune upload failed");
        break;
      }
      const float us = time_best_us(c.st, e0, e1, [&] {
        return launch_self_attention<bf16>(m, c, tiles[k], nk, bk, w.work);
      });
      if (us < 0.f) {
        status = fail(FMD_E_DEVICE, "autotune launch failed");
        break;
      }
      m->tune_all[TS_ATTN][b][k] = us;
      if (best < 0 || us < best_us) best = k, best_us = us;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    FMD_TRY(status);
    m->tune[TS_ATTN][b] = (int8_t)best;
    m->tune_us[TS_ATTN][b] = best_us;
    m->tune_gen++;
  }
  const int qt = attn_tile_for(m, c.Tp);
  const int64_t items = count_items(qt);
  c.qt = qt;
  c.items = items;
  const int64_t all_items = reco_off ? 2 * items : items;
  std::memcpy(hs.off, roff, (size_t)(E + 1) * 8);
  if (build_attention_work(hs.off, hs.off, ids.data(), E, qt, hs.work, &c.bins) != items)
    return fail(FMD_E_INVALID, "token rows beyond 2^31");
  same_truth(c);
  if (reco_off) {
    c.Tt = Tt;
    c.Ttp = round_up(std::max<int64_t>(Tt, 1), kGemmBM);
    c.work_x = items;
    c.sum_nx = sx;
    if (build_attention_work(hs.off, ev->offsets, ids.data(), E, qt, hs.work + items,
                             &c.bins_x) != items)
      return fail(FMD_E_INVALID, "token rows beyond 2^31");
  }
  HIP_TRY(hipMemcpyAsync(w.off, hs.off, (size_t)(E + 1) * 8, hipMemcpyHostToDevice, c.st));
  if (all_items)
    HIP_TRY(hipMemcpyAsync(w.work, hs.work, (size_t)all_items * sizeof(AttnItem),
                           hipMemcpyHostToDevice, c.st));
  FMD_TRY(mark_host_stage(w, c.st));
  FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] { return launch_token_map(c.st, w.off, E, c.T, w.tok_event); }));
  if (ev->on_device) {
    c.u = ev->feat;
  } else {
    HIP_TRY(hipMemcpyAsync(w.u, ev->feat, (size_t)c.Tt * 9 * 4, hipMemcpyHostToDevice, c.st));
    c.u = w.u;
  }
  return FMD_OK;
}

template <typename T>
int truth_cache(fmd_model* m, Call& c) {
  Workspace& w = m->ws;
  const fmd_model_config& cf = m->cfg;
  const int d = cf.d_model, L = cf.n_blocks;
  FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] {
    return launch_truth_encode<T>(c.st, c.u, 9, 9, c.Tt, m->W_tin, m->b_tin, m->g_t, m->s_t, d,
                                  (T*)w.c, d);
  }));
  if (m->kv_hm) {
    // per block: [K | V] rows into a scratch buffer (the MLP hidden buffer, free here), then
    // into the head-major planes the attention kernel reads with contiguous rows
    const int dh = d / cf.n_heads;
    const int64_t plane = w.cap_tok;
    for (int l = 0; l < L; ++l) {
      FMD_TRY(timed(m, c.st, FMD_K_OTHER, 2.0 * c.Tt * d * 2 * d, [&] {
        return launch_gemm<T>(c.st, FMD_K_OTHER, false, EPI_STORE, c.Ttp, 2 * d, d, w.c, d,
                              (const T*)m->Wkv + (size_t)l * 2 * d * d, m->bkv + l * 2 * d,
                              nullptr, nullptr, nullptr, w.hid, 2 * d);
      }));
      FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] {
        return launch_kv_headmajor(c.st, w.hid, c.Tt, d, dh, cf.n_heads,
                                   (char*)w.kv + (size_t)l * 2 * cf.n_heads * plane * dh * sizeof(T),
                                   plane, 0);
      }));
    }
    return FMD_OK;
  }
  FMD_TRY(timed(m, c.st, FMD_K_OTHER, 2.0 * c.Tt * d * 2 * d * L, [&] {
    return launch_gemm<T>(c.st, FMD_K_OTHER, false, EPI_STORE, c.Ttp, 2 * d * L, d, w.c, d,
                          (const T*)m->Wkv, m->bkv, nullptr, nullptr, nullptr, w.kv, 2 * d * L);
  }));
  return FMD_OK;
}

// LayerNorm statistics of every (padded) row of the residual stream.
int row_stats(fmd_model* m, Call& c) {
  if (m->fuse_stats) return FMD_OK;   // the producing residual GEMM wrote them
  Workspace& w = m->ws;
  const int d = m->cfg.d_model;
  return timed(m, c.st, FMD_K_OTHER, 0, [&] { return launch_row_stats(c.st, w.H, d, d, c.Tp, w.stats); });
}

int bucket_of(int64_t Tp) {
  int b = 0;
  while (b + 1 < kTuneBuckets && ((int64_t)1 << (b + 1)) <= Tp) ++b;
  return b;
}

bool full_row_slot(const fmd_model* m, int slot) {
  return m->fuse_stats && (slot == TS_PROJ_RES || slot == TS_DOWN);
}

int tile_for(const fmd_model* m, int slot, int64_t Tp, int N) {
  const int t = m->tune[slot][bucket_of(Tp)];
  if (t >= 0) return t;
  return full_row_slot(m, slot) ? default_tile_rows(N) : default_tile(N);
}

int resid_epi(const fmd_model* m) { return m->fuse_stats ? EPI_RESID_LN : EPI_RESID; }

// Attention query tiles the model's kernel takes (candidates of the autotuner) and the one
// used for a padded token count: the tuned one, else the default.
int attn_tiles(const fmd_model* m, int* tiles) {
  return attention_query_tiles(m->cfg.precision != FMD_FP32,
                               m->cfg.d_model / std::max(m->cfg.n_heads, 1), tiles);
}
int attn_tile_for(const fmd_model* m, int64_t Tp) {
  int tiles[4];
  const int n = attn_tiles(m, tiles);
  const int t = m->tune[TS_ATTN][bucket_of(Tp)];
  if (t >= 0 && t < n) return tiles[t];
  return attention_query_tile(m->cfg.precision != FMD_FP32,
                              m->cfg.d_model / std::max(m->cfg.n_heads, 1), m->cfg.n_heads);
}
// Row tile of the fused QKV / OQC kernels (candidate 0: 64 rows, 1: 128 rows); 64 when the
// call runs a map of 64-row tiles.
int fused_rows_for(const fmd_model* m, const Call& c, int slot) {
  return !c.tiles && m->tune[slot][bucket_of(c.Tp)] == 1 ? 128 : 64;
}

// Launches the GEMM of one tuning slot with a given tiling on the live workspace.
template <typename T>
hipError_t slot_gemm(fmd_model* m, Call& c, int slot, int tile, const DevBlock& B) {
  Workspace& w = m->ws;
  const int d = m->cfg.d_model;
  switch (slot) {
    case TS_QKV:
      return launch_gemm<T>(c.st, FMD_K_GEMM_QKV, true, EPI_STORE, c.Tp, 3 * d, d, w.H, d,
                            (const T*)B.Wqkv, B.bqkv, w.stats, B.g1, B.s1, w.qkv, 3 * d, nullptr, tile);
    case TS_PROJ_RES:
      return launch_gemm<T>(c.st, FMD_K_GEMM_PROJ, false, resid_epi(m), c.Tp, d, d, w.att, d,
                            (const T*)B.Wo, B.bo, nullptr, nullptr, nullptr, w.H, d,
                            m->fuse_stats ? &c.sargs : nullptr, tile);
    case TS_PROJ_LN:
      return launch_gemm<T>(c.st, FMD_K_GEMM_QC, true, EPI_STORE, c.Tp, d, d, w.H, d,
                            (const T*)B.Wqc, B.bqc, w.stats, B.g2, B.s2, w.qc, d, nullptr, tile);
    case TS_UP:
      return launch_gemm<T>(c.st, FMD_K_GEMM_UP, true, EPI_GELU, c.Tp, 4 * d, d, w.H, d,
                            (const T*)B.Wup, B.bup, w.stats, B.g3, B.s3, w.hid, 4 * d, nullptr, tile);
    default:
      return launch_gemm<T>(c.st, FMD_K_GEMM_DOWN, false, resid_epi(m), c.Tp, d, 4 * d, w.hid, 4 * d,
                            (const T*)B.Wdn, B.bdn, nullptr, nullptr, nullptr, w.H, d,
                            m->fuse_stats ? &c.sargs : nullptr, tile);
  }
}

// Autotuner: for every GEMM site not yet tuned for this token-count bucket, time each
// candidate tiling that divides the shape (1 warm-up + 3 timed launches, best of the
// three) and keep the fastest. All tilings give bitwise-identical results (same
// k-slice accumulation order per element), so the choice affects speed only. Runs before
// the first evaluation of a call, while the activation buffers hold nothing that is used
// later (the residual stream is rebuilt by the next input embedding).
// Times one launch sequence: 1 warm-up + 3 timed launches, best of the three, in
// microseconds (negative if a launch failed).
template <typename F>
float time_best_us(hipStream_t st, hipEvent_t e0, hipEvent_t e1, F&& launch) {
  if (launch() != hipSuccess) {
    (void)hipGetLastError();
    return -1.f;
  }
  float best = 1e30f;
  for (int rep = 0; rep < 3; ++rep) {
    float ms = 0.f;
    if (hipEventRecord(e0, st) != hipSuccess || launch() != hipSuccess ||
        hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
      return -1.f;
    best = std::min(best, ms * 1e3f);
  }
  return best;
}

// Fused BF16 path: the row tile (64 or 128 rows) of block 0's QKV kernel and of the OQC
// kernel, timed on the call's shapes and buffers like the GEMM tilings. Both candidates give
// bitwise-identical rows (each row's LayerNorm statistics and products are formed in the
// same order whatever its tile).
int autotune_fused(fmd_model* m, Call& c, int b) {
  Workspace& w = m->ws;
  const DevBlock& B = m->blk[0];
  const int sites[2] = {TS_FQKV, TS_FOQC};
  const int bits[2] = {FMD_FUSED_QKV, FMD_FUSED_OQC};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int status = FMD_OK;
  for (int i = 0; i < 2 && status == FMD_OK; ++i) {
    const int sl = sites[i];
    if (!(m->fused & bits[i]) || m->tune[sl][b] >= 0) continue;
    int best = -1;
    float best_us = 0.f;
    for (int k = 0; k < 2; ++k) {
      const int rows = 64 << k;
      if (c.Tp % rows) continue;
      // block 0's QKV kernel is timed in the form sampler stages run: with the input embedding
      // when that is folded in (calls with per-event times run the plain form with the same
      // row tile)
      const float us = time_best_us(c.st, e0, e1, [&] {
        if (sl == TS_FOQC)
          return launch_fused_oqc(c.st, c.Tp, w.att, B.Fo, B.bo, w.H, B.g2, B.s2, B.Fqc, B.bqc,
                                  w.qc, rows);
        if (m->fused & FMD_FUSED_EMBED)
          return launch_fused_embed_qkv(c.st, c.Tp, w.xs, kStateLd, 9, c.T, w.temb, m->W_xin, w.H,
                                        B.g1, B.s1, B.Fqkv, B.bqkv, w.qkv, rows);
        return launch_fused_qkv(c.st, c.Tp, w.H, B.g1, B.s1, B.Fqkv, B.bqkv, w.qkv, rows);
      });
      if (us < 0.f) {
        status = fail(FMD_E_DEVICE, "autotune launch failed");
        break;
      }
      m->tune_all[sl][b][k] = us;
      if (best < 0 || us < best_us) best = k, best_us = us;
    }
    m->tune[sl][b] = (int8_t)std::max(best, 0);
    m->tune_us[sl][b] = best_us;
    m->tune_gen++;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}

template <typename T>
int autotune(fmd_model* m, Call& c) {
  if (!m->autotune || m->kind != 0) return FMD_OK;   // fixed tiling
  const int b = bucket_of(c.Tp);
  if (std::is_same<T, bf16>::value && m->fused) FMD_TRY(autotune_fused(m, c, b));
  const int blocks_fused = FMD_FUSED_QKV | FMD_FUSED_OQC | FMD_FUSED_MLP;
  if (std::is_same<T, bf16>::value && (m->fused & blocks_fused) == blocks_fused)
    return FMD_OK;   // no GEMM site runs
  const int d = m->cfg.d_model;
  const int N[TS_GEMM] = {3 * d, d, d, 4 * d, d};
  const int K[TS_GEMM] = {d, d, d, d, 4 * d};
  bool any = false;
  for (int sl = 0; sl < TS_GEMM; ++sl) any |= m->tune[sl][b] < 0;
  if (!any) return FMD_OK;
  c.sargs = OdeArgs{};
  c.sargs.stats_out = m->ws.stats;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int status = FMD_OK;
  for (int sl = 0; sl < TS_GEMM && status == FMD_OK; ++sl) {
    if (m->tune[sl][b] >= 0) continue;
    int best = -1;
    float best_us = 0.f;
    for (int t = 0; t < kGemmTiles; ++t) {
      if (!tile_fits(t, c.Tp, N[sl], K[sl], full_row_slot(m, sl))) continue;
      if (slot_gemm<T>(m, c, sl, t, m->blk[0]) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      float run_best = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {
        float ms = 0.f;
        if (hipEventRecord(e0, c.st) != hipSuccess || slot_gemm<T>(m, c, sl, t, m->blk[0]) != hipSuccess ||
            hipEventRecord(e1, c.st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
          status = fail(FMD_E_DEVICE, "autotune launch failed");
          break;
        }
        run_best = std::min(run_best, ms * 1e3f);
      }
      if (status != FMD_OK) break;
      if (t < 8) m->tune_all[sl][b][t] = run_best;
      if (best < 0 || run_best < best_us) best = t, best_us = run_best;
    }
    m->tune[sl][b] = (int8_t)(best >= 0 ? best : full_row_slot(m, sl) ? default_tile_rows(N[sl])
                                                               : default_tile(N[sl]));
    m->tune_us[sl][b] = best_us;
    m->tune_gen++;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return status;
}

// Self-attention of one evaluation over the live workspace, with a work list of query tile qt.
// Q/K/V are head-major [3][heads][Tp][dh] when the fused QKV kernels formed them, row-major
// [Tp][3d] otherwise; the output is head-major [heads][Tp][dh] when the fused OQC kernel reads
// it, row-major [Tp][d] otherwise.
template <typename T>
hipError_t launch_self_attention(fmd_model* m, const Call& c, int qt, int64_t items,
                                 const AttnBins& bins, const AttnItem* work) {
  Workspace& w = m->ws;
  const int d = m->cfg.d_model, Hh = m->cfg.n_heads, dh = d / Hh;
  const size_t es = sizeof(T);
  const int fz = std::is_same<T, bf16>::value ? m->fused : 0;
  const char* qkv = (const char*)w.qkv;
  const bool ohm = (fz & FMD_FUSED_OQC) != 0;
  const int ldo = ohm ? dh : d;
  const int64_t hso = ohm ? c.Tp * dh : dh;
  if (fz & FMD_FUSED_QKV) {
    const int64_t pl = c.Tp * dh;
    return launch_attention<T>(c.st, false, dh, Hh, qt, items, bins, work, (const T*)qkv, dh, pl,
                               (const T*)(qkv + Hh * pl * es), (const T*)(qkv + 2 * Hh * pl * es),
                               dh, pl, (T*)w.att, ldo, hso);
  }
  return launch_attention<T>(c.st, false, dh, Hh, qt, items, bins, work, (const T*)qkv, 3 * d, dh,
                             (const T*)(qkv + d * es), (const T*)(qkv + 2 * d * es), 3 * d, dh,
                             (T*)w.att, ldo, hso);
}

// One evaluation of the velocity network at xs; leaves the residual stream in w.H.
// t_ev: per-event times (device); otherwise the time of the current stage-table entry.
template <typename T>
int net_forward(fmd_model* m, Call& c, const float* t_ev) {
  Workspace& w = m->ws;
  const fmd_model_config& cf = m->cfg;
  const int d = cf.d_model, L = cf.n_blocks, Hh = cf.n_heads, dh = d / Hh;
  const double Td = (double)c.T;
  const size_t es = sizeof(T);
  // algorithmic HBM bytes: a LayerNorm input (FP32 rows + statistics), a residual update
  // (FP32 read and write, plus the next LayerNorm's statistics when fused)
  const double ln_in = Td * (d * 4.0 + 8.0);
  const double resid = Td * (d * 8.0 + (m->fuse_stats ? 8.0 : 0.0));
  char* qkv = (char*)w.qkv;
  char* kv = (char*)w.kv;
  c.sargs = OdeArgs{};
  c.sargs.stats_out = w.stats;
  FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] {
    return launch_time_embed(c.st, t_ev, t_ev ? nullptr : w.desc, w.ctr, 0.f, t_ev ? (int)c.E : 1,
                             m->W_time, m->b_time, m->b_xin, cf.t_embed_dim, d, w.temb);
  }));
  // fused BF16 kernels per block segment (bit 1: LN1 + QKV; bit 2: W_o + residual + LN2 +
  // cross query; bit 4: W_oc + residual + LN3 + MLP + residual; bit 8 with bit 1: the input
  // embedding formed in block 0's QKV kernel); the GEMM kernels otherwise
  const int fz = std::is_same<T, bf16>::value ? m->fused : 0;
  // (stage times only: calls with per-event times keep the embedding kernel)
  const bool embed_in_qkv = (fz & FMD_FUSED_QKV) && (fz & FMD_FUSED_EMBED) && !t_ev && !c.tiles;
  if (!embed_in_qkv)
    FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] {
      return launch_embed(c.st, w.xs, kStateLd, 9, c.T, t_ev ? w.tok_event : nullptr, w.temb,
                          m->W_xin, d, w.H, d, w.stats);
    }));
  const double dd = (double)d;
  bool qkv_ready = false;   // the previous block's MLP kernel formed this block's [Q|K|V]
  for (int l = 0; l < L; ++l) {
    const DevBlock& B = m->blk[l];
    if (fz & FMD_FUSED_QKV) {
      if (l == 0 && embed_in_qkv)
        FMD_TRY(timed(m, c.st, FMD_K_GEMM_QKV, 2.0 * Td * dd * 3 * dd + 2.0 * Td * 9 * dd,
                      Td * (dd * 4 + kStateLd * 4) + (Td + dd) * 3 * dd * es, [&] {
          return launch_fused_embed_qkv(c.st, c.Tp, w.xs, kStateLd, 9, c.T, w.temb, m->W_xin,
                                        w.H, B.g1, B.s1, B.Fqkv, B.bqkv, w.qkv,
                                        fused_rows_for(m, c, TS_FQKV));
        }));
      else if (!qkv_ready)
        FMD_TRY(timed(m, c.st, FMD_K_GEMM_QKV, 2.0 * Td * dd * 3 * dd,
                      Td * dd * 4 + (Td + dd) * 3 * dd * es, [&] {
          return launch_fused_qkv(c.st, c.Tp, w.H, B.g1, B.s1, B.Fqkv, B.bqkv, w.qkv,
                                  fused_rows_for(m, c, TS_FQKV), c.tiles, c.n_tiles);
        }));
    } else {
      if (l > 0) FMD_TRY(row_stats(m, c));
      FMD_TRY(timed(m, c.st, FMD_K_GEMM_QKV, 2.0 * Td * d * 3 * d, ln_in + (Td + d) * 3 * d * es, [&] {
        return launch_gemm<T>(c.st, FMD_K_GEMM_QKV, true, EPI_STORE, c.Tp, 3 * d, d, w.H, d,
                              (const T*)B.Wqkv, B.bqkv, w.stats, B.g1, B.s1, w.qkv, 3 * d, nullptr,
                              tile_for(m, TS_QKV, c.Tp, 3 * d));
      }));
    }
    FMD_TRY(timed(m, c.st, FMD_K_ATTN_SELF, 4.0 * c.sum_n2 * d, Td * 4 * d * es, [&] {
      return launch_self_attention<T>(m, c, c.qt, c.items, c.bins, w.work);
    }));
    if (fz & FMD_FUSED_OQC) {
      FMD_TRY(timed(m, c.st, FMD_K_FUSED_OQC, 2.0 * Td * dd * dd * 2,
                    Td * dd * (es + 8 + es) + 2 * dd * dd * es, [&] {
        return launch_fused_oqc(c.st, c.Tp, w.att, B.Fo, B.bo, w.H, B.g2, B.s2, B.Fqc, B.bqc, w.qc,
                                fused_rows_for(m, c, TS_FOQC), c.tiles, c.n_tiles);
      }));
    } else {
      FMD_TRY(timed(m, c.st, FMD_K_GEMM_PROJ, 2.0 * Td * d * d, (Td + d) * d * es + resid, [&] {
        return launch_gemm<T>(c.st, FMD_K_GEMM_PROJ, false, resid_epi(m), c.Tp, d, d, w.att, d,
                              (const T*)B.Wo, B.bo, nullptr, nullptr, nullptr, w.H, d,
                              m->fuse_stats ? &c.sargs : nullptr, tile_for(m, TS_PROJ_RES, c.Tp, d));
      }));
      FMD_TRY(row_stats(m, c));
      FMD_TRY(timed(m, c.st, FMD_K_GEMM_QC, 2.0 * Td * d * d, ln_in + (Td + d) * d * es, [&] {
        return launch_gemm<T>(c.st, FMD_K_GEMM_QC, true, EPI_STORE, c.Tp, d, d, w.H, d,
                              (const T*)B.Wqc, B.bqc, w.stats, B.g2, B.s2, w.qc, d, nullptr,
                              tile_for(m, TS_PROJ_LN, c.Tp, d));
      }));
    }
    FMD_TRY(timed(m, c.st, FMD_K_ATTN_CROSS, 4.0 * c.sum_nx * d, (Td * 2 + c.Tt * 2.0) * d * es, [&] {
      const size_t o = (size_t)l * 2 * d * es;
      // the cross query is head-major [heads][Tp][dh] when the fused kernel formed it, and
      // the output when the fused MLP kernel reads it
      const bool hm = (fz & FMD_FUSED_OQC) != 0;
      const bool ohm = (fz & FMD_FUSED_MLP) != 0;
      const int ldo = ohm ? dh : d;
      const int64_t hso = ohm ? c.Tp * dh : dh;
      if (m->kv_hm) {   // cache planes [L][K, V][heads][cap rows][dh]
        const int64_t pl = w.cap_tok * dh;
        const char* kb = kv + (size_t)l * 2 * Hh * pl * es;
        return launch_attention<T>(c.st, true, dh, Hh, c.qt, c.items_x, c.bins_x, w.work + c.work_x, (const T*)w.qc,
                                   hm ? dh : d, hm ? c.Tp * dh : dh, (const T*)kb,
                                   (const T*)(kb + Hh * pl * es), dh, pl, (T*)w.att, ldo, hso);
      }
      return launch_attention<T>(c.st, true, dh, Hh, c.qt, c.items_x, c.bins_x, w.work + c.work_x, (const T*)w.qc,
                                 hm ? dh : d, hm ? c.Tp * dh : dh, (const T*)(kv + o),
                                 (const T*)(kv + o + d * es), 2 * d * L, dh, (T*)w.att, ldo, hso);
    }));
    if (fz & FMD_FUSED_MLP) {
      // chained with the next block's LN1 + QKV when that segment is fused too
      const bool chain = (fz & FMD_FUSED_QKV) && l + 1 < L;
      const DevBlock* N = chain ? &m->blk[l + 1] : nullptr;
      // the last block applies the output head and the state update instead of storing H
      const bool fold = l + 1 == L && c.head && c.head->nf == 9;
      const double Tv = (double)c.T;
      FMD_TRY(timed(m, c.st, FMD_K_FUSED_MLP,
                    2.0 * Td * dd * dd * (chain ? 12 : 9) + (fold ? 2.0 * Tv * dd * 9 : 0.0),
                    Td * (dd * (es + (fold ? 4 : 8)) + (fold ? 0 : 8)) + 9 * dd * dd * es +
                        (chain ? Td * 3 * dd * es + 3 * dd * dd * es : 0.0) +
                        (fold ? Tv * 9 * 4 * 5 : 0.0), [&] {
        return launch_fused_mlp(c.st, c.Tp, w.att, B.Foc, B.boc, w.H, B.g3, B.s3, B.Fup, B.bup,
                                B.Fdn, B.bdn, w.stats, chain ? N->g1 : nullptr,
                                chain ? N->s1 : nullptr, chain ? N->Fqkv : nullptr,
                                chain ? N->bqkv : nullptr, chain ? w.qkv : nullptr,
                                fold ? m->g_f : nullptr, fold ? m->s_f : nullptr,
                                fold ? m->Wout_pk : nullptr, fold ? m->bout_pk : nullptr,
                                fold ? c.head : nullptr, m->f8.empty() ? nullptr : &m->f8[l],
                                c.tiles, c.n_tiles);
      }));
      qkv_ready = chain;
      c.head_done = fold;
    } else {
      FMD_TRY(timed(m, c.st, FMD_K_GEMM_PROJ, 2.0 * Td * d * d, (Td + d) * d * es + resid, [&] {
        return launch_gemm<T>(c.st, FMD_K_GEMM_PROJ, false, resid_epi(m), c.Tp, d, d, w.att, d,
                              (const T*)B.Woc, B.boc, nullptr, nullptr, nullptr, w.H, d,
                              m->fuse_stats ? &c.sargs : nullptr, tile_for(m, TS_PROJ_RES, c.Tp, d));
      }));
      FMD_TRY(row_stats(m, c));
      FMD_TRY(timed(m, c.st, FMD_K_GEMM_UP, 2.0 * Td * d * 4 * d, ln_in + (Td + d) * 4 * d * es, [&] {
        return launch_gemm<T>(c.st, FMD_K_GEMM_UP, true, EPI_GELU, c.Tp, 4 * d, d, w.H, d,
                              (const T*)B.Wup, B.bup, w.stats, B.g3, B.s3, w.hid, 4 * d, nullptr,
                              tile_for(m, TS_UP, c.Tp, 4 * d));
      }));
      FMD_TRY(timed(m, c.st, FMD_K_GEMM_DOWN, 2.0 * Td * 4 * d * d, (Td + d) * 4 * d * es + resid, [&] {
        return launch_gemm<T>(c.st, FMD_K_GEMM_DOWN, false, resid_epi(m), c.Tp, d, 4 * d, w.hid,
                              4 * d, (const T*)B.Wdn, B.bdn, nullptr, nullptr, nullptr, w.H, d,
                              m->fuse_stats ? &c.sargs : nullptr, tile_for(m, TS_DOWN, c.Tp, d));
      }));
    }
  }
  return FMD_OK;
}

// Output head with the fused state update. With `direct` the update mode is `mode` (the
// velocity-only hook); otherwise mode, step and output write follow the stage table.
OdeArgs head_args(fmd_model* m, Call& c, bool direct, int mode, float* out, int ldo) {
  Workspace& w = m->ws;
  return OdeArgs{w.x, w.acc, w.xs, out, c.T, kStateLd, ldo, 9, mode, 0.f,
                 direct ? nullptr : w.desc, w.ctr, nullptr};
}

int head(fmd_model* m, Call& c, bool direct, int mode, float* out, int ldo) {
  Workspace& w = m->ws;
  if (m->kind == 1)
    return timed(m, c.st, FMD_K_OTHER, 0, [&] {
      return launch_linear_update(c.st, (float)m->alpha, (float)m->beta, w.desc, w.ctr, c.T, 9,
                                  w.x, w.acc, w.xs, kStateLd, out, ldo);
    });
  FMD_TRY(row_stats(m, c));
  const int d = m->cfg.d_model;
  const OdeArgs ode = head_args(m, c, direct, mode, out, ldo);
  return timed(m, c.st, FMD_K_OTHER, 2.0 * c.T * d * 9, [&] {
    if (head256_supported(d, 9))
      return launch_head256(c.st, w.H, w.stats, m->g_f, m->s_f, m->Wout_pk, m->bout_pk, ode);
    return launch_gemm<float>(c.st, FMD_K_OTHER, true, EPI_ODE, c.Tp, 64, d, w.H, d, m->Wout_pk,
                              m->bout_pk, w.stats, m->g_f, m->s_f, nullptr, 0, &ode);
  });
}

int stages_per_step(int scheme) {
  return scheme == FMD_EULER ? 1 : scheme == FMD_MIDPOINT ? 2 : 4;
}

// Stage i of a schedule (step i / S, stage i % S): evaluation time, step and update mode.
StageDesc stage_desc(const fmd_schedule& s, int i) {
  static const double c_rk4[4] = {0.0, 0.5, 0.5, 1.0};
  const int S = stages_per_step(s.scheme), k = i / S, st = i % S;
  const double h = (s.t1 - s.t0) / s.n_steps;
  StageDesc d;
  if (s.scheme == FMD_EULER) {
    d.t = (float)(s.t0 + k * h);
    d.mode = UPD_EULER;
  } else if (s.scheme == FMD_MIDPOINT) {
    d.t = (float)(s.t0 + (k + 0.5 * st) * h);
    d.mode = st == 0 ? UPD_MID_0 : UPD_MID_1;
  } else {
    d.t = (float)(s.t0 + (k + c_rk4[st]) * h);
    d.mode = UPD_RK4_0 + st;
  }
  d.h = (float)h;
  d.write_out = i == s.n_steps * S - 1;
  return d;
}

// Uploads the stage table of a schedule: stage i = (t, h, update mode, write output).
int upload_stages(fmd_model* m, Call& c, const fmd_schedule* s, int* n_stages) {
  Workspace& w = m->ws;
  Workspace::HostStage& hs = w.hs[w.cur];   // the call's set (made writable by stage_events)
  const int K = s->n_steps, S = stages_per_step(s->scheme);
  const int n = K * S;
  if (n > w.cap_desc) {
    FMD_TRY(grow(w.desc, (size_t)n * sizeof(StageDesc)));
    HIP_TRY(hipDeviceSynchronize());
    w.cap_desc = n;
    w.generation++;
  }
  if (n > hs.cap_desc) {
    FMD_TRY(grow_host(hs.desc, (size_t)n * sizeof(StageDesc)));
    hs.cap_desc = n;
  }
  for (int i = 0; i < n; ++i) hs.desc[i] = stage_desc(*s, i);
  HIP_TRY(hipMemcpyAsync(w.desc, hs.desc, (size_t)n * sizeof(StageDesc), hipMemcpyHostToDevice, c.st));
  FMD_TRY(mark_host_stage(w, c.st));
  FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] { return launch_set_counter(c.st, w.ctr, 0); }));
  *n_stages = n;
  return FMD_OK;
}

// One ODE stage: velocity at the current stage input, fused update, counter advance.
template <typename T>
int run_stage(fmd_model* m, Call& c, float* out, int ldo) {
  const OdeArgs ode = head_args(m, c, false, 0, out, ldo);
  c.head = &ode;
  c.head_done = false;
  const int rc = m->kind == 0 ? net_forward<T>(m, c, nullptr) : FMD_OK;
  c.head = nullptr;
  FMD_TRY(rc);
  if (!c.head_done) FMD_TRY(head(m, c, false, 0, out, ldo));
  return timed(m, c.st, FMD_K_OTHER, 0, [&] { return launch_stage_advance(c.st, m->ws.ctr); });
}

// All stages of a call. With graphs on, one stage is captured into a HIP graph (kernels
// read time, mode and step from the stage table through the device counter) and the graph
// is replayed once per stage; the executable graph is kept for later calls with the same
// shapes, buffers and output pointer.
template <typename T>
int run_stages(fmd_model* m, Call& c, int n_stages, float* out, int ldo) {
  if (!m->graphs || m->timing) {
    for (int i = 0; i < n_stages; ++i) FMD_TRY(run_stage<T>(m, c, out, ldo));
    return FMD_OK;
  }
  const GraphKey key{c.Tp,   c.T,       c.E,    c.items,  out,      ldo, m->ws.generation,
                     m->tune_gen, c.bins, c.items_x, c.work_x, c.bins_x, c.Tt};
  if (!m->gexec || !(key == m->gkey)) {
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    m->gexec = nullptr;
    HIP_TRY(hipStreamBeginCapture(c.st, hipStreamCaptureModeThreadLocal));
    const int st = run_stage<T>(m, c, out, ldo);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(c.st, &g);
    if (st != FMD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (ec != hipSuccess) return fail(FMD_E_DEVICE, "stage capture failed: %s", hipGetErrorString(ec));
    const hipError_t ei = hipGraphInstantiate(&m->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      m->gexec = nullptr;
      return fail(FMD_E_DEVICE, "graph instantiation failed: %s", hipGetErrorString(ei));
    }
    m->gkey = key;
  }
  for (int i = 0; i < n_stages; ++i) HIP_TRY(hipGraphLaunch(m->gexec, c.st));
  return FMD_OK;
}

// Orders the model's private stream after the caller's stream (call start) and the
// caller's stream after the private one (call end), keeping calls asynchronous.
int enter_stream(fmd_model* m, hipStream_t caller, Call& c) {
  if (!m->pstream) {
    HIP_TRY(hipStreamCreateWithFlags(&m->pstream, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&m->ev_in, hipEventDisableTiming));
    HIP_TRY(hipEventCreateWithFlags(&m->ev_out, hipEventDisableTiming));
  }
  HIP_TRY(hipEventRecord(m->ev_in, caller));
  HIP_TRY(hipStreamWaitEvent(m->pstream, m->ev_in, 0));
  c.st = m->pstream;
  return FMD_OK;
}

int leave_stream(fmd_model* m, hipStream_t caller) {
  HIP_TRY(hipEventRecord(m->ev_out, m->pstream));
  HIP_TRY(hipStreamWaitEvent(caller, m->ev_out, 0));
  return FMD_OK;
}

template <typename T>
int simulate_body(fmd_model* m, const fmd_events_in* truth, const float* x0, uint64_t seed,
                  const fmd_schedule* sched, fmd_events_out* reco, Call& c,
                  const int64_t* reco_off) {
  FMD_TRY(stage_events(m, truth, c, reco_off));
  Workspace& w = m->ws;
  int n_stages = 0;
  FMD_TRY(upload_stages(m, c, sched, &n_stages));
  if (x0) {
    const float* src = x0;
    if (!truth->on_device) {
      HIP_TRY(hipMemcpyAsync(w.io, x0, (size_t)c.T * 9 * 4, hipMemcpyHostToDevice, c.st));
      src = w.io;
    }
    FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] { return launch_load_state(c.st, src, 9, c.T, w.x, w.xs, kStateLd); }));
  } else {
    FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] {
      return launch_noise(c.st, seed, w.off, w.tok_event, c.T, 9, w.x, w.xs, kStateLd);
    }));
  }
  float* out = reco->on_device ? reco->feat : w.io;
  if (m->kind == 0) {
    FMD_TRY(truth_cache<T>(m, c));
    FMD_TRY(autotune<T>(m, c));
  }
  FMD_TRY(run_stages<T>(m, c, n_stages, out, 9));
  if (!reco->on_device) {
    HIP_TRY(hipMemcpyAsync(reco->feat, w.io, (size_t)c.T * 9 * 4, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
  }
  return FMD_OK;
}

// Reco multiplicities given by the caller: offsets from 0, non-decreasing, at most n_max
// slots per event, and no reco slot in an event without truth particles (its
// cross-attention would have no key). Sets *T_out to the number of reco slots.
int check_reco_offsets(const fmd_model* m, const fmd_events_in* truth, const int64_t* roff,
                       int64_t* T_out) {
  if (!roff) return fail(FMD_E_INVALID, "null reco offsets");
  if (roff[0] != 0) return fail(FMD_E_INVALID, "reco offsets[0] must be 0");
  for (int64_t e = 0; e < truth->n_events; ++e) {
    const int64_t n = roff[e + 1] - roff[e];
    if (n < 0) return fail(FMD_E_INVALID, "reco offsets decrease at event %lld", (long long)e);
    if (m->kind == 0 && n > m->cfg.n_max)
      return fail(FMD_E_UNSUPPORTED, "event %lld has %lld reco slots, above n_max %d",
                  (long long)e, (long long)n, m->cfg.n_max);
    if (n > 0 && truth->offsets[e + 1] == truth->offsets[e])
      return fail(FMD_E_INVALID, "event %lld has reco slots but no truth particle", (long long)e);
  }
  const int64_t T = roff[truth->n_events];
  if (T > ((int64_t)1 << 31) - 4096) return fail(FMD_E_UNSUPPORTED, "too many reco slots in one call");
  *T_out = T;
  return FMD_OK;
}

int simulate_impl(fmd_model* m, const fmd_events_in* truth, const float* x0, uint64_t seed,
                  const fmd_schedule* sched, fmd_events_out* reco, void* stream,
                  const int64_t* reco_off = nullptr) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  if (m->server) return fail(FMD_E_STATE, "the model is owned by a server");
  Call c{};
  FMD_TRY(check_events(m, truth, &c.T, nullptr));
  if (reco_off) FMD_TRY(check_reco_offsets(m, truth, reco_off, &c.T));
  FMD_TRY(check_schedule(sched));
  if (!reco) return fail(FMD_E_INVALID, "null reco output");
  if (c.T > 0 && !reco->feat) return fail(FMD_E_INVALID, "null reco feature array");
  c.E = truth->n_events;
  if (c.T == 0) return FMD_OK;
  DeviceGuard guard(m->device);
  c.Tp = round_up(c.T, kGemmBM);
  const hipStream_t caller = (hipStream_t)stream;
  FMD_TRY(enter_stream(m, caller, c));
  const int st = m->kind == 0 && m->cfg.precision != FMD_FP32
                     ? simulate_body<bf16>(m, truth, x0, seed, sched, reco, c, reco_off)
                     : simulate_body<float>(m, truth, x0, seed, sched, reco, c, reco_off);
  const int st2 = leave_stream(m, caller);
  return st != FMD_OK ? st : st2;
}

template int truth_cache<float>(fmd_model*, Call&);
template int truth_cache<bf16>(fmd_model*, Call&);
template int autotune<float>(fmd_model*, Call&);
template int autotune<bf16>(fmd_model*, Call&);
template int net_forward<float>(fmd_model*, Call&, const float*);
template int net_forward<bf16>(fmd_model*, Call&, const float*);

}  // namespace eng
}  // namespace fmd

using namespace fmd::eng;

int velocity_body(fmd_model* m, const fmd_events_in* truth, const float* x,
                  const float* t_per_event, float* v, Call& c) {
  FMD_TRY(stage_events(m, truth, c));
  Workspace& w = m->ws;
  const float* xs = x;
  const float* tev = t_per_event;
  if (!truth->on_device) {
    HIP_TRY(hipMemcpyAsync(w.io, x, (size_t)c.T * 9 * 4, hipMemcpyHostToDevice, c.st));
    HIP_TRY(hipMemcpyAsync(w.tev, t_per_event, (size_t)c.E * 4, hipMemcpyHostToDevice, c.st));
    xs = w.io;
    tev = w.tev;
  }
  FMD_TRY(timed(m, c.st, FMD_K_OTHER, 0, [&] { return launch_load_state(c.st, xs, 9, c.T, w.x, w.xs, kStateLd); }));
  float* out = truth->on_device ? v : w.io;
  if (m->cfg.precision != FMD_FP32) {
    FMD_TRY(truth_cache<bf16>(m, c));
    FMD_TRY(autotune<bf16>(m, c));
    FMD_TRY(net_forward<bf16>(m, c, tev));
  } else {
    FMD_TRY(truth_cache<float>(m, c));
    FMD_TRY(autotune<float>(m, c));
    FMD_TRY(net_forward<float>(m, c, tev));
  }
  FMD_TRY(head(m, c, true, UPD_VELOCITY, out, 9));
  if (!truth->on_device) {
    HIP_TRY(hipMemcpyAsync(v, w.io, (size_t)c.T * 9 * 4, hipMemcpyDeviceToHost, c.st));
    HIP_TRY(hipStreamSynchronize(c.st));
  }
  return FMD_OK;
}

// =======================================================================================
// C ABI

extern "C" {

const char* fmd_last_error(void) { return g_err.c_str(); }

size_t fmd_param_count(const fmd_model_config* cfg) {
  if (check_cfg(cfg) != FMD_OK) return 0;
  return walk_params(*cfg, [](int, int, size_t, int64_t, int64_t) {});
}

int fmd_model_create(const fmd_model_config* cfg, const float* params, size_t n_params,
                     fmd_model** out) {
  FMD_TRY(check_cfg(cfg));
  if (!params || !out) return fail(FMD_E_INVALID, "null params or out");
  const size_t need = fmd_param_count(cfg);
  if (n_params != need)
    return fail(FMD_E_INVALID, "parameter vector has %zu values, the config needs %zu", n_params, need);
  fmd_model* m = new fmd_model();
  m->cfg = *cfg;
  std::memset(m->tune, -1, sizeof(m->tune));
  m->fuse_stats = default_tile_rows(cfg->d_model) >= 0;
  std::memset(m->tune_us, 0, sizeof(m->tune_us));
  std::memset(m->tune_all, 0, sizeof(m->tune_all));
  auto bail = [&](int s) {
    fmd_model_destroy(m);
    return s;
  };
  if (hipGetDevice(&m->device) != hipSuccess) return bail(fail(FMD_E_DEVICE, "no HIP device"));
  if (grow(m->params, need * 4) != FMD_OK) return bail(FMD_E_NOMEM);
  if (hipMemcpy(m->params, params, need * 4, hipMemcpyHostToDevice) != hipSuccess)
    return bail(fail(FMD_E_DEVICE, "parameter upload failed"));
  const int64_t d = cfg->d_model, L = cfg->n_blocks;
  const size_t es = elem_size(*cfg);
  const size_t blk_elems = 14 * d * d;
  if (grow(m->packed, (L * blk_elems) * es) != FMD_OK) return bail(FMD_E_NOMEM);
  if (grow(m->Wkv, (size_t)(L * 2 * d * d) * es) != FMD_OK) return bail(FMD_E_NOMEM);
  if (grow(m->bkv, (size_t)(L * 2 * d) * 4) != FMD_OK) return bail(FMD_E_NOMEM);
  if (grow(m->Wout_pk, (size_t)64 * d * 4) != FMD_OK) return bail(FMD_E_NOMEM);
  if (grow(m->bout_pk, (size_t)64 * 4) != FMD_OK) return bail(FMD_E_NOMEM);
  m->fused_ok = cfg->precision != FMD_FP32 &&
                fused_supported(cfg->d_model, cfg->n_heads, cfg->mlp_ratio);
  m->kv_hm = cfg->precision != FMD_FP32 && cfg->d_model == 32 * cfg->n_heads;
  m->fused = m->fused_ok ? FMD_FUSED_ALL : 0;
  if (m->fused_ok && grow(m->frag, (size_t)(L * blk_elems) * 2) != FMD_OK) return bail(FMD_E_NOMEM);
  // FP8 form, per block: e4m3 fragments of W_up and W_dn (4 d^2 bytes each), then the column
  // scales s_up [4d], 1/s_up [4d], s_dn [d], 1/s_dn [d] (FP32)
  const size_t f8_blk = 8 * d * d + (size_t)10 * d * 4;
  if (cfg->precision == FMD_FP8 && grow(m->frag8, (size_t)L * f8_blk) != FMD_OK) return bail(FMD_E_NOMEM);
  if (cfg->precision == FMD_FP8) m->f8.assign(L, Fp8Mlp{});
  m->blk.assign(L, DevBlock{});
  char* pk = (char*)m->packed;
  char* wkv = (char*)m->Wkv;
  int status = FMD_OK;
  auto pack = [&](size_t off, int64_t rows, int64_t cols, void* dst) {
    const float* W = m->params + off;
    hipError_t e = cfg->precision != FMD_FP32
                       ? launch_pack_weight<bf16>(nullptr, W, (int)rows, (int)cols, (bf16*)dst)
                       : launch_pack_weight<float>(nullptr, W, (int)rows, (int)cols, (float*)dst);
    if (e != hipSuccess && status == FMD_OK) status = fail(FMD_E_DEVICE, "weight packing failed");
  };
  // second copy of a block matrix in the fused kernels' fragment layout, at the same
  // element offset inside the block as the packed copy
  char* fr = (char*)m->frag;
  auto pack_frag = [&](size_t off, int64_t rows, int64_t cols, int l, size_t elem_off,
                       void** dst) {
    if (!m->fused_ok) return;
    *dst = fr + ((size_t)l * blk_elems + elem_off) * 2;
    if (launch_pack_frag(nullptr, m->params + off, (int)rows, (int)cols, *dst) != hipSuccess &&
        status == FMD_OK)
      status = fail(FMD_E_DEVICE, "weight packing failed");
  };
  walk_params(*cfg, [&](int id, int l, size_t off, int64_t rows, int64_t cols) {
    const float* p = m->params + off;
    DevBlock* B = l >= 0 ? &m->blk[l] : nullptr;
    char* base = l >= 0 ? pk + (size_t)l * blk_elems * es : nullptr;
    switch (id) {
      case P_W_TIN: m->W_tin = p; break;
      case P_B_TIN: m->b_tin = p; break;
      case P_G_T: m->g_t = p; break;
      case P_S_T: m->s_t = p; break;
      case P_W_XIN: m->W_xin = p; break;
      case P_B_XIN: m->b_xin = p; break;
      case P_W_TIME: m->W_time = p; break;
      case P_B_TIME: m->b_time = p; break;
      case P_G1: B->g1 = p; break;
      case P_S1: B->s1 = p; break;
      case P_G2: B->g2 = p; break;
      case P_S2: B->s2 = p; break;
      case P_G3: B->g3 = p; break;
      case P_S3: B->s3 = p; break;
      case P_B_QKV: B->bqkv = p; break;
      case P_B_O: B->bo = p; break;
      case P_B_QC: B->bqc = p; break;
      case P_B_OC: B->boc = p; break;
      case P_B_UP: B->bup = p; break;
      case P_B_DN: B->bdn = p; break;
      case P_W_QKV:
        B->Wqkv = base;
        pack(off, rows, cols, B->Wqkv);
        pack_frag(off, rows, cols, l, 0, &B->Fqkv);
        break;
      case P_W_O:
        B->Wo = base + 3 * d * d * es;
        pack(off, rows, cols, B->Wo);
        pack_frag(off, rows, cols, l, 3 * d * d, &B->Fo);
        break;
      case P_W_QC:
        B->Wqc = base + 4 * d * d * es;
        pack(off, rows, cols, B->Wqc);
        pack_frag(off, rows, cols, l, 4 * d * d, &B->Fqc);
        break;
      case P_W_OC:
        B->Woc = base + 5 * d * d * es;
        pack(off, rows, cols, B->Woc);
        pack_frag(off, rows, cols, l, 5 * d * d, &B->Foc);
        break;
      case P_W_UP:
        B->Wup = base + 6 * d * d * es;
        pack(off, rows, cols, B->Wup);
        pack_frag(off, rows, cols, l, 6 * d * d, &B->Fup);
        if (cfg->precision == FMD_FP8) {
          char* f = (char*)m->frag8 + (size_t)l * f8_blk;
          float* sc = (float*)(f + 8 * d * d);
          m->f8[l].up = f;
          m->f8[l].up_inv = sc + 4 * d;
          if (launch_pack_frag8(nullptr, p, (int)rows, (int)cols, f, sc, sc + 4 * d) != hipSuccess &&
              status == FMD_OK)
            status = fail(FMD_E_DEVICE, "FP8 weight packing failed");
        }
        break;
      case P_W_DN:
        B->Wdn = base + 10 * d * d * es;
        pack(off, rows, cols, B->Wdn);
        pack_frag(off, rows, cols, l, 10 * d * d, &B->Fdn);
        if (cfg->precision == FMD_FP8) {
          char* f = (char*)m->frag8 + (size_t)l * f8_blk + 4 * d * d;
          float* sc = (float*)((char*)m->frag8 + (size_t)l * f8_blk + 8 * d * d) + 8 * d;
          m->f8[l].dn = f;
          m->f8[l].dn_scale = sc;
          m->f8[l].dn_inv = sc + d;
          if (launch_pack_frag8(nullptr, p, (int)rows, (int)cols, f, sc, sc + d) != hipSuccess &&
              status == FMD_OK)
            status = fail(FMD_E_DEVICE, "FP8 weight packing failed");
        }
        break;
      case P_W_KC: pack(off, rows, cols, wkv + (size_t)l * 2 * d * d * es); break;
      case P_W_VC: pack(off, rows, cols, wkv + ((size_t)l * 2 * d + d) * d * es); break;
      case P_B_KC:
        if (hipMemcpy(m->bkv + l * 2 * d, p, d * 4, hipMemcpyDeviceToDevice) != hipSuccess)
          status = fail(FMD_E_DEVICE, "bias copy failed");
        break;
      case P_B_VC:
        if (hipMemcpy(m->bkv + l * 2 * d + d, p, d * 4, hipMemcpyDeviceToDevice) != hipSuccess)
          status = fail(FMD_E_DEVICE, "bias copy failed");
        break;
      case P_G_F: m->g_f = p; break;
      case P_S_F: m->s_f = p; break;
      case P_W_OUT:
        m->W_out = p;
        if (launch_pack_weight<float>(nullptr, p, (int)rows, (int)cols, m->Wout_pk) != hipSuccess)
          status = fail(FMD_E_DEVICE, "weight packing failed");
        break;
      case P_B_OUT:
        m->b_out = p;
        if (hipMemcpy(m->bout_pk, p, rows * 4, hipMemcpyDeviceToDevice) != hipSuccess)
          status = fail(FMD_E_DEVICE, "bias copy failed");
        break;
      default: break;
    }
  });
  if (status != FMD_OK) return bail(status);
  if (hipDeviceSynchronize() != hipSuccess) return bail(fail(FMD_E_DEVICE, "model setup failed"));
  *out = m;
  return FMD_OK;
}

int fmd_linear_field_create(double alpha, double beta, fmd_model** out) {
  if (!out) return fail(FMD_E_INVALID, "null out");
  if (!std::isfinite(alpha) || !std::isfinite(beta)) return fail(FMD_E_INVALID, "non-finite coefficients");
  fmd_model* m = new fmd_model();
  m->kind = 1;
  m->alpha = alpha;
  m->beta = beta;
  m->cfg.n_max = 1 << 30;
  m->cfg.f_reco = m->cfg.f_truth = 9;
  if (hipGetDevice(&m->device) != hipSuccess) {   // bound on first use if no device yet
    (void)hipGetLastError();
    m->device = 0;
  }
  *out = m;
  return FMD_OK;
}

int fmd_model_destroy(fmd_model* m) {
  if (!m) return FMD_OK;
  if (m->server) return fail(FMD_E_STATE, "destroy the model's server first");
  if (m->kind == 1 && m->ws.cap_tok == 0 && m->ev_pool.empty() && m->trec.empty()) {
    delete m;   // never touched a device
    return FMD_OK;
  }
  DeviceGuard guard(m->device);
  (void)hipDeviceSynchronize();
  flush_timing(m);
  for (hipEvent_t e : m->ev_pool) (void)hipEventDestroy(e);
  if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
  if (m->pstream) (void)hipStreamDestroy(m->pstream);
  if (m->ev_in) (void)hipEventDestroy(m->ev_in);
  if (m->ev_out) (void)hipEventDestroy(m->ev_out);
  free_ws(m->ws);
  if (m->params) (void)hipFree(m->params);
  if (m->packed) (void)hipFree(m->packed);
  if (m->frag) (void)hipFree(m->frag);
  if (m->frag8) (void)hipFree(m->frag8);
  if (m->Wkv) (void)hipFree(m->Wkv);
  if (m->bkv) (void)hipFree(m->bkv);
  if (m->Wout_pk) (void)hipFree(m->Wout_pk);
  if (m->bout_pk) (void)hipFree(m->bout_pk);
  delete m;
  return FMD_OK;
}

int fmd_simulate(fmd_model* m, const fmd_events_in* truth, uint64_t seed,
                 const fmd_schedule* schedule, fmd_events_out* reco, void* hip_stream) {
  return simulate_impl(m, truth, nullptr, seed, schedule, reco, hip_stream);
}

int fmd_simulate_reco(fmd_model* m, const fmd_events_in* truth, const int64_t* reco_offsets,
                      uint64_t seed, const fmd_schedule* schedule, fmd_events_out* reco,
                      void* hip_stream) {
  if (!reco_offsets) return fail(FMD_E_INVALID, "null reco offsets");
  return simulate_impl(m, truth, nullptr, seed, schedule, reco, hip_stream, reco_offsets);
}

int fmd_simulate_from_state(fmd_model* m, const fmd_events_in* truth, const float* x0,
                            const fmd_schedule* schedule, fmd_events_out* reco,
                            void* hip_stream) {
  if (truth && truth->offsets && truth->n_events >= 0 && truth->offsets[truth->n_events] > 0 && !x0)
    return fail(FMD_E_INVALID, "null x0");
  return simulate_impl(m, truth, x0, 0, schedule, reco, hip_stream);
}

int fmd_velocity(fmd_model* m, const fmd_events_in* truth, const float* x,
                 const float* t_per_event, float* v, void* hip_stream) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  if (m->kind != 0) return fail(FMD_E_UNSUPPORTED, "fmd_velocity needs a network model");
  if (m->server) return fail(FMD_E_STATE, "the model is owned by a server");
  Call c{};
  FMD_TRY(check_events(m, truth, &c.T, nullptr));
  c.E = truth->n_events;
  if (c.T == 0) return FMD_OK;
  if (!x || !v || !t_per_event) return fail(FMD_E_INVALID, "null x, v or t_per_event");
  DeviceGuard guard(m->device);
  c.Tp = round_up(c.T, kGemmBM);
  const hipStream_t caller = (hipStream_t)hip_stream;
  FMD_TRY(enter_stream(m, caller, c));
  const int st = velocity_body(m, truth, x, t_per_event, v, c);
  const int st2 = leave_stream(m, caller);
  return st != FMD_OK ? st : st2;
}

int fmd_noise(uint64_t seed, const int64_t* offsets, int64_t n_events, int32_t n_feat,
              float* x0_device, void* hip_stream) {
  if (!offsets || n_events < 0) return fail(FMD_E_INVALID, "bad offsets");
  if (n_feat < 1 || n_feat > 12) return fail(FMD_E_INVALID, "n_feat must be in [1, 12]");
  fmd_events_in ev{n_events, offsets, x0_device, 1};
  int64_t T = 0;
  FMD_TRY(check_events(nullptr, &ev, &T, nullptr));
  if (T == 0) return FMD_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  int64_t* off = nullptr;
  int32_t* tok = nullptr;
  if (hipMalloc((void**)&off, (size_t)(n_events + 1) * 8) != hipSuccess ||
      hipMalloc((void**)&tok, (size_t)T * 4) != hipSuccess) {
    if (off) (void)hipFree(off);
    return fail(FMD_E_NOMEM, "allocation failed");
  }
  int status = FMD_OK;
  if (hipMemcpyAsync(off, offsets, (size_t)(n_events + 1) * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      launch_token_map(st, off, n_events, T, tok) != hipSuccess ||
      launch_noise(st, seed, off, tok, T, n_feat, x0_device, nullptr, n_feat) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    status = fail(FMD_E_DEVICE, "noise kernel failed");
  (void)hipFree(off);
  (void)hipFree(tok);
  return status;
}

int fmd_event_observables(const fmd_events_in* reco, float* ht, float* met, float* iso,
                          void* hip_stream) {
  if (!reco || !reco->offsets || reco->n_events < 0) return fail(FMD_E_INVALID, "bad events");
  const int64_t E = reco->n_events;
  fmd_events_in ev = *reco;
  int64_t T = 0;
  FMD_TRY(check_events(nullptr, &ev, &T, nullptr));
  if (E == 0) return FMD_OK;
  if (!ht || !met || (T > 0 && (!iso || !reco->feat))) return fail(FMD_E_INVALID, "null output");
  hipStream_t st = (hipStream_t)hip_stream;
  // device offsets (and, for host data, device copies) in a grow-only buffer kept between
  // calls; the lock covers the whole call, which ends with the stream synchronized
  static std::mutex mu;
  static void* buf = nullptr;
  static size_t cap = 0;
  std::lock_guard<std::mutex> lock(mu);
  const bool dev = reco->on_device != 0;
  const size_t b_off = (size_t)(E + 1) * 8, b_feat = dev ? 0 : (size_t)T * 9 * 4,
               b_out = dev ? 0 : (size_t)(2 * E + T) * 4;
  const size_t need = ((b_off + 255) & ~(size_t)255) + ((b_feat + 255) & ~(size_t)255) + b_out;
  if (need > cap) {
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    cap = 0;
    if (hipMalloc(&buf, need) != hipSuccess) return fail(FMD_E_NOMEM, "allocation failed");
    cap = need;
  }
  char* p = (char*)buf;
  int64_t* d_off = (int64_t*)p;
  p += (b_off + 255) & ~(size_t)255;
  const float* d_feat = reco->feat;
  float *d_ht = ht, *d_met = met, *d_iso = iso;
  if (!dev) {
    d_feat = (const float*)p;
    p += (b_feat + 255) & ~(size_t)255;
    d_ht = (float*)p;
    d_met = d_ht + E;
    d_iso = d_met + E;
  }
  hipError_t e = hipMemcpyAsync(d_off, reco->offsets, b_off, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !dev && T > 0)
    e = hipMemcpyAsync((void*)d_feat, reco->feat, b_feat, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_event_observables(st, d_feat, 9, d_off, E, d_ht, d_met, d_iso);
  if (e == hipSuccess && !dev) {
    e = hipMemcpyAsync(ht, d_ht, (size_t)E * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(met, d_met, (size_t)E * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess && T > 0)
      e = hipMemcpyAsync(iso, d_iso, (size_t)T * 4, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(FMD_E_DEVICE, "event observables: %s", hipGetErrorString(e));
  return FMD_OK;
}

int fmd_truth_select(const fmd_events_in* truth, double pt_cut_gev, int32_t max_particles,
                     int64_t* offsets_out, float* feat_out, void* hip_stream) {
  if (!truth || !offsets_out) return fail(FMD_E_INVALID, "null argument");
  if (!(pt_cut_gev > 0.0) || max_particles < 0) return fail(FMD_E_INVALID, "bad cut or limit");
  fmd_events_in ev = *truth;
  int64_t T = 0;
  FMD_TRY(check_events(nullptr, &ev, &T, nullptr));
  const int64_t E = truth->n_events;
  offsets_out[0] = 0;
  if (E == 0) return FMD_OK;
  if (T > 0 && !feat_out) return fail(FMD_E_INVALID, "null output");
  hipStream_t st = (hipStream_t)hip_stream;
  static std::mutex mu;
  static void* buf = nullptr;
  static size_t cap = 0;
  std::lock_guard<std::mutex> lock(mu);
  const bool dev = truth->on_device != 0;
  auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const size_t b_off = al((size_t)(E + 1) * 8), b_cnt = al((size_t)E * 4), b_keep = al((size_t)T),
               b_feat = dev ? 0 : al((size_t)T * 9 * 4);
  const size_t need = 2 * b_off + b_cnt + b_keep + 2 * b_feat;
  if (need > cap) {
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    cap = 0;
    if (hipMalloc(&buf, need) != hipSuccess) return fail(FMD_E_NOMEM, "allocation failed");
    cap = need;
  }
  char* p = (char*)buf;
  int64_t* d_off = (int64_t*)p;
  int64_t* d_off2 = (int64_t*)(p + b_off);
  int32_t* d_cnt = (int32_t*)(p + 2 * b_off);
  uint8_t* d_keep = (uint8_t*)(p + 2 * b_off + b_cnt);
  const float* d_in = truth->feat;
  float* d_out = feat_out;
  if (!dev) {
    d_in = (const float*)(p + 2 * b_off + b_cnt + b_keep);
    d_out = (float*)(p + 2 * b_off + b_cnt + b_keep + b_feat);
  }
  const float c0 = (float)std::log(pt_cut_gev / 10.0);
  std::vector<int32_t> cnt((size_t)E);
  hipError_t e = hipMemcpyAsync(d_off, truth->offsets, (size_t)(E + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && !dev && T > 0)
    e = hipMemcpyAsync((void*)d_in, truth->feat, (size_t)T * 9 * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_select_count(st, d_in, 9, d_off, E, c0, max_particles, d_keep, d_cnt);
  if (e == hipSuccess) e = hipMemcpyAsync(cnt.data(), d_cnt, (size_t)E * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess) {
    for (int64_t i = 0; i < E; ++i) offsets_out[i + 1] = offsets_out[i] + cnt[(size_t)i];
    e = hipMemcpyAsync(d_off2, offsets_out, (size_t)(E + 1) * 8, hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) e = launch_select_write(st, d_in, 9, d_off, d_off2, E, d_keep, d_out);
  if (e == hipSuccess && !dev && offsets_out[E] > 0)
    e = hipMemcpyAsync(feat_out, d_out, (size_t)offsets_out[E] * 9 * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(FMD_E_DEVICE, "truth selection: %s", hipGetErrorString(e));
  return FMD_OK;
}

int fmd_reco_multiplicity(const int64_t* truth_offsets, int64_t n_events, uint64_t seed,
                          const fmd_multiplicity_law* law, int32_t n_max, int64_t* reco_offsets_out,
                          void* hip_stream) {
  if (!truth_offsets || !law || !reco_offsets_out || n_events < 0) return fail(FMD_E_INVALID, "null argument");
  if (!(law->loss_prob >= 0.0 && law->loss_prob < 1.0) || !(law->fake_prob >= 0.0 && law->fake_prob < 1.0))
    return fail(FMD_E_INVALID, "probabilities must lie in [0, 1)");
  if (law->fake_trials < 0 || law->fake_trials > 4096) return fail(FMD_E_INVALID, "fake_trials must lie in [0, 4096]");
  if (n_max < 0) return fail(FMD_E_INVALID, "negative n_max");
  if (truth_offsets[0] != 0) return fail(FMD_E_INVALID, "offsets[0] must be 0");
  for (int64_t e = 0; e < n_events; ++e)
    if (truth_offsets[e + 1] < truth_offsets[e]) return fail(FMD_E_INVALID, "offsets decrease at event %lld", (long long)e);
  reco_offsets_out[0] = 0;
  if (n_events == 0) return FMD_OK;
  // floor(p 2^64): exact, and below 2^64 for p < 1
  const uint64_t thr_q = (uint64_t)std::ldexp(law->loss_prob, 64);
  const uint64_t thr_p = (uint64_t)std::ldexp(law->fake_prob, 64);
  hipStream_t st = (hipStream_t)hip_stream;
  static std::mutex mu;
  static void* buf = nullptr;
  static size_t cap = 0;
  std::lock_guard<std::mutex> lock(mu);
  const size_t b_off = ((size_t)(n_events + 1) * 8 + 255) & ~(size_t)255;
  const size_t need = b_off + (size_t)n_events * 4;
  if (need > cap) {
    if (buf) (void)hipFree(buf);
    buf = nullptr;
    cap = 0;
    if (hipMalloc(&buf, need) != hipSuccess) return fail(FMD_E_NOMEM, "allocation failed");
    cap = need;
  }
  int64_t* d_off = (int64_t*)buf;
  int32_t* d_cnt = (int32_t*)((char*)buf + b_off);
  std::vector<int32_t> cnt((size_t)n_events);
  hipError_t e = hipMemcpyAsync(d_off, truth_offsets, (size_t)(n_events + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = launch_reco_counts(st, d_off, n_events, seed, thr_q, thr_p, law->fake_trials, n_max, d_cnt);
  if (e == hipSuccess) e = hipMemcpyAsync(cnt.data(), d_cnt, (size_t)n_events * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(FMD_E_DEVICE, "reco multiplicity: %s", hipGetErrorString(e));
  for (int64_t i = 0; i < n_events; ++i) reco_offsets_out[i + 1] = reco_offsets_out[i] + cnt[(size_t)i];
  return FMD_OK;
}

int fmd_debug_philox(uint64_t key0, uint64_t key1, const uint64_t* counters, int64_t n,
                     uint64_t* out, void* hip_stream) {
  if (n < 0 || (n > 0 && (!counters || !out))) return fail(FMD_E_INVALID, "bad arguments");
  const hipError_t e = launch_philox((hipStream_t)hip_stream, key0, key1, counters, n, out);
  if (e != hipSuccess) return fail(FMD_E_DEVICE, "philox kernel failed: %s", hipGetErrorString(e));
  return FMD_OK;
}

int fmd_pack_padded(const float* padded, const int32_t* lengths, int64_t n_events,
                    int32_t n_max, int32_t f, int64_t* offsets_out, float* feat_out,
                    void* hip_stream) {
  if (n_events < 0 || n_max < 1 || f < 1) return fail(FMD_E_INVALID, "bad sizes");
  if (!offsets_out || (n_events > 0 && (!padded || !lengths || !feat_out)))
    return fail(FMD_E_INVALID, "null pointer");
  const hipError_t e = launch_pack_padded((hipStream_t)hip_stream, padded, lengths, n_events,
                                          n_max, f, offsets_out, feat_out);
  if (e != hipSuccess) return fail(FMD_E_DEVICE, "pack kernel failed: %s", hipGetErrorString(e));
  return FMD_OK;
}

int fmd_timing_enable(fmd_model* m, int32_t enable) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  DeviceGuard guard(m->device);
  flush_timing(m);
  m->timing = enable != 0;
  for (int k = 0; k < FMD_K_COUNT; ++k) m->t_ms[k] = 0, m->t_n[k] = 0, m->t_work[k] = 0, m->t_bytes[k] = 0;
  return FMD_OK;
}

int fmd_timing_read(fmd_model* m, int32_t cls, double* total_ms, int64_t* launches, double* work,
                    double* bytes) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  if (cls < 0 || cls >= FMD_K_COUNT) return fail(FMD_E_INVALID, "unknown kernel class");
  DeviceGuard guard(m->device);
  flush_timing(m);
  if (total_ms) *total_ms = m->t_ms[cls];
  if (launches) *launches = m->t_n[cls];
  if (work) *work = m->t_work[cls];
  if (bytes) *bytes = m->t_bytes[cls];
  return FMD_OK;
}

const char* fmd_kernel_name(fmd_model* m, int32_t cls) {
  (void)m;
  static const char* names[FMD_K_COUNT] = {"k_gemm_qkv",  "k_gemm_proj", "k_gemm_qc",
                                           "k_gemm_up",   "k_gemm_down", "k_fused_oqc",
                                           "k_fused_mlp", "k_attn_self", "k_attn_cross",
                                           "other"};
  if (cls == FMD_K_GEMM_QKV && m && (m->fused & FMD_FUSED_QKV)) return "k_fused_qkv";
  if ((cls == FMD_K_ATTN_SELF || cls == FMD_K_ATTN_CROSS) && m && m->kind == 0 &&
      m->cfg.precision != FMD_FP32 && m->cfg.d_model == 32 * m->cfg.n_heads)
    return cls == FMD_K_ATTN_SELF ? "k_attn32_self" : "k_attn32_cross";
  return cls >= 0 && cls < FMD_K_COUNT ? names[cls] : "";
}

int fmd_graphs_enable(fmd_model* m, int32_t enable) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  m->graphs = enable != 0;
  return FMD_OK;
}

int fmd_fused_enable(fmd_model* m, int32_t mask) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  if (mask < 0 || mask > FMD_FUSED_ALL)
    return fail(FMD_E_INVALID, "fused mask %d not in [0, %d]", mask, (int)FMD_FUSED_ALL);
  if (mask && !m->fused_ok)
    return fail(FMD_E_UNSUPPORTED, "no fused kernels for this configuration (BF16, d_model 256 only)");
  if (m->cfg.precision == FMD_FP8 && !(mask & FMD_FUSED_MLP))
    return fail(FMD_E_UNSUPPORTED, "an FP8 model runs its MLP in the fused kernel");
  if (m->fused != mask) {
    m->fused = mask;
    m->tune_gen++;   // captured graphs hold the other kernel sequence
  }
  return FMD_OK;
}

int fmd_autotune_enable(fmd_model* m, int32_t enable) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  m->autotune = enable != 0;
  return FMD_OK;
}

int fmd_tuning_set(fmd_model* m, int32_t site, int32_t tokens_log2, int32_t candidate) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  if (site < FMD_TUNE_ATTN_QUERY_TILE || site > FMD_TUNE_FUSED_OQC)
    return fail(FMD_E_INVALID, "site %d is not a fused-path site", site);
  if (tokens_log2 < 0 || tokens_log2 >= kTuneBuckets) return fail(FMD_E_INVALID, "bad token bucket");
  int tiles[4];
  const int n = site == FMD_TUNE_ATTN_QUERY_TILE ? attn_tiles(m, tiles) : (m->fused_ok ? 2 : 1);
  if (candidate < 0 || candidate >= n) return fail(FMD_E_INVALID, "candidate %d not in [0, %d)", candidate, n);
  const int sl = TS_ATTN + (site - FMD_TUNE_ATTN_QUERY_TILE);
  m->tune[sl][tokens_log2] = (int8_t)candidate;
  m->tune_us[sl][tokens_log2] = 0.f;
  m->tune_gen++;   // captured graphs hold the previous choice
  return FMD_OK;
}

int fmd_tuning_table(fmd_model* m, char* buf, size_t cap, size_t* needed) {
  if (!m) return fail(FMD_E_INVALID, "null model");
  static const char* slot_names[TS_COUNT] = {"qkv", "proj_residual", "proj_ln", "mlp_up", "mlp_down",
                                             "attn_query_tile", "fused_qkv", "fused_oqc"};
  int tiles[4];
  attn_tiles(m, tiles);
  std::string js = "{\"precision\": \"";
  js += m->cfg.precision == FMD_FP8 ? "fp8" : m->cfg.precision == FMD_BF16 ? "bf16" : "fp32";
  js += "\", \"d_model\": " + std::to_string(m->cfg.d_model) + ", \"entries\": [";
  bool first = true;
  for (int sl = 0; sl < TS_COUNT; ++sl)
    for (int b = 0; b < kTuneBuckets; ++b) {
      if (m->tune[sl][b] < 0) continue;
      // GEMM sites: the tiling; attention: queries per work item (BM) x keys per chunk (BN) x
      // head width (BK); fused kernels: rows per workgroup (BM) x model width (BN) x MFMA depth
      TileDims t{};
      if (sl < TS_GEMM)
        t = tile_dims(m->tune[sl][b]);
      else if (sl == TS_ATTN)
        t = TileDims{tiles[m->tune[sl][b]], 128, m->cfg.d_model / m->cfg.n_heads, 256};
      else
        t = TileDims{64 << m->tune[sl][b], m->cfg.d_model, 16, 512};
      char e[256];
      snprintf(e, sizeof(e),
               "%s{\"site\": \"%s\", \"tokens_log2\": %d, \"tile\": %d, \"BM\": %d, \"BN\": %d, "
               "\"BK\": %d, \"threads\": %d, \"us\": %.1f, \"candidates_us\": {",
               first ? "" : ", ", slot_names[sl], b, (int)m->tune[sl][b], t.BM, t.BN, t.BK, t.threads,
               m->tune_us[sl][b]);
      js += e;
      bool f2 = true;
      for (int k = 0; k < 8; ++k)
        if (m->tune_all[sl][b][k] > 0) {
          snprintf(e, sizeof(e), "%s\"%d\": %.1f", f2 ? "" : ", ", k, m->tune_all[sl][b][k]);
          js += e;
          f2 = false;
        }
      js += "}}";
      first = false;
    }
  js += "]}";
  if (needed) *needed = js.size() + 1;
  if (buf && cap > 0) {
    const size_t n = std::min(cap - 1, js.size());
    std::memcpy(buf, js.data(), n);
    buf[n] = 0;
  }
  return FMD_OK;
}

// ---- test hooks ---------------------------------------------------------------------

int fmd_debug_gemm(int32_t precision, int64_t M, int32_t N, int32_t K, const float* A,
                   const float* W, const float* bias, int32_t ln, const float* g,
                   const float* s, int32_t epi, float* C, int32_t tile, void* hip_stream) {
  if (precision != FMD_FP32 && precision != FMD_BF16) return fail(FMD_E_INVALID, "bad precision");
  if (M < 0 || N <= 0 || K <= 0 || K % 32 || N % 64) return fail(FMD_E_INVALID, "bad GEMM shape");
  if (epi < 0 || epi > 2) return fail(FMD_E_INVALID, "bad epilogue");
  if (M == 0) return FMD_OK;
  if (!A || !W || !C || (ln && (!g || !s))) return fail(FMD_E_INVALID, "null operand");
  hipStream_t st = (hipStream_t)hip_stream;
  const int64_t Mp = round_up(M, kGemmBM);
  if (tile >= kGemmTiles || (tile >= 0 && !tile_fits(tile, Mp, N, K)))
    return fail(FMD_E_UNSUPPORTED, "tiling %d does not divide the shape", tile);
  const int cls = ln && epi == EPI_STORE ? FMD_K_GEMM_QKV : ln && epi == EPI_GELU ? FMD_K_GEMM_UP
                  : !ln && epi == EPI_RESID ? FMD_K_GEMM_DOWN : FMD_K_OTHER;
  if (cls == FMD_K_OTHER && tile != -1 && tile != 0 && tile != 4)
    return fail(FMD_E_UNSUPPORTED, "this epilogue combination has tilings 0 and 4 only");
  const size_t es = precision == FMD_BF16 ? 2 : 4;
  const size_t a_es = ln ? 4 : es;
  const size_t c_es = epi == EPI_RESID ? 4 : es;
  void *Ap = nullptr, *Wt = nullptr, *Cp = nullptr;
  float2* st2 = nullptr;
  int status = FMD_OK;
  if (grow(Ap, (size_t)Mp * K * a_es) || grow(Wt, (size_t)N * K * es) || grow(Cp, (size_t)Mp * N * c_es) ||
      grow(st2, (size_t)Mp * sizeof(float2))) {
    status = FMD_E_NOMEM;
  } else {
    hipError_t e = hipSuccess;
    if (ln) e = hipMemcpyAsync(Ap, A, (size_t)M * K * 4, hipMemcpyDeviceToDevice, st);
    else if (precision == FMD_BF16) e = launch_convert<bf16>(st, A, M * K, (bf16*)Ap);
    else e = hipMemcpyAsync(Ap, A, (size_t)M * K * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = precision == FMD_BF16 ? launch_pack_weight<bf16>(st, W, K, N, (bf16*)Wt)
                                : launch_pack_weight<float>(st, W, K, N, (float*)Wt);
    if (e == hipSuccess && epi == EPI_RESID)
      e = hipMemcpyAsync(Cp, C, (size_t)M * N * 4, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess && ln) {
      if (K % 64 || K > 1024) e = hipErrorInvalidValue;
      else e = launch_row_stats(st, (const float*)Ap, K, K, Mp, st2);
    }
    if (e == hipSuccess)
      e = precision == FMD_BF16
              ? launch_gemm<bf16>(st, cls, ln != 0, epi, Mp, N, K, Ap, K, (const bf16*)Wt, bias, st2, g, s, Cp, N, nullptr, tile)
              : launch_gemm<float>(st, cls, ln != 0, epi, Mp, N, K, Ap, K, (const float*)Wt, bias, st2, g, s, Cp, N, nullptr, tile);
    if (e == hipSuccess) {
      if (epi == EPI_RESID || precision == FMD_FP32)
        e = hipMemcpyAsync(C, Cp, (size_t)M * N * 4, hipMemcpyDeviceToDevice, st);
      else
        e = launch_to_f32<bf16>(st, (const bf16*)Cp, M * N, C);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) status = fail(FMD_E_DEVICE, "debug gemm: %s", hipGetErrorString(e));
  }
  if (Ap) (void)hipFree(Ap);
  if (Wt) (void)hipFree(Wt);
  if (Cp) (void)hipFree(Cp);
  if (st2) (void)hipFree(st2);
  return status;
}

int fmd_debug_attention(int32_t precision, int64_t n_events, const int64_t* q_offsets,
                        const int64_t* kv_offsets, int32_t n_heads, int32_t dh,
                        const float* Q, const float* K, const float* V, float* O,
                        void* hip_stream) {
  if (precision != FMD_FP32 && precision != FMD_BF16) return fail(FMD_E_INVALID, "bad precision");
  if (dh != 16 && dh != 32 && dh != 64) return fail(FMD_E_UNSUPPORTED, "dh must be 16, 32 or 64");
  if (n_heads < 1 || n_events < 0 || !q_offsets || !kv_offsets) return fail(FMD_E_INVALID, "bad arguments");
  if (q_offsets[0] != 0 || kv_offsets[0] != 0) return fail(FMD_E_INVALID, "offsets must start at 0");
  const int qt = attention_query_tile(precision == FMD_BF16, dh, n_heads);   // the default tile
  std::vector<int64_t> ids((size_t)n_events);
  int64_t n_items = 0;
  for (int64_t e = 0; e < n_events; ++e) {
    const int64_t nq = q_offsets[e + 1] - q_offsets[e], nk = kv_offsets[e + 1] - kv_offsets[e];
    if (nq < 0 || nk < 0) return fail(FMD_E_INVALID, "offsets decrease");
    if (nq > 0 && nk == 0) return fail(FMD_E_INVALID, "event %lld has queries but no keys", (long long)e);
    ids[e] = e;
    n_items += (nq + qt - 1) / qt;
  }
  std::vector<AttnItem> work((size_t)n_items);
  AttnBins bins{};
  if (build_attention_work(q_offsets, kv_offsets, ids.data(), n_events, qt, work.data(), &bins) !=
      n_items)
    return fail(FMD_E_INVALID, "rows beyond 2^31");
  const int64_t Tq = q_offsets[n_events], Tk = kv_offsets[n_events];
  if (work.empty()) return FMD_OK;
  if (!Q || !K || !V || !O) return fail(FMD_E_INVALID, "null operand");
  hipStream_t st = (hipStream_t)hip_stream;
  const int ld = n_heads * dh;
  const size_t es = precision == FMD_BF16 ? 2 : 4;
  AttnItem* wk = nullptr;
  void *Qp = nullptr, *Kp = nullptr, *Vp = nullptr, *Op = nullptr;
  int status = FMD_OK;
  if (grow(wk, work.size() * sizeof(AttnItem)) ||
      grow(Qp, (size_t)Tq * ld * es) || grow(Kp, (size_t)Tk * ld * es) || grow(Vp, (size_t)Tk * ld * es) ||
      grow(Op, (size_t)Tq * ld * es)) {
    status = FMD_E_NOMEM;
  } else {
    hipError_t e = hipMemcpy(wk, work.data(), work.size() * sizeof(AttnItem), hipMemcpyHostToDevice);
    if (precision == FMD_BF16) {
      if (e == hipSuccess) e = launch_convert<bf16>(st, Q, Tq * ld, (bf16*)Qp);
      if (e == hipSuccess) e = launch_convert<bf16>(st, K, Tk * ld, (bf16*)Kp);
      if (e == hipSuccess) e = launch_convert<bf16>(st, V, Tk * ld, (bf16*)Vp);
      if (e == hipSuccess)
        e = launch_attention<bf16>(st, false, dh, n_heads, qt, (int64_t)work.size(), bins, wk, (const bf16*)Qp, ld,
                                   dh, (const bf16*)Kp, (const bf16*)Vp, ld, dh, (bf16*)Op, ld, dh);
      if (e == hipSuccess) e = launch_to_f32<bf16>(st, (const bf16*)Op, Tq * ld, O);
    } else {
      if (e == hipSuccess)
        e = launch_attention<float>(st, false, dh, n_heads, qt, (int64_t)work.size(), bins, wk, Q, ld, dh, K, V, ld,
                                    dh, O, ld, dh);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) status = fail(FMD_E_DEVICE, "debug attention: %s", hipGetErrorString(e));
  }
  void* bufs[] = {wk, Qp, Kp, Vp, Op};
  for (void* p : bufs)
    if (p) (void)hipFree(p);
  return status;
}

}  // extern "C"
