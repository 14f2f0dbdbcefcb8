// Continuous-batching server for flow-matching sampling requests.
//
// Requests (a set of truth events, a seed and a schedule) arrive at any time. A worker
// thread runs the device loop:
//   admission  FIFO; a request is admitted when a contiguous range of max(truth particles,
//              reco slots) rows is free in the device token pool, whose size is the HBM
//              budget divided by the per-token footprint. Admission draws the noise of its
//              reco slots, encodes its truth particles and fills its cross-attention K/V
//              cache, all in its pool range (reco slot rows and truth rows both count from
//              the range start). These stay resident until the request completes.
//   iteration  one velocity evaluation over the pool prefix that holds resident events.
//              Every event carries its own stage-table entry (time, step, Euler/RK4 stage),
//              so requests with different schedules and at different points of their
//              integration share one launch of each kernel. Gaps between requests are
//              dummy segments whose rows are never read by a live event and are not
//              updated.
//   completion when a request's events finish their last stage, its rows are copied back,
//              its pool range is released and waiters are woken.
// The loop is pipelined by one iteration: the host plans and enqueues iteration i + 1
// (admission work, work lists, kernels, copy-out) before it waits for iteration i to end, so
// the device does not idle while the host builds the next work lists. Everything the host
// hands to the device in flight goes through pinned staging buffers, two sets used in turn;
// a finished request keeps its pool range until its rows have reached host memory.
// An event's noise is keyed by (request seed, event index in the request, slot). GEMM
// rows are independent and attention stays within an event. So a request's result is
// bitwise the same alone and in any mix of other requests.
#include <time.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "engine_impl.h"
#include "gemm_body.h"

using namespace fmd;
using namespace fmd::eng;

namespace {

uint64_t now_ns() {
  timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (uint64_t)ts.tv_sec * 1000000000ull + (uint64_t)ts.tv_nsec;
}

struct Req {
  uint64_t id = 0;
  std::vector<int64_t> off;     // [n + 1] truth offsets
  std::vector<int64_t> roff;    // [n + 1] reco offsets (equal to off unless given)
  std::vector<float> feat;      // [T, 9]
  uint64_t seed = 0;
  fmd_schedule sched{};
  int64_t T = 0, Tr = 0;        // truth particles, reco slots
  int64_t rows = 0, base = -1;  // pool rows max(T, Tr) and the first of them
  int64_t n_events = 0;
  int stage = 0, n_stages = 0;  // all events of a request advance together
  std::vector<float> out;       // [Tr, 9] result
  fmd_request_stats stats{};
  int status = FMD_PENDING;
  std::string error;
};

// First-fit allocator of contiguous row ranges with coalescing of freed ranges.
struct Pool {
  int64_t cap = 0;
  std::map<int64_t, int64_t> free_;   // start -> length
  void init(int64_t c) {
    cap = c;
    free_.clear();
    if (c > 0) free_[0] = c;
  }
  int64_t alloc(int64_t n) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const int64_t s = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[s + n] = len - n;
      return s;
    }
    return -1;
  }
  void release(int64_t s, int64_t n) {
    auto it = free_.emplace(s, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

constexpr int64_t kPoolSlack = 256;   // rows past the pool so padded GEMM tiles stay inside
// Pool ranges are whole 64-row tiles, so that a tile holds rows of one request or none: the
// fused kernels then run only the tiles of resident requests.
constexpr int64_t kTile = 64;
int64_t pool_rows(const Req* r) { return round_up(std::max<int64_t>(r->rows, 1), kTile); }

// Pinned host buffers of one iteration: its CSR offsets, attention work lists, stage table,
// per-event times, and the reco offsets and truth features of the requests it admits.
struct Staging {
  int64_t* off = nullptr;
  AttnItem* work = nullptr;
  StageDesc* desc = nullptr;
  float* tev = nullptr;
  int32_t* tiles = nullptr;
  char* adm = nullptr;
  size_t cap_off = 0, cap_work = 0, cap_desc = 0, cap_tev = 0, cap_tiles = 0, cap_adm = 0;
};

// Grow-only pinned buffer of at least n elements (contents are not kept).
template <typename P>
int reserve_pinned(P*& p, size_t& cap, size_t n) {
  if (n <= cap) return FMD_OK;
  const size_t want = std::max(n, cap + cap / 2);
  FMD_TRY(grow_host(p, want * sizeof(P)));
  cap = want;
  return FMD_OK;
}

void free_staging(Staging& g) {
  void* ps[] = {g.off, g.work, g.desc, g.tev, g.tiles, g.adm};
  for (void* p : ps)
    if (p) (void)hipHostFree(p);
  g = Staging{};
}

// One enqueued iteration whose completion the host has not yet handled.
struct InFlight {
  int set;                       // staging set and event pair
  std::vector<Req*> finished;    // requests whose last stage ran in it
};

}  // namespace

struct fmd_server {
  fmd_model* m = nullptr;
  fmd_server_config cfg{};
  int64_t pool_tokens = 0;
  size_t bytes_per_token = 0;
  Pool pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> queue;
  std::map<uint64_t, Req*> reqs;       // every request not yet collected
  std::vector<Req*> resident;
  int64_t resident_tokens = 0;
  uint64_t next_id = 1;
  bool stop = false;
  int dead = FMD_OK;                   // device failure of the worker
  std::string dead_msg;
  std::thread worker;
  hipStream_t st = nullptr;
  // admission scratch (one request at a time)
  int64_t* adm_off = nullptr;
  int32_t* adm_tok = nullptr;
  int64_t adm_cap_ev = 0, adm_cap_tok = 0;
  // pinned staging of the two iterations that can be in flight, and the output rows
  Staging stg[2];
  float* out_pin = nullptr;            // [pool rows, 9]: a finished request's rows by pool row
  int32_t* d_tiles = nullptr;          // [pool rows / 64]: 64-row tiles of an iteration
  hipEvent_t ev_start[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
  // counters
  uint64_t iterations = 0, rows_processed = 0, rows_live = 0, busy_ns = 0;
};

namespace {

// Device bytes one resident token costs: ODE state, residual stream and LayerNorm
// statistics, activations, truth features and encoding, cross K/V cache, output.
size_t bytes_per_token(const fmd_model_config& c) {
  const size_t d = c.d_model, L = c.n_blocks, es = c.precision == FMD_FP32 ? 4 : 2;
  return 3 * kStateLd * 4 + d * 4 + sizeof(float2) + 4 + (3 * d + d + d + 4 * d + d) * es +
         2 * d * L * es + 9 * 4 * 2;
}

// Enqueues the admission of r: noise, truth encoding and cross K/V cache in its pool range.
// roff_pin / feat_pin: its reco offsets and truth features in pinned staging.
template <typename T>
int admit_device(fmd_server* S, Req* r, const int64_t* roff_pin, const float* feat_pin) {
  fmd_model* m = S->m;
  Workspace& w = m->ws;
  const int d = m->cfg.d_model, L = m->cfg.n_blocks;
  const int64_t E = r->n_events, nT = r->T, nR = r->Tr, b = r->base;
  if (E + 1 > S->adm_cap_ev) {   // (a reallocation waits for the device to go idle)
    FMD_TRY(grow(S->adm_off, (size_t)(E + 1) * 8));
    S->adm_cap_ev = E + 1;
  }
  if (nR > S->adm_cap_tok) {
    FMD_TRY(grow(S->adm_tok, (size_t)nR * 4));
    S->adm_cap_tok = nR;
  }
  // noise of the reco slots, keyed by (seed, event, slot)
  HIP_TRY(hipMemcpyAsync(S->adm_off, roff_pin, (size_t)(E + 1) * 8, hipMemcpyHostToDevice, S->st));
  HIP_TRY(launch_token_map(S->st, S->adm_off, E, nR, S->adm_tok));
  HIP_TRY(launch_noise(S->st, r->seed, S->adm_off, S->adm_tok, nR, 9, w.x + b * kStateLd,
                       w.xs + b * kStateLd, kStateLd));
  if (nT == 0) return FMD_OK;
  HIP_TRY(hipMemcpyAsync(w.u + b * 9, feat_pin, (size_t)nT * 9 * 4, hipMemcpyHostToDevice, S->st));
  const size_t es = sizeof(T);
  T* cb = (T*)w.c + b * d;
  HIP_TRY(launch_truth_encode<T>(S->st, w.u + b * 9, 9, 9, nT, m->W_tin, m->b_tin, m->g_t, m->s_t,
                                 d, cb, d));
  // K/V cache of the request's rows; padded rows past its end recompute identical values
  // for neighbours (a pure function of their own truth encoding) or fill unused rows.
  if (m->kv_hm) {   // per block into scratch rows, then the request's rows of the planes
    const int H = m->cfg.n_heads, dh = d / H;
    for (int l = 0; l < L; ++l) {
      HIP_TRY(launch_gemm<T>(S->st, FMD_K_OTHER, false, EPI_STORE, round_up(nT, kGemmBM), 2 * d,
                             d, cb, d, (const T*)m->Wkv + (size_t)l * 2 * d * d,
                             m->bkv + l * 2 * d, nullptr, nullptr, nullptr, w.hid, 2 * d));
      HIP_TRY(launch_kv_headmajor(S->st, w.hid, nT, d, dh, H,
                                  (char*)w.kv + (size_t)l * 2 * H * w.cap_tok * dh * es,
                                  w.cap_tok, b));
    }
    return FMD_OK;
  }
  HIP_TRY(launch_gemm<T>(S->st, FMD_K_OTHER, false, EPI_STORE, round_up(nT, kGemmBM), 2 * d * L, d,
                         cb, d, (const T*)m->Wkv, m->bkv, nullptr, nullptr, nullptr,
                         (char*)w.kv + (size_t)b * 2 * d * L * es, 2 * d * L));
  return FMD_OK;
}

// Enqueues one iteration over all resident requests, with the host data of staging set k and
// the completion event ev_done[k]; moves the requests whose last stage it runs to `finished`.
template <typename T>
int iterate(fmd_server* S, int k, std::vector<Req*>& finished) {
  fmd_model* m = S->m;
  Workspace& w = m->ws;
  Staging& g = S->stg[k];
  std::vector<Req*> res = S->resident;
  std::sort(res.begin(), res.end(), [](Req* a, Req* b) { return a->base < b->base; });
  // segments: dummy gaps and real events, in pool order
  std::vector<int64_t> off{0};
  std::vector<StageDesc> desc;
  std::vector<float> tev;
  std::vector<std::pair<int64_t, int64_t>> real;   // (segment index, length)
  std::vector<int64_t> kv0, kvn;                   // per segment: first truth row, count
  double sum_n2 = 0, sum_nx = 0;
  int64_t pos = 0, items = 0, live = 0;
  std::vector<int32_t> tiles;   // the 64-row tiles of the resident requests' ranges
  for (Req* r : res) {
    for (int64_t t = r->base / kTile; t < (r->base + pool_rows(r)) / kTile; ++t) tiles.push_back((int32_t)t);
    if (r->base > pos) {
      off.push_back(r->base);
      desc.push_back(StageDesc{0.f, 0.f, UPD_NONE, 0});
      tev.push_back(0.f);
      kv0.push_back(0);
      kvn.push_back(0);
      pos = r->base;
    }
    const StageDesc sd = stage_desc(r->sched, r->stage);
    for (int64_t e = 0; e < r->n_events; ++e) {
      const int64_t n = r->roff[e + 1] - r->roff[e], nt = r->off[e + 1] - r->off[e];
      if (n == 0) continue;
      real.emplace_back((int64_t)desc.size(), n);
      kv0.push_back(r->base + r->off[e]);
      kvn.push_back(nt);
      off.push_back(pos + n);
      desc.push_back(sd);
      tev.push_back(sd.t);
      pos += n;
      live += n;
      sum_n2 += (double)n * (double)n;
      sum_nx += (double)n * (double)nt;
    }
  }
  const int64_t E = (int64_t)desc.size(), span = pos;
  if (span == 0) return FMD_OK;
  // work items of the query tile tuned for this size (the default where none is)
  const int qt = attn_tile_for(m, round_up(span, kGemmBM));
  for (const auto& rs : real) items += (rs.second + qt - 1) / qt;
  // self-attention items, then cross-attention items (reco queries, truth keys)
  FMD_TRY(ensure_ws(m, span, E, 2 * items));
  FMD_TRY(reserve_pinned(g.off, g.cap_off, (size_t)E + 1));
  FMD_TRY(reserve_pinned(g.work, g.cap_work, (size_t)(2 * items)));
  FMD_TRY(reserve_pinned(g.desc, g.cap_desc, (size_t)E));
  FMD_TRY(reserve_pinned(g.tev, g.cap_tev, (size_t)E));
  FMD_TRY(reserve_pinned(g.tiles, g.cap_tiles, tiles.size()));
  // the last request's tiles may reach past the span (its range is rounded to whole tiles)
  const int64_t Tp = round_up(span, kGemmBM);
  while (!tiles.empty() && (int64_t)tiles.back() * kTile >= Tp) tiles.pop_back();
  std::memcpy(g.tiles, tiles.data(), tiles.size() * 4);
  std::memcpy(g.off, off.data(), (size_t)(E + 1) * 8);
  std::memcpy(g.desc, desc.data(), (size_t)E * sizeof(StageDesc));
  std::memcpy(g.tev, tev.data(), (size_t)E * 4);
  AttnBins bins{}, bins_x{};
  {
    std::vector<int64_t> ids(real.size());
    for (size_t i = 0; i < real.size(); ++i) ids[i] = real[i].first;
    if (build_attention_work(off.data(), off.data(), ids.data(), (int64_t)real.size(),
                             qt, g.work, &bins) != items ||
        build_attention_work_kv(off.data(), kv0.data(), kvn.data(), ids.data(),
                                (int64_t)real.size(), qt, g.work + items, &bins_x) != items)
      return fail(FMD_E_INVALID, "token rows beyond 2^31");
  }
  if (E > w.cap_desc) {   // (the reallocation waits for the device to go idle)
    FMD_TRY(grow(w.desc, (size_t)E * sizeof(StageDesc)));
    w.cap_desc = (int)E;
  }
  HIP_TRY(hipMemcpyAsync(w.off, g.off, (size_t)(E + 1) * 8, hipMemcpyHostToDevice, S->st));
  HIP_TRY(hipMemcpyAsync(w.work, g.work, (size_t)(2 * items) * sizeof(AttnItem), hipMemcpyHostToDevice, S->st));
  HIP_TRY(hipMemcpyAsync(w.desc, g.desc, (size_t)E * sizeof(StageDesc), hipMemcpyHostToDevice, S->st));
  HIP_TRY(hipMemcpyAsync(w.tev, g.tev, (size_t)E * 4, hipMemcpyHostToDevice, S->st));
  HIP_TRY(hipMemcpyAsync(S->d_tiles, g.tiles, tiles.size() * 4, hipMemcpyHostToDevice, S->st));

  Call c{};
  c.st = S->st;
  c.E = E;
  c.T = span;
  c.Tp = round_up(span, kGemmBM);
  c.qt = qt;
  c.items = items;
  c.bins = bins;
  c.sum_n2 = sum_n2;
  same_truth(c);
  c.items_x = items;
  c.work_x = items;
  c.bins_x = bins_x;
  c.sum_nx = sum_nx;
  c.u = w.u;
  c.tiles = S->d_tiles;
  c.n_tiles = (int64_t)tiles.size();
  HIP_TRY(launch_token_map(S->st, w.off, E, span, w.tok_event));
  FMD_TRY(autotune<T>(m, c));
  const OdeArgs ode{w.x, w.acc, w.xs, w.io, span, kStateLd, 9, 9, 0, 0.f, w.desc, nullptr, w.tok_event};
  c.head = &ode;
  FMD_TRY(net_forward<T>(m, c, w.tev));
  c.head = nullptr;
  const int d = m->cfg.d_model;
  if (!c.head_done) {   // else the last block's MLP kernel applied the head
    FMD_TRY(row_stats(m, c));
    if (head256_supported(d, 9))
      HIP_TRY(launch_head256(S->st, w.H, w.stats, m->g_f, m->s_f, m->Wout_pk, m->bout_pk, ode));
    else
      HIP_TRY(launch_gemm<float>(S->st, FMD_K_OTHER, true, EPI_ODE, c.Tp, 64, d, w.H, d,
                                 m->Wout_pk, m->bout_pk, w.stats, m->g_f, m->s_f, nullptr, 0,
                                 &ode));
  }
  // a finished request's rows go to its pool rows of the pinned output staging
  for (Req* r : res)
    if (r->stage == r->n_stages - 1) {
      HIP_TRY(hipMemcpyAsync(S->out_pin + r->base * 9, w.io + r->base * 9, (size_t)r->Tr * 9 * 4,
                             hipMemcpyDeviceToHost, S->st));
      finished.push_back(r);
    }
  HIP_TRY(hipEventRecord(S->ev_done[k], S->st));
  for (Req* r : res) r->stage++;
  S->iterations++;
  S->rows_processed += span;
  S->rows_live += live;
  return FMD_OK;
}

void fail_all(fmd_server* S, int status, const std::string& msg) {
  // caller holds the lock
  for (auto& kv : S->reqs) {
    Req* r = kv.second;
    if (r->status == FMD_PENDING) {
      r->status = status;
      r->error = msg;
      r->stats.t_done_ns = now_ns();
    }
  }
  S->queue.clear();
  S->resident.clear();
  S->cv_done.notify_all();
}

// Handles the end of an enqueued iteration: waits for its event, copies the finished
// requests' rows from the pinned staging, releases their pool ranges and wakes waiters.
int complete(fmd_server* S, const InFlight& f) {
  HIP_TRY(hipEventSynchronize(S->ev_done[f.set]));
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, S->ev_start[f.set], S->ev_done[f.set]) == hipSuccess)
    S->busy_ns += (uint64_t)((double)ms * 1e6);
  for (Req* r : f.finished)
    if (r->Tr) std::memcpy(r->out.data(), S->out_pin + r->base * 9, (size_t)r->Tr * 9 * 4);
  std::lock_guard<std::mutex> lk(S->mu);
  const uint64_t t = now_ns();
  for (Req* r : f.finished) {
    r->status = FMD_OK;
    r->stats.t_done_ns = t;
    S->pool.release(r->base, pool_rows(r));
    S->resident_tokens -= r->rows;
  }
  if (!f.finished.empty()) S->cv_done.notify_all();
  return FMD_OK;
}

void worker_main(fmd_server* S) {
  fmd_model* m = S->m;
  DeviceGuard guard(m->device);
  const bool bf = m->cfg.precision != FMD_FP32;
  std::deque<InFlight> inflight;   // at most two: the one just enqueued and its predecessor
  int k = 0;                       // staging set of the next iteration
  for (;;) {
    std::vector<Req*> admitted;
    bool work = false;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv_work.wait(lk, [&] {
        return S->stop || !S->queue.empty() || !S->resident.empty() || !inflight.empty();
      });
      if (S->stop) {
        lk.unlock();
        (void)hipStreamSynchronize(S->st);   // no copy may still target the staging
        lk.lock();
        fail_all(S, FMD_E_STATE, "server destroyed before the request completed");
        return;
      }
      while (!S->queue.empty()) {
        Req* r = S->queue.front();
        if (S->cfg.max_requests > 0 && (int64_t)S->resident.size() >= S->cfg.max_requests) break;
        if (S->cfg.max_tokens_per_iter > 0 && !S->resident.empty() &&
            S->resident_tokens + r->rows > S->cfg.max_tokens_per_iter)
          break;
        const int64_t b = S->pool.alloc(pool_rows(r));
        if (b < 0) break;
        S->queue.pop_front();
        r->base = b;
        r->stats.t_admit_ns = now_ns();
        S->resident.push_back(r);
        S->resident_tokens += r->rows;
        admitted.push_back(r);
      }
      work = !S->resident.empty();
    }
    int st = FMD_OK;
    if (work) {
      // set k was last used two iterations ago, and that iteration has been completed
      Staging& g = S->stg[k];
      size_t need = 0;
      for (Req* r : admitted) need += (size_t)(r->n_events + 1) * 8 + (size_t)r->T * 9 * 4;
      st = reserve_pinned(g.adm, g.cap_adm, need);
      if (st == FMD_OK && hipEventRecord(S->ev_start[k], S->st) != hipSuccess)
        st = fail(FMD_E_DEVICE, "event record failed");
      size_t o = 0;
      for (Req* r : admitted) {
        if (st != FMD_OK) break;
        int64_t* ro = (int64_t*)(g.adm + o);
        std::memcpy(ro, r->roff.data(), (size_t)(r->n_events + 1) * 8);
        o += (size_t)(r->n_events + 1) * 8;
        float* fe = (float*)(g.adm + o);
        std::memcpy(fe, r->feat.data(), (size_t)r->T * 9 * 4);
        o += (size_t)r->T * 9 * 4;
        st = bf ? admit_device<bf16>(S, r, ro, fe) : admit_device<float>(S, r, ro, fe);
      }
      InFlight f{k, {}};
      if (st == FMD_OK) st = bf ? iterate<bf16>(S, k, f.finished) : iterate<float>(S, k, f.finished);
      if (st == FMD_OK) {
        std::lock_guard<std::mutex> lk(S->mu);
        for (Req* r : f.finished) S->resident.erase(std::find(S->resident.begin(), S->resident.end(), r));
        inflight.push_back(std::move(f));
        k ^= 1;
      }
    }
    // complete the previous iteration while the one just enqueued runs (or everything, when
    // nothing new was enqueued)
    while (st == FMD_OK && (inflight.size() > 1 || (!work && !inflight.empty()))) {
      st = complete(S, inflight.front());
      inflight.pop_front();
    }
    if (st != FMD_OK) {
      const std::string msg = fmd_last_error();
      (void)hipStreamSynchronize(S->st);
      std::lock_guard<std::mutex> lk(S->mu);
      S->dead = st;
      S->dead_msg = msg;
      fail_all(S, st, S->dead_msg);
      return;
    }
  }
}

// Device and pinned resources of a server (its stream must be idle).
void release_resources(fmd_server* S) {
  if (S->st) (void)hipStreamDestroy(S->st);
  S->st = nullptr;
  for (int i = 0; i < 2; ++i) {
    if (S->ev_start[i]) (void)hipEventDestroy(S->ev_start[i]);
    if (S->ev_done[i]) (void)hipEventDestroy(S->ev_done[i]);
    free_staging(S->stg[i]);
  }
  if (S->out_pin) (void)hipHostFree(S->out_pin);
  if (S->adm_off) (void)hipFree(S->adm_off);
  if (S->adm_tok) (void)hipFree(S->adm_tok);
  if (S->d_tiles) (void)hipFree(S->d_tiles);
  S->d_tiles = nullptr;
  S->out_pin = nullptr;
  S->adm_off = nullptr;
  S->adm_tok = nullptr;
}

// Copies a finished request out and forgets it (caller holds the lock).
int collect(fmd_server* S, Req* r, float* reco, fmd_request_stats* stats) {
  const int status = r->status;
  if (stats) *stats = r->stats;
  if (status == FMD_OK && reco && r->Tr) std::memcpy(reco, r->out.data(), (size_t)r->Tr * 9 * 4);
  const std::string err = r->error;
  S->reqs.erase(r->id);
  delete r;
  if (status != FMD_OK) return fail(status, "%s", err.c_str());
  return FMD_OK;
}

}  // namespace

extern "C" {

int fmd_server_create(fmd_model* m, const fmd_server_config* cfg, fmd_server** out) {
  if (!m || !cfg || !out) return fail(FMD_E_INVALID, "null argument");
  if (m->kind != 0) return fail(FMD_E_UNSUPPORTED, "the server needs a network model");
  if (m->server) return fail(FMD_E_STATE, "the model already has a server");
  if (cfg->max_requests < 0 || cfg->max_tokens_per_iter < 0)
    return fail(FMD_E_INVALID, "negative limits");
  const size_t bpt = bytes_per_token(m->cfg);
  const int64_t pool = ((int64_t)(cfg->hbm_budget_bytes / bpt) - kPoolSlack) / kTile * kTile;
  if (pool < kTile)
    return fail(FMD_E_BUDGET, "HBM budget below one 64-row tile (%zu bytes per row)", bpt);
  DeviceGuard guard(m->device);
  fmd_server* S = new fmd_server();
  S->m = m;
  S->cfg = *cfg;
  S->pool_tokens = pool;
  S->bytes_per_token = bpt;
  S->pool.init(pool);
  int st = ensure_ws(m, pool + kPoolSlack, 1, 1);
  if (st == FMD_OK && hipStreamCreateWithFlags(&S->st, hipStreamNonBlocking) != hipSuccess)
    st = fail(FMD_E_DEVICE, "stream creation failed");
  for (int i = 0; i < 2 && st == FMD_OK; ++i)
    if (hipEventCreate(&S->ev_start[i]) != hipSuccess || hipEventCreate(&S->ev_done[i]) != hipSuccess)
      st = fail(FMD_E_DEVICE, "event creation failed");
  if (st == FMD_OK) st = grow_host(S->out_pin, (size_t)(pool + kPoolSlack) * 9 * 4);
  if (st == FMD_OK) st = grow(S->d_tiles, (size_t)(pool / kTile + 1) * 4);
  if (st != FMD_OK) {
    release_resources(S);
    delete S;
    return st;
  }
  m->server = S;
  S->worker = std::thread(worker_main, S);
  *out = S;
  return FMD_OK;
}

namespace {
int submit(fmd_server* S, const fmd_events_in* truth, const int64_t* reco_offsets, uint64_t seed,
           const fmd_schedule* sched, uint64_t* req_id) {
  if (!S || !req_id) return fail(FMD_E_INVALID, "null argument");
  int64_t T = 0, Tr = 0;
  FMD_TRY(check_events(S->m, truth, &T, nullptr));
  Tr = T;
  if (reco_offsets) FMD_TRY(check_reco_offsets(S->m, truth, reco_offsets, &Tr));
  FMD_TRY(check_schedule(sched));
  if (truth->on_device) return fail(FMD_E_INVALID, "the server takes host event arrays");
  const int64_t rows = std::max(T, Tr);
  if (rows > S->pool_tokens)
    return fail(FMD_E_BUDGET, "request of %lld rows exceeds the pool of %lld", (long long)rows,
                (long long)S->pool_tokens);
  if (S->cfg.max_tokens_per_iter > 0 && rows > S->cfg.max_tokens_per_iter)
    return fail(FMD_E_BUDGET, "request of %lld rows exceeds max_tokens_per_iter", (long long)rows);
  Req* r = new Req();
  r->off.assign(truth->offsets, truth->offsets + truth->n_events + 1);
  if (reco_offsets)
    r->roff.assign(reco_offsets, reco_offsets + truth->n_events + 1);
  else
    r->roff = r->off;
  r->feat.assign(truth->feat, truth->feat + T * 9);
  r->seed = seed;
  r->sched = *sched;
  r->T = T;
  r->Tr = Tr;
  r->rows = rows;
  r->n_events = truth->n_events;
  r->n_stages = sched->n_steps * stages_per_step(sched->scheme);
  r->out.assign((size_t)Tr * 9, 0.f);
  r->stats.t_submit_ns = now_ns();
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->dead != FMD_OK || S->stop) {
    delete r;
    return fail(FMD_E_STATE, "server is not running: %s", S->dead_msg.c_str());
  }
  r->id = S->next_id++;
  S->reqs[r->id] = r;
  if (Tr == 0) {       // nothing to integrate
    r->status = FMD_OK;
    r->stats.t_admit_ns = r->stats.t_done_ns = r->stats.t_submit_ns;
  } else {
    S->queue.push_back(r);
    S->cv_work.notify_one();
  }
  *req_id = r->id;
  return FMD_OK;
}
}  // namespace

int fmd_server_submit(fmd_server* S, const fmd_events_in* truth, uint64_t seed,
                      const fmd_schedule* sched, uint64_t* req_id) {
  return submit(S, truth, nullptr, seed, sched, req_id);
}

int fmd_server_submit_reco(fmd_server* S, const fmd_events_in* truth,
                           const int64_t* reco_offsets, uint64_t seed,
                           const fmd_schedule* sched, uint64_t* req_id) {
  if (!reco_offsets) return fail(FMD_E_INVALID, "null reco offsets");
  return submit(S, truth, reco_offsets, seed, sched, req_id);
}

int fmd_server_poll(fmd_server* S, uint64_t req_id, float* reco, fmd_request_stats* stats) {
  if (!S) return fail(FMD_E_INVALID, "null server");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return fail(FMD_E_STATE, "unknown request %llu", (unsigned long long)req_id);
  if (it->second->status == FMD_PENDING) return FMD_PENDING;
  return collect(S, it->second, reco, stats);
}

int fmd_server_wait(fmd_server* S, uint64_t req_id, float* reco, fmd_request_stats* stats) {
  if (!S) return fail(FMD_E_INVALID, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->reqs.find(req_id);
  if (it == S->reqs.end()) return fail(FMD_E_STATE, "unknown request %llu", (unsigned long long)req_id);
  Req* r = it->second;
  S->cv_done.wait(lk, [&] { return r->status != FMD_PENDING; });
  return collect(S, r, reco, stats);
}

int fmd_server_get_info(fmd_server* S, fmd_server_info* info) {
  if (!S || !info) return fail(FMD_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(S->mu);
  info->pool_tokens = S->pool_tokens;
  info->bytes_per_token = (int64_t)S->bytes_per_token;
  info->queued_requests = (int64_t)S->queue.size();
  info->resident_requests = (int64_t)S->resident.size();
  info->resident_tokens = S->resident_tokens;
  info->iterations = (int64_t)S->iterations;
  info->rows_processed = (int64_t)S->rows_processed;
  info->busy_ns = (int64_t)S->busy_ns;
  info->rows_live = (int64_t)S->rows_live;
  return FMD_OK;
}

int fmd_server_destroy(fmd_server* S) {
  if (!S) return FMD_OK;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
  }
  S->cv_work.notify_all();
  if (S->worker.joinable()) S->worker.join();
  DeviceGuard guard(S->m->device);
  if (S->st) (void)hipStreamSynchronize(S->st);
  release_resources(S);
  for (auto& kv : S->reqs) delete kv.second;
  S->m->server = nullptr;
  delete S;
  return FMD_OK;
}

}  // extern "C"
