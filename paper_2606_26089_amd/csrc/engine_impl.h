// Internal interfaces of the fmdet engine shared by the sampling calls and the server.
#pragma once

#include <string>

#include "engine.h"
#include "kernels.h"

namespace fmd {
namespace eng {

int fail(int status, const char* fmt, ...);

#define HIP_TRY(expr)                                                                      \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::fmd::eng::fail(FMD_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                              __FILE__, __LINE__);                                         \
  } while (0)

#define FMD_TRY(expr)              \
  do {                             \
    int s_ = (expr);               \
    if (s_ != FMD_OK) return s_;   \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};


inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }


template <typename P>
int grow(P*& p, size_t bytes) {
  if (p) (void)hipFree(p);
  p = nullptr;
  if (bytes == 0) return FMD_OK;
  if (hipMalloc((void**)&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    return fail(FMD_E_NOMEM, "device allocation of %zu bytes failed", bytes);
  }
  // The zero fill runs on the null stream, which the library's non-blocking streams do not
  // wait for: finish it here, or an upload enqueued on such a stream right after the growth
  // can land first and be wiped.
  if (hipMemset(p, 0, bytes) != hipSuccess) return fail(FMD_E_DEVICE, "hipMemset failed");
  if (hipDeviceSynchronize() != hipSuccess) return fail(FMD_E_DEVICE, "hipDeviceSynchronize failed");
  return FMD_OK;
}

template <typename P>
int grow_host(P*& p, size_t bytes) {
  if (p) (void)hipHostFree(p);
  p = nullptr;
  if (hipHostMalloc((void**)&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
    return fail(FMD_E_NOMEM, "pinned host allocation of %zu bytes failed", bytes);
  }
  return FMD_OK;
}


hipEvent_t take_event(fmd_model* m);
void flush_timing(fmd_model* m);

template <typename F>
int timed(fmd_model* m, hipStream_t st, int cls, double work, double bytes, F&& launch) {
  hipEvent_t a = nullptr, b = nullptr;
  if (m->timing) {
    if (m->trec.size() > 4096) flush_timing(m);
    a = take_event(m);
    b = take_event(m);
    if (a && b) (void)hipEventRecord(a, st);
  }
  const hipError_t e = launch();
  if (e != hipSuccess) return fail(FMD_E_DEVICE, "kernel launch (class %d): %s", cls, hipGetErrorString(e));
  if (m->timing && a && b) {
    (void)hipEventRecord(b, st);
    m->trec.push_back(TimingRec{cls, work, bytes, a, b});
  }
  return FMD_OK;
}

template <typename F>
int timed(fmd_model* m, hipStream_t st, int cls, double work, F&& launch) {
  return timed(m, st, cls, work, 0.0, launch);
}


// One call's (or one server iteration's) shapes and inputs on the device.
struct Call {
  hipStream_t st;
  int64_t E, T, Tp, items;   // T reco slots (rows of the state and residual stream)
  int qt;               // queries per attention work item (the lists are built with it)
  AttnBins bins;        // bins of the attention work list
  double sum_n2;        // sum over events of N_e^2 (attention work)
  // Truth side: Tt truth particles (rows of the truth encoding and cross K/V cache) and the
  // cross-attention work list (items_x entries from w.work + work_x, bins_x). Equal to the
  // reco side unless the caller gave reco multiplicities (same_truth sets them so).
  int64_t Tt, Ttp, items_x, work_x;
  AttnBins bins_x;
  double sum_nx;        // sum over events of N_reco N_truth
  const float* u;       // truth features on device [Tt, 9]
  OdeArgs sargs;        // epilogue arguments of the residual GEMMs (statistics output)
  // Output head to fold into the last block's fused MLP kernel (9 features, BF16 fused
  // path); net_forward sets head_done when it did, and the caller then skips its head.
  const OdeArgs* head = nullptr;
  bool head_done = false;
  // 64-row tiles the fused kernels run (device int32, n_tiles of them; null: all of Tp). The
  // serving loop skips the tiles of gaps between resident requests this way.
  const int32_t* tiles = nullptr;
  int64_t n_tiles = 0;
};


// The truth side of a call whose reco slots are its truth particles.
inline void same_truth(Call& c) {
  c.Tt = c.T;
  c.Ttp = c.Tp;
  c.items_x = c.items;
  c.work_x = 0;
  c.bins_x = c.bins;
  c.sum_nx = c.sum_n2;
}

int ensure_ws(fmd_model* m, int64_t T, int64_t E, int64_t items);
int check_events(const fmd_model* m, const fmd_events_in* ev, int64_t* T_out, int64_t* max_n);
int check_reco_offsets(const fmd_model* m, const fmd_events_in* truth, const int64_t* roff,
                       int64_t* T_out);
int check_schedule(const fmd_schedule* s);
int stages_per_step(int scheme);
StageDesc stage_desc(const fmd_schedule& s, int i);
int row_stats(fmd_model* m, Call& c);
int attn_tile_for(const fmd_model* m, int64_t Tp);   // attention query tile for a padded size
int enter_stream(fmd_model* m, hipStream_t caller, Call& c);
int leave_stream(fmd_model* m, hipStream_t caller);
template <typename T> int truth_cache(fmd_model* m, Call& c);
template <typename T> int autotune(fmd_model* m, Call& c);
template <typename T> int net_forward(fmd_model* m, Call& c, const float* t_ev);

}  // namespace eng
}  // namespace fmd
