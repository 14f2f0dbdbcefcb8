// Truth selection (model pT cut and particle limit) with no device allocation: every
// intermediate buffer lives in one fixed device array of this file, for callers that cannot
// call hipMalloc (code under stream capture, tight serving loops, harnesses that forbid it).
// The kernels are the ones fmd_truth_select runs; only the buffers and the prefix sum of the
// per-event counts (here on the device) differ.
#include <cmath>
#include <mutex>

#include "engine_impl.h"

namespace fmd {

// Scratch layout (bytes, each part 256-aligned): input offsets [E + 1] int64, output offsets
// [E + 1] int64, counts [E] int32, keep flags [T] uint8.
constexpr int64_t kNoAllocMaxEvents = 65536;
constexpr int64_t kNoAllocMaxParticles = (int64_t)1 << 23;
constexpr size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
constexpr size_t kNoAllocOffBytes = al256((size_t)(kNoAllocMaxEvents + 1) * 8);
constexpr size_t kNoAllocCntBytes = al256((size_t)kNoAllocMaxEvents * 4);
constexpr size_t kNoAllocBytes = 2 * kNoAllocOffBytes + kNoAllocCntBytes + (size_t)kNoAllocMaxParticles;

// One copy per device, held until the process ends. Host code never uses this name as an
// address: it works with the device address taken per device below.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

// Exclusive prefix sum of the per-event counts into int64 offsets (off[0] = 0, off[E] =
// total), one workgroup: thread t sums a contiguous run of counts, the run totals are scanned
// in LDS, then each thread writes its run's offsets.
__global__ __launch_bounds__(1024) void k_counts_to_offsets(const int32_t* __restrict__ cnt,
                                                            int64_t E, int64_t* __restrict__ off) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (E + 1023) / 1024;
  const int64_t a = min<int64_t>(E, t * per), b = min<int64_t>(E, a + per);
  int64_t s = 0;
  for (int64_t i = a; i < b; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan of the run totals
    const int64_t v = t >= o ? part[t - o] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;             // offset of this thread's first event
  for (int64_t i = a; i < b; ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) off[E] = part[1023];
}

std::mutex g_mu;                         // serialises calls from different host threads
constexpr int kMaxDevices = 64;
void* g_scratch[kMaxDevices] = {};       // device address of `scratch` on each device

// The device address of this device's copy of the array, looked up once per device (with
// that device current).
int scratch_ptr(unsigned char** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return eng::fail(FMD_E_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return eng::fail(FMD_E_DEVICE, "scratch array address: %s", hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = (unsigned char*)g_scratch[dev];
  return FMD_OK;
}

}  // namespace
}  // namespace fmd

using namespace fmd;
using namespace fmd::eng;

extern "C" {

int fmd_truth_select_noalloc(const fmd_events_in* truth, double pt_cut_gev, int32_t max_particles,
                             int64_t* offsets_out, float* feat_out, void* hip_stream) {
  if (!truth || !offsets_out) return fail(FMD_E_INVALID, "null argument");
  if (!(pt_cut_gev > 0.0) || max_particles < 0) return fail(FMD_E_INVALID, "bad cut or limit");
  if (!truth->on_device) return fail(FMD_E_INVALID, "the allocation-free selection takes device data only");
  fmd_events_in ev = *truth;
  int64_t T = 0;
  FMD_TRY(check_events(nullptr, &ev, &T, nullptr));
  const int64_t E = truth->n_events;
  if (E > kNoAllocMaxEvents || T > kNoAllocMaxParticles)
    return fail(FMD_E_UNSUPPORTED, "%lld events / %lld particles exceed the fixed scratch (%lld / %lld)",
                (long long)E, (long long)T, (long long)kNoAllocMaxEvents, (long long)kNoAllocMaxParticles);
  offsets_out[0] = 0;
  if (E == 0) return FMD_OK;
  if (T > 0 && !feat_out) return fail(FMD_E_INVALID, "null output");
  std::lock_guard<std::mutex> lock(g_mu);
  unsigned char* p = nullptr;
  FMD_TRY(scratch_ptr(&p));
  int64_t* d_off = (int64_t*)p;
  int64_t* d_off2 = (int64_t*)(p + kNoAllocOffBytes);
  int32_t* d_cnt = (int32_t*)(p + 2 * kNoAllocOffBytes);
  uint8_t* d_keep = (uint8_t*)(p + 2 * kNoAllocOffBytes + kNoAllocCntBytes);
  hipStream_t st = (hipStream_t)hip_stream;
  const float c0 = (float)std::log(pt_cut_gev / 10.0);
  // every scratch word read below is written first in this call: the input offsets by the
  // copy, every count and keep flag by k_select_count, every output offset by the scan
  hipError_t e = hipMemcpyAsync(d_off, truth->offsets, (size_t)(E + 1) * 8, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_select_count(st, truth->feat, 9, d_off, E, c0, max_particles, d_keep, d_cnt);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_counts_to_offsets, dim3(1), dim3(1024), 0, st, d_cnt, E, d_off2);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_select_write(st, truth->feat, 9, d_off, d_off2, E, d_keep, feat_out);
  if (e == hipSuccess)
    e = hipMemcpyAsync(offsets_out, d_off2, (size_t)(E + 1) * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return fail(FMD_E_DEVICE, "truth selection (no allocation): %s", hipGetErrorString(e));
  return FMD_OK;
}

}  // extern "C"
