// Host-side engine state behind the fmd C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <string>
#include <vector>

#include "../../include/fmd.h"
#include "common.h"
#include "kernels.h"

namespace fmd {

// Per-block device pointers. Matrices are packed transposed ([N][K]) in the compute type.
struct DevBlock {
  const float *g1, *s1, *g2, *s2, *g3, *s3;
  const float *bqkv, *bo, *bqc, *boc, *bup, *bdn;
  void *Wqkv, *Wo, *Wqc, *Woc, *Wup, *Wdn;
  void *Fqkv, *Fo, *Fqc, *Foc, *Fup, *Fdn;   // BF16 MFMA fragment layout (fused kernels)
};

// Device buffers of one call, grown on demand and reused across calls.
struct Workspace {
  int64_t cap_tok = 0, cap_ev = 0, cap_items = 0;
  size_t elem = 0;                 // bytes per compute-type element
  float *x = nullptr, *acc = nullptr, *xs = nullptr;    // [Tp, 16] FP32 ODE state
  float* H = nullptr;              // [Tp, d] FP32 residual stream
  void* qkv = nullptr;             // [Tp, 3d] T
  void* att = nullptr;             // [Tp, d] T   attention output
  void* qc = nullptr;              // [Tp, d] T   cross-attention queries
  void* hid = nullptr;             // [Tp, 4d] T  MLP hidden
  void* c = nullptr;               // [Tp, d] T   truth encoding
  void* kv = nullptr;              // [Tp, L*2d] T cross K/V cache
  float* u = nullptr;              // [Tp, 9] truth features (host inputs are staged here)
  float* io = nullptr;             // [Tp, 9] staging of host state / outputs
  float* temb = nullptr;           // [max(E,1), d] time embedding
  float* tev = nullptr;            // [E] per-event time
  float2* stats = nullptr;         // [Tp] LayerNorm (mean, rstd) of the rows of H
  int32_t* tok_event = nullptr;    // [Tp]
  int64_t* off = nullptr;          // [E + 1]
  AttnItem* work = nullptr;        // attention work list
  StageDesc* desc = nullptr;       // [stages] stage table of the call
  int32_t* ctr = nullptr;          // current stage index (device)
  // Pinned staging of the host-built arrays a call uploads (offsets, attention work lists,
  // stage table), two sets used by alternate calls. A set's event is recorded after the
  // copies that read it; a call waits on it before rewriting the set, so it only waits for
  // the uploads of the call two calls back, never for the device work of the last one.
  struct HostStage {
    int64_t* off = nullptr;
    AttnItem* work = nullptr;
    StageDesc* desc = nullptr;
    int64_t cap_ev = 0, cap_items = 0, cap_desc = 0;
    hipEvent_t ev = nullptr;
    bool live = false;             // ev recorded and not yet waited for
  } hs[2];
  int cur = 0;                     // set of the current call
  int cap_desc = 0;
  uint64_t generation = 0;         // bumped whenever a buffer is reallocated
};

// What a captured stage graph depends on besides buffer contents.
struct GraphKey {
  int64_t Tp, T, E, items;
  const float* out;
  int ldo;
  uint64_t ws_gen, tune_gen;
  AttnBins bins;  // kernel arguments and grid size of the attention launches
  int64_t items_x, work_x;   // cross-attention list: size and offset in the work buffer
  AttnBins bins_x;
  int64_t Tt;                // truth rows (the reco side may differ in size)
  bool operator==(const GraphKey& o) const {
    return Tp == o.Tp && T == o.T && E == o.E && items == o.items && out == o.out &&
           ldo == o.ldo && ws_gen == o.ws_gen && tune_gen == o.tune_gen &&
           std::memcmp(&bins, &o.bins, sizeof(AttnBins)) == 0 && items_x == o.items_x &&
           work_x == o.work_x && std::memcmp(&bins_x, &o.bins_x, sizeof(AttnBins)) == 0 &&
           Tt == o.Tt;
  }
};

// Sites the autotuner chooses a variant for: the GEMM sites (a tiling of the matrix-core
// GEMM kernel), then on the fused BF16 path the attention query tile (work items of 64 or
// 128 queries) and the row tile of the fused QKV and OQC kernels (64 or 128 rows).
enum TuneSlot { TS_QKV = 0, TS_PROJ_RES = 1, TS_PROJ_LN = 2, TS_UP = 3, TS_DOWN = 4, TS_GEMM = 5,
                TS_ATTN = 5, TS_FQKV = 6, TS_FOQC = 7, TS_COUNT = 8 };
constexpr int kTuneBuckets = 40;   // floor(log2(padded token count))

struct TimingRec {
  int cls;
  double work, bytes;
  hipEvent_t a, b;
};

}  // namespace fmd

struct fmd_model {
  int kind = 0;                    // 0 network, 1 linear test field
  double alpha = 0, beta = 0;
  fmd_model_config cfg{};
  int device = 0;
  float* params = nullptr;         // flat FP32 copy on device
  void* packed = nullptr;          // packed matrices in the compute type
  void* frag = nullptr;            // fragment-layout BF16 matrices of the fused kernels
  void* frag8 = nullptr;           // FP8 form: e4m3 fragments of W_up, W_dn and column scales
  std::vector<fmd::Fp8Mlp> f8;     // FP8 form: per block pointers into frag8
  bool fused_ok = false;           // the fused block kernels exist for this configuration
  bool kv_hm = false;              // cross K/V cache head-major [L][2][heads][cap][dh]
  int fused = 0;                   // segments that use them (FMD_FUSED_* bits)
  float* bkv = nullptr;            // [L * 2d] cross K/V biases
  float* Wout_pk = nullptr;        // [64][d] output head, transposed, rows >= f_reco zero (FP32)
  float* bout_pk = nullptr;        // [64] output bias, zero-padded
  void* Wkv = nullptr;             // [L * 2d][d] cross K/V weights (packed)
  std::vector<fmd::DevBlock> blk;
  const float *W_tin, *b_tin, *g_t, *s_t, *W_xin, *b_xin, *W_time, *b_time, *g_f, *s_f, *W_out,
      *b_out;
  fmd::Workspace ws;
  bool fuse_stats = false;         // residual GEMMs emit the next LayerNorm's row statistics
  int autotune = 1;                // 1: time the candidate tilings on first use of a size bucket
  uint64_t tune_gen = 0;
  int graphs = 1;                  // 1: capture one ODE stage as a HIP graph and replay it
  hipStream_t pstream = nullptr;   // private stream of the model (captured, non-blocking)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraphExec_t gexec = nullptr;
  fmd::GraphKey gkey{};
  fmd_server* server = nullptr;    // attached server (the model's own calls are refused)
  int8_t tune[fmd::TS_COUNT][fmd::kTuneBuckets];   // chosen tiling, -1 = not tuned yet
  float tune_us[fmd::TS_COUNT][fmd::kTuneBuckets]; // its measured time
  float tune_all[fmd::TS_COUNT][fmd::kTuneBuckets][8];   // every candidate's time (0: not run)
  bool timing = false;
  std::vector<fmd::TimingRec> trec;
  std::vector<hipEvent_t> ev_pool;
  double t_ms[FMD_K_COUNT] = {0};
  int64_t t_n[FMD_K_COUNT] = {0};
  double t_work[FMD_K_COUNT] = {0};
  double t_bytes[FMD_K_COUNT] = {0};
};
