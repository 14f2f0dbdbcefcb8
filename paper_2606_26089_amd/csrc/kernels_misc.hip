// Bandwidth-bound kernels of the sampling path: CSR token map, Philox noise, truth
// encoder, time and input embeddings, the fused output head + ODE update, ragged
// packing and parameter packing.
#include "common.h"
#include "kernels.h"

namespace fmd {

// ---------------------------------------------------------------------------------------
// Token -> event map of a CSR batch: the largest e with off[e] <= r (empty events skipped).
__global__ void k_token_map(const int64_t* __restrict__ off, int64_t E, int64_t T,
                            int32_t* __restrict__ tok_event) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T) return;
  int64_t lo = 0, hi = E;  // off[lo] <= r < off[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (off[mid] <= r) lo = mid; else hi = mid;
  }
  tok_event[r] = (int32_t)lo;
}

hipError_t launch_token_map(hipStream_t st, const int64_t* off, int64_t E, int64_t T,
                            int32_t* tok_event) {
  if (T <= 0) return hipSuccess;
  const int64_t blocks = (T + 255) / 256;
  hipLaunchKernelGGL(k_token_map, dim3((unsigned)blocks), dim3(256), 0, st, off, E, T, tok_event);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): two 64x64->128 multiplies per round,
// Weyl-sequence key schedule, ten rounds.
struct Philox4x64 {
  uint64_t c[4];
};

__device__ __forceinline__ Philox4x64 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2,
                                                   uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  Philox4x64 o;
  o.c[0] = c0; o.c[1] = c1; o.c[2] = c2; o.c[3] = c3;
  return o;
}

// u = ((w >> 41) + 1/2) 2^-23: exact in FP32, strictly inside (0, 1).
__device__ __forceinline__ float u23(uint64_t w) {
  return ((float)(uint32_t)(w >> 41) + 0.5f) * 1.1920928955078125e-07f;
}

__global__ void k_noise(uint64_t seed, const int64_t* __restrict__ off,
                        const int32_t* __restrict__ tok_event, int64_t T, int n_feat,
                        float* __restrict__ x, float* __restrict__ xs, int ldx) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= T) return;
  const int32_t e = tok_event[r];
  const uint64_t slot = (uint64_t)(r - off[e]);
  float z[12];
  const int nb = (n_feat + 3) >> 2;
  for (int b = 0; b < 3; ++b) {
    if (b >= nb) break;
    const Philox4x64 w = philox4x64_10((uint64_t)b, slot, (uint64_t)e, 0ull, seed, 0ull);
#pragma unroll
    for (int p = 0; p < 2; ++p) {
      const float ua = u23(w.c[2 * p]), ub = u23(w.c[2 * p + 1]);
      const float rad = sqrtf(-2.0f * logf(ua));
      float sn, cs;
      sincospif(2.0f * ub, &sn, &cs);
      z[4 * b + 2 * p] = rad * cs;
      z[4 * b + 2 * p + 1] = rad * sn;
    }
  }
  float* xr = x + r * ldx;
  for (int f = 0; f < ldx; ++f) xr[f] = f < n_feat ? z[f] : 0.0f;
  if (xs) {
    float* sr = xs + r * ldx;
    for (int f = 0; f < ldx; ++f) sr[f] = f < n_feat ? z[f] : 0.0f;
  }
}

hipError_t launch_noise(hipStream_t st, uint64_t seed, const int64_t* off,
                        const int32_t* tok_event, int64_t T, int n_feat, float* x, float* xs,
                        int ldx) {
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_noise, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st, seed, off,
                     tok_event, T, n_feat, x, xs, ldx);
  return hipGetLastError();
}

__global__ void k_philox(uint64_t k0, uint64_t k1, const uint64_t* __restrict__ ctr, int64_t n,
                         uint64_t* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t* c = ctr + 4 * i;
  const Philox4x64 w = philox4x64_10(c[0], c[1], c[2], c[3], k0, k1);
  for (int k = 0; k < 4; ++k) out[4 * i + k] = w.c[k];
}

hipError_t launch_philox(hipStream_t st, uint64_t k0, uint64_t k1, const uint64_t* ctr,
                         int64_t n, uint64_t* out) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k0, k1, ctr, n,
                     out);
  return hipGetLastError();
}

__global__ void k_load_state(const float* __restrict__ src, int f, int64_t T,
                             float* __restrict__ x, float* __restrict__ xs, int ldx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * ldx) return;
  const int64_t r = i / ldx;
  const int c = (int)(i % ldx);
  const float v = c < f ? src[r * f + c] : 0.0f;
  x[i] = v;
  if (xs) xs[i] = v;
}

hipError_t launch_load_state(hipStream_t st, const float* src, int f, int64_t T, float* x,
                             float* xs, int ldx) {
  if (T <= 0) return hipSuccess;
  const int64_t n = T * ldx;
  hipLaunchKernelGGL(k_load_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, f,
                     T, x, xs, ldx);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Truth encoder c = LN_t(u W_tin + b_tin): one wave per particle; lane owns columns
// lane + 64 j. Statistics are two-pass in registers.
constexpr int kMaxDPerLane = 16;   // d_model <= 1024

template <typename T>
__global__ __launch_bounds__(256) void k_truth_encode(
    const float* __restrict__ u, int ldu, int f, int64_t T_, const float* __restrict__ W,
    const float* __restrict__ b, const float* __restrict__ g, const float* __restrict__ s,
    int d, T* __restrict__ c, int ldc) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= T_) return;
  float uf[16];
  for (int k = 0; k < f; ++k) uf[k] = u[r * ldu + k];
  const int nj = d >> 6;
  float y[kMaxDPerLane];
  float sum = 0.f;
#pragma unroll
  for (int jj = 0; jj < kMaxDPerLane; ++jj) {
    if (jj < nj) {
      const int j = lane + 64 * jj;
      float a = b[j];
      for (int k = 0; k < f; ++k) a = fmaf(uf[k], W[k * d + j], a);
      y[jj] = a;
      sum += a;
    }
  }
  const float mean = wave_sum(sum) / d;
  float q = 0.f;
#pragma unroll
  for (int jj = 0; jj < kMaxDPerLane; ++jj)
    if (jj < nj) { const float dv = y[jj] - mean; q = fmaf(dv, dv, q); }
  const float rstd = rsqrtf(wave_sum(q) / d + kLnEps);
#pragma unroll
  for (int jj = 0; jj < kMaxDPerLane; ++jj)
    if (jj < nj) {
      const int j = lane + 64 * jj;
      c[r * ldc + j] = from_f32<T>((y[jj] - mean) * rstd * g[j] + s[j]);
    }
}

template <typename T>
hipError_t launch_truth_encode(hipStream_t st, const float* u, int ldu, int f, int64_t T_,
                               const float* W, const float* b, const float* g,
                               const float* s, int d, T* c, int ldc) {
  if (T_ <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_truth_encode<T>, dim3((unsigned)((T_ + 3) / 4)), dim3(256), 0, st, u,
                     ldu, f, T_, W, b, g, s, d, c, ldc);
  return hipGetLastError();
}
template hipError_t launch_truth_encode<float>(hipStream_t, const float*, int, int, int64_t,
                                               const float*, const float*, const float*,
                                               const float*, int, float*, int);
template hipError_t launch_truth_encode<bf16>(hipStream_t, const float*, int, int, int64_t,
                                              const float*, const float*, const float*,
                                              const float*, int, bf16*, int);

// ---------------------------------------------------------------------------------------
// Time embedding: temb[e, j] = b_xin[j] + b_time[j] + sum_k phi_k(t_e) W_time[k, j] with
// phi = [sin(w_k t) | cos(w_k t)], w_k = 10000^(-k/(E/2)). One block per event.
__global__ __launch_bounds__(256) void k_time_embed(const float* __restrict__ t_ev,
                                                    const StageDesc* __restrict__ desc,
                                                    const int32_t* __restrict__ ctr,
                                                    float t_uniform, const float* __restrict__ W,
                                                    const float* __restrict__ b_time,
                                                    const float* __restrict__ b_xin, int E_dim,
                                                    int d, float* __restrict__ temb) {
  __shared__ float phi[64];
  const int e = blockIdx.x;
  const float t = t_ev ? t_ev[e] : desc ? desc[*ctr].t : t_uniform;
  const int half = E_dim >> 1;
  if (threadIdx.x < half) {
    // ln(10000) / half scales the exponent
    const float w = expf(-(float)threadIdx.x * (9.210340371976184f / (float)half));
    float sn, cs;
    sincosf(w * t, &sn, &cs);
    phi[threadIdx.x] = sn;
    phi[threadIdx.x + half] = cs;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < d; j += blockDim.x) {
    float a = 0.f;
    for (int k = 0; k < E_dim; ++k) a = fmaf(phi[k], W[k * d + j], a);
    temb[(int64_t)e * d + j] = (a + b_time[j]) + b_xin[j];
  }
}

hipError_t launch_time_embed(hipStream_t st, const float* t_ev, const StageDesc* desc,
                             const int32_t* ctr, float t_uniform, int n, const float* W_time,
                             const float* b_time, const float* b_xin, int E_dim, int d,
                             float* temb) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_time_embed, dim3(n), dim3(256), 0, st, t_ev, desc, ctr, t_uniform, W_time,
                     b_time, b_xin, E_dim, d, temb);
  return hipGetLastError();
}

__global__ void k_set_counter(int32_t* ctr, int32_t v) { *ctr = v; }
__global__ void k_stage_advance(int32_t* ctr) { *ctr += 1; }

hipError_t launch_set_counter(hipStream_t st, int32_t* ctr, int32_t v) {
  hipLaunchKernelGGL(k_set_counter, dim3(1), dim3(1), 0, st, ctr, v);
  return hipGetLastError();
}

hipError_t launch_stage_advance(hipStream_t st, int32_t* ctr) {
  hipLaunchKernelGGL(k_stage_advance, dim3(1), dim3(1), 0, st, ctr);
  return hipGetLastError();
}

// Input embedding H = xs W_xin + temb, one wave per token (lane owns columns lane + 64 j),
// with the row's LayerNorm statistics for the first block.
__global__ __launch_bounds__(256) void k_embed(const float* __restrict__ xs, int ldx, int f,
                                               int64_t T, const int32_t* __restrict__ tok_event,
                                               const float* __restrict__ temb,
                                               const float* __restrict__ W, int d,
                                               float* __restrict__ H, int ldh,
                                               float2* __restrict__ stats) {
  const int lane = threadIdx.x & 63;
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= T) return;
  const float* te = temb + (tok_event ? (int64_t)tok_event[r] * d : 0);
  float xv[16];
  for (int k = 0; k < f; ++k) xv[k] = xs[r * ldx + k];
  const int nj = d >> 6;
  float y[kMaxDPerLane];
  float sum = 0.f;
#pragma unroll
  for (int jj = 0; jj < kMaxDPerLane; ++jj)
    if (jj < nj) {
      const int j = lane + 64 * jj;
      float a = te[j];
      for (int k = 0; k < f; ++k) a = fmaf(xv[k], W[k * d + j], a);
      y[jj] = a;
      sum += a;
      H[r * ldh + j] = a;
    }
  const float mean = wave_sum(sum) / d;
  float q = 0.f;
#pragma unroll
  for (int jj = 0; jj < kMaxDPerLane; ++jj)
    if (jj < nj) { const float dv = y[jj] - mean; q = fmaf(dv, dv, q); }
  const float var = wave_sum(q) / d;
  if (lane == 0) stats[r] = make_float2(mean, rsqrtf(var + kLnEps));
}

// The same for d = 256 and 9 input features, built for memory-level parallelism: a wave
// embeds kEmbTok consecutive tokens, lane l owning columns 4l .. 4l + 3 (16-byte loads and
// stores), with W_xin kept in registers across the tokens and the token inputs read by
// scalar loads. Each output is formed in the same order as above (temb first, then the
// features in order), so H is identical; the statistics reductions of all tokens of the
// wave run side by side.
constexpr int kEmbTok = 8;
constexpr int kEmbF = 9;
__global__ __launch_bounds__(256) void k_embed256(const float* __restrict__ xs, int ldx,
                                                  int64_t T, const int32_t* __restrict__ tok_event,
                                                  const float* __restrict__ temb,
                                                  const float* __restrict__ W,
                                                  float* __restrict__ H, int ldh,
                                                  float2* __restrict__ stats) {
  constexpr int D = 256;
  const int lane = threadIdx.x & 63;
  const int64_t r0 =
      ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * kEmbTok;
  if (r0 >= T) return;
  float4 w[kEmbF];
#pragma unroll
  for (int k = 0; k < kEmbF; ++k) w[k] = *(const float4*)(W + k * D + 4 * lane);
  float4 a[kEmbTok];
  float part[kEmbTok];
#pragma unroll
  for (int t = 0; t < kEmbTok; ++t) {
    const int64_t r = r0 + t;
    a[t] = make_float4(0.f, 0.f, 0.f, 0.f);
    part[t] = 0.f;
    if (r < T) {
      const float* te = temb + (tok_event ? (int64_t)tok_event[r] * D : 0);
      float4 v = *(const float4*)(te + 4 * lane);
#pragma unroll
      for (int k = 0; k < kEmbF; ++k) {
        const float x = xs[r * ldx + k];
        v.x = fmaf(x, w[k].x, v.x);
        v.y = fmaf(x, w[k].y, v.y);
        v.z = fmaf(x, w[k].z, v.z);
        v.w = fmaf(x, w[k].w, v.w);
      }
      *(float4*)(H + r * ldh + 4 * lane) = v;
      a[t] = v;
      part[t] = (v.x + v.y) + (v.z + v.w);
    }
  }
  float mean[kEmbTok];
#pragma unroll
  for (int t = 0; t < kEmbTok; ++t) mean[t] = wave_sum(part[t]) * (1.0f / D);
#pragma unroll
  for (int t = 0; t < kEmbTok; ++t) {
    const float dx = a[t].x - mean[t], dy = a[t].y - mean[t], dz = a[t].z - mean[t],
                dw = a[t].w - mean[t];
    part[t] = fmaf(dw, dw, fmaf(dz, dz, fmaf(dy, dy, dx * dx)));
  }
#pragma unroll
  for (int t = 0; t < kEmbTok; ++t) {
    const float var = wave_sum(part[t]) * (1.0f / D);
    if (lane == 0 && r0 + t < T) stats[r0 + t] = make_float2(mean[t], rsqrtf(var + kLnEps));
  }
}

hipError_t launch_embed(hipStream_t st, const float* xs, int ldx, int f, int64_t T,
                        const int32_t* tok_event, const float* temb, const float* W_xin,
                        int d, float* H, int ldh, float2* stats) {
  if (T <= 0) return hipSuccess;
  if (d == 256 && f == kEmbF && ldh % 4 == 0) {
    const int64_t waves = (T + kEmbTok - 1) / kEmbTok;
    hipLaunchKernelGGL(k_embed256, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, xs, ldx,
                       T, tok_event, temb, W_xin, H, ldh, stats);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_embed, dim3((unsigned)((T + 3) / 4)), dim3(256), 0, st, xs, ldx, f, T,
                     tok_event, temb, W_xin, d, H, ldh, stats);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
__global__ void k_linear_update(float alpha, float beta, const StageDesc* __restrict__ desc,
                                const int32_t* __restrict__ ctr, int64_t T, int f,
                                float* __restrict__ x, float* __restrict__ acc,
                                float* __restrict__ xs, int ldx, float* __restrict__ out,
                                int ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T * f) return;
  const StageDesc sd = desc[*ctr];
  const int64_t r = i / f;
  const int k = (int)(i % f);
  const int64_t o = r * ldx + k;
  const float v = (alpha + beta * sd.t) * xs[o];
  ode_update(sd.mode, sd.h, v, x + o, acc + o, xs + o,
             out && sd.write_out ? out + r * ldo + k : nullptr);
}

hipError_t launch_linear_update(hipStream_t st, float alpha, float beta, const StageDesc* desc,
                                const int32_t* ctr, int64_t T, int f, float* x, float* acc,
                                float* xs, int ldx, float* out, int ldo) {
  if (T <= 0) return hipSuccess;
  const int64_t n = T * f;
  hipLaunchKernelGGL(k_linear_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, alpha,
                     beta, desc, ctr, T, f, x, acc, xs, ldx, out, ldo);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Parameter packing and conversions.
template <typename T>
__global__ void k_pack_weight(const float* __restrict__ W, int K, int N, T* __restrict__ Wt) {
  __shared__ float tile[32][33];
  const int k0 = blockIdx.y * 32, n0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 256 threads: 32 x 8
  for (int i = ty; i < 32; i += 8) {
    const int k = k0 + i, n = n0 + tx;
    tile[i][tx] = (k < K && n < N) ? W[(int64_t)k * N + n] : 0.f;
  }
  __syncthreads();
  for (int i = ty; i < 32; i += 8) {
    const int n = n0 + i, k = k0 + tx;
    if (n < N && k < K) Wt[(int64_t)n * K + k] = from_f32<T>(tile[tx][i]);
  }
}

template <typename T>
hipError_t launch_pack_weight(hipStream_t st, const float* W, int K, int N, T* Wt) {
  dim3 grid((N + 31) / 32, (K + 31) / 32);
  hipLaunchKernelGGL(k_pack_weight<T>, grid, dim3(256), 0, st, W, K, N, Wt);
  return hipGetLastError();
}
template hipError_t launch_pack_weight<float>(hipStream_t, const float*, int, int, float*);
template hipError_t launch_pack_weight<bf16>(hipStream_t, const float*, int, int, bf16*);

template <typename T>
__global__ void k_convert(const float* __restrict__ src, int64_t n, T* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = from_f32<T>(src[i]);
}
template <typename T>
__global__ void k_to_f32(const T* __restrict__ src, int64_t n, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = to_f32(src[i]);
}

template <typename T>
hipError_t launch_convert(hipStream_t st, const float* src, int64_t n, T* dst) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_convert<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, n,
                     dst);
  return hipGetLastError();
}
template <typename T>
hipError_t launch_to_f32(hipStream_t st, const T* src, int64_t n, float* dst) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_f32<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, n,
                     dst);
  return hipGetLastError();
}
template hipError_t launch_convert<float>(hipStream_t, const float*, int64_t, float*);
template hipError_t launch_convert<bf16>(hipStream_t, const float*, int64_t, bf16*);
template hipError_t launch_to_f32<float>(hipStream_t, const float*, int64_t, float*);
template hipError_t launch_to_f32<bf16>(hipStream_t, const bf16*, int64_t, float*);

// ---------------------------------------------------------------------------------------
// Ragged packing: padded [E, n_max, f] + lengths -> CSR offsets + rows. Lengths are
// clamped to [0, n_max], so the output never exceeds E * n_max rows.
// One block computes the exclusive prefix sum (chunks of 1024 with a running carry).
__device__ __forceinline__ int64_t clamp_len(int32_t v, int n_max) {
  return v < 0 ? 0 : (v > n_max ? n_max : v);
}

__global__ __launch_bounds__(1024) void k_scan_lengths(const int32_t* __restrict__ len,
                                                       int64_t E, int n_max,
                                                       int64_t* __restrict__ off) {
  __shared__ int64_t buf[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < E; base += 1024) {
    const int64_t i = base + threadIdx.x;
    buf[threadIdx.x] = i < E ? clamp_len(len[i], n_max) : 0;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {          // Hillis-Steele inclusive scan
      const int64_t v = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
      __syncthreads();
      buf[threadIdx.x] += v;
      __syncthreads();
    }
    if (i < E) off[i + 1] = carry + buf[threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 1023) carry += buf[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) off[0] = 0;
}

__global__ void k_scatter_rows(const float* __restrict__ padded, const int32_t* __restrict__ len,
                               const int64_t* __restrict__ off, int64_t E, int n_max, int f,
                               float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // (e, slot, feature)
  const int64_t per_event = (int64_t)n_max * f;
  if (i >= E * per_event) return;
  const int64_t e = i / per_event;
  const int64_t rem = i % per_event;
  const int slot = (int)(rem / f), k = (int)(rem % f);
  if (slot < clamp_len(len[e], n_max)) out[(off[e] + slot) * f + k] = padded[i];
}

hipError_t launch_pack_padded(hipStream_t st, const float* padded, const int32_t* lengths,
                              int64_t E, int n_max, int f, int64_t* off_out, float* feat_out) {
  hipLaunchKernelGGL(k_scan_lengths, dim3(1), dim3(1024), 0, st, lengths, E, n_max, off_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || E == 0) return e;
  const int64_t n = E * n_max * f;
  hipLaunchKernelGGL(k_scatter_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, padded,
                     lengths, off_out, E, n_max, f, feat_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Output head for d = 256 and 9 features: v = LN_f(H) W_out + b_out followed by the ODE
// update of the state (the same update as the GEMM head's epilogue). The product has only
// nine columns, so it runs on the vector ALUs in FP32 instead of a matrix tile padded to 64
// columns: half a wave per token (lane i of the half owns columns 4i .. 4i+3 and 128 + 4i ..
// 131 + 4i, coalesced 16-byte loads), W_out, gain and shift in registers, the nine dot
// products reduced over the half wave by DPP rotations inside 16-lane rows and one
// permlane16 swap between the two rows. Lanes 0..8 of a half then update feature i.
namespace {
constexpr int kHeadIter = 4;     // token pairs per wave
constexpr int kHeadF = 9;

template <int CTRL>
__device__ __forceinline__ float dpp_add(float v) {
  return v + __builtin_amdgcn_update_dpp(0.f, v, CTRL, 0xF, 0xF, false);
}

// Sum over the 32 lanes of each half wave, left in every lane of the half; the same
// addition tree for both halves and for every lane.
__device__ __forceinline__ float half_wave_sum(float v) {
  v = dpp_add<0x128>(v);   // row_ror 8
  v = dpp_add<0x124>(v);   // row_ror 4
  v = dpp_add<0x122>(v);   // row_ror 2
  v = dpp_add<0x121>(v);   // row_ror 1
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false,
                                                  false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
}  // namespace

__global__ __launch_bounds__(256) void k_head256(const float* __restrict__ H,
                                                 const float2* __restrict__ stats,
                                                 const float* __restrict__ g,
                                                 const float* __restrict__ s,
                                                 const float* __restrict__ Wt,
                                                 const float* __restrict__ b, OdeArgs ode) {
  constexpr int D = 256;
  const int lane = threadIdx.x & 63, half = lane >> 5, i = lane & 31;
  const int64_t p0 =
      ((int64_t)blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6)) * kHeadIter;
  const int64_t T = ode.m_valid;
  if (2 * p0 >= T) return;
  float4 hv[kHeadIter][2];
  float2 st[kHeadIter];
#pragma unroll
  for (int it = 0; it < kHeadIter; ++it) {
    const int64_t r = min(2 * (p0 + it) + half, T - 1);
#pragma unroll
    for (int j = 0; j < 2; ++j) hv[it][j] = *(const float4*)(H + r * D + 128 * j + 4 * i);
    st[it] = stats[r];
  }
  float4 gv[2], sv[2], w[kHeadF][2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    gv[j] = *(const float4*)(g + 128 * j + 4 * i);
    sv[j] = *(const float4*)(s + 128 * j + 4 * i);
#pragma unroll
    for (int c = 0; c < kHeadF; ++c) w[c][j] = *(const float4*)(Wt + c * D + 128 * j + 4 * i);
  }
  int mode = ode.mode;
  float h = ode.h;
  float* out = ode.out;
  if (ode.desc && !ode.tok_event) {
    const StageDesc sd = ode.desc[*ode.ctr];
    mode = sd.mode;
    h = sd.h;
    if (!sd.write_out) out = nullptr;
  }
  const float bias = i < kHeadF ? b[i] : 0.f;
#pragma unroll
  for (int it = 0; it < kHeadIter; ++it) {
    const int64_t r = 2 * (p0 + it) + half;
    float part[kHeadF];
#pragma unroll
    for (int c = 0; c < kHeadF; ++c) part[c] = 0.f;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const float y[4] = {fmaf((hv[it][j].x - st[it].x) * st[it].y, gv[j].x, sv[j].x),
                          fmaf((hv[it][j].y - st[it].x) * st[it].y, gv[j].y, sv[j].y),
                          fmaf((hv[it][j].z - st[it].x) * st[it].y, gv[j].z, sv[j].z),
                          fmaf((hv[it][j].w - st[it].x) * st[it].y, gv[j].w, sv[j].w)};
#pragma unroll
      for (int c = 0; c < kHeadF; ++c) {
        part[c] = fmaf(y[0], w[c][j].x, part[c]);
        part[c] = fmaf(y[1], w[c][j].y, part[c]);
        part[c] = fmaf(y[2], w[c][j].z, part[c]);
        part[c] = fmaf(y[3], w[c][j].w, part[c]);
      }
    }
    float v = 0.f;
#pragma unroll
    for (int c = 0; c < kHeadF; ++c) {
      const float tot = half_wave_sum(part[c]);
      v = i == c ? tot : v;
    }
    if (i < kHeadF && r < T) {
      const int64_t o = r * ode.ldx + i;
      if (ode.tok_event) {
        const StageDesc sd = ode.desc[ode.tok_event[r]];
        ode_update(sd.mode, sd.h, v + bias, ode.x + o, ode.acc + o, ode.xs + o,
                   out && sd.write_out ? out + r * ode.ldo + i : nullptr);
      } else {
        ode_update(mode, h, v + bias, ode.x + o, ode.acc + o, ode.xs + o,
                   out ? out + r * ode.ldo + i : nullptr);
      }
    }
  }
}

bool head256_supported(int d, int nf) { return d == 256 && nf == kHeadF; }

hipError_t launch_head256(hipStream_t st, const float* H, const float2* stats, const float* g,
                          const float* s, const float* Wt, const float* b, const OdeArgs& ode) {
  if (ode.nf != kHeadF) return hipErrorInvalidValue;
  if (ode.m_valid <= 0) return hipSuccess;
  const int64_t waves = (ode.m_valid + 2 * kHeadIter - 1) / (2 * kHeadIter);
  hipLaunchKernelGGL(k_head256, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, H, stats, g,
                     s, Wt, b, ode);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// One block's cross K/V rows [rows][2d] (K | V, row-major, pitch 2d) into head-major planes:
// element (row, s, head, i) -> dst[((s * n_heads + head) * plane + row0 + row) * dh + i],
// s = 0 for K, 1 for V. 16-byte copies.
__global__ void k_kv_headmajor(const bf16* __restrict__ src, int64_t rows, int d, int dh,
                               int n_heads, bf16* __restrict__ dst, int64_t plane, int64_t row0) {
  const int per_row = 2 * d / 8;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * per_row) return;
  const int64_t row = t / per_row;
  const int col = (int)(t % per_row) * 8;
  const int sel = col / d, head = (col % d) / dh, i = col % dh;
  *(u32x4*)(dst + ((int64_t)(sel * n_heads + head) * plane + row0 + row) * dh + i) =
      *(const u32x4*)(src + row * 2 * d + col);
}

hipError_t launch_kv_headmajor(hipStream_t st, const void* src, int64_t rows, int d, int dh,
                               int n_heads, void* dst, int64_t plane, int64_t row0) {
  if (rows <= 0) return hipSuccess;
  if (dh % 8 || d % dh || row0 + rows > plane) return hipErrorInvalidValue;
  const int64_t n = rows * (2 * d / 8);
  hipLaunchKernelGGL(k_kv_headmajor, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                     (const bf16*)src, rows, d, dh, n_heads, (bf16*)dst, plane, row0);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Event observables of reconstructed events (Sec. 2.4, event post-processing): H_T and MET
// per event, and the isolation of every electron and muon: the pT sum of the event's other
// particles inside Delta R < 0.4, over the lepton's pT. One workgroup per event. pT, the
// trigonometric terms and every sum are FP64; the class maximum and the cone test are taken
// in FP32 with separate multiplies and adds (integer decisions in the input's precision).
// The event's particles stream through LDS in tiles of kObsTile; each thread takes
// particles i = tid, tid + 256, ... and sums its cone members in order of j.
namespace {
constexpr int kObsTile = 1024;
constexpr float kObsTwoPi = (float)(2.0 * 3.14159265358979323846);
constexpr float kObsInvTwoPi = (float)(1.0 / (2.0 * 3.14159265358979323846));

__device__ __forceinline__ int obs_class(const float* f) {
  int c = 0;
  float best = f[3];
#pragma unroll
  for (int k = 1; k < 5; ++k)
    if (f[3 + k] > best) best = f[3 + k], c = k;    // first maximum
  return c;
}

__device__ __forceinline__ bool obs_in_cone(float eta_i, float phi_i, float eta_j, float phi_j) {
#pragma clang fp contract(off)
  const float deta = eta_i - eta_j;
  const float d = phi_i - phi_j;
  const float dphi = d - kObsTwoPi * rintf(d * kObsInvTwoPi);
  return deta * deta + dphi * dphi < 0.16f;
}

__device__ __forceinline__ double obs_block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) t += red[q];       // the same order in every thread
  return t;
}
}  // namespace

__global__ __launch_bounds__(256) void k_event_observables(const float* __restrict__ feat,
                                                           int ldf,
                                                           const int64_t* __restrict__ off,
                                                           float* __restrict__ ht,
                                                           float* __restrict__ met,
                                                           float* __restrict__ iso) {
  __shared__ double s_pt[kObsTile];
  __shared__ float s_eta[kObsTile], s_phi[kObsTile];
  __shared__ double red[4];
  const int e = blockIdx.x, tid = threadIdx.x;
  const int64_t a = off[e], n = off[e + 1] - a;
  double h = 0.0, px = 0.0, py = 0.0;
  for (int64_t i = tid; i < n; i += 256) {
    const float* f = feat + (a + i) * ldf;
    const double pt = 10.0 * exp((double)f[0]);
    const double phi = (double)f[2];
    h += pt;
    px += pt * cos(phi);
    py += pt * sin(phi);
  }
  h = obs_block_sum(h, red);
  px = obs_block_sum(px, red);
  py = obs_block_sum(py, red);
  if (tid == 0) {
    ht[e] = (float)h;
    met[e] = (float)sqrt(px * px + py * py);
  }
  for (int64_t i0 = 0; i0 < n; i0 += 256) {
    const int64_t i = i0 + tid;
    bool lep = false;
    double pt_i = 0.0;
    float eta_i = 0.f, phi_i = 0.f;
    if (i < n) {
      const float* f = feat + (a + i) * ldf;
      const int c = obs_class(f);
      lep = c == 1 || c == 2;                      // electron, muon
      pt_i = 10.0 * exp((double)f[0]);
      eta_i = f[1];
      phi_i = f[2];
    }
    double sum = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kObsTile) {
      const int nt = (int)min<int64_t>(kObsTile, n - j0);
      __syncthreads();
      for (int j = tid; j < nt; j += 256) {
        const float* f = feat + (a + j0 + j) * ldf;
        s_pt[j] = 10.0 * exp((double)f[0]);
        s_eta[j] = f[1];
        s_phi[j] = f[2];
      }
      __syncthreads();
      if (lep)
        for (int j = 0; j < nt; ++j)
          if (j0 + j != i && obs_in_cone(eta_i, phi_i, s_eta[j], s_phi[j])) sum += s_pt[j];
    }
    if (i < n) iso[a + i] = lep ? (float)(sum / pt_i) : __builtin_nanf("");
  }
}

hipError_t launch_event_observables(hipStream_t st, const float* feat, int ldf,
                                    const int64_t* off_device, int64_t n_events, float* ht,
                                    float* met, float* iso) {
  if (n_events <= 0) return hipSuccess;
  if (n_events > 0x7fffffff || ldf < 8) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_event_observables, dim3((unsigned)n_events), dim3(256), 0, st, feat, ldf,
                     off_device, ht, met, iso);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------------------
// Truth preprocessing before the sampler: the model's pT cut and particle limit (stream
// compaction per event). Pass 1, one workgroup per event: a particle survives when
// x0 > c0 (x0 = ln(pT / 10 GeV), c0 = ln(cut / 10 GeV) in float32); if more than `limit`
// survive, a survivor is kept when fewer than `limit` survivors rank before it (larger x0,
// or equal x0 and an earlier position). Writes keep[row] and the event's count. Pass 2
// writes the kept rows in input order at the event's output offset (a block-wide prefix
// sum of the keep flags).
namespace {
constexpr int kSelTile = 1024;
}  // namespace

__global__ __launch_bounds__(256) void k_select_count(const float* __restrict__ feat, int ldf,
                                                      const int64_t* __restrict__ off, float c0,
                                                      int limit, uint8_t* __restrict__ keep,
                                                      int32_t* __restrict__ cnt) {
  __shared__ float s_x[kSelTile];
  __shared__ int s_n;
  const int e = blockIdx.x, tid = threadIdx.x;
  const int64_t a = off[e], n = off[e + 1] - a;
  if (tid == 0) s_n = 0;
  __syncthreads();
  int mine = 0;
  for (int64_t i = tid; i < n; i += 256) mine += feat[(a + i) * ldf] > c0;
  atomicAdd(&s_n, mine);                 // LDS atomic: an integer count, order-free
  __syncthreads();
  const int surv = s_n;
  const bool all = surv <= limit;
  for (int64_t i0 = 0; i0 < n; i0 += 256) {
    const int64_t i = i0 + tid;
    const float xi = i < n ? feat[(a + i) * ldf] : 0.f;
    const bool si = i < n && xi > c0;
    int rank = 0;
    if (!all) {
      for (int64_t j0 = 0; j0 < n; j0 += kSelTile) {
        const int nt = (int)min<int64_t>(kSelTile, n - j0);
        __syncthreads();
        for (int j = tid; j < nt; j += 256) s_x[j] = feat[(a + j0 + j) * ldf];
        __syncthreads();
        if (si)
          for (int j = 0; j < nt; ++j) {
            const float xj = s_x[j];
            rank += xj > c0 && (xj > xi || (xj == xi && j0 + j < i));
          }
      }
    }
    if (i < n) keep[a + i] = si && (all || rank < limit);
  }
  if (tid == 0) cnt[e] = all ? surv : limit;
}

__global__ __launch_bounds__(256) void k_select_write(const float* __restrict__ feat, int ldf,
                                                      const int64_t* __restrict__ off,
                                                      const int64_t* __restrict__ off_out,
                                                      const uint8_t* __restrict__ keep,
                                                      float* __restrict__ out) {
  __shared__ int s_tot[4];
  const int e = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t a = off[e], n = off[e + 1] - a;
  int64_t base = off_out[e];
  for (int64_t i0 = 0; i0 < n; i0 += 256) {
    const int64_t i = i0 + tid;
    const bool k = i < n && keep[a + i];
    // block prefix of the flags: ballot within the wave, wave totals through LDS
    const uint64_t bal = __ballot(k);
    const int before_w = __popcll(bal & ((lane ? (~0ull >> (64 - lane)) : 0ull)));
    __syncthreads();
    if (lane == 0) s_tot[wave] = __popcll(bal);
    __syncthreads();
    int before = before_w;
    for (int q = 0; q < wave; ++q) before += s_tot[q];
    if (k) {
      const float* src = feat + (a + i) * ldf;
      float* dst = out + (base + before) * ldf;
      for (int f = 0; f < ldf; ++f) dst[f] = src[f];
    }
    base += s_tot[0] + s_tot[1] + s_tot[2] + s_tot[3];
  }
}

// Reco multiplicity per event (a stand-in law; the model can emit particles that match no
// truth particle, Sec. 2.2): N_reco = min(n_max, N - lost + fakes) for N > 0 truth particles,
// else 0. lost counts the words w_i, i < N, below thr_q (each truth particle missed with
// probability q), fakes the words w_(N + j), j < M, below thr_p (M trials of probability p).
// The words are those of Philox4x64-10 with key (seed, 1) at counters (c, e, 0, 0), four per
// counter in order. One wave per event: lane l takes counters l, l + 64, ...; the integer
// counts are summed across the wave (order-free).
__global__ __launch_bounds__(64) void k_reco_counts(const int64_t* __restrict__ off, int64_t E,
                                                    uint64_t seed, uint64_t thr_q, uint64_t thr_p,
                                                    int M, int n_max, int32_t* __restrict__ cnt) {
  const int64_t e = blockIdx.x;
  if (e >= E) return;
  const int lane = threadIdx.x;
  const int64_t n = off[e + 1] - off[e];
  if (n <= 0) {
    if (lane == 0) cnt[e] = 0;
    return;
  }
  const int64_t words = n + M, ctrs = (words + 3) / 4;
  int lost = 0, fakes = 0;
  for (int64_t c = lane; c < ctrs; c += 64) {
    const Philox4x64 w = philox4x64_10((uint64_t)c, (uint64_t)e, 0ull, 0ull, seed, 1ull);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t i = 4 * c + k;
      if (i < n) lost += w.c[k] < thr_q;
      else if (i < words) fakes += w.c[k] < thr_p;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lost += __shfl_xor(lost, o, 64);
    fakes += __shfl_xor(fakes, o, 64);
  }
  if (lane == 0) cnt[e] = (int32_t)min<int64_t>(n_max, n - lost + fakes);
}

hipError_t launch_reco_counts(hipStream_t st, const int64_t* off, int64_t n_events, uint64_t seed,
                              uint64_t thr_q, uint64_t thr_p, int fake_trials, int n_max,
                              int32_t* cnt) {
  if (n_events <= 0) return hipSuccess;
  if (n_events > 0x7fffffff || fake_trials < 0 || n_max < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reco_counts, dim3((unsigned)n_events), dim3(64), 0, st, off, n_events, seed,
                     thr_q, thr_p, fake_trials, n_max, cnt);
  return hipGetLastError();
}

hipError_t launch_select_count(hipStream_t st, const float* feat, int ldf, const int64_t* off,
                               int64_t n_events, float c0, int limit, uint8_t* keep,
                               int32_t* cnt) {
  if (n_events <= 0) return hipSuccess;
  if (n_events > 0x7fffffff || limit < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_select_count, dim3((unsigned)n_events), dim3(256), 0, st, feat, ldf, off,
                     c0, limit, keep, cnt);
  return hipGetLastError();
}

hipError_t launch_select_write(hipStream_t st, const float* feat, int ldf, const int64_t* off,
                               const int64_t* off_out, int64_t n_events, const uint8_t* keep,
                               float* out) {
  if (n_events <= 0) return hipSuccess;
  if (n_events > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_select_write, dim3((unsigned)n_events), dim3(256), 0, st, feat, ldf, off,
                     off_out, keep, out);
  return hipGetLastError();
}

}  // namespace fmd
