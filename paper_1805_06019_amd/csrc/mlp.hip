// The encoder's per-block network (learned encoder control): inference,
// batch gradient and Adam update, hand-written for CDNA4.
//
// 16 features -> 64 ReLU -> 64 ReLU -> 37 logits (10 threshold classes, 27
// range classes).  Parameters W1[64][16], b1[64], W2[64][64], b2[64],
// W3[37][64], b3[37]; inference and gradients read them as bfloat16 and
// accumulate in float32.  The network is tiny (7,653 parameters).
// Inference runs one row per lane with the parameters, unpacked once per
// call to float32, read through the scalar unit (they are the same for every
// lane), so each multiply-add takes its weight from a scalar register; the
// gradient kernel keeps all parameters and a tile of 128 rows' activations
// in LDS and forms each weight gradient as a 128-long dot product over the
// tile.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "internal.h"

namespace {

constexpr int kIn = 16, kH = 64, kOut = 37, kCls = 10, kRng = 27;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;
static_assert(kParams == LFC_MLP_PARAMS, "parameter count");
constexpr int kThreads = 256;
constexpr int kTile = 128;   // rows per gradient workgroup

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// float32 -> bfloat16, round to nearest, ties to even (NaN stays NaN)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0;
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ void load_weights(const uint16_t *w, float *sw) {
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) sw[i] = bf16_to_f32(w[i]);
}

// ---------------------------------------------------------------------------
// inference: one row per lane, parameters through the scalar unit
// ---------------------------------------------------------------------------
typedef const __attribute__((address_space(4))) float *uniform_f32;

__global__ __launch_bounds__(kThreads) void k_mlp_unpack(const uint16_t *w, float *wf) {
  const int i = blockIdx.x * kThreads + threadIdx.x;
  if (i < kParams) wf[i] = bf16_to_f32(w[i]);
}

struct InferArgs {
  const float *wf;   // the parameters as float32 (k_mlp_unpack)
  const float *x;
  int64_t n;
  int8_t *cls, *rng;
  float *conf, *logits;
};

__global__ __launch_bounds__(kThreads) void k_mlp_infer(InferArgs a) {
  const uniform_f32 sw = (uniform_f32)a.wf;
  {
    // one row per lane and no loop over rows, so that the parameter loads stay
    // at their uses instead of being hoisted out of a loop into registers
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= a.n) return;
    float x[kIn];
    const float4 *xr = reinterpret_cast<const float4 *>(a.x + r * kIn);
#pragma unroll
    for (int k = 0; k < kIn / 4; k++) {
      const float4 t = xr[k];
      x[4 * k] = t.x;
      x[4 * k + 1] = t.y;
      x[4 * k + 2] = t.z;
      x[4 * k + 3] = t.w;
    }
    float h1[kH];
#pragma unroll
    for (int j = 0; j < kH; j++) {
      float acc = sw[oB1 + j];
#pragma unroll
      for (int k = 0; k < kIn; k++) acc += sw[oW1 + j * kIn + k] * x[k];
      h1[j] = fmaxf(acc, 0.0f);
    }
    float h2[kH];
#pragma unroll
    for (int j = 0; j < kH; j++) {
      float acc = sw[oB2 + j];
#pragma unroll
      for (int k = 0; k < kH; k++) acc += sw[oW2 + j * kH + k] * h1[k];
      h2[j] = fmaxf(acc, 0.0f);
    }
    float z[kOut];
#pragma unroll
    for (int o = 0; o < kOut; o++) {
      float acc = sw[oB3 + o];
#pragma unroll
      for (int k = 0; k < kH; k++) acc += sw[oW3 + o * kH + k] * h2[k];
      z[o] = acc;
    }
    if (a.logits)
#pragma unroll
      for (int o = 0; o < kOut; o++) a.logits[r * kOut + o] = z[o];
    // heads: argmax (ties to the lower class)
    float best_t = z[0], best_r = z[kCls];
    int ct = 0, cr = 0;
#pragma unroll
    for (int o = 1; o < kCls; o++)
      if (z[o] > best_t) {
        best_t = z[o];
        ct = o;
      }
#pragma unroll
    for (int o = 1; o < kRng; o++)
      if (z[kCls + o] > best_r) {
        best_r = z[kCls + o];
        cr = o;
      }
    a.cls[r] = (int8_t)ct;
    a.rng[r] = (int8_t)cr;
    if (a.conf) {
      float den = 0.0f;
#pragma unroll
      for (int o = 0; o < kCls; o++) den += expf(z[o] - best_t);
      a.conf[r] = 1.0f / den;
    }
  }
}

// ---------------------------------------------------------------------------
// inference on the matrix cores: bf16 operands, fp32 accumulation
// ---------------------------------------------------------------------------
// Each wave runs tiles of 32 rows through v_mfma_f32_32x32x16_bf16: lane l
// supplies row l%32 of A with K elements 8*(l/32)..+7, column l%32 of B with
// the same K elements, and receives D[8*(r/4) + 4*(l/32) + r%4][l%32] in its
// register r.  The weights (as B operands) stay in registers for the wave's
// life; each layer's output goes through the wave's LDS (bias, ReLU, rounded
// to bf16) to become the next layer's A operand.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kMfmaWaves = 4;

__device__ __forceinline__ bf16x8 load_bf16x8(const uint16_t *p) {
  const uint4 v = *reinterpret_cast<const uint4 *>(p);
  bf16x8 r;
  __builtin_memcpy(&r, &v, sizeof r);
  return r;
}

__global__ __launch_bounds__(64 * kMfmaWaves) void k_mlp_infer_mfma(InferArgs a, const uint16_t *w) {
  __shared__ __attribute__((aligned(16))) __bf16 sh[kMfmaWaves][2][32][kH];   // layer outputs
  __shared__ float sz[kMfmaWaves][32][kOut + 3];   // logits
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, col = lane & 31, kh = lane >> 5;
  // B operands: W1 (K 16) as 2 column tiles; W2, W3 (K 64) as 4 K steps x 2 tiles
  bf16x8 b1[2], b2[4][2], b3[4][2];
  float bias1[2], bias2[2], bias3[2];
  const bf16x8 zero8 = {};
#pragma unroll
  for (int t = 0; t < 2; t++) {
    const int j = t * 32 + col;
    b1[t] = load_bf16x8(w + oW1 + j * kIn + kh * 8);
    bias1[t] = bf16_to_f32(w[oB1 + j]);
    bias2[t] = bf16_to_f32(w[oB2 + j]);
    bias3[t] = j < kOut ? bf16_to_f32(w[oB3 + j]) : 0.0f;
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
      b2[ks][t] = load_bf16x8(w + oW2 + j * kH + ks * 16 + kh * 8);
      b3[ks][t] = j < kOut ? load_bf16x8(w + oW3 + j * kH + ks * 16 + kh * 8) : zero8;
    }
  }
  const int64_t tiles = (a.n + 31) / 32;
  for (int64_t tile = (int64_t)blockIdx.x * kMfmaWaves + wv; tile < tiles; tile += (int64_t)gridDim.x * kMfmaWaves) {
    const int64_t r0 = tile * 32, row = r0 + col;
    // layer 1: A = this lane's row, features 8*kh..+7, rounded to bf16
    bf16x8 a1;
    if (row < a.n) {
      const float4 u = *reinterpret_cast<const float4 *>(a.x + row * kIn + kh * 8);
      const float4 v = *reinterpret_cast<const float4 *>(a.x + row * kIn + kh * 8 + 4);
      a1[0] = (__bf16)u.x, a1[1] = (__bf16)u.y, a1[2] = (__bf16)u.z, a1[3] = (__bf16)u.w;
      a1[4] = (__bf16)v.x, a1[5] = (__bf16)v.y, a1[6] = (__bf16)v.z, a1[7] = (__bf16)v.w;
    } else {
      a1 = zero8;
    }
    // d -> bias, ReLU, bf16 into the wave's LDS rows
    auto store_act = [&](const f32x16 &d, float bias, int t, int buf) {
#pragma unroll
      for (int r = 0; r < 16; r++) sh[wv][buf][8 * (r / 4) + 4 * kh + (r % 4)][t * 32 + col] = (__bf16)fmaxf(d[r] + bias, 0.0f);
    };
#pragma unroll
    for (int t = 0; t < 2; t++) {
      f32x16 d = {};
      d = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b1[t], d, 0, 0, 0);
      store_act(d, bias1[t], t, 0);
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);   // LDS writes of this wave done before its reads
    __builtin_amdgcn_wave_barrier();
    // layer 2
    f32x16 d2[2] = {{}, {}};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
      const bf16x8 a2 = *reinterpret_cast<const bf16x8 *>(&sh[wv][0][col][ks * 16 + kh * 8]);
#pragma unroll
      for (int t = 0; t < 2; t++) d2[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2, b2[ks][t], d2[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 2; t++) store_act(d2[t], bias2[t], t, 1);
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    // layer 3 (columns 37..63 are zero weights)
    f32x16 d3[2] = {{}, {}};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
      const bf16x8 a3 = *reinterpret_cast<const bf16x8 *>(&sh[wv][1][col][ks * 16 + kh * 8]);
#pragma unroll
      for (int t = 0; t < 2; t++) d3[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a3, b3[ks][t], d3[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 2; t++)
#pragma unroll
      for (int r = 0; r < 16; r++) {
        const int j = t * 32 + col;
        if (j < kOut) sz[wv][8 * (r / 4) + 4 * kh + (r % 4)][j] = d3[t][r] + bias3[t];
      }
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    // heads: lane i < 32 takes row i
    if (lane < 32 && r0 + lane < a.n) {
      const float *z = sz[wv][lane];
      const int64_t rr = r0 + lane;
      float bt = z[0], br = z[kCls];
      int ct = 0, cr = 0;
      for (int o = 1; o < kCls; o++)
        if (z[o] > bt) {
          bt = z[o];
          ct = o;
        }
      for (int o = 1; o < kRng; o++)
        if (z[kCls + o] > br) {
          br = z[kCls + o];
          cr = o;
        }
      a.cls[rr] = (int8_t)ct;
      a.rng[rr] = (int8_t)cr;
      if (a.conf) {
        float den = 0.0f;
        for (int o = 0; o < kCls; o++) den += expf(z[o] - bt);
        a.conf[rr] = 1.0f / den;
      }
      if (a.logits)
        for (int o = 0; o < kOut; o++) a.logits[rr * kOut + o] = z[o];
    }
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------------------
// batch gradient: 128 rows per workgroup, activations in LDS
// ---------------------------------------------------------------------------
struct GradArgs {
  const uint16_t *w;
  const float *x;
  const int8_t *cls, *rng;
  int n;
  float *part;   // [gridDim.x][kParams + 1]: partial gradient sums, then the partial loss
};

__global__ __launch_bounds__(kThreads) void k_mlp_grad(GradArgs a) {
  extern __shared__ float smem[];
  float *sw = smem;                      // [kParams]
  float *X = sw + kParams;               // [kTile][kIn]
  float *H1 = X + kTile * kIn;           // [kTile][kH], later dL/d(pre-activation 1)
  float *H2 = H1 + kTile * kH;           // [kTile][kH], later dL/d(pre-activation 2)
  float *Z = H2 + kTile * kH;            // [kTile][kOut], logits, later dL/dz
  float *red = Z + kTile * kOut;         // [kTile] row losses
  const int t = threadIdx.x, r0 = blockIdx.x * kTile;
  const int rows = min(kTile, a.n - r0);
  const float inv_n = 1.0f / (float)a.n;
  load_weights(a.w, sw);
  for (int i = t; i < kTile * kIn; i += kThreads) {
    const int r = i / kIn;
    X[i] = r < rows ? a.x[(size_t)(r0 + r) * kIn + i % kIn] : 0.0f;
  }
  __syncthreads();
  // forward: lane t computes unit j = t % 64 for rows t/64, t/64 + 4, ...
  const int j = t % kH, rq = t / kH;
  for (int r = rq; r < kTile; r += kThreads / kH) {
    float acc = sw[oB1 + j];
    for (int k = 0; k < kIn; k++) acc += sw[oW1 + j * kIn + k] * X[r * kIn + k];
    H1[r * kH + j] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  for (int r = rq; r < kTile; r += kThreads / kH) {
    float acc = sw[oB2 + j];
    for (int k = 0; k < kH; k++) acc += sw[oW2 + j * kH + k] * H1[r * kH + k];
    H2[r * kH + j] = fmaxf(acc, 0.0f);
  }
  __syncthreads();
  if (j < kOut)
    for (int r = rq; r < kTile; r += kThreads / kH) {
      float acc = sw[oB3 + j];
      for (int k = 0; k < kH; k++) acc += sw[oW3 + j * kH + k] * H2[r * kH + k];
      Z[r * kOut + j] = acc;
    }
  __syncthreads();
  // softmax cross-entropy of both heads, one lane per row; dL/dz in place
  // (scaled by 1/n: the batch mean)
  if (t < kTile) {
    float *z = Z + t * kOut;
    float loss = 0.0f;
    if (t < rows) {
      const int yc = a.cls[r0 + t], yr = a.rng[r0 + t];
      if (yc < 0 || yc >= kCls || yr < 0 || yr >= kRng) {
        loss = __builtin_nanf("");
        for (int o = 0; o < kOut; o++) z[o] = 0.0f;
      } else {
        for (int h = 0; h < 2; h++) {
          const int o0 = h ? kCls : 0, no = h ? kRng : kCls, y = h ? yr : yc;
          float m = z[o0];
          for (int o = 1; o < no; o++) m = fmaxf(m, z[o0 + o]);
          float den = 0.0f;
          for (int o = 0; o < no; o++) den += expf(z[o0 + o] - m);
          loss += logf(den) + m - z[o0 + y];
          const float inv = 1.0f / den;
          for (int o = 0; o < no; o++) z[o0 + o] = (expf(z[o0 + o] - m) * inv - (o == y ? 1.0f : 0.0f)) * inv_n;
        }
      }
    } else {
      for (int o = 0; o < kOut; o++) z[o] = 0.0f;
    }
    red[t] = loss;
  }
  __syncthreads();
  float *part = a.part + (size_t)blockIdx.x * (kParams + 1);
  // dW3, db3
  for (int e = t; e < kOut * (kH + 1); e += kThreads) {
    const int o = e / (kH + 1), k = e % (kH + 1);
    float acc = 0.0f;
    if (k < kH)
      for (int r = 0; r < kTile; r++) acc += Z[r * kOut + o] * H2[r * kH + k];
    else
      for (int r = 0; r < kTile; r++) acc += Z[r * kOut + o];
    part[k < kH ? oW3 + o * kH + k : oB3 + o] = acc;
  }
  if (t == 0) {
    float l = 0.0f;
    for (int r = 0; r < kTile; r++) l += red[r];
    part[kParams] = l * inv_n;
  }
  __syncthreads();
  // back through layer 3 and the second ReLU
  for (int r = rq; r < kTile; r += kThreads / kH) {
    float acc = 0.0f;
    for (int o = 0; o < kOut; o++) acc += Z[r * kOut + o] * sw[oW3 + o * kH + j];
    H2[r * kH + j] = H2[r * kH + j] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  // dW2, db2
  for (int e = t; e < kH * (kH + 1); e += kThreads) {
    const int o = e / (kH + 1), k = e % (kH + 1);
    float acc = 0.0f;
    if (k < kH)
      for (int r = 0; r < kTile; r++) acc += H2[r * kH + o] * H1[r * kH + k];
    else
      for (int r = 0; r < kTile; r++) acc += H2[r * kH + o];
    part[k < kH ? oW2 + o * kH + k : oB2 + o] = acc;
  }
  __syncthreads();
  // back through layer 2 and the first ReLU
  for (int r = rq; r < kTile; r += kThreads / kH) {
    float acc = 0.0f;
    for (int o = 0; o < kH; o++) acc += H2[r * kH + o] * sw[oW2 + o * kH + j];
    H1[r * kH + j] = H1[r * kH + j] > 0.0f ? acc : 0.0f;
  }
  __syncthreads();
  // dW1, db1
  for (int e = t; e < kH * (kIn + 1); e += kThreads) {
    const int o = e / (kIn + 1), k = e % (kIn + 1);
    float acc = 0.0f;
    if (k < kIn)
      for (int r = 0; r < kTile; r++) acc += H1[r * kH + o] * X[r * kIn + k];
    else
      for (int r = 0; r < kTile; r++) acc += H1[r * kH + o];
    part[k < kIn ? oW1 + o * kIn + k : oB1 + o] = acc;
  }
}

// sum of the workgroups' partials, parameter by parameter (and the loss)
__global__ __launch_bounds__(kThreads) void k_mlp_reduce(const float *part, int nwg, float *grad, float *loss) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p > kParams) return;
  float acc = 0.0f;
  for (int w = 0; w < nwg; w++) acc += part[(size_t)w * (kParams + 1) + p];
  if (p < kParams)
    grad[p] = acc;
  else
    loss[0] = acc;
}

struct AdamArgs {
  float *master;
  uint16_t *w;
  float *m, *v;
  const float *grad;
  float lr, beta1, beta2, eps, c1, c2;   // c1 = 1/(1-beta1^t), c2 = 1/(1-beta2^t)
};

__global__ __launch_bounds__(kThreads) void k_mlp_adam(AdamArgs a) {
  const int p = blockIdx.x * kThreads + threadIdx.x;
  if (p >= kParams) return;
  const float g = a.grad[p];
  const float m = a.beta1 * a.m[p] + (1.0f - a.beta1) * g;
  const float v = a.beta2 * a.v[p] + (1.0f - a.beta2) * g * g;
  a.m[p] = m;
  a.v[p] = v;
  const float w = a.master[p] - a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
  a.master[p] = w;
  a.w[p] = f32_to_bf16(w);
}

lfc_status mlp_check(const void *p, size_t need, size_t align, const char *who, const char *what) {
  if (!p) return lfc::fail(LFC_E_INVALID, std::string(who) + ": null " + what);
  if (reinterpret_cast<uintptr_t>(p) % align)
    return lfc::fail(LFC_E_INVALID, std::string(who) + ": " + what + " is not " + std::to_string(align) + "-byte aligned");
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void *>(p)) != hipSuccess || !base) {
    (void)hipGetLastError();
    return lfc::fail(LFC_E_INVALID, std::string(who) + ": " + what + " is not device memory");
  }
  const size_t off = static_cast<const char *>(p) - static_cast<const char *>(base);
  if (off + need > size) return lfc::fail(LFC_E_INVALID, std::string(who) + ": " + what + " is too small");
  return LFC_OK;
}

lfc_status mlp_launched(const char *who) {
  const hipError_t he = hipGetLastError();
  if (he != hipSuccess) return lfc::fail(LFC_E_HIP, std::string(who) + ": launch failed: " + hipGetErrorString(he));
  return LFC_OK;
}

constexpr size_t kGradLds = sizeof(float) * (kParams + kTile * (kIn + 2 * kH + kOut + 1));

lfc_status infer_launch(const uint16_t *w, const float *x, int64_t n, int8_t *cls, int8_t *rng, float *conf,
                        float *logits, hipStream_t s) {
  if (n == 0) return LFC_OK;
  if (n > (int64_t)0x7FFFFFFF * kThreads) return lfc::fail(LFC_E_INVALID, "lfc_mlp_infer: too many rows");
  // the float32 parameters live in stream-ordered scratch for this call
  float *wf = nullptr;
  if (hipMallocAsync(reinterpret_cast<void **>(&wf), sizeof(float) * kParams, s) != hipSuccess) {
    (void)hipGetLastError();
    return lfc::fail(LFC_E_NOMEM, "lfc_mlp_infer: scratch for the parameters");
  }
  hipLaunchKernelGGL(k_mlp_unpack, dim3((kParams + kThreads - 1) / kThreads), dim3(kThreads), 0, s, w, wf);
  lfc_status st = mlp_launched("lfc_mlp_infer");
  if (st == LFC_OK) {
    const int64_t blocks = (n + kThreads - 1) / kThreads;   // n < 2^31 * 256, checked by the callers
    InferArgs a{wf, x, n, cls, rng, conf, logits};
    hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)blocks), dim3(kThreads), 0, s, a);
    st = mlp_launched("lfc_mlp_infer");
  }
  if (hipFreeAsync(wf, s) != hipSuccess && st == LFC_OK) st = lfc::fail(LFC_E_HIP, "lfc_mlp_infer: scratch release");
  return st;
}

}  // namespace

extern "C" lfc_status lfc_mlp_infer(const uint16_t *d_w, const float *d_x, int64_t n, int8_t *d_cls, int8_t *d_rng,
                                    float *d_conf, float *d_logits, hipStream_t s) {
  return lfc_mlp_infer_ex(d_w, d_x, n, d_cls, d_rng, d_conf, d_logits, LFC_MLP_FP32, s);
}

extern "C" lfc_status lfc_mlp_infer_ex(const uint16_t *d_w, const float *d_x, int64_t n, int8_t *d_cls, int8_t *d_rng,
                                       float *d_conf, float *d_logits, int32_t precision, hipStream_t s) {
  const char *who = "lfc_mlp_infer";
  if (precision != LFC_MLP_FP32 && precision != LFC_MLP_BF16)
    return lfc::fail(LFC_E_INVALID, "lfc_mlp_infer: unknown precision");
  if (n < 0) return lfc::fail(LFC_E_INVALID, "lfc_mlp_infer: n < 0");
  if (lfc_status st = mlp_check(d_w, sizeof(uint16_t) * kParams, 2, who, "d_w")) return st;
  if (n == 0) return LFC_OK;
  if (lfc_status st = mlp_check(d_x, sizeof(float) * kIn * (size_t)n, 16, who, "d_x")) return st;
  if (lfc_status st = mlp_check(d_cls, (size_t)n, 1, who, "d_cls")) return st;
  if (lfc_status st = mlp_check(d_rng, (size_t)n, 1, who, "d_rng")) return st;
  if (d_conf)
    if (lfc_status st = mlp_check(d_conf, sizeof(float) * (size_t)n, 4, who, "d_conf")) return st;
  if (d_logits)
    if (lfc_status st = mlp_check(d_logits, sizeof(float) * kOut * (size_t)n, 4, who, "d_logits")) return st;
  if (precision == LFC_MLP_FP32) return infer_launch(d_w, d_x, n, d_cls, d_rng, d_conf, d_logits, s);
  if (reinterpret_cast<uintptr_t>(d_w) % 16)
    return lfc::fail(LFC_E_INVALID, "lfc_mlp_infer: bf16 inference needs 16-byte aligned weights");
  const int64_t tiles = (n + 31) / 32;
  const int64_t blocks = std::min<int64_t>((tiles + kMfmaWaves - 1) / kMfmaWaves, 4096);
  InferArgs a{nullptr, d_x, n, d_cls, d_rng, d_conf, d_logits};
  hipLaunchKernelGGL(k_mlp_infer_mfma, dim3((unsigned)blocks), dim3(64 * kMfmaWaves), 0, s, a, d_w);
  return mlp_launched(who);
}

extern "C" lfc_status lfc_mlp_grad(const uint16_t *d_w, const float *d_x, const int8_t *d_cls, const int8_t *d_rng,
                                   int32_t n, float *d_part, float *d_grad, float *d_loss, hipStream_t s) {
  const char *who = "lfc_mlp_grad";
  if (n < 1) return lfc::fail(LFC_E_INVALID, "lfc_mlp_grad: n < 1");
  const int nwg = (n + kTile - 1) / kTile;
  if (lfc_status st = mlp_check(d_w, sizeof(uint16_t) * kParams, 2, who, "d_w")) return st;
  if (lfc_status st = mlp_check(d_x, sizeof(float) * kIn * (size_t)n, 4, who, "d_x")) return st;
  if (lfc_status st = mlp_check(d_cls, (size_t)n, 1, who, "d_cls")) return st;
  if (lfc_status st = mlp_check(d_rng, (size_t)n, 1, who, "d_rng")) return st;
  if (lfc_status st = mlp_check(d_part, sizeof(float) * (kParams + 1) * (size_t)nwg, 4, who, "d_part")) return st;
  if (lfc_status st = mlp_check(d_grad, sizeof(float) * kParams, 4, who, "d_grad")) return st;
  if (lfc_status st = mlp_check(d_loss, sizeof(float), 4, who, "d_loss")) return st;
  GradArgs a{d_w, d_x, d_cls, d_rng, n, d_part};
  hipLaunchKernelGGL(k_mlp_grad, dim3(nwg), dim3(kThreads), kGradLds, s, a);
  if (lfc_status st = mlp_launched(who)) return st;
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kParams + 1 + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     (const float *)d_part, nwg, d_grad, d_loss);
  return mlp_launched(who);
}

extern "C" lfc_status lfc_mlp_adam(float *d_master, uint16_t *d_w, float *d_m, float *d_v, const float *d_grad,
                                   int32_t step, float lr, float beta1, float beta2, float eps, hipStream_t s) {
  const char *who = "lfc_mlp_adam";
  if (step < 1) return lfc::fail(LFC_E_INVALID, "lfc_mlp_adam: step < 1");
  if (lfc_status st = mlp_check(d_master, sizeof(float) * kParams, 4, who, "d_master")) return st;
  if (lfc_status st = mlp_check(d_w, sizeof(uint16_t) * kParams, 2, who, "d_w")) return st;
  if (lfc_status st = mlp_check(d_m, sizeof(float) * kParams, 4, who, "d_m")) return st;
  if (lfc_status st = mlp_check(d_v, sizeof(float) * kParams, 4, who, "d_v")) return st;
  if (lfc_status st = mlp_check(d_grad, sizeof(float) * kParams, 4, who, "d_grad")) return st;
  const double c1 = 1.0 / (1.0 - std::pow((double)beta1, step)), c2 = 1.0 / (1.0 - std::pow((double)beta2, step));
  AdamArgs a{d_master, d_w, d_m, d_v, d_grad, lr, beta1, beta2, eps, (float)c1, (float)c2};
  hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + kThreads - 1) / kThreads), dim3(kThreads), 0, s, a);
  return mlp_launched(who);
}

namespace lfc {

// The encoder's inference over host rows: staged through stream-ordered
// device memory, then back to the host.
lfc_status mlp_infer_rows(const void *d_w, const float *feat, int64_t n, int8_t *cls, int8_t *rng, float *conf,
                          hipStream_t s) {
  if (n == 0) return LFC_OK;
  if (lfc_status st = mlp_check(d_w, sizeof(uint16_t) * kParams, 2, "lfc_encode_ctl", "d_mlp")) return st;
  char *d = nullptr;
  const size_t fx = sizeof(float) * kIn * (size_t)n, bytes = fx + sizeof(float) * (size_t)n + 2 * (size_t)n;
  if (hipMallocAsync(reinterpret_cast<void **>(&d), bytes, s) != hipSuccess) {
    (void)hipGetLastError();
    return fail(LFC_E_NOMEM, "lfc_encode_ctl: device memory for the network's rows");
  }
  float *dx = reinterpret_cast<float *>(d), *dconf = reinterpret_cast<float *>(d + fx);
  int8_t *dcls = reinterpret_cast<int8_t *>(d + fx + sizeof(float) * (size_t)n), *drng = dcls + n;
  lfc_status st = LFC_OK;
  if (hipMemcpyAsync(dx, feat, fx, hipMemcpyHostToDevice, s) != hipSuccess)
    st = fail(LFC_E_HIP, "lfc_encode_ctl: copy of the features");
  if (st == LFC_OK) st = infer_launch(static_cast<const uint16_t *>(d_w), dx, n, dcls, drng, dconf, nullptr, s);
  if (st == LFC_OK && (hipMemcpyAsync(cls, dcls, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
                       hipMemcpyAsync(rng, drng, (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess ||
                       hipMemcpyAsync(conf, dconf, sizeof(float) * (size_t)n, hipMemcpyDeviceToHost, s) != hipSuccess))
    st = fail(LFC_E_HIP, "lfc_encode_ctl: copy of the classes");
  if (hipFreeAsync(d, s) != hipSuccess && st == LFC_OK) st = fail(LFC_E_HIP, "lfc_encode_ctl: release");
  if (hipStreamSynchronize(s) != hipSuccess && st == LFC_OK) st = fail(LFC_E_HIP, "lfc_encode_ctl: synchronize");
  return st;
}

}  // namespace lfc
