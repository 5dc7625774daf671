// BC1 latents as trainable parameters (Sec. 3.2, Eqs. 1-3).
//
// During training the paper keeps every BC1 texture as floating-point
// tensors, endpoints and per-texel interpolation weights, and obtains the
// BC1 values by a sigmoid followed by quantisation to the field widths
// (5, 6, 5 bits for the endpoints, 2 bits for the weight), with the
// quantisation transparent to gradients. Here one level of W x H texels
// is a float array [H/4][W/4][22] of logits per block:
//   e0 (r, g, b), e1 (r, g, b), alpha[16] (texel (x, y) of the block at 4y + x).
// Codes: E = round(sigmoid(e) (2^b - 1)), w = round(sigmoid(alpha) 3), and
// the texel value per channel is ((3 - w) E0 + w E1) / (3 (2^b - 1)): the
// four-colour BC1 palette, so the same texels come out of real BC1 blocks
// (ntc_qat_export_bc1) through the ordinary decoder.
//
// A code is decided by comparing the logit with the FP32 logits of the
// rounding midpoints (k + 1/2) / (2^b - 1), computed on the host in double
// precision: sigmoid is monotonic, so this is the rounding of the sigmoid
// without evaluating it, and the decision depends only on the input and a
// correctly rounded constant.
#include <hip/hip_runtime.h>

#include <cmath>

#include "ntc_device.hpp"
#include "ntc_internal.hpp"

namespace ntc {

namespace {

constexpr int kQatParams = 22;

struct QatArgs {
  const float *params;  // [bh][bw][22]
  const float *grad;    // texel gradients [h][w][3] (backward)
  float *texels;        // [h][w][3] (forward) or parameter gradients [bh][bw][22] (backward)
  uint2 *blocks;        // [bh][bw] (export)
  int32_t w, h, bw, bh;
  QatTables t;
};

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

// Code of logit x on M + 1 levels: the number of midpoint logits mid[0..M-1]
// at or below x. A candidate from the FP32 sigmoid (within one level of the
// answer: its error is far below 1 / (2M)) is corrected by the exact
// comparisons. NaN gives 0.
__device__ __forceinline__ int quant_code(float x, const float *mid, int M) {
  const float s = sigmoidf(x) * (float)M;
  int c = s >= 0.0f ? (int)rintf(fminf(s, (float)M)) : 0;
#pragma unroll
  for (int i = 0; i < 2; ++i)
    if (c > 0 && !(x >= mid[c - 1])) --c;
#pragma unroll
  for (int i = 0; i < 2; ++i)
    if (c < M && x >= mid[c]) ++c;
  return c;
}

// Endpoint codes of a block as red | blue << 8 | green << 16 (the field
// order of the decoder's numerators).
__device__ __forceinline__ uint32_t endpoint_codes(const float *p, const QatTables &t) {
  const uint32_t r = (uint32_t)quant_code(p[0], t.mid5, 31);
  const uint32_t g = (uint32_t)quant_code(p[1], t.mid6, 63);
  const uint32_t b = (uint32_t)quant_code(p[2], t.mid5, 31);
  return r | (b << 8) | (g << 16);
}

// One thread per texel.
__global__ __launch_bounds__(256) void qat_texels_kernel(QatArgs a) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)a.w * a.h) return;
  const int i = (int)(id % a.w), j = (int)(id / a.w);
  const float *p = a.params + ((int64_t)(j >> 2) * a.bw + (i >> 2)) * kQatParams;
  const uint32_t e0 = endpoint_codes(p, a.t), e1 = endpoint_codes(p + 3, a.t);
  const uint32_t w = (uint32_t)quant_code(p[6 + 4 * (j & 3) + (i & 3)], a.t.mid2, 3);
  // numerators over 6 (2^b - 1), as the BC1 decoder forms them; one
  // rounding of the exact quotient (a double quotient of these small
  // integers is never a float32 rounding tie)
  const uint32_t n = 2u * (3u - w) * e0 + 2u * w * e1;
  float *o = a.texels + id * 3;
  o[0] = (float)((double)(n & 255u) / 186.0);
  o[1] = (float)((double)(n >> 16) / 378.0);
  o[2] = (float)((double)((n >> 8) & 255u) / 186.0);
}

// One thread per block: gradients with the quantisation passed through,
//   dL/dE0_c = sum_t (1 - w_t/3) g_tc, dL/dE1_c = sum_t (w_t/3) g_tc,
//   dL/dw_t = sum_c (E1_c - E0_c) g_tc  (values E, w/3 in [0, 1]),
// each times the sigmoid's derivative at its logit.
__global__ __launch_bounds__(256) void qat_backward_kernel(QatArgs a) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)a.bw * a.bh) return;
  const int bx = (int)(id % a.bw), by = (int)(id / a.bw);
  const float *p = a.params + id * kQatParams;
  float *gp = a.texels + id * kQatParams;
  const uint32_t e0 = endpoint_codes(p, a.t), e1 = endpoint_codes(p + 3, a.t);
  const float ev0[3] = {numer_r(e0) * (1.0f / 31.0f), numer_g(e0) * (1.0f / 63.0f), numer_b(e0) * (1.0f / 31.0f)};
  const float ev1[3] = {numer_r(e1) * (1.0f / 31.0f), numer_g(e1) * (1.0f / 63.0f), numer_b(e1) * (1.0f / 31.0f)};
  float g0[3] = {0.f, 0.f, 0.f}, g1[3] = {0.f, 0.f, 0.f};
  for (int t = 0; t < 16; ++t) {
    const int i = 4 * bx + (t & 3), j = 4 * by + (t >> 2);
    const float *g = a.grad + ((int64_t)j * a.w + i) * 3;
    const float wv = (float)quant_code(p[6 + t], a.t.mid2, 3) * (1.0f / 3.0f);
    float ga = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      g0[c] = fmaf(1.0f - wv, g[c], g0[c]);
      g1[c] = fmaf(wv, g[c], g1[c]);
      ga = fmaf(ev1[c] - ev0[c], g[c], ga);
    }
    const float s = sigmoidf(p[6 + t]);
    gp[6 + t] = s * (1.0f - s) * ga;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float s0 = sigmoidf(p[c]), s1 = sigmoidf(p[3 + c]);
    gp[c] = s0 * (1.0f - s0) * g0[c];
    gp[3 + c] = s1 * (1.0f - s1) * g1[c];
  }
}

// One thread per block: BC1 words whose four-colour decode gives the
// quantised texels. The palette of (c0, c1) in four-colour mode (c0 > c1)
// is indexed 0: E0, 1: E1, 2: (2 E0 + E1) / 3, 3: (E0 + 2 E1) / 3, so weight
// w maps to index {0, 2, 3, 1}[w]; with c0 < c1 the endpoints swap and w
// becomes 3 - w; equal endpoints make every weight give E0 (index 0).
__global__ __launch_bounds__(256) void qat_export_kernel(QatArgs a) {
  const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= (int64_t)a.bw * a.bh) return;
  const float *p = a.params + id * kQatParams;
  uint32_t c[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const uint32_t r = (uint32_t)quant_code(p[3 * e], a.t.mid5, 31);
    const uint32_t g = (uint32_t)quant_code(p[3 * e + 1], a.t.mid6, 63);
    const uint32_t b = (uint32_t)quant_code(p[3 * e + 2], a.t.mid5, 31);
    c[e] = (r << 11) | (g << 5) | b;
  }
  const bool swap = c[0] < c[1];
  uint32_t idx = 0;
  if (c[0] != c[1]) {
    for (int t = 0; t < 16; ++t) {
      uint32_t w = (uint32_t)quant_code(p[6 + t], a.t.mid2, 3);
      if (swap) w = 3u - w;
      idx |= ((0x78u >> (2u * w)) & 3u) << (2u * t);  // {0, 2, 3, 1}[w]
    }
  }
  const uint32_t lo = swap ? (c[1] | (c[0] << 16)) : (c[0] | (c[1] << 16));
  a.blocks[id] = make_uint2(lo, idx);
}

QatArgs qat_args(const float *params, int w, int h) {
  QatArgs a{};
  a.params = params;
  a.w = w;
  a.h = h;
  a.bw = w / 4;
  a.bh = h / 4;
  a.t = qat_tables();
  return a;
}

}  // namespace

QatTables qat_tables() {
  static QatTables t = [] {
    QatTables q{};
    auto fill = [](float *mid, int M) {
      for (int k = 0; k < M; ++k) {
        const double p = (k + 0.5) / M;
        mid[k] = (float)std::log(p / (1.0 - p));
      }
    };
    fill(q.mid5, 31);
    fill(q.mid6, 63);
    fill(q.mid2, 3);
    return q;
  }();
  return t;
}

hipError_t launch_qat_texels(const float *params, int w, int h, float *texels, hipStream_t st) {
  QatArgs a = qat_args(params, w, h);
  a.texels = texels;
  const int64_t n = (int64_t)w * h;
  hipLaunchKernelGGL(qat_texels_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_qat_backward(const float *params, int w, int h, const float *grad_texels, float *grad_params,
                               hipStream_t st) {
  QatArgs a = qat_args(params, w, h);
  a.grad = grad_texels;
  a.texels = grad_params;
  const int64_t n = (int64_t)a.bw * a.bh;
  hipLaunchKernelGGL(qat_backward_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_qat_export(const float *params, int w, int h, uint64_t *blocks, hipStream_t st) {
  QatArgs a = qat_args(params, w, h);
  a.blocks = reinterpret_cast<uint2 *>(blocks);
  const int64_t n = (int64_t)a.bw * a.bh;
  hipLaunchKernelGGL(qat_export_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace ntc
